"""Device buffers for the GPU tests, allocated through the HIP runtime the
library itself loaded (ctypes), so their pointers are valid for the library.
They expose what qpgpu.qp_create_device reads from an array: data_ptr(),
numel(), dtype, is_contiguous(), is_cuda."""
import ctypes as C

import numpy as np

from paper_2405_03584_amd import qpgpu

_H2D = 1   # hipMemcpyHostToDevice


def runtime():
    qpgpu.load_library()
    return C.CDLL("libamdhip64.so.7")   # resolves to the runtime already loaded


class DeviceArray:
    def __init__(self, host):
        a = np.ascontiguousarray(host)
        self._rt = runtime()
        self.dtype = str(a.dtype)
        self._n = int(a.size)
        self._p = C.c_void_p()
        assert self._rt.hipMalloc(C.byref(self._p), C.c_size_t(max(a.nbytes, 8))) == 0
        if a.nbytes:
            assert self._rt.hipMemcpy(self._p, C.c_void_p(a.ctypes.data), C.c_size_t(a.nbytes), _H2D) == 0

    is_cuda = True

    def data_ptr(self) -> int:
        return int(self._p.value)

    def numel(self) -> int:
        return self._n

    def is_contiguous(self) -> bool:
        return True

    def free(self):
        if self._p:
            self._rt.hipFree(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        self.free()


def csr_on_device(M):
    return (DeviceArray(np.asarray(M.indptr, dtype=np.int64)), DeviceArray(np.asarray(M.indices, dtype=np.int32)),
            DeviceArray(np.asarray(M.data, dtype=np.float64)), tuple(int(v) for v in M.shape))
