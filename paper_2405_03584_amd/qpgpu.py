"""ctypes binding of libqpgpu.so (include/qpgpu.h), same names as the C ABI.

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  The library must be built (``python -m paper_2405_03584_amd.build``);
loading fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqpgpu.so")

QP_OK, QP_ERR_INVALID, QP_ERR_NOMEM, QP_ERR_DEVICE, QP_ERR_NOT_CONVERGED, QP_ERR_NUMERIC = range(6)
QP_FP64, QP_FP32, QP_BF16 = 0, 1, 2
STATUS_NAMES = {0: "QP_OK", 1: "QP_ERR_INVALID", 2: "QP_ERR_NOMEM", 3: "QP_ERR_DEVICE",
                4: "QP_ERR_NOT_CONVERGED", 5: "QP_ERR_NUMERIC"}
PRECISIONS = {"fp64": QP_FP64, "fp32": QP_FP32, "bf16": QP_BF16}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class qp_csr(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", _lp), ("col_idx", _ip), ("val", _dp)]


class qp_hessian(C.Structure):
    _fields_ = [("gamma", C.c_double), ("p", _dp), ("k", C.c_int32), ("U", _dp), ("w", _dp)]


class qp_range(C.Structure):
    _fields_ = [("lo", _dp), ("hi", _dp)]


class qp_settings(C.Structure):
    _fields_ = [("precision", C.c_int32), ("refine_steps", C.c_int32), ("pcg_tol", C.c_double),
                ("pcg_max_iter", C.c_int32), ("mu0", C.c_double), ("mu_tol", C.c_double),
                ("tau", C.c_double), ("max_ipm_iter", C.c_int32), ("step_mode", C.c_int32),
                ("scale_objective", C.c_int32), ("schedule", C.c_int32), ("timing", C.c_int32),
                ("log_level", C.c_int32), ("precond", C.c_int32), ("spmv_format", C.c_int32),
                ("refine_tol", C.c_double), ("graphs", C.c_int32), ("kkt_system", C.c_int32),
                ("batch_mode", C.c_int32)]


class qp_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("ipm_iters", C.c_int32), ("pcg_iters", C.c_int64),
                ("pcg_solves", C.c_int32), ("pcg_capped", C.c_int32), ("mu", C.c_double),
                ("rnorm", C.c_double), ("zeta", C.c_double), ("objective", C.c_double),
                ("pcg_relres", C.c_double), ("t_solve_ms", C.c_double), ("t_pcg_ms", C.c_double),
                ("t_spmv_fwd_ms", C.c_double), ("t_spmv_bwd_ms", C.c_double),
                ("n_spmv_fwd", C.c_int64), ("n_spmv_bwd", C.c_int64), ("spmv_format", C.c_int32),
                ("prec_fallbacks", C.c_int32), ("eps_d", C.c_double), ("eps_p", C.c_double),
                ("eps_c", C.c_double), ("gap", C.c_double), ("prec_tier", C.c_int32),
                ("spmv_schedule", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = ["qp_default_settings", "qp_create", "qp_create_device", "qp_solve", "qp_solve_from", "qp_update_hessian",
           "qp_newton_step", "qp_operator_apply", "qp_operator_apply_noalloc", "qp_solve_batch", "qp_last_error",
           "qp_destroy", "qp_sizes"]

_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libqpgpu.so and declare its signatures.  Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libqpgpu.so not built ({path}); run python -m paper_2405_03584_amd.build")
    lib = C.CDLL(path)
    lib.qp_default_settings.argtypes = [C.POINTER(qp_settings)]
    lib.qp_default_settings.restype = None
    lib.qp_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(qp_hessian), C.POINTER(qp_csr), _dp,
                              C.POINTER(qp_csr), C.POINTER(qp_range), C.POINTER(qp_range),
                              C.POINTER(qp_settings), C.c_void_p]
    lib.qp_create.restype = C.c_int
    lib.qp_create_device.argtypes = lib.qp_create.argtypes
    lib.qp_create_device.restype = C.c_int
    lib.qp_solve.argtypes = [C.c_void_p, _dp, _dp, _dp, C.POINTER(qp_info)]
    lib.qp_solve.restype = C.c_int
    lib.qp_solve_from.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.POINTER(qp_info)]
    lib.qp_solve_from.restype = C.c_int
    lib.qp_update_hessian.argtypes = [C.c_void_p, C.POINTER(qp_hessian)]
    lib.qp_update_hessian.restype = C.c_int
    lib.qp_newton_step.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.POINTER(qp_info)]
    lib.qp_newton_step.restype = C.c_int
    lib.qp_operator_apply.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_int32, C.c_int32,
                                      C.POINTER(qp_info)]
    lib.qp_operator_apply.restype = C.c_int
    lib.qp_operator_apply_noalloc.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_int32, C.c_void_p]
    lib.qp_operator_apply_noalloc.restype = C.c_int
    lib.qp_solve_batch.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(_dp), C.POINTER(qp_info)]
    lib.qp_solve_batch.restype = C.c_int
    lib.qp_last_error.argtypes = [C.c_void_p]
    lib.qp_last_error.restype = C.c_char_p
    lib.qp_destroy.argtypes = [C.c_void_p]
    lib.qp_destroy.restype = None
    lib.qp_sizes.argtypes = [C.c_void_p, _ip, _ip, _ip, _lp, _lp]
    lib.qp_sizes.restype = None
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray], t=_dp):
    return None if a is None else a.ctypes.data_as(t)


class QPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def qp_default_settings(**overrides) -> qp_settings:
    s = qp_settings()
    load_library().qp_default_settings(C.byref(s))
    for k, v in overrides.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        setattr(s, k, v)
    return s


def _csr_struct(M, keep: list) -> qp_csr:
    indptr = np.ascontiguousarray(M.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(M.indices, dtype=np.int32)
    data = _f64(M.data)
    keep += [indptr, indices, data]
    return qp_csr(int(M.shape[0]), int(M.shape[1]), int(data.shape[0]),
                  _ptr(indptr, _lp), _ptr(indices, _ip), _ptr(data))


class QPHandle:
    """Owns one qp_handle.  Arrays are copied to the device by qp_create."""

    def __init__(self, handle: C.c_void_p, n: int, m: int):
        self._h = handle
        self.n, self.m = n, m

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None):
            load_library().qp_destroy(self._h)
            self._h = None

    def last_error(self) -> str:
        return load_library().qp_last_error(self._h).decode()


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def qp_create(gamma: float, p, J, W, A=None, A_lo=None, A_hi=None, x_lo=None, x_hi=None,
              U=None, w=None, settings: Optional[qp_settings] = None, stream=None) -> QPHandle:
    """Create a handle (qp_create).  J, A: scipy CSR matrices with sorted
    indices; bounds as arrays with +-inf for absent sides; stream: a torch
    stream (its HIP stream is used) or None for a library-owned stream."""
    lib = load_library()
    keep: list = []
    p = _f64(p)
    n = p.shape[0]
    k = 0 if U is None else int(np.asarray(U).shape[1])
    Uf = None if U is None else np.asfortranarray(U, dtype=np.float64).ravel(order="F")
    wf = None if w is None else _f64(w)
    keep += [p, Uf, wf]
    H = qp_hessian(float(gamma), _ptr(p), k, _ptr(Uf), _ptr(wf))
    Js = _csr_struct(J, keep)
    Wf = _f64(W)
    keep.append(Wf)
    As = None
    b = None
    m = 0
    if A is not None and A.shape[0] > 0:
        As = _csr_struct(A, keep)
        m = int(A.shape[0])
        lo = None if A_lo is None else _f64(A_lo)
        hi = None if A_hi is None else _f64(A_hi)
        keep += [lo, hi]
        b = qp_range(_ptr(lo), _ptr(hi))
    xl = None if x_lo is None else _f64(x_lo)
    xh = None if x_hi is None else _f64(x_hi)
    keep += [xl, xh]
    bnd = qp_range(_ptr(xl), _ptr(xh))
    h = C.c_void_p()
    st = lib.qp_create(C.byref(h), C.byref(H), C.byref(Js), _ptr(Wf),
                       C.byref(As) if As is not None else None,
                       C.byref(b) if b is not None else None, C.byref(bnd),
                       C.byref(settings) if settings is not None else None, _stream_handle(stream))
    if st != QP_OK:
        raise QPError(st, lib.qp_last_error(None).decode())
    return QPHandle(h, n, m)


def hip_runtimes_mapped() -> list:
    """Paths of the HIP runtime libraries (libamdhip64) mapped into this
    process.  Device pointers are shared between the library and a caller
    only when there is exactly one."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 6 and "libamdhip64" in parts[-1]:
                    paths.add(os.path.realpath(parts[-1]))
    except OSError:
        pass
    return sorted(paths)


_DEV_DTYPES = {"f64": ("torch.float64", "float64"), "i64": ("torch.int64", "int64"),
               "i32": ("torch.int32", "int32")}


def _dev_ptr(a, kind: str, count: int, name: str):
    """Device address of a contiguous device array with `count` entries of
    `kind`: any object with data_ptr(), numel(), dtype and is_contiguous()
    (a torch tensor on the GPU, or a buffer of the same runtime)."""
    if a is None:
        return None
    if str(a.dtype) not in _DEV_DTYPES[kind]:
        raise TypeError(f"{name}: dtype {a.dtype}, expected {_DEV_DTYPES[kind][1]}")
    if int(a.numel()) != count:
        raise ValueError(f"{name}: {int(a.numel())} entries, expected {count}")
    if not a.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    if hasattr(a, "is_cuda") and not a.is_cuda:
        raise ValueError(f"{name}: not in device memory")
    return C.cast(C.c_void_p(int(a.data_ptr())), _dp if kind == "f64" else (_lp if kind == "i64" else _ip))


def qp_create_device(gamma: float, p, J, W, A=None, A_lo=None, A_hi=None, x_lo=None, x_hi=None,
                     U=None, w=None, settings: Optional[qp_settings] = None, stream=None) -> QPHandle:
    """qp_create_device: the problem's arrays already in device memory.
    J and A are (indptr int64, indices int32, data float64, (rows, cols))
    tuples of device arrays; p, W, bounds, U (n*k, column-major, flat) and w
    are float64 device arrays.  The library and the arrays' allocator must
    share one HIP runtime: with torch, import torch before this module loads
    the library (checked here)."""
    lib = load_library()
    rt = hip_runtimes_mapped()
    if len(rt) > 1:
        raise RuntimeError("two HIP runtimes in this process (" + ", ".join(rt) + "): device pointers of one "
                           "are not valid in the other; load the library after the allocating framework")
    Jp, Ji, Jd, (nJ, n) = J
    nnzJ = int(Jd.numel())
    k = 0 if U is None else int(U.numel()) // n
    H = qp_hessian(float(gamma), _dev_ptr(p, "f64", n, "p"), k, _dev_ptr(U, "f64", n * k, "U") if k else None,
                   _dev_ptr(w, "f64", k, "w") if k else None)
    Js = qp_csr(int(nJ), int(n), nnzJ, _dev_ptr(Jp, "i64", nJ + 1, "J.indptr"),
                _dev_ptr(Ji, "i32", nnzJ, "J.indices"), _dev_ptr(Jd, "f64", nnzJ, "J.data"))
    As = b = None
    m = 0
    if A is not None:
        Ap, Ai, Ad, (m, nA) = A
        if nA != n:
            raise ValueError("A must have n columns")
        nnzA = int(Ad.numel())
        As = qp_csr(int(m), int(n), nnzA, _dev_ptr(Ap, "i64", m + 1, "A.indptr"),
                    _dev_ptr(Ai, "i32", nnzA, "A.indices"), _dev_ptr(Ad, "f64", nnzA, "A.data"))
        b = qp_range(_dev_ptr(A_lo, "f64", m, "A_lo"), _dev_ptr(A_hi, "f64", m, "A_hi"))
    bnd = qp_range(_dev_ptr(x_lo, "f64", n, "x_lo"), _dev_ptr(x_hi, "f64", n, "x_hi"))
    h = C.c_void_p()
    st = lib.qp_create_device(C.byref(h), C.byref(H), C.byref(Js), _dev_ptr(W, "f64", nJ, "W"),
                              C.byref(As) if As is not None else None,
                              C.byref(b) if b is not None else None, C.byref(bnd),
                              C.byref(settings) if settings is not None else None, _stream_handle(stream))
    if st != QP_OK:
        raise QPError(st, lib.qp_last_error(None).decode())
    return QPHandle(h, int(n), int(m))


def qp_create_from_problem(prob, settings: Optional[qp_settings] = None, stream=None) -> QPHandle:
    """qp_create for an object with the fields of qpsynth.QPProblem."""
    return qp_create(prob.gamma, prob.p, prob.J, prob.W, prob.A, prob.A_lo, prob.A_hi,
                     prob.x_lo, prob.x_hi, prob.U, prob.w, settings, stream)


@dataclass
class SolveResult:
    status: int
    x: np.ndarray
    lam_A: np.ndarray
    lam_x: np.ndarray
    info: dict


def qp_solve(h: QPHandle, raise_on_error: bool = False) -> SolveResult:
    lib = load_library()
    x = np.zeros(h.n)
    lA = np.zeros(max(h.m, 1))
    lx = np.zeros(h.n)
    info = qp_info()
    st = lib.qp_solve(h._h, _ptr(x), _ptr(lA), _ptr(lx), C.byref(info))
    if raise_on_error and st not in (QP_OK,):
        raise QPError(st, h.last_error())
    return SolveResult(st, x, lA[:h.m], lx, info.as_dict())


def qp_solve_from(h: QPHandle, x0, raise_on_error: bool = False) -> SolveResult:
    """qp_solve started at the primal point x0 (None = the default start)."""
    lib = load_library()
    x0f = None if x0 is None else _f64(x0)
    if x0f is not None and x0f.shape != (h.n,):
        raise ValueError(f"x0 must have shape ({h.n},)")
    x = np.zeros(h.n)
    lA = np.zeros(max(h.m, 1))
    lx = np.zeros(h.n)
    info = qp_info()
    st = lib.qp_solve_from(h._h, _ptr(x0f), _ptr(x), _ptr(lA), _ptr(lx), C.byref(info))
    if raise_on_error and st not in (QP_OK,):
        raise QPError(st, h.last_error())
    return SolveResult(st, x, lA[:h.m], lx, info.as_dict())


def qp_update_hessian(h: QPHandle, gamma: float, p, U=None, w=None) -> None:
    """Replace the objective (gamma, p, U, w) of a handle (qp_update_hessian)."""
    lib = load_library()
    p = _f64(p)
    k = 0 if U is None else int(np.asarray(U).shape[1])
    Uf = None if U is None else np.asfortranarray(U, dtype=np.float64).ravel(order="F")
    wf = None if w is None else _f64(w)
    if p.shape != (h.n,) or (k > 0 and (np.asarray(U).shape[0] != h.n or wf is None or wf.shape != (k,))):
        raise ValueError("p must have n entries, U shape (n, k) and w k entries")
    H = qp_hessian(float(gamma), _ptr(p), k, _ptr(Uf), _ptr(wf))
    st = lib.qp_update_hessian(h._h, C.byref(H))
    if st != QP_OK:
        raise QPError(st, h.last_error())


def qp_solve_batch(handles, raise_on_error: bool = False):
    """Solve several handles together (qp_solve_batch).  Returns (status,
    list of x arrays, list of info dicts)."""
    lib = load_library()
    count = len(handles)
    hs = (C.c_void_p * count)(*[h._h for h in handles])
    xs_np = [np.zeros(h.n) for h in handles]
    xs = (_dp * count)(*[_ptr(x) for x in xs_np])
    infos = (qp_info * count)()
    st = lib.qp_solve_batch(hs, count, xs, infos)
    if raise_on_error and st != QP_OK:
        raise QPError(st, lib.qp_last_error(None).decode())
    return st, xs_np, [infos[i].as_dict() for i in range(count)]


def qp_newton_step(h: QPHandle, sigma_x, sigma_A, rhs):
    lib = load_library()
    sx = _f64(sigma_x)
    sa = None if sigma_A is None else _f64(sigma_A)
    r = _f64(rhs)
    dx = np.zeros(h.n)
    info = qp_info()
    st = lib.qp_newton_step(h._h, _ptr(sx), _ptr(sa), _ptr(r), _ptr(dx), C.byref(info))
    return st, dx, info.as_dict()


def qp_operator_apply(h: QPHandle, sigma_x, sigma_A, v, precision=QP_FP64, reps: int = 1):
    lib = load_library()
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    sx = _f64(sigma_x)
    sa = None if sigma_A is None else _f64(sigma_A)
    vv = _f64(v)
    y = np.zeros(h.n)
    info = qp_info()
    st = lib.qp_operator_apply(h._h, _ptr(sx), _ptr(sa), _ptr(vv), _ptr(y), int(precision), int(reps),
                               C.byref(info))
    if st != QP_OK:
        raise QPError(st, h.last_error())
    return y, info.as_dict()


def qp_operator_apply_noalloc(h: QPHandle, sigma_x, sigma_A, v, y, precision=QP_FP64, stream=None) -> int:
    """qp_operator_apply_noalloc: y = K v with every vector in device memory
    (float64 device arrays: torch tensors or buffers of the same HIP
    runtime), enqueued on `stream` (None: the handle's stream) without any
    allocation.  Returns the status; the product is complete once the stream
    has reached it."""
    lib = load_library()
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    sx = _dev_ptr(sigma_x, "f64", h.n, "sigma_x")
    sa = _dev_ptr(sigma_A, "f64", h.m, "sigma_A") if h.m > 0 else None
    vv = _dev_ptr(v, "f64", h.n, "v")
    yy = _dev_ptr(y, "f64", h.n, "y")
    return lib.qp_operator_apply_noalloc(h._h, sx, sa, vv, yy, int(precision), _stream_handle(stream))


def qp_sizes(h: QPHandle):
    lib = load_library()
    n, m, nJ = C.c_int32(), C.c_int32(), C.c_int32()
    nnzJ, nnzA = C.c_int64(), C.c_int64()
    lib.qp_sizes(h._h, C.byref(n), C.byref(m), C.byref(nJ), C.byref(nnzJ), C.byref(nnzA))
    return n.value, m.value, nJ.value, nnzJ.value, nnzA.value
