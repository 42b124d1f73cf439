"""The C ABI library loads, exports every declared symbol, and rejects bad
input before any GPU call (these run without a GPU)."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import qpsynth
from paper_2405_03584_amd import qpgpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "qpgpu.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qp_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = qpgpu.load_library()
    names = declared_functions()
    assert "qp_create" in names and "qp_solve" in names and "qp_newton_step" in names
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(qpgpu.EXPORTS) >= set(names)


def test_default_settings():
    s = qpgpu.qp_default_settings()
    assert s.pcg_tol == 1e-8 and s.mu_tol == 1e-10 and s.tau == 0.995
    assert s.precision == qpgpu.QP_FP64 and s.refine_steps == 6 and s.max_ipm_iter == 200
    assert s.refine_tol == 1e-3 and s.graphs == 1


def _expect_invalid(**kw):
    p = qpsynth.config1(0)
    args = dict(gamma=p.gamma, p=p.p, J=p.J, W=p.W, A=p.A, A_lo=p.A_lo, A_hi=p.A_hi,
                x_lo=p.x_lo, x_hi=p.x_hi)
    args.update(kw)
    with pytest.raises(qpgpu.QPError) as e:
        qpgpu.qp_create(**args)
    assert e.value.status == qpgpu.QP_ERR_INVALID, str(e.value)
    return str(e.value)


def test_invalid_inputs_rejected_before_device():
    p = qpsynth.config1(0)
    W = p.W.copy(); W[5] = -1.0
    assert "W" in _expect_invalid(W=W)
    lo = p.x_lo.copy(); lo[3] = 20.0
    assert "lo > hi" in _expect_invalid(x_lo=lo)
    assert "gamma" in _expect_invalid(gamma=-1.0)
    pp = p.p.copy(); pp[0] = np.nan
    assert "p" in _expect_invalid(p=pp)
    J = p.J.copy(); J.data = J.data.copy(); J.data[7] = np.inf
    assert "non-finite" in _expect_invalid(J=J)
    J2 = p.J.copy(); J2.indices = J2.indices.copy()
    J2.indices[0], J2.indices[1] = J2.indices[1], J2.indices[0]
    assert "increasing" in _expect_invalid(J=J2)
    J3 = p.J.copy(); J3.indices = J3.indices.copy(); J3.indices[-1] = 10_000
    assert "out of range" in _expect_invalid(J=J3)
    A = sp.csr_matrix(np.ones((3, 7)))
    assert "cols" in _expect_invalid(A=A, A_lo=np.zeros(3), A_hi=np.ones(3))
    s = qpgpu.qp_default_settings(tau=1.5)
    assert "tau" in _expect_invalid(settings=s)
    s = qpgpu.qp_default_settings(schedule=7)
    assert "schedule" in _expect_invalid(settings=s)
    s = qpgpu.qp_default_settings(refine_tol=1e-9)   # below pcg_tol
    assert "refine_tol" in _expect_invalid(settings=s)
    s = qpgpu.qp_default_settings(graphs=2)
    assert "graphs" in _expect_invalid(settings=s)


def test_no_gpu_gives_device_error_not_crash():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    p = qpsynth.config1(0)
    with pytest.raises(qpgpu.QPError) as e:
        qpgpu.qp_create_from_problem(p)
    assert e.value.status == qpgpu.QP_ERR_DEVICE


def test_sequence_entry_points_reject_null_handle():
    """qp_update_hessian / qp_solve_from return QP_ERR_INVALID for a NULL
    handle without touching a device."""
    import ctypes as C
    lib = qpgpu.load_library()
    p = np.zeros(4)
    H = qpgpu.qp_hessian(1e-3, p.ctypes.data_as(C.POINTER(C.c_double)), 0, None, None)
    assert lib.qp_update_hessian(None, C.byref(H)) == qpgpu.QP_ERR_INVALID
    x = np.zeros(4)
    assert lib.qp_solve_from(None, None, x.ctypes.data_as(C.POINTER(C.c_double)), None, None,
                             None) == qpgpu.QP_ERR_INVALID


def test_sqp_sequence_shares_constraints_and_grows_rank():
    base = qpsynth.config1(0)
    seq = qpsynth.sqp_sequence(base, 4)
    assert [q.k for q in seq] == [0, 2, 4, 6]
    for t, q in enumerate(seq):
        assert q.J is base.J and q.A is base.A and q.W is base.W
        if t >= 2:   # earlier columns are kept
            np.testing.assert_array_equal(q.U[:, :2 * (t - 1)], seq[t - 1].U)
        if q.k:
            assert np.all(q.w > 0) and q.U.flags.f_contiguous
    again = qpsynth.sqp_sequence(base, 4)
    np.testing.assert_array_equal(again[3].p, seq[3].p)


def test_noalloc_scratch_symbol_is_registrable():
    """The static scratch array of qp_operator_apply_noalloc must reach the
    device code object as a global symbol: the HIP runtime registers every
    __device__ variable at load time and cannot find a local one (the whole
    library would then fail to load on a GPU)."""
    import subprocess
    import tempfile
    llvm = "/opt/rocm/llvm/bin"
    tools = [os.path.join(llvm, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not all(os.path.exists(t) for t in tools):
        pytest.skip("ROCm LLVM tools not present")
    lib = qpgpu.LIB_PATH
    with tempfile.TemporaryDirectory() as d:
        fat, co = os.path.join(d, "lib.fat"), os.path.join(d, "lib.co")
        subprocess.run([tools[0], f"--dump-section=.hip_fatbin={fat}", lib], check=True)
        subprocess.run([tools[1], "--unbundle", "--type=o", f"--input={fat}",
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"], check=True)
        syms = subprocess.run([tools[2], "-s", co], check=True, capture_output=True, text=True).stdout
    rows = [ln.split() for ln in syms.splitlines() if ln.strip().endswith("scratch") and "uses_flat" not in ln]
    assert rows, "scratch array missing from the device code object"
    for r in rows:
        assert r[3] == "OBJECT" and r[4] == "GLOBAL", r
        assert int(r[2]) == 32 * 1024 * 1024, r
