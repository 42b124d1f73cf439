"""qp_operator_apply_noalloc: the operator product with every vector in
device memory and its intermediates in the library's static scratch array
(no allocation).  Checked through the C ABI against qp_operator_apply (same
kernels: identical bits) and against the oracle's condensed operator (the
operator bars of the parity tests), on two calls in a row on one GPU, the
second with a smaller problem than the first, so the second reads nothing the
first left in the shared scratch; and the size limit is enforced."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import qpsynth
from devarray import DeviceArray, runtime
from paper_2405_03584_amd import qpgpu

pytestmark = pytest.mark.gpu

_D2H = 2   # hipMemcpyDeviceToHost


def _abs_op(prob, sigma_x, sigma_A):
    J = abs(prob.J).toarray()
    K = J.T @ (prob.W[:, None] * J) + prob.gamma * np.eye(prob.n)
    K[np.diag_indices(prob.n)] += sigma_x
    if prob.m:
        Ad = abs(prob.A).toarray()
        K += (Ad * sigma_A[:, None]).T @ Ad
    return K


def _noalloc(h, prob, it, prec):
    """One no-alloc product on the handle's stream; returns y on the host."""
    rt = runtime()
    sx = DeviceArray(it["sigma_x"])
    sa = DeviceArray(it["sigma_A"]) if prob.m else None
    v = DeviceArray(it["v"])
    y = DeviceArray(np.full(prob.n, np.nan))
    st = qpgpu.qp_operator_apply_noalloc(h, sx, sa, v, y, precision=prec)
    assert st == qpgpu.QP_OK, h.last_error()
    assert rt.hipDeviceSynchronize() == 0
    out = np.empty(prob.n)
    assert rt.hipMemcpy(C.c_void_p(out.ctypes.data), C.c_void_p(y.data_ptr()), C.c_size_t(out.nbytes), _D2H) == 0
    return out


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_noalloc_matches_operator_apply_twice_second_smaller(prec):
    # first a line-format band QP, then a smaller CSR QP (n = 200)
    cases = [qpsynth.config2(scale=0.05), qpsynth.config1(3)]
    assert cases[1].n < cases[0].n
    for prob in cases:
        print(f"noalloc {prec} on {prob.name} n={prob.n} m={prob.m}", flush=True)
        it = qpsynth.random_iterate(prob, 11)
        sA = it["sigma_A"] if prob.m else None
        h = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(precision=prec))
        ref_lib, _ = qpgpu.qp_operator_apply(h, it["sigma_x"], sA, it["v"], precision=prec)
        y = _noalloc(h, prob, it, prec)
        assert np.array_equal(y, ref_lib)
        K = oracle.condensed_operator_dense(prob, it["sigma_x"], sA)
        ref = K @ it["v"]
        bound = _abs_op(prob, it["sigma_x"], sA) @ np.abs(it["v"])
        if prec == "fp64":
            c = 1e-12
        else:
            Lj = np.diff(prob.J.indptr).max()
            Lt = np.diff(prob.J.tocsc().indptr).max()
            c = 2 * 2.0 ** -8 + (Lj + Lt + 2) * 2.0 ** -24
        assert np.all(np.abs(y - ref) <= c * bound + 1e-300), float((np.abs(y - ref) / bound).max())
        h.close()


def test_noalloc_rejects_what_it_cannot_serve():
    # a low-precision copy that is not resident
    prob = qpsynth.config1(0)
    h = qpgpu.qp_create_from_problem(prob)
    it = qpsynth.random_iterate(prob, 3)
    sx, sa, v, y = (DeviceArray(it["sigma_x"]), DeviceArray(it["sigma_A"]), DeviceArray(it["v"]),
                    DeviceArray(np.zeros(prob.n)))
    assert qpgpu.qp_operator_apply_noalloc(h, sx, sa, v, y, precision="fp32") == qpgpu.QP_ERR_INVALID
    assert "resident" in h.last_error()
    h.close()
    # more J rows than the 32 MiB scratch holds (CSR: one double per row)
    nJ, n = 4_300_000, 8
    J = sp.csr_matrix((np.ones(nJ), (np.arange(nJ), np.arange(nJ) % n)), shape=(nJ, n))
    J.sort_indices()
    print("noalloc size limit: CSR J with 4.3M rows", flush=True)
    hb = qpgpu.qp_create(1e-3, np.zeros(n), J, np.ones(nJ), x_lo=np.zeros(n), x_hi=np.ones(n),
                         settings=qpgpu.qp_default_settings(spmv_format=1))
    sx, v, y = DeviceArray(np.zeros(n)), DeviceArray(np.ones(n)), DeviceArray(np.zeros(n))
    assert qpgpu.qp_operator_apply_noalloc(hb, sx, None, v, y) == qpgpu.QP_ERR_INVALID
    assert "too large" in hb.last_error()
    hb.close()
