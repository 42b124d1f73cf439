"""GPU parity of the doubly augmented system (kkt_system = 1): PCG with the
Jacobi preconditioner on eq. (2x2_augmented) of the paper (Section 4), its x
part taken as the search direction.

* Newton step: for the condensed system (H + Sigma_x + A^T diag(sigA) A) dx =
  rhs the library poses the doubly augmented one with one side per row
  (B = -A, D = 1/sigA, r_2 = 0), whose x part is that dx.  PCG stops on the
  augmented residual; the condensed residual of dx is then r_x - B^T D^-1 r_l,
  at most (1 + ||A^T diag(sigA)||) times the PCG tolerance (times ||rhs||).
* Whole solves against the oracle at the bars of tests/bars.py.
"""
import numpy as np
import pytest

import oracle
import qpsynth
from bars import check_solve_vs_oracle
from paper_2405_03584_amd import qpgpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["cfg1", "band", "tiny12"])
@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_augmented_newton_step_matches_cholesky(which, prec):
    prob = {"cfg1": lambda: qpsynth.config1(0), "band": lambda: qpsynth.config2(scale=0.02),
            "tiny12": lambda: qpsynth.tiny(12)}[which]()
    it = qpsynth.random_iterate(prob, 11)
    tol = 1e-10
    s = qpgpu.qp_default_settings(kkt_system=1, precision=prec, pcg_tol=tol, pcg_max_iter=50000)
    h = qpgpu.qp_create_from_problem(prob, settings=s)
    st, dx, info = qpgpu.qp_newton_step(h, it["sigma_x"], it["sigma_A"], it["rhs"])
    print(f"augmented newton step on {prob.name} {prec}: pcg {info['pcg_iters']}", flush=True)
    assert st == qpgpu.QP_OK, info
    K = oracle.condensed_operator_dense(prob, it["sigma_x"], it["sigma_A"])
    ref = oracle.newton_solve_dense(K, it["rhs"])
    res = np.linalg.norm(K @ dx - it["rhs"]) / np.linalg.norm(it["rhs"])
    amp = 1.0 + np.linalg.norm(prob.A.toarray().T * it["sigma_A"][None, :], 2)
    assert res <= 10 * amp * tol, (res, amp)
    cond = np.linalg.cond(K)
    assert np.linalg.norm(dx - ref) <= 10 * amp * tol * cond * np.linalg.norm(ref)
    # the same step through the condensed system
    hc = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(precision=prec, pcg_tol=tol,
                                                                                 pcg_max_iter=50000))
    stc, dxc, infoc = qpgpu.qp_newton_step(hc, it["sigma_x"], it["sigma_A"], it["rhs"])
    assert stc == qpgpu.QP_OK
    print(f"  condensed: pcg {infoc['pcg_iters']}", flush=True)


@pytest.mark.parametrize("inst", range(5))
def test_augmented_solve_config1(inst):
    prob = qpsynth.config1(inst)
    h = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(kkt_system=1))
    res = qpgpu.qp_solve(h)
    print(f"{prob.name}: ipm {res.info['ipm_iters']} pcg {res.info['pcg_iters']}", flush=True)
    ref = oracle.solve(prob)
    check_solve_vs_oracle(prob, res, ref, "fp64")


@pytest.mark.parametrize("inst", [0, 3, 12, 21, 33, 42])
def test_augmented_solve_tiny(inst):
    """Every kind of side (two-sided, one-sided, absent) on rows of A: absent
    sides keep their zero row of B."""
    prob = qpsynth.tiny(inst)
    h = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(kkt_system=1))
    res = qpgpu.qp_solve(h)
    ref = oracle.solve(prob)
    check_solve_vs_oracle(prob, res, ref, "fp64")


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_augmented_solve_band(prec):
    """Line format, rows of A with an upper side only."""
    prob = qpsynth.config2(scale=0.02)
    h = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(kkt_system=1, precision=prec))
    res = qpgpu.qp_solve(h)
    print(f"{prob.name} {prec}: ipm {res.info['ipm_iters']} pcg {res.info['pcg_iters']} "
          f"format {res.info['spmv_format']}", flush=True)
    assert res.info["spmv_format"] == 1
    ref = oracle.solve(prob)
    check_solve_vs_oracle(prob, res, ref, prec)


def test_augmented_graph_replays_match_direct_launches():
    prob = qpsynth.config1(2)
    a = qpgpu.qp_solve(qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(kkt_system=1,
                                                                                              graphs=1)))
    b = qpgpu.qp_solve(qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(kkt_system=1,
                                                                                              graphs=0)))
    assert a.status == b.status == qpgpu.QP_OK
    assert np.array_equal(a.x, b.x) and a.info["pcg_iters"] == b.info["pcg_iters"]
