"""Parity bars of the GPU tests against the FP64 oracle, per precision.

* x: ||x - x_oracle||_inf <= 1e-7 (1 + ||x_oracle||_inf) when the PCG
  operator holds J in FP64, and <= 1e-5 (absolute, the mixed-precision
  target) with FP32 or BF16 values.  The FP64 bar is relative to the
  solution's size because the oracle itself pins x only that far at its
  stopping rule (mu_tol = 1e-10): its own minimiser moves by 4.4e-7 on the
  n = 1000 band QP when mu_tol is tightened to 1e-13, and by 4.6e-7 on the
  ragged-lines QP with the BLAS thread count (||x||_inf = 50 on both);
* objective: |f - f_oracle| <= 1e-10 |f_oracle| (FP64) or 1e-6 |f_oracle|
  (FP32, BF16), plus the gap the stopping rule itself allows both solvers:
  at exit every scaled lambda_i s_i is below 2 mu_tol, so the objective of
  either is within 2 m_tot mu_tol zeta of the optimum (original units);
* KKT certificate of the returned point <= 1e-9, computed by the oracle from
  (x, lam_x, lam_A) and by the library on the device (qp_info), the two
  agreeing to 1e-11.
"""
import numpy as np

import oracle

X_BAR = {"fp64": 1e-7, "fp32": 1e-5, "bf16": 1e-5}
OBJ_REL_BAR = {"fp64": 1e-10, "fp32": 1e-6, "bf16": 1e-6}
CERT_BAR = 1e-9
CERT_AGREE = 1e-11


def x_bar(prec, x_ref) -> float:
    """The x bar of the precision for a reference solution x_ref."""
    if prec == "fp64":
        return X_BAR["fp64"] * (1.0 + float(np.abs(x_ref).max(initial=0.0)))
    return X_BAR[prec]


def m_tot(prob) -> int:
    t = int(np.isfinite(prob.x_lo).sum() + np.isfinite(prob.x_hi).sum())
    if prob.A is not None and prob.m > 0:
        t += int(np.isfinite(prob.A_lo).sum() + np.isfinite(prob.A_hi).sum())
    return t


def gap_bound(prob, zeta, mu_tol=1e-10) -> float:
    return 2.0 * m_tot(prob) * mu_tol * zeta


def check_certificate(prob, res):
    """Oracle certificate of the returned point <= CERT_BAR, and the device's
    own certificate (qp_info) equal to it within CERT_AGREE."""
    cert = oracle.kkt_certificate(prob, res.x, res.lam_x, res.lam_A if prob.m else None)
    assert cert.worst() <= CERT_BAR, cert
    info = res.info
    for k in ("eps_d", "eps_p", "eps_c", "gap"):
        assert info[k] <= CERT_BAR, (k, info[k])
        assert abs(info[k] - getattr(cert, k)) <= CERT_AGREE, (k, info[k], getattr(cert, k))
    return cert


def check_solve(prob, res, x_ref, f_ref, zeta, prec="fp64", status_ok=True):
    """The bars above for one solve.  Returns (max |x - x_ref|, certificate)."""
    if status_ok:
        assert res.status == 0, res.info
    dx = float(np.abs(res.x - x_ref).max()) if prob.n else 0.0
    assert dx <= x_bar(prec, x_ref), (prec, dx, x_bar(prec, x_ref))
    dobj = abs(res.info["objective"] - f_ref)
    assert dobj <= OBJ_REL_BAR[prec] * abs(f_ref) + gap_bound(prob, zeta), (prec, dobj, f_ref)
    cert = check_certificate(prob, res)
    return dx, cert


def check_solve_vs_oracle(prob, res, ref, prec="fp64"):
    """check_solve against an oracle.solve result."""
    return check_solve(prob, res, ref.x, ref.objective, ref.zeta, prec)
