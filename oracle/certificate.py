"""KKT optimality certificate and brute-force active-set solver.

TEST INFRASTRUCTURE ONLY (see ``oracle/ipm_dense.py``).

Both work from the QP of eq. (qp) directly and share nothing with the interior
point iteration: the certificate measures how far a point (x, y) is from the
KKT conditions of the QP (eq. (perturbed_KKT) with mu = 0), and the brute-force
solver enumerates active sets, so either can pin a solver's answer.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .ipm_dense import hessian_apply


@dataclass
class Certificate:
    eps_d: float      # scaled stationarity residual
    eps_p: float      # scaled primal infeasibility
    eps_c: float      # largest multiplier * slack product, relative to the objective size
    gap: float        # relative primal-dual objective gap
    sign_ok: bool     # multipliers only on finite sides
    objective: float

    def worst(self) -> float:
        if not self.sign_ok:
            return np.inf
        return max(self.eps_d, self.eps_p, self.eps_c, self.gap)


def kkt_certificate(prob, x: np.ndarray, y_x: np.ndarray, y_A: Optional[np.ndarray]) -> Certificate:
    """Certificate of (x, y) for eq. (qp) with combined multipliers.

    ``y_x[j] = lambda_ux[j] - lambda_lx[j]`` and ``y_A[i] = lambda_uA[i] -
    lambda_lA[i]``: positive where the upper side binds, negative where the
    lower side binds.  Stationarity reads H x + p + y_x + A^T y_A = 0.
    """
    n = prob.n
    Hx = hessian_apply(prob, x)
    f = float(0.5 * x @ Hx + prob.p @ x)
    y_x = np.asarray(y_x, dtype=np.float64)
    lam_ux, lam_lx = np.maximum(y_x, 0.0), np.maximum(-y_x, 0.0)
    rH = Hx + prob.p + y_x
    dscale = [np.abs(Hx).max(initial=0.0), np.abs(prob.p).max(initial=0.0),
              np.abs(y_x).max(initial=0.0)]
    cvals = [np.abs(prob.x_lo[np.isfinite(prob.x_lo)]), np.abs(prob.x_hi[np.isfinite(prob.x_hi)])]
    sign_ok = bool(np.all(lam_lx[~np.isfinite(prob.x_lo)] == 0.0)
                   and np.all(lam_ux[~np.isfinite(prob.x_hi)] == 0.0))
    viol = [np.maximum(prob.x_lo - x, 0.0), np.maximum(x - prob.x_hi, 0.0)]
    with np.errstate(invalid="ignore"):
        comp = [np.where(lam_lx > 0, lam_lx * (x - prob.x_lo), 0.0),
                np.where(lam_ux > 0, lam_ux * (prob.x_hi - x), 0.0)]
    dual_c = float(np.sum(lam_lx[lam_lx > 0] * prob.x_lo[lam_lx > 0])
                   - np.sum(lam_ux[lam_ux > 0] * prob.x_hi[lam_ux > 0]))
    if prob.A is not None and prob.m > 0:
        y_A = np.asarray(y_A, dtype=np.float64)
        lam_uA, lam_lA = np.maximum(y_A, 0.0), np.maximum(-y_A, 0.0)
        Aty = prob.A.T @ y_A
        Ax = prob.A @ x
        rH = rH + Aty
        dscale.append(np.abs(Aty).max(initial=0.0))
        cvals += [np.abs(prob.A_lo[np.isfinite(prob.A_lo)]), np.abs(prob.A_hi[np.isfinite(prob.A_hi)])]
        sign_ok = sign_ok and bool(np.all(lam_lA[~np.isfinite(prob.A_lo)] == 0.0)
                                   and np.all(lam_uA[~np.isfinite(prob.A_hi)] == 0.0))
        viol += [np.maximum(prob.A_lo - Ax, 0.0), np.maximum(Ax - prob.A_hi, 0.0)]
        with np.errstate(invalid="ignore"):
            comp += [np.where(lam_lA > 0, lam_lA * (Ax - prob.A_lo), 0.0),
                     np.where(lam_uA > 0, lam_uA * (prob.A_hi - Ax), 0.0)]
        dual_c += float(np.sum(lam_lA[lam_lA > 0] * prob.A_lo[lam_lA > 0])
                        - np.sum(lam_uA[lam_uA > 0] * prob.A_hi[lam_uA > 0]))
    eps_d = float(np.abs(rH).max(initial=0.0) / (1.0 + max(dscale)))
    cscale = 1.0 + max((float(c.max()) for c in cvals if c.size), default=0.0)
    eps_p = float(max((float(v.max()) for v in viol if v.size), default=0.0) / cscale)
    # multiplier * slack has the units of the objective: measure it, and the
    # gap, against the size of the objective's two terms
    oscale = 1.0 + 0.5 * abs(float(x @ Hx)) + abs(float(prob.p @ x))
    eps_c = float(max((float(np.abs(c).max()) for c in comp if c.size), default=0.0)) / oscale
    # dual objective of the QP: -1/2 x^T H x + c^T lambda
    d = -0.5 * float(x @ Hx) + dual_c
    gap = abs(f - d) / oscale
    return Certificate(eps_d=eps_d, eps_p=eps_p, eps_c=eps_c, gap=gap, sign_ok=sign_ok,
                       objective=f)


@dataclass
class BruteForceResult:
    x: np.ndarray
    y_x: np.ndarray
    y_A: np.ndarray
    objective: float
    candidates: int


def bruteforce_qp(prob, feas_tol: float = 1e-12, max_candidates: int = 2_000_000) -> BruteForceResult:
    """Exact minimiser of a tiny QP by enumerating active sets.

    For every choice of {inactive, lower bound active, upper bound active} per
    variable and per row of A (only finite sides, at most n active), solve the
    equality-constrained QP by its KKT system (least squares when the active
    rows are dependent), keep the primal-feasible points and return the one
    with the least objective.  The QP is strictly convex (H >= gamma I), so the
    minimiser over the true active set's affine hull is the global optimum and
    it is among the feasible candidates.
    """
    H = np.eye(prob.n) * prob.gamma + (prob.J.T @ (prob.W[:, None] * prob.J.toarray()))
    if prob.U is not None and prob.U.shape[1] > 0:
        H = H + (prob.U * prob.w) @ prob.U.T
    n = prob.n
    rows = [np.eye(n)[j] for j in range(n)]
    lo = list(prob.x_lo)
    hi = list(prob.x_hi)
    if prob.A is not None and prob.m > 0:
        Ad = prob.A.toarray()
        rows += [Ad[i] for i in range(prob.m)]
        lo += list(prob.A_lo)
        hi += list(prob.A_hi)
    R = np.array(rows)
    lo, hi = np.array(lo), np.array(hi)
    options = []
    for i in range(len(rows)):
        o = [0]
        if np.isfinite(lo[i]):
            o.append(-1)
        if np.isfinite(hi[i]) and not (np.isfinite(lo[i]) and hi[i] == lo[i]):
            o.append(1)
        options.append(o)
    total = int(np.prod([len(o) for o in options]))
    if total > max_candidates:
        raise ValueError(f"too many active sets ({total})")
    scale = 1.0 + max(np.abs(lo[np.isfinite(lo)]).max(initial=0.0),
                      np.abs(hi[np.isfinite(hi)]).max(initial=0.0))
    best = None
    count = 0
    for choice in itertools.product(*options):
        act = [i for i, c in enumerate(choice) if c != 0]
        if len(act) > n:
            continue
        count += 1
        E = R[act]
        e = np.array([lo[i] if choice[i] < 0 else hi[i] for i in act])
        k = len(act)
        KKT = np.zeros((n + k, n + k))
        KKT[:n, :n] = H
        KKT[:n, n:] = E.T
        KKT[n:, :n] = E
        rhs = np.concatenate([-prob.p, e])
        sol, *_ = np.linalg.lstsq(KKT, rhs, rcond=None)
        if np.linalg.norm(KKT @ sol - rhs) > 1e-9 * (1.0 + np.linalg.norm(rhs)):
            continue
        x = sol[:n]
        v = R @ x
        if np.any(v < lo - feas_tol * scale) or np.any(v > hi + feas_tol * scale):
            continue
        f = 0.5 * x @ H @ x + prob.p @ x
        if best is None or f < best[0] - 1e-14 * (1 + abs(f)):
            # multipliers: H x + p + E^T nu = 0, nu_i = y of that row
            y = np.zeros(len(rows))
            y[act] = sol[n:]
            best = (f, x, y)
    if best is None:
        raise RuntimeError("no feasible active set")
    f, x, y = best
    return BruteForceResult(x=x, y_x=y[:n], y_A=y[n:], objective=float(f), candidates=count)
