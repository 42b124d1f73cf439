"""FP64 dense-Cholesky interior point method: the test oracle.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything under
``oracle/``.  The GPU library never links, imports or calls it.

What it computes (Section 3.1 and Section 4 of the paper):

* the QP of eq. (qp): min 1/2 x^T H x + p^T x  s.t.  l <= A x <= u, with the
  variable bounds kept apart from the rows of A (Section 4, before
  eq. (2x2_reduced)).  Four constraint groups g in {lx, ux, lA, uA}, each
  written G_g x >= c_g with a slack s_g = G_g x - c_g >= 0 and a multiplier
  lambda_g >= 0:

      lx: G = rows of I,   c = l_x        ux: G = rows of -I,  c = -u_x
      lA: G = rows of A,   c = l_A        uA: G = rows of -A,  c = -u_A

  Only rows with a finite bound form a group row.  With G = -A, c = -u this is
  r_u = -A x - s_u + u, the form of eq. (qp_barrier) and of the third block row
  of eq. (newton_system) (eq. (perturbed_KKT) prints the s_u sign flipped).
* residuals of eq. (perturbed_KKT):  r_H = H x + p - sum_g G_g^T lambda_g,
  r_g = G_g x - s_g - c_g,  r_c,g = lambda_g * s_g - mu;
* the Newton system eq. (newton_system), reduced by block elimination to the
  condensed (Schur complement) system

      (H + sum_g G_g^T Sigma_g G_g) dx = -(H x + p) + sum_g G_g^T (mu/s_g - Sigma_g r_g),
      Sigma_g = lambda_g / s_g,

  which is the Schur complement of the doubly augmented system
  eq. (2x2_augmented) with respect to its D block (Q = H + Sigma_x,
  B^T D^{-1} B = A^T Sigma_A A).  Solved here by dense Cholesky;
* Algorithm 1: direction, separate primal and dual step lengths (fraction to
  the boundary), update of x, lambda, s, residuals, and the barrier rule
  "if ||r|| < mu: if mu <= mu_tol return; mu <- mu/10".

Readings where the paper is silent (the same values are the GPU library's
defaults): the objective is divided by zeta = max(1, ||H x0 + p||_inf), the
gradient size at the start point, before iterating (multipliers are scaled
back on return; the minimiser is unchanged), so that mu_tol is measured in
units where the multipliers are of order one; initial point x0 = bound midpoint (or bound +-1, or 0),
s0 = max(G x0 - c, 1), lambda0 = 1, mu0 = s0^T lambda0 / m_tot; fraction to
the boundary tau = 0.995; mu_tol = 1e-10; ||r|| is the infinity norm of the
stacked scaled residuals r_H/(1 + ||p||_inf + ||Hx||_inf),
r_g/(1 + ||c||_inf) and the unscaled r_c.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

GROUPS = ("lx", "ux", "lA", "uA")


@dataclass
class OracleSettings:
    mu0: Optional[float] = None       # None: average complementarity of the start point
    mu_tol: float = 1e-10
    tau: float = 0.995
    max_ipm_iter: int = 200
    step_mode: str = "separate"       # "separate" (Algorithm 1) or "equal"


@dataclass
class OracleResult:
    x: np.ndarray
    s: Dict[str, np.ndarray]
    lam: Dict[str, np.ndarray]
    mu: float
    iters: int
    converged: bool
    objective: float
    history: List[dict] = field(default_factory=list)
    zeta: float = 1.0


# ----------------------------------------------------------------------------
# problem pieces
# ----------------------------------------------------------------------------

def hessian_dense(prob) -> np.ndarray:
    """H = gamma*I + J^T diag(W) J + U diag(w) U^T as a dense array
    (eq. (bfgs_hessian) with a diagonal-plus-least-squares H_0)."""
    n = prob.n
    JtWJ = (prob.J.T @ sp.diags(prob.W) @ prob.J).toarray()
    H = JtWJ
    H[np.diag_indices(n)] += prob.gamma
    if prob.U is not None and prob.U.shape[1] > 0:
        U = np.asarray(prob.U)
        H += (U * prob.w[None, :]) @ U.T
    return H


def objective(prob, x: np.ndarray, H: Optional[np.ndarray] = None) -> float:
    """f(x) = 1/2 x^T H x + p^T x (eq. (qp))."""
    Hx = H @ x if H is not None else hessian_apply(prob, x)
    return float(0.5 * x @ Hx + prob.p @ x)


def hessian_apply(prob, x: np.ndarray) -> np.ndarray:
    """H x from the factors, without forming H (used by the certificate)."""
    y = prob.gamma * x + prob.J.T @ (prob.W * (prob.J @ x))
    if prob.U is not None and prob.U.shape[1] > 0:
        y = y + prob.U @ (prob.w * (prob.U.T @ x))
    return y


@dataclass
class Groups:
    """Row index sets of the four constraint groups and their c_g."""
    idx: Dict[str, np.ndarray]
    c: Dict[str, np.ndarray]
    A: Optional[np.ndarray]           # dense A (m x n) or None

    def G(self, g: str, x: np.ndarray) -> np.ndarray:
        """G_g x."""
        i = self.idx[g]
        if len(i) == 0:
            return np.zeros(0)
        if g == "lx":
            return x[i]
        if g == "ux":
            return -x[i]
        if g == "lA":
            return self.A[i] @ x
        return -(self.A[i] @ x)

    def GT(self, g: str, y: np.ndarray, n: int) -> np.ndarray:
        """G_g^T y as an n-vector."""
        i = self.idx[g]
        out = np.zeros(n)
        if len(i) == 0:
            return out
        if g == "lx":
            np.add.at(out, i, y)
        elif g == "ux":
            np.add.at(out, i, -y)
        elif g == "lA":
            out = self.A[i].T @ y
        else:
            out = -(self.A[i].T @ y)
        return out

    def gram(self, g: str, sigma: np.ndarray, n: int) -> np.ndarray:
        """G_g^T diag(sigma) G_g, dense n x n."""
        i = self.idx[g]
        if g in ("lx", "ux"):
            K = np.zeros((n, n))
            K[i, i] += sigma
            return K
        Ai = self.A[i]
        return (Ai * sigma[:, None]).T @ Ai

    def m_tot(self) -> int:
        return sum(len(self.idx[g]) for g in GROUPS)

    def c_scale(self) -> float:
        vals = [np.abs(self.c[g]) for g in GROUPS if len(self.c[g])]
        return 1.0 + (max(float(v.max()) for v in vals) if vals else 0.0)


def make_groups(prob) -> Groups:
    lx = np.flatnonzero(np.isfinite(prob.x_lo))
    ux = np.flatnonzero(np.isfinite(prob.x_hi))
    if prob.A is not None and prob.m > 0:
        lA = np.flatnonzero(np.isfinite(prob.A_lo))
        uA = np.flatnonzero(np.isfinite(prob.A_hi))
        Ad = prob.A.toarray()
        cA_l, cA_u = prob.A_lo[lA], -prob.A_hi[uA]
    else:
        lA = uA = np.zeros(0, dtype=np.int64)
        Ad = None
        cA_l = cA_u = np.zeros(0)
    return Groups(idx={"lx": lx, "ux": ux, "lA": lA, "uA": uA},
                  c={"lx": prob.x_lo[lx], "ux": -prob.x_hi[ux], "lA": cA_l, "uA": cA_u},
                  A=Ad)


def initial_point(prob, G: Groups):
    """Start point (the paper only asks for positive slacks, Section 3.1)."""
    lo, hi = prob.x_lo, prob.x_hi
    x = np.zeros(prob.n)
    both = np.isfinite(lo) & np.isfinite(hi)
    only_lo = np.isfinite(lo) & ~np.isfinite(hi)
    only_hi = ~np.isfinite(lo) & np.isfinite(hi)
    x[both] = 0.5 * (lo[both] + hi[both])
    x[only_lo] = lo[only_lo] + 1.0
    x[only_hi] = hi[only_hi] - 1.0
    s = {g: np.maximum(G.G(g, x) - G.c[g], 1.0) for g in GROUPS}
    lam = {g: np.ones(len(G.idx[g])) for g in GROUPS}
    return x, s, lam


# ----------------------------------------------------------------------------
# one IPM iteration, step by step
# ----------------------------------------------------------------------------

def residuals(prob, G: Groups, H: np.ndarray, x, s, lam, mu):
    """eq. (perturbed_KKT) for the four groups."""
    n = prob.n
    Hx = H @ x
    rH = Hx + prob.p
    for g in GROUPS:
        rH = rH - G.GT(g, lam[g], n)
    rg = {g: G.G(g, x) - s[g] - G.c[g] for g in GROUPS}
    rc = {g: lam[g] * s[g] - mu for g in GROUPS}
    return Hx, rH, rg, rc


def residual_norm(prob, G: Groups, Hx, rH, rg, rc) -> float:
    """Infinity norm of the stacked scaled residuals (the ||r|| of Algorithm 1)."""
    dscale = 1.0 + max(np.abs(prob.p).max(initial=0.0), np.abs(Hx).max(initial=0.0))
    v = np.abs(rH).max(initial=0.0) / dscale
    cs = G.c_scale()
    for g in GROUPS:
        v = max(v, np.abs(rg[g]).max(initial=0.0) / cs, np.abs(rc[g]).max(initial=0.0))
    return float(v)


def condensed_matrix(prob, G: Groups, H: np.ndarray, sigma: Dict[str, np.ndarray]) -> np.ndarray:
    """K = H + sum_g G_g^T Sigma_g G_g (dense)."""
    K = H.copy()
    for g in GROUPS:
        if len(G.idx[g]):
            K += G.gram(g, sigma[g], prob.n)
    return K


def newton_direction(prob, G: Groups, H, x, s, lam, mu, Hx, rg):
    """Solve eq. (newton_system) through its condensed form (dense Cholesky),
    then recover ds and dlambda for every group."""
    n = prob.n
    sigma = {g: lam[g] / s[g] for g in GROUPS}
    K = condensed_matrix(prob, G, H, sigma)
    rhs = -(Hx + prob.p)
    for g in GROUPS:
        if len(G.idx[g]):
            rhs = rhs + G.GT(g, mu / s[g] - sigma[g] * rg[g], n)
    cf = sla.cho_factor(K, lower=True, check_finite=False)
    dx = sla.cho_solve(cf, rhs, check_finite=False)
    ds = {g: G.G(g, dx) + rg[g] for g in GROUPS}
    dlam = {g: -lam[g] + mu / s[g] - sigma[g] * ds[g] for g in GROUPS}
    return dx, ds, dlam


def max_step(v: Dict[str, np.ndarray], dv: Dict[str, np.ndarray], tau: float) -> float:
    """Largest alpha in (0, 1] with v + alpha*dv staying positive, scaled by tau
    (fraction to the boundary)."""
    a = 1.0
    for g in GROUPS:
        neg = dv[g] < 0
        if np.any(neg):
            a = min(a, tau * float(np.min(-v[g][neg] / dv[g][neg])))
    return a


def objective_scale(prob, H: np.ndarray) -> float:
    """zeta = max(1, ||H x0 + p||_inf) at the start point x0."""
    G = make_groups(prob)
    x0, _, _ = initial_point(prob, G)
    return max(1.0, float(np.abs(H @ x0 + prob.p).max(initial=0.0)))


def solve(prob, settings: Optional[OracleSettings] = None, H: Optional[np.ndarray] = None,
          record: bool = False, progress=None) -> OracleResult:
    """Algorithm 1 with a dense Cholesky Newton solve, on the objective
    divided by zeta (see the module docstring).  ``progress(iter, mu, rnorm)``,
    when given, is called after every iteration (it only reports)."""
    import copy
    st = settings or OracleSettings()
    if H is None:
        H = hessian_dense(prob)
    zeta = objective_scale(prob, H)
    sprob = copy.copy(prob)
    sprob.p = prob.p / zeta
    H = H / zeta
    res = _solve_scaled(sprob, st, H, record, progress)
    res.lam = {g: v * zeta for g, v in res.lam.items()}
    res.objective = res.objective * zeta
    res.zeta = zeta
    return res


def _solve_scaled(prob, st: OracleSettings, H: np.ndarray, record: bool, progress=None) -> OracleResult:
    G = make_groups(prob)
    x, s, lam = initial_point(prob, G)
    m_tot = G.m_tot()
    if st.mu0 is not None:
        mu = st.mu0
    elif m_tot > 0:
        mu = float(sum(s[g] @ lam[g] for g in GROUPS) / m_tot)
    else:
        mu = st.mu_tol
    Hx, rH, rg, rc = residuals(prob, G, H, x, s, lam, mu)
    hist = []
    converged = False
    it = 0
    for it in range(1, st.max_ipm_iter + 1):
        dx, ds, dlam = newton_direction(prob, G, H, x, s, lam, mu, Hx, rg)
        a_x = max_step(s, ds, st.tau)
        a_l = max_step(lam, dlam, st.tau)
        if st.step_mode == "equal":
            a_x = a_l = min(a_x, a_l)
        x = x + a_x * dx
        lam = {g: lam[g] + a_l * dlam[g] for g in GROUPS}
        s = {g: s[g] + a_x * ds[g] for g in GROUPS}
        Hx, rH, rg, rc = residuals(prob, G, H, x, s, lam, mu)
        rn = residual_norm(prob, G, Hx, rH, rg, rc)
        if progress is not None:
            progress(it, mu, rn)
        if record:
            hist.append({"iter": it, "mu": mu, "rnorm": rn, "alpha_x": a_x, "alpha_l": a_l,
                         "min_s": min((s[g].min() for g in GROUPS if len(s[g])), default=np.inf),
                         "min_l": min((lam[g].min() for g in GROUPS if len(lam[g])), default=np.inf)})
        if rn < mu:
            if mu <= st.mu_tol:
                converged = True
                break
            mu = mu / 10.0
    return OracleResult(x=x, s=s, lam=lam, mu=mu, iters=it, converged=converged,
                        objective=float(0.5 * x @ Hx + prob.p @ x), history=hist)


# ----------------------------------------------------------------------------
# pieces the GPU parity tests compare against
# ----------------------------------------------------------------------------

def condensed_operator_dense(prob, sigma_x: np.ndarray, sigma_A: Optional[np.ndarray],
                             H: Optional[np.ndarray] = None) -> np.ndarray:
    """K = H + diag(sigma_x) + A^T diag(sigma_A) A for given per-variable and
    per-row weights (the operator PCG runs on, north of eq. (2x2_augmented))."""
    K = (hessian_dense(prob) if H is None else H).copy()
    K[np.diag_indices(prob.n)] += sigma_x
    if prob.A is not None and prob.m > 0 and sigma_A is not None:
        Ad = prob.A.toarray()
        K += (Ad * sigma_A[:, None]).T @ Ad
    return K


def newton_solve_dense(K: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """dx = K^{-1} rhs by dense Cholesky."""
    cf = sla.cho_factor(K, lower=True, check_finite=False)
    return sla.cho_solve(cf, rhs, check_finite=False)


def lambda_A_combined(res: OracleResult, prob) -> np.ndarray:
    """lambda_uA - lambda_lA scattered to the m rows of A (one multiplier per
    row; positive when the upper bound is active)."""
    G = make_groups(prob)
    out = np.zeros(prob.m)
    out[G.idx["uA"]] += res.lam["uA"]
    out[G.idx["lA"]] -= res.lam["lA"]
    return out


def lambda_x_combined(res: OracleResult, prob) -> np.ndarray:
    """lambda_ux - lambda_lx scattered to the n variables."""
    G = make_groups(prob)
    out = np.zeros(prob.n)
    out[G.idx["ux"]] += res.lam["ux"]
    out[G.idx["lx"]] -= res.lam["lx"]
    return out
