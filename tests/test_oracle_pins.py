"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

P1  the paper's literal Newton system (eq. (newton_system)), its 2x2 reduced
    form (eq. (2x2_reduced)) and its doubly augmented form (eq. (2x2_augmented))
    give the same direction as the oracle's condensed solve, and the condensed
    operator the GPU tests compare with is the Schur complement of the literal
    Newton matrix;
P2  brute-force active-set enumeration (n <= 8);
P3  closed form x = clip(-p/gamma, l, u) when H = gamma*I;
P4  scipy's bounded least squares (BVLS) and NNLS for box-constrained
    least-squares QPs;
P5  unconstrained x = -H^{-1} p;
P6  the KKT certificate, itself pinned on exact solutions and on perturbed ones;
P7  iterate invariants;
plus hand-solved QPs in tests/golden/handsolved.json and planted mistakes that
the pins must catch.
"""
import json
import os

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import oracle
import qpsynth
from oracle import ipm_dense
from qpsynth import QPProblem

HERE = os.path.dirname(os.path.abspath(__file__))


def _gap_bound(res, prob, mu_tol=1e-10):
    """Objective error allowed by the stopping rule: at exit every scaled
    lambda_i*s_i is below 2*mu_tol, so s^T lambda <= 2*m_tot*mu_tol*zeta in the
    original units, plus rounding."""
    m_tot = sum(len(v) for v in res.lam.values())
    return 2.0 * m_tot * mu_tol * res.zeta


def _combined(res, prob):
    return (oracle.lambda_x_combined(res, prob),
            oracle.lambda_A_combined(res, prob) if prob.m else None)


# ----------------------------------------------------------------------------
# P2: brute force on the tiny set
# ----------------------------------------------------------------------------

TINY = list(range(48))


@pytest.mark.parametrize("inst", TINY)
def test_p2_tiny_matches_bruteforce(inst):
    prob = qpsynth.tiny(inst)
    res = oracle.solve(prob)
    bf = oracle.bruteforce_qp(prob)
    assert res.converged
    assert np.abs(res.x - bf.x).max() <= 1e-8
    assert abs(res.objective - bf.objective) <= 1e-10 * (1 + abs(bf.objective)) + _gap_bound(res, prob)
    cert = oracle.kkt_certificate(prob, res.x, *_combined(res, prob))
    assert cert.worst() <= 1e-9, cert


# ----------------------------------------------------------------------------
# P6: the certificate itself
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("inst", [0, 3, 12, 42])
def test_p6_certificate_zero_at_exact_solution_and_large_off_it(inst):
    prob = qpsynth.tiny(inst)
    bf = oracle.bruteforce_qp(prob)
    yA = bf.y_A if prob.m else None
    cert = oracle.kkt_certificate(prob, bf.x, bf.y_x, yA)
    assert cert.worst() <= 1e-9, cert
    assert abs(cert.objective - bf.objective) <= 1e-12 * (1 + abs(bf.objective))
    # a moved point breaks stationarity
    c2 = oracle.kkt_certificate(prob, bf.x + 1e-3, bf.y_x, yA)
    assert c2.worst() > 1e-7
    # a multiplier of the wrong sign on an absent side is flagged
    y_bad = bf.y_x.copy()
    free = ~np.isfinite(prob.x_lo) & ~np.isfinite(prob.x_hi)
    if np.any(free):
        j = int(np.flatnonzero(free)[0])
        y_bad[j] = 1.0
        assert oracle.kkt_certificate(prob, bf.x, y_bad, yA).worst() == np.inf


# ----------------------------------------------------------------------------
# P3, P4, P5: closed forms and library routines
# ----------------------------------------------------------------------------

def _box_prob(n, J, W, p, lo, hi, gamma=1e-3):
    return QPProblem(gamma=gamma, p=p, J=sp.csr_matrix(J), W=W, x_lo=lo, x_hi=hi)


def test_p3_identity_hessian_is_clipping():
    rng = np.random.default_rng(7)
    n = 30
    p = rng.uniform(-0.02, 0.02, size=n)
    lo = rng.uniform(-5, 0, size=n)
    hi = lo + rng.uniform(0.5, 10, size=n)
    lo[:5] = -np.inf
    hi[5:10] = np.inf
    prob = _box_prob(n, np.zeros((1, n)), np.ones(1), p, lo, hi)
    res = oracle.solve(prob)
    x_ref = np.clip(-p / prob.gamma, lo, hi)
    assert np.abs(res.x - x_ref).max() <= 1e-8 * (1 + np.abs(x_ref).max())


def test_p4_bvls_box_least_squares():
    rng = np.random.default_rng(11)
    nJ, n = 60, 12
    J = np.where(rng.uniform(size=(nJ, n)) < 0.4, rng.lognormal(size=(nJ, n)), 0.0)
    W = rng.uniform(0.5, 2, size=nJ)
    p = rng.normal(size=n) * 20
    lo, hi = np.zeros(n), np.full(n, 3.0)
    prob = _box_prob(n, J, W, p, lo, hi)
    res = oracle.solve(prob)
    # normal equations of [W^1/2 J; sqrt(g) I] x ~ [0; -p/sqrt(g)] are (J^T W J + g I) x = -p
    M = np.vstack([np.sqrt(W)[:, None] * J, np.sqrt(prob.gamma) * np.eye(n)])
    y = np.concatenate([np.zeros(nJ), -p / np.sqrt(prob.gamma)])
    ref = so.lsq_linear(M, y, bounds=(lo, hi), method="bvls", tol=1e-14)
    assert np.abs(res.x - ref.x).max() <= 1e-7


def test_p4_nnls_nonnegative_least_squares():
    rng = np.random.default_rng(12)
    nJ, n = 50, 10
    J = np.where(rng.uniform(size=(nJ, n)) < 0.5, rng.lognormal(size=(nJ, n)), 0.0)
    W = rng.uniform(0.5, 2, size=nJ)
    p = rng.normal(size=n) * 20
    prob = _box_prob(n, J, W, p, np.zeros(n), np.full(n, np.inf))
    res = oracle.solve(prob)
    M = np.vstack([np.sqrt(W)[:, None] * J, np.sqrt(prob.gamma) * np.eye(n)])
    y = np.concatenate([np.zeros(nJ), -p / np.sqrt(prob.gamma)])
    x_ref, _ = so.nnls(M, y, maxiter=10000)
    assert np.abs(res.x - x_ref).max() <= 1e-7


def test_p5_unconstrained_is_linear_solve():
    prob = qpsynth.config1(0)
    n = prob.n
    free = QPProblem(gamma=prob.gamma, p=prob.p, J=prob.J, W=prob.W,
                     x_lo=np.full(n, -np.inf), x_hi=np.full(n, np.inf))
    res = oracle.solve(free)
    H = free.J.T.toarray() @ (free.W[:, None] * free.J.toarray()) + free.gamma * np.eye(n)
    x_ref = np.linalg.solve(H, -free.p)
    assert res.converged
    assert np.abs(res.x - x_ref).max() <= 1e-9 * (1 + np.abs(x_ref).max())


# ----------------------------------------------------------------------------
# hand-solved fixtures
# ----------------------------------------------------------------------------

def _load_handsolved():
    with open(os.path.join(HERE, "golden", "handsolved.json")) as f:
        return json.load(f)["cases"]


def _arr(v):
    return np.array([np.nan if e is None else e for e in v], dtype=float)


def _handsolved_problem(c):
    g = c["gamma"]
    J = np.array(c["J"], dtype=float)
    W = np.array(c["W"], dtype=float)
    H0 = J.T @ (W[:, None] * J)
    fac = 1.0
    if "p_over_1pg" in c:
        fac = 1 + g
        p = fac * np.array(c["p_over_1pg"], dtype=float)
    elif "p_over_2pg" in c:
        fac = 2 + g
        p = fac * np.array(c["p_over_2pg"], dtype=float)
    else:
        p = np.array(c["p"], dtype=float)
    assert np.allclose(H0 + g * np.eye(len(p)), fac * np.eye(len(p))) or fac == 1.0
    lo = np.nan_to_num(_arr(c["x_lo"]), nan=-np.inf)
    hi = np.nan_to_num(_arr(c["x_hi"]), nan=np.inf)
    A = A_lo = A_hi = None
    if c.get("A") is not None:
        A = sp.csr_matrix(np.array(c["A"], dtype=float))
        A_lo = np.nan_to_num(_arr(c["A_lo"]), nan=-np.inf)
        A_hi = np.nan_to_num(_arr(c["A_hi"]), nan=np.inf)
    prob = QPProblem(gamma=g, p=p, J=sp.csr_matrix(J), W=W, x_lo=lo, x_hi=hi,
                     A=A, A_lo=A_lo, A_hi=A_hi, name=c["name"])
    f = c["f"] if "f" in c else fac * c.get("f_over_1pg", c.get("f_over_2pg"))
    return prob, np.array(c["x"], dtype=float), f


@pytest.mark.parametrize("case", _load_handsolved(), ids=lambda c: c["name"])
def test_handsolved(case):
    prob, x_ref, f_ref = _handsolved_problem(case)
    res = oracle.solve(prob)
    assert res.converged
    assert np.abs(res.x - x_ref).max() <= 1e-8
    assert abs(res.objective - f_ref) <= 1e-10 * (1 + abs(f_ref)) + _gap_bound(res, prob)
    # the brute force agrees on these too
    bf = oracle.bruteforce_qp(prob)
    assert np.abs(bf.x - x_ref).max() <= 1e-10


def test_equality_row_lo_equals_hi():
    """A row with lo == hi: min (1+g)/2 |x|^2 s.t. x1 - x2 = 1 has x = (1/2, -1/2)."""
    g = 1e-3
    prob = QPProblem(gamma=g, p=np.zeros(2), J=sp.csr_matrix(np.eye(2)), W=np.ones(2),
                     x_lo=np.full(2, -np.inf), x_hi=np.full(2, np.inf),
                     A=sp.csr_matrix(np.array([[1.0, -1.0]])), A_lo=np.array([1.0]),
                     A_hi=np.array([1.0]))
    res = oracle.solve(prob)
    assert res.converged
    assert np.abs(res.x - np.array([0.5, -0.5])).max() <= 1e-8


# ----------------------------------------------------------------------------
# P1: the paper's Newton system forms agree with the condensed solve
# ----------------------------------------------------------------------------

def _random_state(prob, seed):
    rng = np.random.default_rng(seed)
    G = ipm_dense.make_groups(prob)
    x = rng.uniform(-1, 1, size=prob.n)
    s = {g: rng.uniform(0.1, 3, size=len(G.idx[g])) for g in ipm_dense.GROUPS}
    lam = {g: rng.uniform(0.1, 3, size=len(G.idx[g])) for g in ipm_dense.GROUPS}
    mu = float(rng.uniform(0.01, 1))
    return G, x, s, lam, mu


def _literal_newton_matrix(prob, s, lam, x, mu):
    """eq. (newton_system) written with the paper's single constraint matrix
    R = [I; A] and l <= R x <= u (bounds are rows of R), assembled as the
    5x5 block matrix over (dx, dlambda_l, dlambda_u, ds_l, ds_u), with its
    right-hand side.  Returns (M, rhs, block offsets)."""
    n = prob.n
    H = ipm_dense.hessian_dense(prob)
    R = np.eye(n) if prob.m == 0 else np.vstack([np.eye(n), prob.A.toarray()])
    lo = prob.x_lo if prob.m == 0 else np.concatenate([prob.x_lo, prob.A_lo])
    hi = prob.x_hi if prob.m == 0 else np.concatenate([prob.x_hi, prob.A_hi])
    L = np.flatnonzero(np.isfinite(lo))
    U = np.flatnonzero(np.isfinite(hi))
    # the oracle orders group rows bounds first, then rows of A: same as L, U here
    s_l = np.concatenate([s["lx"], s["lA"]])
    s_u = np.concatenate([s["ux"], s["uA"]])
    l_l = np.concatenate([lam["lx"], lam["lA"]])
    l_u = np.concatenate([lam["ux"], lam["uA"]])
    RL, RU = R[L], R[U]
    nl, nu = len(L), len(U)
    r_H = H @ x + prob.p - RL.T @ l_l + RU.T @ l_u
    r_l = RL @ x - s_l - lo[L]
    r_u = -RU @ x - s_u + hi[U]
    r_c1 = l_l * s_l - mu
    r_c2 = l_u * s_u - mu
    N = n + 2 * nl + 2 * nu
    M = np.zeros((N, N))
    o = [0, n, n + nl, n + nl + nu, n + 2 * nl + nu, N]
    M[o[0]:o[1], o[0]:o[1]] = H
    M[o[0]:o[1], o[1]:o[2]] = -RL.T
    M[o[0]:o[1], o[2]:o[3]] = RU.T
    M[o[1]:o[2], o[0]:o[1]] = RL
    M[o[1]:o[2], o[3]:o[4]] = -np.eye(nl)
    M[o[2]:o[3], o[0]:o[1]] = -RU
    M[o[2]:o[3], o[4]:o[5]] = -np.eye(nu)
    M[o[3]:o[4], o[1]:o[2]] = np.diag(s_l)
    M[o[3]:o[4], o[3]:o[4]] = np.diag(l_l)
    M[o[4]:o[5], o[2]:o[3]] = np.diag(s_u)
    M[o[4]:o[5], o[4]:o[5]] = np.diag(l_u)
    return M, -np.concatenate([r_H, r_l, r_u, r_c1, r_c2]), o


@pytest.mark.parametrize("inst", [0, 1, 2, 12, 42, 54])
def test_p1_full_newton_system(inst):
    """The literal eq. (newton_system), solved densely, against the oracle's
    condensed solve and recovery."""
    prob = qpsynth.tiny(inst)
    n = prob.n
    G, x, s, lam, mu = _random_state(prob, 100 + inst)
    H = ipm_dense.hessian_dense(prob)
    M, rhs, o = _literal_newton_matrix(prob, s, lam, x, mu)
    sol = np.linalg.solve(M, rhs)
    dx_full = sol[:n]
    dl_l, dl_u = sol[o[1]:o[2]], sol[o[2]:o[3]]
    ds_l, ds_u = sol[o[3]:o[4]], sol[o[4]:o[5]]

    Hx, rH, rg, rc = ipm_dense.residuals(prob, G, H, x, s, lam, mu)
    dx, ds, dlam = ipm_dense.newton_direction(prob, G, H, x, s, lam, mu, Hx, rg)
    sc = 1 + np.abs(sol).max()
    assert np.abs(dx - dx_full).max() <= 1e-10 * sc
    assert np.abs(np.concatenate([dlam["lx"], dlam["lA"]]) - dl_l).max() <= 1e-10 * sc
    assert np.abs(np.concatenate([dlam["ux"], dlam["uA"]]) - dl_u).max() <= 1e-10 * sc
    assert np.abs(np.concatenate([ds["lx"], ds["lA"]]) - ds_l).max() <= 1e-10 * sc
    assert np.abs(np.concatenate([ds["ux"], ds["uA"]]) - ds_u).max() <= 1e-10 * sc


@pytest.mark.parametrize("inst", [0, 2, 12, 42])
def test_p1_reduced_and_doubly_augmented(inst):
    """eq. (2x2_reduced) and eq. (2x2_augmented) with Q = H + S^-1 Lambda
    (bounds), B = [A_L; -A_U], D = Lambda^-1 S (rows of A).  The paper leaves
    r1, r2 to its companion work; eliminating eq. (newton_system) gives
    r2 = -(r_g + r_c/lambda) on the rows of A and
    r1 = -r_H - sum_bounds G^T S^-1 (r_c + Lambda r_g)."""
    prob = qpsynth.tiny(inst)
    if prob.m == 0:
        pytest.skip("needs rows of A")
    n = prob.n
    G, x, s, lam, mu = _random_state(prob, 200 + inst)
    H = ipm_dense.hessian_dense(prob)
    Hx, rH, rg, rc = ipm_dense.residuals(prob, G, H, x, s, lam, mu)
    Ad = prob.A.toarray()
    B = np.vstack([Ad[G.idx["lA"]], -Ad[G.idx["uA"]]])
    Dd = np.concatenate([s["lA"] / lam["lA"], s["uA"] / lam["uA"]])
    Q = H.copy()
    Q[G.idx["lx"], G.idx["lx"]] += lam["lx"] / s["lx"]
    Q[G.idx["ux"], G.idx["ux"]] += lam["ux"] / s["ux"]
    r2 = -np.concatenate([rg["lA"] + rc["lA"] / lam["lA"], rg["uA"] + rc["uA"] / lam["uA"]])
    r1 = -rH.copy()
    for g in ("lx", "ux"):
        r1 -= G.GT(g, (rc[g] + lam[g] * rg[g]) / s[g], n)
    k = B.shape[0]
    M = np.block([[Q, -B.T], [B, np.diag(Dd)]])
    red = np.linalg.solve(M, np.concatenate([r1, r2]))
    Ma = np.block([[Q + 2 * B.T @ np.diag(1 / Dd) @ B, B.T], [B, np.diag(Dd)]])
    aug = np.linalg.solve(Ma, np.concatenate([r1 + 2 * B.T @ (r2 / Dd), r2]))
    # the doubly augmented matrix is symmetric positive definite
    assert np.allclose(Ma, Ma.T)
    assert np.all(np.linalg.eigvalsh(Ma) > 0)
    dx, ds, dlam = ipm_dense.newton_direction(prob, G, H, x, s, lam, mu, Hx, rg)
    dlA = np.concatenate([dlam["lA"], dlam["uA"]])
    sc = 1 + np.abs(red).max()
    for sol in (red, aug):
        assert np.abs(sol[:n] - dx).max() <= 1e-9 * sc
        assert np.abs(sol[n:n + k] - dlA).max() <= 1e-9 * sc


@pytest.mark.parametrize("inst", [0, 1, 2, 5, 12, 17, 42, 54])
def test_p1_condensed_operator_is_schur_complement(inst):
    """condensed_operator_dense(prob, sigma_x, sigma_A) -- the operator every
    GPU operator and Newton-step test compares with -- equals the Schur
    complement onto dx of the literal eq. (newton_system) matrix, eliminated
    here numerically (M11 - M12 M22^-1 M21), with sigma_x = Sigma_lx + Sigma_ux
    per variable and sigma_A = Sigma_lA + Sigma_uA per row of A, Sigma_g =
    lambda_g / s_g.  Variables and rows without a finite side get weight 0."""
    prob = qpsynth.tiny(inst)
    n = prob.n
    G, x, s, lam, mu = _random_state(prob, 300 + inst)
    M, _, o = _literal_newton_matrix(prob, s, lam, x, mu)
    K_schur = M[:n, :n] - M[:n, n:] @ np.linalg.solve(M[n:, n:], M[n:, :n])
    sig_x = np.zeros(n)
    sig_x[G.idx["lx"]] += lam["lx"] / s["lx"]
    sig_x[G.idx["ux"]] += lam["ux"] / s["ux"]
    sig_A = None
    if prob.m:
        sig_A = np.zeros(prob.m)
        sig_A[G.idx["lA"]] += lam["lA"] / s["lA"]
        sig_A[G.idx["uA"]] += lam["uA"] / s["uA"]
    K = oracle.condensed_operator_dense(prob, sig_x, sig_A)
    assert np.abs(K - K_schur).max() <= 1e-12 * (1 + np.abs(K_schur).max())
    # and against the condensed matrix of the oracle's own iteration (pinned by
    # the solves above), with the groups' weights kept apart
    Kc = ipm_dense.condensed_matrix(prob, G, ipm_dense.hessian_dense(prob),
                                    {g: lam[g] / s[g] for g in ipm_dense.GROUPS})
    assert np.abs(K - Kc).max() <= 1e-13 * (1 + np.abs(Kc).max())


def test_p1_condensed_operator_catches_planted_mistakes(monkeypatch):
    """The Schur-complement pin above fails for each plausible slip in the
    operator: a dropped A^T Sigma_A A term, sqrt(Sigma_A) in place of Sigma_A,
    a dropped Sigma_x, and the row weights counted twice (lower and upper
    sides merged twice)."""
    prob = qpsynth.tiny(12)
    assert prob.m > 0 and prob.n != prob.m
    n = prob.n
    G, x, s, lam, mu = _random_state(prob, 312)
    M, _, o = _literal_newton_matrix(prob, s, lam, x, mu)
    K_schur = M[:n, :n] - M[:n, n:] @ np.linalg.solve(M[n:, n:], M[n:, :n])
    sig_x = np.zeros(n)
    sig_x[G.idx["lx"]] += lam["lx"] / s["lx"]
    sig_x[G.idx["ux"]] += lam["ux"] / s["ux"]
    sig_A = np.zeros(prob.m)
    sig_A[G.idx["lA"]] += lam["lA"] / s["lA"]
    sig_A[G.idx["uA"]] += lam["uA"] / s["uA"]
    H = ipm_dense.hessian_dense(prob)
    Ad = prob.A.toarray()
    mutants = [H + np.diag(sig_x),
               H + np.diag(sig_x) + (Ad * np.sqrt(sig_A)[:, None]).T @ Ad,
               H + (Ad * sig_A[:, None]).T @ Ad,
               H + np.diag(sig_x) + 2.0 * (Ad * sig_A[:, None]).T @ Ad]
    for Km in mutants:
        assert np.abs(Km - K_schur).max() > 1e-6 * (1 + np.abs(K_schur).max())


# ----------------------------------------------------------------------------
# P7: invariants along the path; config 1 certificates
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("inst", range(5))
def test_p7_invariants_and_certificate_config1(inst):
    prob = qpsynth.config1(inst)
    res = oracle.solve(prob, record=True)
    assert res.converged and res.iters <= 200
    mus = [h["mu"] for h in res.history]
    assert all(b <= a for a, b in zip(mus, mus[1:]))
    for h in res.history:
        assert 0 < h["alpha_x"] <= 1 and 0 < h["alpha_l"] <= 1
        assert h["min_s"] > 0 and h["min_l"] > 0
    cert = oracle.kkt_certificate(prob, res.x, *_combined(res, prob))
    assert cert.worst() <= 1e-9, cert


# ----------------------------------------------------------------------------
# planted mistakes: each must make a pin fail (the oracle is mutated on the CPU)
# ----------------------------------------------------------------------------

def _mutant_fails(monkeypatch, patch):
    with monkeypatch.context() as mp:
        patch(mp)
        for inst in (0, 2, 12):
            prob = qpsynth.tiny(inst)
            bf = oracle.bruteforce_qp(prob)
            try:
                res = oracle.solve(prob, oracle.OracleSettings(max_ipm_iter=60))
            except Exception:
                return True
            if (not res.converged) or np.abs(res.x - bf.x).max() > 1e-8:
                return True
    return False


def test_planted_mistakes_are_caught(monkeypatch):
    orig_res = ipm_dense.residuals
    orig_dir = ipm_dense.newton_direction

    def flip_ru_sign(mp):
        def bad(prob, G, H, x, s, lam, mu):
            Hx, rH, rg, rc = orig_res(prob, G, H, x, s, lam, mu)
            rg = dict(rg)
            rg["uA"] = G.G("uA", x) + s["uA"] - G.c["uA"]
            return Hx, rH, rg, rc
        mp.setattr(ipm_dense, "residuals", bad)

    def drop_sigma_r_term(mp):
        def bad(prob, G, H, x, s, lam, mu, Hx, rg):
            return orig_dir(prob, G, H, x, s, lam, mu, Hx, {g: 0 * v for g, v in rg.items()})
        mp.setattr(ipm_dense, "newton_direction", bad)

    def transpose_hessian_term(mp):
        orig_h = ipm_dense.hessian_dense

        def bad(prob):
            H = orig_h(prob)
            return H + np.triu(np.ones_like(H), 1) * 1e-2
        mp.setattr(ipm_dense, "hessian_dense", bad)

    def wrong_dlambda_sign(mp):
        def bad(prob, G, H, x, s, lam, mu, Hx, rg):
            dx, ds, dlam = orig_dir(prob, G, H, x, s, lam, mu, Hx, rg)
            sig = {g: lam[g] / s[g] for g in dlam}
            return dx, ds, {g: -lam[g] + mu / s[g] + sig[g] * ds[g] for g in dlam}
        mp.setattr(ipm_dense, "newton_direction", bad)

    for patch in (flip_ru_sign, drop_sigma_r_term, transpose_hessian_term, wrong_dlambda_sign):
        assert _mutant_fails(monkeypatch, patch), patch.__name__


# ----------------------------------------------------------------------------
# generators: determinism and shapes
# ----------------------------------------------------------------------------

def test_generators_are_deterministic():
    a, b = qpsynth.config1(3), qpsynth.config1(3)
    assert a.J.data.tobytes() == b.J.data.tobytes()
    assert a.A_hi.tobytes() == b.A_hi.tobytes()
    c, d = qpsynth.config2(scale=0.05), qpsynth.config2(scale=0.05)
    assert c.J.indices.tobytes() == d.J.indices.tobytes()
    assert c.p.tobytes() == d.p.tobytes()


def test_config_shapes():
    p1 = qpsynth.config1(0)
    assert p1.J.shape == (2000, 200) and p1.J.nnz == 20000
    assert p1.A.shape == (50, 200) and p1.A.nnz == 10000
    p2 = qpsynth.config2(scale=0.1)
    rl = np.diff(p2.J.indptr)
    assert p2.J.shape[0] % 64 == 0
    # rows of one 64-voxel line share a column pattern
    blk = p2.J.indptr[:65]
    assert np.all(np.diff(blk) == rl[0])
    cl = np.diff(p2.J.tocsc().indptr)
    assert cl.min() >= 64 * 31 and cl.max() <= 64 * 32
    # bfloat16 keeps 8 significant bits: spacing 2^-7 on [1, 2); ties go to even
    bf = qpsynth.round_to_bf16(np.array([1.0, 1.00390625, 1.01171875, 1.0040, 1.0029296875]))
    assert list(bf) == [1.0, 1.0, 1.015625, 1.0078125, 1.0]
