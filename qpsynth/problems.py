"""Seeded synthetic QP instances shaped like the paper's radiotherapy QP sub-problems.

The paper measures on QPs exported from a commercial treatment planning system
(Section 5.2, Table 1), which are not available; these generators stand in for
them.  They produce the data of the QP of Section 3.1, eq. (qp),

    min 1/2 x^T H x + p^T x   s.t.  lo_A <= A x <= hi_A,  lo_x <= x <= hi_x,

with H = gamma*I + J^T diag(W) J + U diag(w) U^T, the quasi-Newton form of
eq. (bfgs_hessian) with a dose-influence least-squares term in H_0.

This module only draws data.  It holds none of the interior point method or
conjugate gradient arithmetic; both the oracle and the GPU path receive the
arrays it returns.  Every draw goes through ``numpy.random.default_rng(seed)``
(PCG64) in the order documented on each function, so equal seeds give equal
bytes on any machine with the same numpy.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class QPProblem:
    """One QP instance.  Infinite bounds are +-inf (an absent constraint)."""

    gamma: float
    p: np.ndarray                      # (n,)   linear term
    J: sp.csr_matrix                   # (nJ, n) dose-influence matrix, float64
    W: np.ndarray                      # (nJ,)  diagonal weights, > 0
    x_lo: np.ndarray                   # (n,)
    x_hi: np.ndarray                   # (n,)
    A: Optional[sp.csr_matrix] = None  # (m, n) linear constraints
    A_lo: Optional[np.ndarray] = None  # (m,)
    A_hi: Optional[np.ndarray] = None  # (m,)
    U: Optional[np.ndarray] = None     # (n, k) column-major (Fortran order)
    w: Optional[np.ndarray] = None     # (k,)   weights of the low-rank term, >= 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.p.shape[0])

    @property
    def m(self) -> int:
        return 0 if self.A is None else int(self.A.shape[0])

    @property
    def k(self) -> int:
        return 0 if self.U is None else int(self.U.shape[1])


# ----------------------------------------------------------------------------
# helpers (data only)
# ----------------------------------------------------------------------------

def _csr(indptr, indices, data, shape) -> sp.csr_matrix:
    M = sp.csr_matrix((data, indices, indptr), shape=shape)
    M.has_sorted_indices = True
    return M


def round_to_bf16(v: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 value (ties to even).

    Goes through binary32 with round-to-odd (truncate, then set the last bit
    when any dropped bit was set), then rounds the binary32 pattern to its top
    16 bits with round-to-nearest-even; rounding to odd first keeps the two
    steps equal to one correct rounding.  Used only to *define* problem data
    whose values are bfloat16 numbers (finite, within the binary32 normal
    range, or zero).
    """
    v = np.ascontiguousarray(v, dtype=np.float64)
    d = v.view(np.uint64)
    sign = d >> np.uint64(63)
    e = ((d >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1023 + 127
    m = d & np.uint64((1 << 52) - 1)
    normal = (e >= 1) & (e <= 254)
    b = ((sign << np.uint64(31)) | (np.clip(e, 0, 255).astype(np.uint64) << np.uint64(23))
         | (m >> np.uint64(29)))
    b = b | ((m & np.uint64((1 << 29) - 1)) != 0).astype(np.uint64)
    b = np.where(normal, b, v.astype(np.float32).view(np.uint32).astype(np.uint64))
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    b = (b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    out = (b.astype(np.uint32) << np.uint32(16)).view(np.float32)
    return out.astype(np.float64)


def _linear_term(J: sp.csr_matrix, W: np.ndarray, x_t: np.ndarray) -> np.ndarray:
    """p = -J^T W (J x_t): the least-squares target d = J x_t made a linear term."""
    return -(J.T @ (W * (J @ x_t)))


def _feasible_rhs(A: sp.csr_matrix, x0: np.ndarray, s0: np.ndarray) -> np.ndarray:
    """b = A x0 + s0, so that x0 satisfies A x <= b with slack s0 > 0."""
    return A @ x0 + s0


# ----------------------------------------------------------------------------
# "64-voxel band" dose-influence structure
# ----------------------------------------------------------------------------

def band_dose_pattern(rng: np.random.Generator, n_spots: int, Z: int, Y: int,
                      total_lines: int, X: int = 64):
    """Column structure of a banded dose-influence matrix.

    Voxel rows form a Z x Y x X grid with X the fastest axis; a *line* is one
    (z, y) pair and owns the X consecutive rows z*Y*X + y*X + (0..X-1).  Each
    spot (column) covers ``b_j`` lines, the nearest to its centre, and every
    covered line gives one band of X consecutive nonzero rows.

    Draw order: (1) centres, 2*n_spots uniforms (z then y per spot),
    (2) a permutation of the spots deciding who gets ceil(beta) lines.

    Returns (line_ptr, line_spots): CSR of the (lines x spots) incidence, with
    sorted spot ids in each line.
    """
    n_lines = Z * Y
    cz = rng.uniform(0.0, Z, size=n_spots)
    cy = rng.uniform(0.0, Y, size=n_spots)
    # sort spots by centre: coarse z slab first, then y
    order = np.lexsort((cy, np.floor(cz)))
    cz, cy = cz[order], cy[order]
    base = total_lines // n_spots
    extra = total_lines - base * n_spots
    b = np.full(n_spots, base, dtype=np.int64)
    b[rng.permutation(n_spots)[:extra]] += 1

    bmax = int(b.max())
    if bmax > n_lines:
        raise ValueError("more lines per spot than lines in the grid")

    def nearest(czc, cyc, rad):
        oz, oy = np.meshgrid(np.arange(-rad, rad + 1), np.arange(-rad, rad + 1), indexing="ij")
        oz, oy = oz.ravel(), oy.ravel()
        iz = np.floor(czc)[:, None].astype(np.int64) + oz[None, :]
        iy = np.floor(cyc)[:, None].astype(np.int64) + oy[None, :]
        valid = (iz >= 0) & (iz < Z) & (iy >= 0) & (iy < Y)
        d2 = (iz + 0.5 - czc[:, None]) ** 2 + (iy + 0.5 - cyc[:, None]) ** 2
        d2 = np.where(valid, d2, np.inf)
        line = np.where(valid, iz * Y + iy, n_lines)
        # nearest first, ties by line id
        o = np.lexsort((line, d2), axis=1)
        return np.take_along_axis(line, o, axis=1), valid.sum(axis=1)

    rad0 = int(np.ceil(np.sqrt(bmax))) + 3
    pairs_line = np.empty(int(b.sum()), dtype=np.int64)
    pairs_spot = np.empty(int(b.sum()), dtype=np.int64)
    pos = 0
    chunk = 4096
    for s0 in range(0, n_spots, chunk):
        s1 = min(n_spots, s0 + chunk)
        lines, nvalid = nearest(cz[s0:s1], cy[s0:s1], rad0)
        short = np.flatnonzero(nvalid < b[s0:s1])
        fixed = {}
        rad = rad0
        while short.size:
            rad *= 2
            l2, v2 = nearest(cz[s0:s1][short], cy[s0:s1][short], rad)
            ok = v2 >= b[s0:s1][short]
            for r, row in zip(short[ok], l2[ok]):
                fixed[int(r)] = row
            short = short[~ok]
        for r in range(s1 - s0):
            bj = int(b[s0 + r])
            sel = fixed[r][:bj] if r in fixed else lines[r, :bj]
            pairs_line[pos:pos + bj] = sel
            pairs_spot[pos:pos + bj] = s0 + r
            pos += bj
    o = np.lexsort((pairs_spot, pairs_line))
    pairs_line, pairs_spot = pairs_line[o], pairs_spot[o]
    line_ptr = np.zeros(n_lines + 1, dtype=np.int64)
    np.add.at(line_ptr, pairs_line + 1, 1)
    line_ptr = np.cumsum(line_ptr)
    return line_ptr, pairs_spot.astype(np.int32)


def band_dose_matrix(rng: np.random.Generator, n_spots: int, Z: int, Y: int,
                     nnz_target: int, X: int = 64, value_dtype=np.float64):
    """Banded dose-influence CSR matrix of (Z*Y*X) x n_spots, lognormal(0,1) values.

    Draw order: the pattern (``band_dose_pattern``), then nnz lognormal values
    in CSR order.
    """
    assert nnz_target % X == 0
    total_lines = nnz_target // X
    line_ptr, line_spots = band_dose_pattern(rng, n_spots, Z, Y, total_lines, X)
    n_lines = Z * Y
    line_len = np.diff(line_ptr)
    rows = n_lines * X
    row_len = np.repeat(line_len, X)
    indptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(row_len, out=indptr[1:])
    nnz = int(indptr[-1])
    assert nnz == nnz_target
    indices = np.empty(nnz, dtype=np.int32)
    for ell in range(n_lines):
        a, c = int(line_ptr[ell]), int(line_ptr[ell + 1])
        L = c - a
        if L == 0:
            continue
        r0 = ell * X
        start = int(indptr[r0])
        indices[start:start + L * X] = np.tile(line_spots[a:c], X)
    data = rng.lognormal(0.0, 1.0, size=nnz).astype(value_dtype, copy=False)
    return _csr(indptr, indices, data, (rows, n_spots))


def random_sparse(rng: np.random.Generator, rows: int, cols: int, nnz_per_row: int,
                  values: str = "normal") -> sp.csr_matrix:
    """Each row gets ``nnz_per_row`` distinct random columns (sorted).

    Draw order: per row, a column choice (without replacement); then all values
    in CSR order.
    """
    k = nnz_per_row
    indptr = np.arange(rows + 1, dtype=np.int64) * k
    indices = np.empty(rows * k, dtype=np.int32)
    for i in range(rows):
        indices[i * k:(i + 1) * k] = np.sort(rng.choice(cols, size=k, replace=False))
    if values == "normal":
        data = rng.standard_normal(rows * k)
    else:
        data = rng.lognormal(0.0, 1.0, size=rows * k)
    return _csr(indptr, indices, data, (rows, cols))


# ----------------------------------------------------------------------------
# the benchmark configurations
# ----------------------------------------------------------------------------

GAMMA = 1e-3


def config1(instance: int = 0) -> QPProblem:
    """n=200 spots; J 2000x200 at 5% (uniform random positions, lognormal(0,1));
    W ~ U[0.5,2]; A 50x200 dense N(0,1); A x <= b with b = A x0 + U[0.1,1],
    x0 ~ U[0,1]; bounds 0 <= x <= 10; p = -J^T W J x_t, x_t ~ U[-2, 12].

    Seed 1000 + instance.  Draw order: J positions, J values, W, A, x0, s0, x_t.
    """
    seed = 1000 + instance
    rng = np.random.default_rng(seed)
    n, nJ, m, hi = 200, 2000, 50, 10.0
    nnz = nJ * n // 20
    pos = np.sort(rng.choice(nJ * n, size=nnz, replace=False))
    r, c = pos // n, (pos % n).astype(np.int32)
    indptr = np.zeros(nJ + 1, dtype=np.int64)
    np.add.at(indptr, r + 1, 1)
    indptr = np.cumsum(indptr)
    val = rng.lognormal(0.0, 1.0, size=nnz)
    J = _csr(indptr, c, val, (nJ, n))
    W = rng.uniform(0.5, 2.0, size=nJ)
    Ad = rng.standard_normal((m, n))
    A = sp.csr_matrix(Ad)
    A.has_sorted_indices = True
    x0 = rng.uniform(0.0, 1.0, size=n)
    s0 = rng.uniform(0.1, 1.0, size=m)
    x_t = rng.uniform(-0.2 * hi, 1.2 * hi, size=n)
    b = _feasible_rhs(A, x0, s0)
    return QPProblem(gamma=GAMMA, p=_linear_term(J, W, x_t), J=J, W=W,
                     x_lo=np.zeros(n), x_hi=np.full(n, hi),
                     A=A, A_lo=np.full(m, -np.inf), A_hi=b,
                     name=f"config1[{instance}]", meta={"seed": seed})


def config2(seed: int = 2000, scale: float = 1.0) -> QPProblem:
    """n=20,000 spots; J 400,000x20,000 with 40M nnz in 64-voxel bands (grid
    50x125x64, 31.25 lines per spot), lognormal(0,1); W ~ U[0.5,2]; A
    2,000x20,000 at 2% (400 per row) N(0,1); A x <= b as in config1; bounds
    [0, 50].  ``scale`` < 1 shrinks every dimension (for quick tests): n, the
    grid's z extent and m scale together so nnz per row stays about 100.

    Draw order: J (pattern, values), W, A (pattern, values), x0, s0, x_t.
    """
    rng = np.random.default_rng(seed)
    n = int(round(20000 * scale))
    Z = max(2, int(round(50 * scale)))
    Y = 125
    m = max(1, int(round(2000 * scale)))
    total_lines = int(round(n * 31.25))
    J = band_dose_matrix(rng, n, Z, Y, total_lines * 64)
    W = rng.uniform(0.5, 2.0, size=J.shape[0])
    A = random_sparse(rng, m, n, max(1, n // 50))
    hi = 50.0
    x0 = rng.uniform(0.0, 1.0, size=n)
    s0 = rng.uniform(0.1, 1.0, size=m)
    x_t = rng.uniform(-0.2 * hi, 1.2 * hi, size=n)
    return QPProblem(gamma=GAMMA, p=_linear_term(J, W, x_t), J=J, W=W,
                     x_lo=np.zeros(n), x_hi=np.full(n, hi),
                     A=A, A_lo=np.full(m, -np.inf), A_hi=_feasible_rhs(A, x0, s0),
                     name=f"config2(scale={scale})", meta={"seed": seed, "scale": scale})


def irregular_bands(seed: int = 2100, scale: float = 0.05, drop: float = 0.15, trim: int = 23) -> QPProblem:
    """A banded-dose QP whose bands are irregular, as measured dose matrices
    are: the config2 pattern at `scale`, each nonzero of J dropped with
    probability `drop` (so the 64 rows of a line no longer share one column
    list), and the last `trim` rows removed (the row count is then not a
    multiple of 64).  The rest as config2.

    Draw order: J (pattern, values), the drop mask, W, A (pattern, values),
    x0, s0, x_t.
    """
    rng = np.random.default_rng(seed)
    n = int(round(20000 * scale))
    Z = max(2, int(round(50 * scale)))
    m = max(1, int(round(2000 * scale)))
    J = band_dose_matrix(rng, n, Z, 125, int(round(n * 31.25)) * 64).tocoo()
    keep = rng.uniform(size=J.nnz) >= drop
    J = sp.csr_matrix((J.data[keep], (J.row[keep], J.col[keep])), shape=J.shape)[:J.shape[0] - trim]
    J.sort_indices()
    W = rng.uniform(0.5, 2.0, size=J.shape[0])
    A = random_sparse(rng, m, n, max(1, n // 50))
    hi = 50.0
    x0 = rng.uniform(0.0, 1.0, size=n)
    s0 = rng.uniform(0.1, 1.0, size=m)
    x_t = rng.uniform(-0.2 * hi, 1.2 * hi, size=n)
    return QPProblem(gamma=GAMMA, p=_linear_term(J, W, x_t), J=J, W=W,
                     x_lo=np.zeros(n), x_hi=np.full(n, hi),
                     A=A, A_lo=np.full(m, -np.inf), A_hi=_feasible_rhs(A, x0, s0),
                     name=f"irregular_bands(scale={scale}, drop={drop})",
                     meta={"seed": seed, "scale": scale, "drop": drop, "trim": trim})


def config5(seed: int = 5000, scale: float = 1.0) -> QPProblem:
    """n=60,000; J 2,000,000x60,000 with 200M nnz (grid 125x250x64, ~52.1 lines
    per spot), values lognormal(0,1) *rounded to bfloat16* (the problem is
    defined by the bfloat16 values); U 60,000x20 with N(0,1)/sqrt(n) entries,
    w ~ U[0.1,1]; A 6,000x60,000 at 1% (600 per row); bounds [0, 50].

    Draw order: J (pattern, values), W, U, w, A, x0, s0, x_t.
    """
    rng = np.random.default_rng(seed)
    n = int(round(60000 * scale))
    Z = max(2, int(round(125 * scale)))
    Y = 250
    m = max(1, int(round(6000 * scale)))
    total_lines = int(round(200_000_000 * scale)) // 64
    J = band_dose_matrix(rng, n, Z, Y, total_lines * 64)
    J.data = round_to_bf16(J.data)
    W = rng.uniform(0.5, 2.0, size=J.shape[0])
    k = 20
    U = np.asfortranarray(rng.standard_normal((n, k)) / np.sqrt(n))
    w = rng.uniform(0.1, 1.0, size=k)
    A = random_sparse(rng, m, n, max(1, n // 100))
    hi = 50.0
    x0 = rng.uniform(0.0, 1.0, size=n)
    s0 = rng.uniform(0.1, 1.0, size=m)
    x_t = rng.uniform(-0.2 * hi, 1.2 * hi, size=n)
    p = _linear_term(J, W, x_t) - U @ (w * (U.T @ x_t))
    return QPProblem(gamma=GAMMA, p=p, J=J, W=W,
                     x_lo=np.zeros(n), x_hi=np.full(n, hi),
                     A=A, A_lo=np.full(m, -np.inf), A_hi=_feasible_rhs(A, x0, s0),
                     U=U, w=w, name=f"config5(scale={scale})",
                     meta={"seed": seed, "scale": scale})


def config4_sizes(seed: int = 4000, count: int = 64):
    """Sizes n_k ~ U_int[2000, 20000] rounded down to a multiple of 16."""
    rng = np.random.default_rng(seed)
    n = rng.integers(2000, 20001, size=count)
    return (n // 16) * 16


def config4_instance(index: int, seed: int = 4000, count: int = 64) -> QPProblem:
    """Member ``index`` of the 64-QP batch: n_k spots, J 20n_k x n_k at 0.5%
    (64-voxel bands, 0.1 n_k/64 lines per spot), m_k = n_k/10 at 2%, bounds
    [0, 50].  Each member has its own stream seed*100 + index."""
    n = int(config4_sizes(seed, count)[index])
    rng = np.random.default_rng(seed * 100 + index)
    rows = 20 * n
    n_lines = rows // 64
    Y = int(np.ceil(np.sqrt(n_lines)))
    Z = n_lines // Y
    # keep whole lines only: Z*Y <= n_lines; rows of the trailing partial z-row
    # are absent
    nnz_target = int(round(0.005 * rows)) * n
    nnz_target -= nnz_target % 64
    J = band_dose_matrix(rng, n, Z, Y, nnz_target)
    W = rng.uniform(0.5, 2.0, size=J.shape[0])
    m = n // 10
    A = random_sparse(rng, m, n, max(1, n // 50))
    hi = 50.0
    x0 = rng.uniform(0.0, 1.0, size=n)
    s0 = rng.uniform(0.1, 1.0, size=m)
    x_t = rng.uniform(-0.2 * hi, 1.2 * hi, size=n)
    return QPProblem(gamma=GAMMA, p=_linear_term(J, W, x_t), J=J, W=W,
                     x_lo=np.zeros(n), x_hi=np.full(n, hi),
                     A=A, A_lo=np.full(m, -np.inf), A_hi=_feasible_rhs(A, x0, s0),
                     name=f"config4[{index}]", meta={"seed": seed, "index": index})


def tiny(instance: int) -> QPProblem:
    """Small instance for brute-force checks: n in [1, 8]; J 10n x n at 50%;
    m in [0, 4]; bounds of every kind (two-sided, one-sided, absent) on x and
    on the rows of A, all strictly satisfied at a drawn point x0.

    Seed 90000 + instance.  Draw order: n, m, J mask, J values, W, bound kinds
    of x, bound kinds of A rows, A, x0, slacks, x_t, bound widths.
    """
    seed = 90000 + instance
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    m = int(rng.integers(0, 5))
    nJ = 10 * n
    mask = rng.uniform(size=(nJ, n)) < 0.5
    vals = rng.lognormal(0.0, 1.0, size=(nJ, n))
    J = sp.csr_matrix(np.where(mask, vals, 0.0))
    J.has_sorted_indices = True
    W = rng.uniform(0.5, 2.0, size=nJ)
    kind_x = rng.integers(0, 4, size=n)      # 0 both, 1 lower, 2 upper, 3 free
    kind_a = rng.integers(0, 3, size=m)      # 0 both, 1 lower, 2 upper
    Ad = rng.standard_normal((m, n))
    x0 = rng.uniform(-1.0, 1.0, size=n)
    sl = rng.uniform(0.1, 1.0, size=(2, n + m))
    x_t = rng.uniform(-4.0, 4.0, size=n)
    wid = rng.uniform(0.5, 3.0, size=(2, n + m))
    x_lo = np.where((kind_x == 0) | (kind_x == 1), x0 - sl[0, :n] * wid[0, :n], -np.inf)
    x_hi = np.where((kind_x == 0) | (kind_x == 2), x0 + sl[1, :n] * wid[1, :n], np.inf)
    A = sp.csr_matrix(Ad) if m > 0 else None
    if A is not None:
        A.has_sorted_indices = True
        ax0 = Ad @ x0
        A_lo = np.where((kind_a == 0) | (kind_a == 1), ax0 - sl[0, n:] * wid[0, n:], -np.inf)
        A_hi = np.where((kind_a == 0) | (kind_a == 2), ax0 + sl[1, n:] * wid[1, n:], np.inf)
    else:
        A_lo = A_hi = None
    return QPProblem(gamma=GAMMA, p=_linear_term(J, W, x_t), J=J, W=W,
                     x_lo=x_lo, x_hi=x_hi, A=A, A_lo=A_lo, A_hi=A_hi,
                     name=f"tiny[{instance}]", meta={"seed": seed})


def long_rows(seed: int = 96000) -> QPProblem:
    """CSR row-length edge cases: n = 2600 spots, J 900 x 2600 with row lengths
    U_int[0, 60), 200 of them set to 0 (empty rows), and 12 rows longer than
    2048 entries (lengths U_int[2049, 2600), the first of them a full row of
    2600); positions uniform without repeats, values lognormal(0, 1); W ~
    U[0.5, 2]; A 40 x 2600 with N(0,1) entries at 5%, A x <= b feasible at x0
    ~ U[0,1]; bounds [0, 10]; p = -J^T W J x_t, x_t ~ U[0, 5].

    Draw order: row lengths, the empty rows, the long rows, their lengths,
    then per row its positions; values; W; A's mask and entries; x0; s0; x_t."""
    rng = np.random.default_rng(seed)
    n, nJ, m = 2600, 900, 40
    counts = rng.integers(0, 60, nJ)
    counts[rng.choice(nJ, 200, replace=False)] = 0
    longr = rng.choice(nJ, 12, replace=False)
    counts[longr] = rng.integers(2049, n, 12)
    counts[longr[0]] = n
    indptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    indices = np.concatenate([np.sort(rng.choice(n, int(c), replace=False)) for c in counts]).astype(np.int32)
    data = rng.lognormal(0.0, 1.0, int(indptr[-1]))
    J = _csr(indptr, indices, data, (nJ, n))
    W = rng.uniform(0.5, 2.0, nJ)
    mask = rng.random((m, n)) < 0.05
    A = sp.csr_matrix(np.where(mask, rng.standard_normal((m, n)), 0.0))
    x0 = rng.uniform(0.0, 1.0, n)
    s0 = rng.uniform(0.1, 1.0, m)
    x_t = rng.uniform(0.0, 5.0, n)
    return QPProblem(gamma=GAMMA, p=_linear_term(J, W, x_t), J=J, W=W,
                     x_lo=np.zeros(n), x_hi=np.full(n, 10.0),
                     A=A, A_lo=np.full(m, -np.inf), A_hi=_feasible_rhs(A, x0, s0),
                     name="long_rows", meta={"seed": seed})


def ragged_lines(seed: int = 95000) -> QPProblem:
    """Line-format edge cases: n = 400 spots, eight 64-row lines with 0, 1, 5,
    130, 300, 64, 3 and 0 slots (empty lines, the first and the last included;
    lines longer than four wavefronts of 32 held slots, with remainders); W
    uniform [0.5, 2]; A 20 x 400 with 40 normal entries per row, b feasible at
    x0; bounds [0, 50].

    Draw order: per line, its spots (without replacement, sorted); J values;
    W; A; x0; slacks; x_t.
    """
    rng = np.random.default_rng(seed)
    n, X = 400, 64
    lens = [0, 1, 5, 130, 300, 64, 3, 0]
    cols = [np.sort(rng.choice(n, size=L, replace=False)) for L in lens]
    rows = X * len(lens)
    indptr = np.zeros(rows + 1, dtype=np.int64)
    for ell, L in enumerate(lens):
        for r in range(X):
            indptr[ell * X + r + 1] = indptr[ell * X + r] + L
    indices = np.concatenate([np.tile(c, X) for c in cols]).astype(np.int32)
    data = rng.lognormal(0.0, 1.0, size=int(indptr[-1]))
    J = _csr(indptr, indices, data, (rows, n))
    W = rng.uniform(0.5, 2.0, size=rows)
    m = 20
    A = random_sparse(rng, m, n, 40)
    x0 = rng.uniform(0.0, 1.0, size=n)
    s0 = rng.uniform(0.1, 1.0, size=m)
    x_t = rng.uniform(-10.0, 60.0, size=n)
    return QPProblem(gamma=GAMMA, p=_linear_term(J, W, x_t), J=J, W=W,
                     x_lo=np.zeros(n), x_hi=np.full(n, 50.0),
                     A=A, A_lo=np.full(m, -np.inf), A_hi=_feasible_rhs(A, x0, s0),
                     name="ragged_lines", meta={"seed": seed})


def random_iterate(prob: QPProblem, seed: int):
    """Random positive slacks/multipliers and a random x, mu for operator and
    Newton-system checks.  Returns dict with x, mu and per-row sigma values."""
    rng = np.random.default_rng(seed)
    n, m = prob.n, prob.m
    return {
        "x": rng.uniform(-1.0, 1.0, size=n),
        "sigma_x": np.exp(rng.uniform(-4.0, 4.0, size=n)),
        "sigma_A": np.exp(rng.uniform(-4.0, 4.0, size=m)),
        "v": rng.standard_normal(n),
        "rhs": rng.standard_normal(n),
    }


def sqp_sequence(base: QPProblem, steps: int, seed: int = 77000) -> list:
    """A sequence of QP sub-problems as an SQP run produces them (Section 3.2):
    J, W, A and the bounds of ``base`` throughout; sub-problem t has a
    quasi-Newton term U_t w_t U_t^T with 2t columns (each step appends two
    columns of N(0,1)/sqrt(n) entries and keeps the earlier ones, w ~
    U[0.1, 1]) and the linear term p_t = base.p * (1 + 0.05 N(0,1)) -
    U_t (w_t * U_t^T x_g), x_g ~ U[lo, hi] drawn once.  Sub-problem 0 has no
    low-rank term.

    Draw order: x_g, then per step t >= 1: two U columns, two w entries,
    the p perturbation (step 0 draws its perturbation first).
    """
    rng = np.random.default_rng(seed)
    n = base.n
    lo = np.where(np.isfinite(base.x_lo), base.x_lo, -1.0)
    hi = np.where(np.isfinite(base.x_hi), base.x_hi, 1.0)
    x_g = rng.uniform(lo, hi)
    cols, ws = [], []
    out = []
    for t in range(steps):
        if t > 0:
            cols.append(rng.standard_normal((n, 2)) / np.sqrt(n))
            ws.append(rng.uniform(0.1, 1.0, size=2))
        pert = 1.0 + 0.05 * rng.standard_normal(n)
        if cols:
            U = np.asfortranarray(np.hstack(cols))
            w = np.concatenate(ws)
            p = base.p * pert - U @ (w * (U.T @ x_g))
        else:
            U, w = None, None
            p = base.p * pert
        out.append(QPProblem(gamma=base.gamma, p=p, J=base.J, W=base.W, x_lo=base.x_lo, x_hi=base.x_hi,
                             A=base.A, A_lo=base.A_lo, A_hi=base.A_hi, U=U, w=w,
                             name=f"{base.name}/sqp[{t}]", meta={"seed": seed, "step": t}))
    return out
