"""Host preparation code of the library (validation helpers, transposes, value
rounding, the line format), compiled with g++ for the CPU: no GPU needed."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import qpsynth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_03584_amd", "csrc")


@pytest.fixture(scope="module")
def hp(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("hp") / "libhp.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", os.path.join(ROOT, "include"),
                    "-I", CSRC, os.path.join(CSRC, "host_prep.cpp"),
                    os.path.join(ROOT, "tests", "host_prep_harness.cpp"), "-o", out], check=True)
    return C.CDLL(out)


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def test_transpose_matches_scipy(hp):
    M = qpsynth.config1(0).J
    ptr = M.indptr.astype(np.int32); col = M.indices.astype(np.int32); val = M.data.copy()
    optr = np.zeros(M.shape[1] + 1, np.int32); ocol = np.zeros(M.nnz, np.int32); oval = np.zeros(M.nnz)
    hp.hp_transpose(M.shape[0], M.shape[1], _p(ptr, C.c_int), _p(col, C.c_int), _p(val, C.c_double),
                    _p(optr, C.c_int), _p(ocol, C.c_int), _p(oval, C.c_double))
    T = M.T.tocsr()
    T.sort_indices()
    assert np.array_equal(optr, T.indptr) and np.array_equal(ocol, T.indices)
    assert np.array_equal(oval, T.data)


def _bf16_bruteforce(v):
    """Nearest bfloat16 by enumeration of the two neighbours (ties to even)."""
    out = np.empty(v.shape, np.uint16)
    for i, x in enumerate(v):
        f = np.float32(x)
        b = int(np.array([f], np.float32).view(np.uint32)[0]) >> 16
        cands = [(b - 1) & 0xFFFF, b, (b + 1) & 0xFFFF]
        best = None
        for c in cands:
            val = float(np.array([c << 16], np.uint32).view(np.float32)[0])
            if not np.isfinite(val):
                continue
            d = abs(val - x)
            key = (d, c & 1)
            if best is None or key < best[0]:
                best = (key, c)
        out[i] = best[1]
    return out


def test_bf16_round_to_nearest_even(hp):
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.lognormal(0, 1, 3000), -rng.lognormal(0, 3, 1000),
                        [1.0, 1.00390625, 1.01171875, 1.0 + 2 ** -8 + 2 ** -40, 0.0, 3.0e38]])
    out = np.zeros(v.shape, np.uint16)
    hp.hp_bf16(_p(v, C.c_double), _p(out, C.c_ushort), C.c_long(v.size))
    ref = _bf16_bruteforce(v)
    assert np.array_equal(out, ref)
    # the generator's rounding agrees with the library's
    gen = qpsynth.round_to_bf16(v[:-1])
    lib = (out[:-1].astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert np.array_equal(gen, lib)


def _line_format(hp, M, R=64, max_fill=2.0):
    ptr = M.indptr.astype(np.int32); col = M.indices.astype(np.int32); val = M.data.copy()
    L = -(-M.shape[0] // R)
    cap = int(max_fill * M.nnz / R) + 4 * L + 1   # real slots within the budget, plus group padding
    lptr = np.zeros(L + 1, np.int32); lcol = np.zeros(cap, np.int32); lval = np.zeros(cap * R)
    sptr = np.zeros(M.shape[1] + 1, np.int32); sline = np.zeros(cap, np.int32)
    sslot = np.zeros(cap, np.int32); ns = C.c_int(0)
    ok = hp.hp_line_format(M.shape[0], M.shape[1], _p(ptr, C.c_int), _p(col, C.c_int), _p(val, C.c_double), R,
                           C.c_double(max_fill), cap, _p(lptr, C.c_int), _p(lcol, C.c_int), _p(lval, C.c_double),
                           _p(sptr, C.c_int), _p(sline, C.c_int), _p(sslot, C.c_int), C.byref(ns))
    assert ok != -1
    n = ns.value
    nreal = int(sptr[-1]) if ok == 1 else 0   # the per-spot lists name real slots only
    return ok, L, lptr, lcol[:n], lval[:n * R], sptr, sline[:nreal], sslot[:nreal]


def _reconstruct(M, L, lptr, lcol, lval, R=64):
    rows, cols, vals = [], [], []
    for l in range(L):
        for k in range(lptr[l], lptr[l + 1]):
            for r in range(R):
                if R * l + r < M.shape[0]:
                    rows.append(R * l + r); cols.append(lcol[k]); vals.append(lval[k * R + r])
                else:
                    assert lval[k * R + r] == 0.0   # padding rows of the last line hold nothing
    return sp.csr_matrix((vals, (rows, cols)), shape=M.shape)


def _check_spot_lists(M, lcol, sptr, sline, sslot, R=64):
    # per-spot (line, slot) lists are the transpose of the line incidence, lines increasing
    for j in range(0, M.shape[1], 37):
        ls = sline[sptr[j]:sptr[j + 1]]
        assert np.all(np.diff(ls) > 0)
        assert np.all(lcol[sslot[sptr[j]:sptr[j + 1]]] == j)
        col_rows = M.tocsc()[:, j].indices
        assert np.array_equal(np.unique(col_rows // R), ls)


def _check_slot_groups(lptr, lcol, lval, real, R=64):
    """Lines hold whole groups of 4 slots; the padding slots repeat the
    line's last real column and hold zeros."""
    for l in range(len(lptr) - 1):
        a, b = lptr[l], lptr[l + 1]
        assert (b - a) % 4 == 0 and (b - a) - real[l] in range(4)
        for k in range(a + real[l], b):
            assert lcol[k] == lcol[a + real[l] - 1]
            assert not np.any(lval[k * R:(k + 1) * R])


def test_line_format_reconstructs_banded_matrix(hp):
    M = qpsynth.config2(scale=0.02).J
    ok, L, lptr, lcol, lval, sptr, sline, sslot = _line_format(hp, M, max_fill=1.0)
    assert ok == 1
    real = [len(np.unique(M[64 * l:64 * (l + 1)].indices)) for l in range(L)]
    assert sum(real) * 64 == M.nnz             # the bands share their column lists: only group padding
    _check_slot_groups(lptr, lcol, lval, real)
    assert (_reconstruct(M, L, lptr, lcol, lval) != M).nnz == 0
    _check_spot_lists(M, lcol, sptr, sline, sslot)


def test_line_format_pads_rows_that_miss_columns(hp):
    """A banded matrix with 15% of its entries dropped at random and a row
    count that is not a multiple of 64: each line stores the union of its
    rows' columns, zeros where a row lacks one, and empty padding rows."""
    M = qpsynth.config2(scale=0.02).J.tocoo()
    keep = np.random.default_rng(4).uniform(size=M.nnz) >= 0.15
    M = sp.csr_matrix((M.data[keep], (M.row[keep], M.col[keep])), shape=M.shape)[:M.shape[0] - 23]
    M.sort_indices()
    ok, L, lptr, lcol, lval, sptr, sline, sslot = _line_format(hp, M)
    assert ok == 1 and L == -(-M.shape[0] // 64)
    real = [len(np.unique(M[64 * l:64 * (l + 1)].indices)) for l in range(L)]
    assert M.nnz < 64 * sum(real) <= 2 * M.nnz
    _check_slot_groups(lptr, lcol, lval, real)
    assert (_reconstruct(M, L, lptr, lcol, lval) != M).nnz == 0
    # each line's list starts with exactly the union of its rows' columns, sorted
    for l in range(L):
        union = np.unique(M[64 * l:64 * (l + 1)].indices)
        assert np.array_equal(lcol[lptr[l]:lptr[l] + len(union)], union)
    _check_spot_lists(M, lcol, sptr, sline, sslot)
    # a fill budget below what the lines need refuses the format
    assert _line_format(hp, M, max_fill=1.0)[0] == 0


def test_line_format_rejects_unstructured(hp):
    M = qpsynth.config1(0).J   # 2000 x 200 at 5%, uniform positions: a line's rows share almost nothing
    assert _line_format(hp, M)[0] == 0


def _row_blocks(hp, counts, max_nnz, max_rows):
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    rows = len(counts)
    cap = rows + 1
    out = np.zeros(2 * (cap + 1), np.int32)
    nb = hp.hp_row_blocks(rows, _p(ptr, C.c_int), max_nnz, max_rows, cap, _p(out, C.c_int))
    assert nb >= 0
    return ptr, out[:2 * (nb + 1)].reshape(-1, 2)


@pytest.mark.parametrize("case", ["short", "mixed", "empty_rows", "long_only", "none"])
def test_row_blocks_cover_every_row_once(hp, case):
    """Nonzero-balanced row blocks of the streamed forward pass: consecutive,
    covering every row once, each within the nonzero and row limits or a
    single longer row, and maximal (the next row would break a limit)."""
    rng = np.random.default_rng(7)
    counts = {"short": rng.integers(0, 40, 3000),
              "mixed": np.where(rng.random(800) < 0.05, rng.integers(2049, 9000, 800), rng.integers(0, 300, 800)),
              "empty_rows": np.zeros(1000, np.int64),
              "long_only": rng.integers(2049, 5000, 40),
              "none": np.zeros(0, np.int64)}[case]
    max_nnz, max_rows = 2048, 256
    ptr, blk = _row_blocks(hp, counts, max_nnz, max_rows)
    rows = len(counts)
    assert blk[0].tolist() == [0, 0] and blk[-1].tolist() == [rows, int(ptr[rows])]
    for (r0, e0), (r1, e1) in zip(blk[:-1], blk[1:]):
        assert r1 > r0 and e0 == ptr[r0] and e1 == ptr[r1]
        nnz, nr = e1 - e0, r1 - r0
        assert (nnz <= max_nnz and nr <= max_rows) or (nr == 1 and nnz > max_nnz)
        if r1 < rows and nnz <= max_nnz:   # maximal: one more row would not fit
            assert nr == max_rows or ptr[r1 + 1] - e0 > max_nnz
    if rows == 0:
        assert len(blk) == 1

