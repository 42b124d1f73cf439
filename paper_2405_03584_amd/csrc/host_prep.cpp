// Host-side preparation of QP data (no HIP calls).
#include "host_prep.h"

#include <cmath>
#include <algorithm>
#include <cstring>
#include <limits>

namespace qpg {

std::string check_csr(const qp_csr* M, const char* name, int32_t expect_cols) {
    std::string nm(name);
    if (!M) return nm + " is NULL";
    if (M->rows < 0 || M->cols < 0) return nm + ": negative dimension";
    if (expect_cols >= 0 && M->cols != expect_cols)
        return nm + ": cols does not match the number of variables";
    if (M->nnz < 0 || M->nnz >= (int64_t(1) << 31)) return nm + ": nnz must be in [0, 2^31)";
    if (!M->row_ptr) return nm + ": row_ptr is NULL";
    if (M->nnz > 0 && (!M->col_idx || !M->val)) return nm + ": col_idx/val is NULL";
    if (M->row_ptr[0] != 0) return nm + ": row_ptr[0] != 0";
    if (M->row_ptr[M->rows] != M->nnz) return nm + ": row_ptr[rows] != nnz";
    for (int32_t i = 0; i < M->rows; ++i) {
        int64_t a = M->row_ptr[i], c = M->row_ptr[i + 1];
        if (c < a) return nm + ": row_ptr decreases at row " + std::to_string(i);
        int32_t prev = -1;
        for (int64_t k = a; k < c; ++k) {
            int32_t j = M->col_idx[k];
            if (j < 0 || j >= M->cols)
                return nm + ": column index out of range in row " + std::to_string(i);
            if (j <= prev)
                return nm + ": column indices not strictly increasing in row " + std::to_string(i);
            prev = j;
            if (!std::isfinite(M->val[k])) return nm + ": non-finite value in row " + std::to_string(i);
        }
    }
    return "";
}

HostCsr to_host_csr(const qp_csr* M) {
    HostCsr h;
    h.rows = M->rows;
    h.cols = M->cols;
    h.ptr.resize(size_t(M->rows) + 1);
    for (int32_t i = 0; i <= M->rows; ++i) h.ptr[i] = static_cast<int32_t>(M->row_ptr[i]);
    h.col.assign(M->col_idx, M->col_idx + M->nnz);
    h.val.assign(M->val, M->val + M->nnz);
    return h;
}

HostCsr transpose(const HostCsr& M) {
    HostCsr T;
    T.rows = M.cols;
    T.cols = M.rows;
    T.ptr.assign(size_t(M.cols) + 1, 0);
    const int64_t nnz = M.nnz();
    for (int64_t k = 0; k < nnz; ++k) T.ptr[size_t(M.col[k]) + 1]++;
    for (int32_t j = 0; j < M.cols; ++j) T.ptr[j + 1] += T.ptr[j];
    T.col.resize(nnz);
    T.val.resize(nnz);
    std::vector<int32_t> next(T.ptr.begin(), T.ptr.end() - 1);
    for (int32_t i = 0; i < M.rows; ++i) {
        for (int32_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
            int32_t j = M.col[k];
            int32_t dst = next[j]++;
            T.col[dst] = i;
            T.val[dst] = M.val[k];
        }
    }
    return T;
}

bool build_line_format(const HostCsr& M, int32_t R, LineFormat& lf, double max_fill) {
    if (R <= 0 || M.rows == 0) return false;
    const int32_t L = (M.rows + R - 1) / R;   // the last line may have fewer rows (padded with empty ones)
    const double budget = max_fill * double(M.nnz());
    // each line's column list: the union of its rows' sorted lists, padded to
    // a multiple of kLineSlotAlign slots (repeats of its last column, zero
    // values: the packed low-precision loads read whole slot groups)
    std::vector<int32_t> lptr(size_t(L) + 1, 0), lcol, lreal(size_t(L), 0);
    std::vector<int32_t> scratch;
    int64_t real = 0;
    for (int32_t l = 0; l < L; ++l) {
        const int32_t r0 = l * R, r1 = std::min(M.rows, r0 + R);
        scratch.assign(M.col.begin() + M.ptr[r0], M.col.begin() + M.ptr[r1]);
        std::sort(scratch.begin(), scratch.end());
        scratch.erase(std::unique(scratch.begin(), scratch.end()), scratch.end());
        lreal[l] = int32_t(scratch.size());
        real += int64_t(scratch.size());
        while (scratch.size() % kLineSlotAlign) scratch.push_back(scratch.back());
        lcol.insert(lcol.end(), scratch.begin(), scratch.end());
        lptr[l + 1] = int32_t(lcol.size());
        if (double(real) * R > budget) return false;   // too many stored zeros
    }
    LineFormat f;
    f.R = R;
    f.lines = L;
    f.cols = M.cols;
    f.ptr = std::move(lptr);
    f.col = std::move(lcol);
    f.val.assign(f.col.size() * size_t(R), 0.0);
    for (int32_t l = 0; l < L; ++l) {
        const int32_t* lc = f.col.data() + f.ptr[l];
        const int32_t len = lreal[l];
        for (int32_t r = 0; r < R && l * R + r < M.rows; ++r) {
            const int32_t row = l * R + r;
            int32_t k = 0;   // both lists sorted: one merge walk
            for (int32_t e = M.ptr[row]; e < M.ptr[row + 1]; ++e) {
                while (k < len && lc[k] < M.col[e]) ++k;
                f.val[(size_t(f.ptr[l]) + k) * R + r] = M.val[e];
            }
        }
    }
    // transpose of the (line x spot) incidence, counting sort over spots
    f.sptr.assign(size_t(M.cols) + 1, 0);
    for (int32_t l = 0; l < L; ++l)
        for (int32_t k = f.ptr[l]; k < f.ptr[l] + lreal[l]; ++k) f.sptr[size_t(f.col[k]) + 1]++;
    for (int32_t j = 0; j < M.cols; ++j) f.sptr[j + 1] += f.sptr[j];
    f.sline.resize(size_t(real));
    f.sslot.resize(size_t(real));
    std::vector<int32_t> next(f.sptr.begin(), f.sptr.end() - 1);
    for (int32_t l = 0; l < L; ++l)
        for (int32_t k = f.ptr[l]; k < f.ptr[l] + lreal[l]; ++k) {
            const int32_t j = f.col[k];
            const int32_t d = next[j]++;
            f.sline[d] = l;
            f.sslot[d] = k;
        }
    lf = std::move(f);
    return true;
}

void build_row_blocks(const std::vector<int32_t>& ptr, int32_t rows, int32_t max_nnz, int32_t max_rows,
                      std::vector<int32_t>& out) {
    out.clear();
    int32_t r = 0;
    while (r < rows) {
        out.push_back(r);
        out.push_back(ptr[r]);
        const int32_t start = r;
        const int32_t e0 = ptr[r];
        ++r;   // the first row always fits (alone when longer than max_nnz)
        while (r < rows && r - start < max_rows && int64_t(ptr[r + 1]) - e0 <= max_nnz) ++r;
    }
    out.push_back(rows);
    out.push_back(rows > 0 ? ptr[rows] : 0);
}

// binary64 -> binary32 with round to nearest, ties to even.  The C++ cast
// rounds with the current rounding mode, which is round-to-nearest-even by
// default; values beyond the float range become +-inf.
uint32_t f64_to_f32_bits(double v) {
    float f = static_cast<float>(v);
    uint32_t b;
    std::memcpy(&b, &f, 4);
    return b;
}

// binary64 -> bfloat16 (1 sign, 8 exponent, 7 fraction bits), round to
// nearest, ties to even.  Rounding twice to nearest (to binary32, then to
// bfloat16) can round a value that is not a tie as if it were one; rounding the
// first step to odd instead (truncate, then set the last bit when anything was
// dropped) makes the second round-to-nearest-even step exact (Boldo and
// Melquiond, "Emulation of FMA and correctly rounded sums: proved algorithms
// using rounding to odd", IEEE TC 2008).  Inputs outside the binary32 normal
// range go through the plain cast (zero, or values the format cannot hold).
uint16_t f64_to_bf16_bits(double v) {
    uint64_t d;
    std::memcpy(&d, &v, 8);
    const uint64_t sign = d >> 63;
    const int64_t e = int64_t((d >> 52) & 0x7FF) - 1023 + 127;
    const uint64_t m = d & ((uint64_t(1) << 52) - 1);
    uint32_t b;
    if (e >= 1 && e <= 254) {
        b = uint32_t(sign << 31) | uint32_t(e << 23) | uint32_t(m >> 29);
        if (m & ((uint64_t(1) << 29) - 1)) b |= 1u;      // round to odd
    } else {
        b = f64_to_f32_bits(v);
    }
    const uint32_t lsb = (b >> 16) & 1u;
    b += 0x7FFFu + lsb;                                   // nearest, ties to even
    return static_cast<uint16_t>(b >> 16);
}

double bf16_bits_to_f64(uint16_t h) {
    uint32_t b = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &b, 4);
    return static_cast<double>(f);
}

std::string validate_settings(const qp_settings* s) {
    if (!s) return "";
    if (s->precision < QP_FP64 || s->precision > QP_BF16) return "settings.precision out of range";
    if (s->refine_steps < 0 || s->refine_steps > 16) return "settings.refine_steps must be in [0, 16]";
    if (!(s->pcg_tol > 0.0) || !(s->pcg_tol < 1.0)) return "settings.pcg_tol must be in (0, 1)";
    if (!(s->refine_tol >= s->pcg_tol) || !(s->refine_tol < 1.0))
        return "settings.refine_tol must be in [pcg_tol, 1)";
    if (s->pcg_max_iter < 1) return "settings.pcg_max_iter must be >= 1";
    if (!std::isfinite(s->mu0)) return "settings.mu0 must be finite";
    if (!(s->mu_tol > 0.0)) return "settings.mu_tol must be > 0";
    if (!(s->tau > 0.0) || !(s->tau < 1.0)) return "settings.tau must be in (0, 1)";
    if (s->max_ipm_iter < 1) return "settings.max_ipm_iter must be >= 1";
    if (s->step_mode != 0 && s->step_mode != 1) return "settings.step_mode must be 0 or 1";
    if (s->schedule != 0 && s->schedule != 1 && s->schedule != 4 && s->schedule != 8 && s->schedule != 16 &&
        s->schedule != 32 && s->schedule != 64)
        return "settings.schedule must be 0, 1, 4, 8, 16, 32 or 64";
    if (s->precond != 0 && s->precond != 1) return "settings.precond must be 0 or 1";
    if (s->graphs != 0 && s->graphs != 1) return "settings.graphs must be 0 or 1";
    if (s->spmv_format != 0 && s->spmv_format != 1) return "settings.spmv_format must be 0 or 1";
    if (s->kkt_system != 0 && s->kkt_system != 1) return "settings.kkt_system must be 0 or 1";
    if (s->batch_mode != 0 && s->batch_mode != 1) return "settings.batch_mode must be 0 or 1";
    return "";
}

static std::string check_range(const double* lo, const double* hi, int64_t len, const char* what) {
    for (int64_t i = 0; i < len; ++i) {
        double l = lo ? lo[i] : -INFINITY;
        double u = hi ? hi[i] : INFINITY;
        if (std::isnan(l) || std::isnan(u)) return std::string(what) + ": NaN bound";
        if (l == INFINITY || u == -INFINITY) return std::string(what) + ": bound of the wrong infinite sign";
        if (l > u) return std::string(what) + ": lo > hi at index " + std::to_string(i);
    }
    return "";
}

std::string validate_hessian(const qp_hessian* H, int32_t n) {
    if (!H) return "H is NULL";
    if (!(H->gamma >= 0.0) || !std::isfinite(H->gamma)) return "H.gamma must be finite and >= 0";
    if (!H->p) return "H.p is NULL";
    for (int32_t j = 0; j < n; ++j)
        if (!std::isfinite(H->p[j])) return "H.p has a non-finite entry";
    if (H->k < 0) return "H.k < 0";
    if (H->k > 0) {
        if (!H->U || !H->w) return "H.U / H.w is NULL with k > 0";
        for (int64_t i = 0; i < int64_t(n) * H->k; ++i)
            if (!std::isfinite(H->U[i])) return "H.U has a non-finite entry";
        for (int32_t c = 0; c < H->k; ++c)
            if (!(H->w[c] >= 0.0) || !std::isfinite(H->w[c])) return "H.w must be finite and >= 0";
    }
    return "";
}

std::string validate_problem(const qp_hessian* H, const qp_csr* J, const double* W,
                             const qp_csr* A, const qp_range* b, const qp_range* bounds,
                             const qp_settings* s) {
    if (!H) return "H is NULL";
    if (!J) return "J is NULL";
    std::string e = check_csr(J, "J", -1);
    if (!e.empty()) return e;
    const int32_t n = J->cols;
    if (n <= 0) return "the problem needs at least one variable (J->cols > 0)";
    e = validate_hessian(H, n);
    if (!e.empty()) return e;
    if (J->rows > 0 && !W) return "W is NULL";
    for (int32_t i = 0; i < J->rows; ++i)
        if (!(W[i] >= 0.0) || !std::isfinite(W[i])) return "W must be finite and >= 0";
    if (A) {
        e = check_csr(A, "A", n);
        if (!e.empty()) return e;
        if (A->rows > 0 && !b) return "b (row bounds of A) is NULL";
        if (A->rows > 0) {
            e = check_range(b->lo, b->hi, A->rows, "b");
            if (!e.empty()) return e;
        }
    }
    if (bounds) {
        e = check_range(bounds->lo, bounds->hi, n, "bounds");
        if (!e.empty()) return e;
    }
    return validate_settings(s);
}

}  // namespace qpg
