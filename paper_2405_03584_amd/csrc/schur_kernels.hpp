// Constraint-block preconditioner for the condensed Newton system.
//
// The PCG operator is K = Hs + Sigma_x + A^T Sigma_A A (Hs = H/zeta).  Jacobi
// (the paper's preconditioner, Section 4.1.2) treats the A^T Sigma_A A term by
// its diagonal only; once rows of A become active (Sigma_A -> infinity) the
// Jacobi-scaled operator gains eigenvalues of order H/Sigma_A and PCG stalls.
// Here the H part keeps its Jacobi diagonal D = diag(Hs + Sigma_x) while the
// constraint block is taken exactly:
//
//   P = D + A^T Sigma_A A,
//   P^{-1} r = D^{-1} r - D^{-1} A^T Sigma^{1/2} S^{-1} Sigma^{1/2} A D^{-1} r,
//   S = I + Sigma^{1/2} A D^{-1} A^T Sigma^{1/2}        (m x m, SPD, eigenvalues >= 1)
//
// (Sherman-Morrison-Woodbury).  S is formed densely without atomics, factored
// by a blocked Cholesky (its pivots cannot drop below 1), inverted through the
// triangular inverse, and applied as one dense symmetric matrix-vector product
// per PCG iteration.  Only the "strong" rows of A enter the dense block: a
// row i with M_ii = Sigma_i sum_j A_ij^2 / D_j below 1 changes P little and is
// folded into the Jacobi diagonal instead (D_j += Sigma_i A_ij^2), so the
// dense block has k <= m rows, about the number of active constraints late in
// the IPM.  Dense k x k storage is row-major with leading dimension ld = k
// rounded up to 32; padding rows/columns hold the identity.
#pragma once

#include "device_common.hpp"

namespace qpg {

constexpr int TS = 32;   // tile edge of the dense kernels

constexpr double kStrongRow = 1.0;   // M_ii threshold for the dense block

// M_ii = Sigma_i sum_j A_ij^2 / D_j (a wavefront per row) and the strong flag.
__global__ __launch_bounds__(256) void k_row_strength(const int* Ap, const int* Ac, const double* Av,
                                                      const double* D, const double* sigA, int m, int* flag,
                                                      const int* stop) {
    if (stop && *stop) return;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= m) return;
    double s = 0.0;
    for (int e = Ap[i] + lane; e < Ap[i + 1]; e += 64) {
        const double a = Av[e];
        s += a * a / D[Ac[e]];
    }
    s = group_sum<double, 64>(s);
    if (lane == 0) flag[i] = (sigA[i] * s >= kStrongRow) ? 1 : 0;
}

// Deterministic compaction by one block: pos[i] = rank of strong row i (or
// -1), idx[r] = i, count in *k_out.
__global__ __launch_bounds__(1024) void k_compact(const int* flag, int m, int* pos, int* idx, int* k_out,
                                                  const int* stop) {
    __shared__ int sh[1024];
    if (stop && *stop) return;
    int base = 0;
    for (int c0 = 0; c0 < m; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const int f = (i < m) ? flag[i] : 0;
        sh[threadIdx.x] = f;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
            const int v = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += v;
            __syncthreads();
        }
        if (i < m) {
            const int r = base + sh[threadIdx.x] - f;
            pos[i] = f ? r : -1;
            if (f) idx[r] = i;
        }
        const int tot = sh[1023];
        __syncthreads();
        base += tot;
    }
    if (threadIdx.x == 0) *k_out = base;
}

// Dw_j = dh_j + sum over weak rows i of Sigma_i A_ij^2 (rows of A^T, G = 16).
__global__ __launch_bounds__(256) void k_fold_weak(const int* Atp, const int* Atc, const double* Atv,
                                                   const double* sigA, const int* pos, const double* dh,
                                                   int n, double* Dw, const int* stop) {
    if (stop && *stop) return;
    const int j = blockIdx.x * 16 + (threadIdx.x >> 4);
    const int lane = threadIdx.x & 15;
    if (j >= n) return;
    double s = 0.0;
    for (int e = Atp[j] + lane; e < Atp[j + 1]; e += 16) {
        const int i = Atc[e];
        if (pos[i] < 0) {
            const double a = Atv[e];
            s += a * a * sigA[i];
        }
    }
    s = group_sum<double, 16>(s);
    if (lane == 0) Dw[j] = dh[j] + s;
}

// S = I + Sigma^{1/2} A_s D^{-1} A_s^T Sigma^{1/2} over the k strong rows: one
// wavefront per strong row r (row i = idx[r] of A), the row accumulated in
// LDS.  For each nonzero A_ij of row i (in column order), the strong entries
// of column j of A (row j of the stored A^T) are added with weight A_ij/D_j;
// within one column all row indices differ, so no two lanes touch the same
// LDS word in a step, and steps of one wavefront execute in order.
__global__ __launch_bounds__(64) void k_schur_form(const int* __restrict__ Ap, const int* __restrict__ Ac,
                                                  const double* __restrict__ Av, const int* __restrict__ Atp,
                                                  const int* __restrict__ Atc, const double* __restrict__ Atv,
                                                  const double* __restrict__ D, const double* __restrict__ sigA,
                                                  const int* __restrict__ pos, const int* __restrict__ idx, int k,
                                                  int ld, double* __restrict__ S, const int* stop) {
    extern __shared__ double acc[];
    if (stop && *stop) return;
    const int r = blockIdx.x;
    const int lane = threadIdx.x;
    for (int c = lane; c < ld; c += 64) acc[c] = 0.0;
    __syncthreads();
    if (r < k) {
        const int i = idx[r];
        const int e0 = Ap[i], e1 = Ap[i + 1];
        for (int e = e0; e < e1; ++e) {
            const int j = Ac[e];
            const double c = Av[e] / D[j];
            for (int f = Atp[j] + lane; f < Atp[j + 1]; f += 64) {
                const int q = pos[Atc[f]];
                if (q >= 0) acc[q] += c * Atv[f];
            }
        }
    }
    __syncthreads();
    const double si = (r < k) ? sqrt(sigA[idx[r]]) : 0.0;
    for (int c = lane; c < ld; c += 64) {
        double v = (r < k && c < k) ? si * sqrt(sigA[idx[c]]) * acc[c] : 0.0;
        if (c == r) v += 1.0;
        S[size_t(r) * ld + c] = v;
    }
}

// ---- blocked Cholesky S = L L^T, L overwriting the lower triangle -------------

// Diagonal tile b: unblocked Cholesky in LDS, then its inverse (forward
// substitution on the identity), stored in Linv[b].
__global__ __launch_bounds__(256) void k_chol_diag(double* S, int ld, int b, double* Linv, const int* stop) {
    __shared__ double a[TS][TS + 1];
    __shared__ double x[TS][TS + 1];
    if (stop && *stop) return;
    const int t = threadIdx.x;
    const size_t base = size_t(b) * TS * ld + size_t(b) * TS;
    for (int e = t; e < TS * TS; e += 256) a[e / TS][e % TS] = S[base + size_t(e / TS) * ld + e % TS];
    __syncthreads();
    for (int j = 0; j < TS; ++j) {
        if (t == 0) {
            const double d = a[j][j];
            // S has eigenvalues >= 1, so d >= 1 in exact arithmetic; the
            // guard only keeps a rounding accident from producing NaN.
            a[j][j] = (d > 0.0 && __builtin_isfinite(d)) ? sqrt(d) : 1.0;
        }
        __syncthreads();
        if (t > j && t < TS) a[t][j] /= a[j][j];
        __syncthreads();
        for (int e = t; e < TS * TS; e += 256) {
            const int r = e / TS, c = e % TS;
            if (c > j && r >= c) a[r][c] -= a[r][j] * a[c][j];
        }
        __syncthreads();
    }
    if (t < TS) {
        const int c = t;
        for (int r = 0; r < TS; ++r) {
            if (r < c) {
                x[r][c] = 0.0;
            } else {
                double s = (r == c) ? 1.0 : 0.0;
                for (int k = c; k < r; ++k) s -= a[r][k] * x[k][c];
                x[r][c] = s / a[r][r];
            }
        }
    }
    __syncthreads();
    for (int e = t; e < TS * TS; e += 256) {
        const int r = e / TS, c = e % TS;
        S[base + size_t(r) * ld + c] = (c <= r) ? a[r][c] : 0.0;
        Linv[size_t(b) * TS * TS + e] = x[r][c];
    }
}

// Panel: L_ib = S_ib L_bb^{-T} for row tiles i = b+1+blockIdx.x.
__global__ __launch_bounds__(256) void k_chol_panel(double* S, int ld, int b, const double* Linv, const int* stop) {
    __shared__ double a[TS][TS + 1];
    __shared__ double v[TS][TS + 1];
    if (stop && *stop) return;
    const int i = b + 1 + blockIdx.x;
    const int t = threadIdx.x;
    const size_t base = size_t(i) * TS * ld + size_t(b) * TS;
    for (int e = t; e < TS * TS; e += 256) {
        a[e / TS][e % TS] = S[base + size_t(e / TS) * ld + e % TS];
        v[e / TS][e % TS] = Linv[size_t(b) * TS * TS + e];
    }
    __syncthreads();
    for (int e = t; e < TS * TS; e += 256) {
        const int r = e / TS, c = e % TS;
        double s = 0.0;
        for (int k = 0; k <= c; ++k) s += a[r][k] * v[c][k];   // (L^-T)_{kc} = Linv_{ck}, zero for k > c
        S[base + size_t(r) * ld + c] = s;
    }
}

// Trailing update S_ij -= L_ib L_jb^T for b < j <= i.
__global__ __launch_bounds__(256) void k_chol_update(double* S, int ld, int b, const int* stop) {
    __shared__ double li[TS][TS + 1];
    __shared__ double lj[TS][TS + 1];
    if (stop && *stop) return;
    const int i = b + 1 + blockIdx.x, j = b + 1 + blockIdx.y;
    if (j > i) return;
    const int t = threadIdx.x;
    const size_t bi = size_t(i) * TS * ld + size_t(b) * TS;
    const size_t bj = size_t(j) * TS * ld + size_t(b) * TS;
    for (int e = t; e < TS * TS; e += 256) {
        li[e / TS][e % TS] = S[bi + size_t(e / TS) * ld + e % TS];
        lj[e / TS][e % TS] = S[bj + size_t(e / TS) * ld + e % TS];
    }
    __syncthreads();
    const size_t out = size_t(i) * TS * ld + size_t(j) * TS;
    for (int e = t; e < TS * TS; e += 256) {
        const int r = e / TS, c = e % TS;
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < TS; ++k) s += li[r][k] * lj[c][k];
        S[out + size_t(r) * ld + c] -= s;
    }
}

// ---- inverse: X = L^{-1} (lower), then S^{-1} = X^T X ---------------------------

// Row tile i of X: X_ib = -L_ii^{-1} sum_{k=b}^{i-1} L_ik X_kb for b = blockIdx.x < i.
// The diagonal tiles X_bb = L_bb^{-1} are written by k_trinv_diag.
__global__ __launch_bounds__(256) void k_trinv_row(const double* S, int ld, int i, const double* Linv,
                                                   double* X, const int* stop) {
    __shared__ double l[TS][TS + 1];
    __shared__ double xk[TS][TS + 1];
    if (stop && *stop) return;
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = b; k < i; ++k) {
        __syncthreads();
        const size_t sl = size_t(i) * TS * ld + size_t(k) * TS;
        const size_t sx = size_t(k) * TS * ld + size_t(b) * TS;
        for (int e = t; e < TS * TS; e += 256) {
            l[e / TS][e % TS] = S[sl + size_t(e / TS) * ld + e % TS];
            xk[e / TS][e % TS] = X[sx + size_t(e / TS) * ld + e % TS];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            const int r = e / TS, c = e % TS;
            double s = 0.0;
            for (int kk = 0; kk < TS; ++kk) s += l[r][kk] * xk[kk][c];
            acc[q] += s;
        }
    }
    __syncthreads();
    // y -> LDS, then X_ib = -Linv_ii * y
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q;
        xk[e / TS][e % TS] = acc[q];
        l[e / TS][e % TS] = Linv[size_t(i) * TS * TS + e];
    }
    __syncthreads();
    const size_t ox = size_t(i) * TS * ld + size_t(b) * TS;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q;
        const int r = e / TS, c = e % TS;
        double s = 0.0;
        for (int kk = 0; kk <= r; ++kk) s += l[r][kk] * xk[kk][c];
        X[ox + size_t(r) * ld + c] = -s;
    }
}

__global__ __launch_bounds__(256) void k_trinv_diag(const double* Linv, int ld, int T, double* X, const int* stop) {
    if (stop && *stop) return;
    const int b = blockIdx.x;
    if (b >= T) return;
    for (int e = threadIdx.x; e < TS * TS; e += 256)
        X[size_t(b) * TS * ld + size_t(b) * TS + size_t(e / TS) * ld + e % TS] = Linv[size_t(b) * TS * TS + e];
}

// Sinv tile (I, J), J <= I: sum_{K >= I} X_KI^T X_KJ; written to (I,J) and (J,I).
__global__ __launch_bounds__(256) void k_inv_product(const double* X, int ld, int T, double* Sinv, const int* stop) {
    __shared__ double xi[TS][TS + 1];
    __shared__ double xj[TS][TS + 1];
    if (stop && *stop) return;
    const int I = blockIdx.x, J = blockIdx.y;
    if (J > I) return;
    const int t = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int K = I; K < T; ++K) {
        __syncthreads();
        const size_t a = size_t(K) * TS * ld + size_t(I) * TS;
        const size_t c = size_t(K) * TS * ld + size_t(J) * TS;
        for (int e = t; e < TS * TS; e += 256) {
            xi[e / TS][e % TS] = X[a + size_t(e / TS) * ld + e % TS];
            xj[e / TS][e % TS] = X[c + size_t(e / TS) * ld + e % TS];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            const int r = e / TS, cc = e % TS;
            double s = 0.0;
            for (int k = 0; k < TS; ++k) s += xi[k][r] * xj[k][cc];
            acc[q] += s;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q;
        const int r = e / TS, c = e % TS;
        Sinv[(size_t(I) * TS + r) * ld + size_t(J) * TS + c] = acc[q];
        if (I != J) Sinv[(size_t(J) * TS + c) * ld + size_t(I) * TS + r] = acc[q];
    }
}

}  // namespace qpg
