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
// (Sherman-Morrison-Woodbury).  S is formed densely without atomics, inverted
// in place by a block Gauss-Jordan sweep (its pivots cannot drop below 1), and
// applied as one dense symmetric matrix-vector product per PCG iteration.  Only the "strong" rows of A enter the dense block: a
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

// ---- in-place inverse by a block Gauss-Jordan sweep ------------------------------
//
// For each pivot tile b (TS x TS):  P = S_bb^{-1};  S_bj <- P S_bj;
// S_ij <- S_ij - S_ib (P S_bj);  S_ib <- -S_ib P;  S_bb <- P  (i, j != b).
// After the last pivot S holds S^{-1}.  Every pivot is a Schur complement of
// S, and S has eigenvalues >= 1, so every pivot tile has eigenvalues >= 1: no
// pivoting is needed.  A step is two launches:
//   k_gj_panel  (T blocks)   block j inverts the pivot tile in LDS (every
//               block redundantly: no single-workgroup launch on the critical
//               path), forms Q_j = P S_bj (Q_b = P) and copies the old column
//               tile C_j = S_jb; both go to panel buffers in the operand
//               layouts of the matrix cores;
//   k_gj_apply  (T x T tiles, a wavefront per tile)  S_ij <- S_ij - C_i Q_j,
//               S_ib <- -C_i Q_b, S_bj <- Q_j, the products on FP64 MFMA
//               16x16x4.
// The dense contraction (T^3 tile products per inversion) runs on the matrix
// cores; the panels make every tile of a step independent of the others.

using f64x4 = double __attribute__((ext_vector_type(4)));

// Operand layouts of v_mfma_f64_16x16x4f64 for a 32 x 32 tile, 1024 doubles:
//   left operand (A, 16 x 4 per step):  X[16a + l%16][4s + l/16] at ((a*8 + s)*64 + l)
//   right operand (B, 4 x 16 per step): X[4s + l/16][16c + l%16] at ((c*8 + s)*64 + l)
// and the result (16 x 16 per block): lane l, element r holds
//   D[l/16 + 4r][l%16].
__device__ __forceinline__ int frag_left(int row, int col) {
    return ((row >> 4) * 8 + (col >> 2)) * 64 + (row & 15) + 16 * (col & 3);
}
__device__ __forceinline__ int frag_right(int row, int col) {
    return ((col >> 4) * 8 + (row >> 2)) * 64 + (col & 15) + 16 * (row & 3);
}

// C (TS x TS, in registers: element e = t + 256q) = A * B for LDS tiles.
__device__ __forceinline__ void tile_mm(const double (*a)[TS + 1], const double (*b)[TS + 1], double out[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q;
        const int r = e / TS, c = e % TS;
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < TS; ++k) s += a[r][k] * b[k][c];
        out[q] = s;
    }
}

__device__ __forceinline__ void tile_load(double (*dst)[TS + 1], const double* S, int ld, int ti, int tj) {
    const size_t base = size_t(ti) * TS * ld + size_t(tj) * TS;
    for (int e = threadIdx.x; e < TS * TS; e += 256) dst[e / TS][e % TS] = S[base + size_t(e / TS) * ld + e % TS];
}

// Step b, panels: block j of T.  Qf, Cf: T tiles of 1024 doubles each.
__global__ __launch_bounds__(256) void k_gj_panel(const double* S, int ld, int b, double* Qf, double* Cf,
                                                  const int* stop) {
    __shared__ double a[TS][TS + 1];
    __shared__ double sb[TS][TS + 1];
    if (stop && *stop) return;
    const int j = blockIdx.x;
    tile_load(a, S, ld, b, b);
    if (j != b) tile_load(sb, S, ld, b, j);
    __syncthreads();
    // Gauss-Jordan inversion of the pivot tile in LDS, four entries per thread
    for (int jj = 0; jj < TS; ++jj) {
        const double pv = a[jj][jj];
        double f[4], ajc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q;
            f[q] = a[e / TS][jj];
            ajc[q] = a[jj][e % TS];
        }
        __syncthreads();
        // pivots are >= 1 in exact arithmetic; the guard keeps a rounding
        // accident from spreading NaN through the preconditioner
        const double pinv = (pv > 0.0 && __builtin_isfinite(pv)) ? 1.0 / pv : 1.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int r = e / TS, c = e % TS;
            const double rowj = (c == jj) ? pinv : ajc[q] * pinv;
            if (r == jj) a[r][c] = rowj;
            else a[r][c] = (c == jj) ? -f[q] * pinv : a[r][c] - f[q] * rowj;
        }
        __syncthreads();
    }
    double* q = Qf + size_t(j) * TS * TS;
    if (j == b) {
        for (int e = threadIdx.x; e < TS * TS; e += 256) q[frag_right(e / TS, e % TS)] = a[e / TS][e % TS];
    } else {
        double out[4];
        tile_mm(a, sb, out);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = threadIdx.x + 256 * k;
            q[frag_right(e / TS, e % TS)] = out[k];
        }
        // old column tile S_jb, left-operand layout
        double* c = Cf + size_t(j) * TS * TS;
        const size_t base = size_t(j) * TS * ld + size_t(b) * TS;
        for (int e = threadIdx.x; e < TS * TS; e += 256)
            c[frag_left(e / TS, e % TS)] = S[base + size_t(e / TS) * ld + e % TS];
    }
}

// Step b, update: a wavefront per tile (i, j); blocks of four wavefronts take
// 2 x 2 tiles.  Grid ((T+1)/2, (T+1)/2).
__global__ __launch_bounds__(256) void k_gj_apply(double* S, int ld, int T, int b, const double* Qf,
                                                  const double* Cf, const int* stop) {
    if (stop && *stop) return;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int i = 2 * blockIdx.y + (w >> 1), j = 2 * blockIdx.x + (w & 1);
    if (i >= T || j >= T) return;   // whole wavefronts
    double* tile = S + size_t(i) * TS * ld + size_t(j) * TS;
    const double* q = Qf + size_t(j) * TS * TS;
    if (i == b) {   // new pivot row: S_bj = Q_j
#pragma unroll
        for (int ra = 0; ra < 2; ++ra)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * ra + (l >> 4) + 4 * r, col = 16 * cb + (l & 15);
                    tile[size_t(row) * ld + col] = q[frag_right(row, col)];
                }
        return;
    }
    const double* c = Cf + size_t(i) * TS * TS;
    f64x4 acc[2][2];
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[ra][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < TS / 4; ++s) {
        const double a0 = c[(0 * 8 + s) * 64 + l], a1 = c[(1 * 8 + s) * 64 + l];
        const double b0 = q[(0 * 8 + s) * 64 + l], b1 = q[(1 * 8 + s) * 64 + l];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * ra + (l >> 4) + 4 * r, col = 16 * cb + (l & 15);
                double* dst = tile + size_t(row) * ld + col;
                *dst = (j == b) ? -acc[ra][cb][r] : *dst - acc[ra][cb][r];
            }
}

// Sinv = (S + S^T)/2: the sweep's result is symmetric up to rounding; PCG
// wants an exactly symmetric preconditioner.
__global__ __launch_bounds__(256) void k_symmetrize(const double* S, int ld, double* Sinv, const int* stop) {
    if (stop && *stop) return;
    const size_t N = size_t(ld) * ld;
    for (size_t e = size_t(blockIdx.x) * 256 + threadIdx.x; e < N; e += size_t(gridDim.x) * 256) {
        const size_t r = e / ld, c = e % ld;
        Sinv[e] = 0.5 * (S[e] + S[c * ld + r]);
    }
}

}  // namespace qpg
