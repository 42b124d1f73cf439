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

#include "ipm_kernels.hpp"

namespace qpg {

constexpr int TS = TS_PREC;   // tile edge of the dense kernels (the preconditioner kernels use the same)

constexpr double kStrongRow = 1.0;   // M_ii threshold for the dense block

// M_ii = Sigma_i sum_j A_ij^2 / D_j (a wavefront per row), kept in mii, and
// the strong flag.
__global__ __launch_bounds__(256) void k_row_strength(const int* Ap, const int* Ac, const double* Av,
                                                      const double* D, const double* sigA, int m, int* flag,
                                                      double* mii, const int* stop) {
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
    if (lane == 0) {
        const double mi = sigA[i] * s;
        mii[i] = mi;
        flag[i] = (mi >= kStrongRow) ? 1 : 0;
    }
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

// Per strong row r, what the per-iteration kernels read in one load: the
// range of row idx[r] in A (ext[2r], ext[2r+1]) and sqrt(Sigma) of it (sq[r]);
// rows r in [k, rows) get an empty range and 0.  With tau > 0 the block
// takes Sigma_i min(1, tau / M_ii) in place of Sigma_i, so that no diagonal
// entry of S exceeds 1 + tau: the capped block, the preconditioner used once
// the exact one has lost definiteness to rounding (its correction cancels
// D^-1 in the row space of the active rows when Sigma / D passes about 1e8).
__global__ __launch_bounds__(256) void k_strong_rows(const int* Ap, const int* idx, const double* sigA,
                                                     const double* mii, double tau, const int* kdev, int rows,
                                                     int* ext, double* sq, const int* stop) {
    if (stop && *stop) return;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    const int k = *kdev;
    int e0 = 0, e1 = 0;
    double q = 0.0;
    if (r < k) {
        const int i = idx[r];
        e0 = Ap[i];
        e1 = Ap[i + 1];
        const double sig = sigA[i];
        q = sqrt((tau > 0.0 && mii[i] > tau) ? sig * (tau / mii[i]) : sig);
    }
    ext[2 * r] = e0;
    ext[2 * r + 1] = e1;
    sq[r] = q;
}

// Dw_j = dh_j + sum over weak rows i of Sigma_i A_ij^2 (rows of A^T, G = 16),
// and column j's strong entries compacted in row order: their ranks and
// values at scr/scv[Atp[j] ...], their count in scnt[j] (for k_schur_form).
__global__ __launch_bounds__(256) void k_fold_weak(const int* Atp, const int* Atc, const double* Atv,
                                                   const double* sigA, const int* pos, const double* dh,
                                                   int n, double* Dw, int* scr, double* scv, int* scnt,
                                                   const int* stop) {
    if (stop && *stop) return;
    const int j = blockIdx.x * 16 + (threadIdx.x >> 4);
    const int lane = threadIdx.x & 15;
    const int gshift = threadIdx.x & 48;   // this group's first lane in the wavefront
    if (j >= n) return;                    // whole groups
    const int e0 = Atp[j], e1 = Atp[j + 1];
    double s = 0.0;
    int cnt = 0;
    for (int base = e0; base < e1; base += 16) {   // trip count uniform over the group
        const int e = base + lane;
        const bool in = e < e1;
        const int i = in ? Atc[e] : 0;
        const int r = in ? pos[i] : -1;
        const double a = in ? Atv[e] : 0.0;
        if (in && r < 0) s += a * a * sigA[i];
        const unsigned mask = unsigned(__ballot(in && r >= 0) >> gshift) & 0xFFFFu;
        if (in && r >= 0) {
            const int at = e0 + cnt + __popc(mask & ((1u << lane) - 1u));
            scr[at] = r;
            scv[at] = a;
        }
        cnt += __popc(mask);
    }
    s = group_sum<double, 16>(s);
    if (lane == 0) {
        Dw[j] = dh[j] + s;
        scnt[j] = cnt;
    }
}

// S = I + Sigma^{1/2} A_s D^{-1} A_s^T Sigma^{1/2} over the k strong rows: one
// workgroup of NW wavefronts per strong row r (row i = idx[r] of A), the
// wavefronts taking contiguous parts of the row's nonzeros, each with its own
// copy of the output row in LDS.  For each nonzero A_ij (in column order), the
// strong entries of column j of A (compacted by k_fold_weak) are added with
// weight A_ij/D_j; within one column all row indices differ, so no two lanes
// touch the same LDS word in a step, and steps of one wavefront execute in
// order.  The NW copies are summed in a fixed order at the end.
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_schur_form(const int* __restrict__ Ap, const int* __restrict__ Ac,
                                                       const double* __restrict__ Av, const int* __restrict__ Atp,
                                                       const int* __restrict__ scr, const double* __restrict__ scv,
                                                       const int* __restrict__ scnt,
                                                       const double* __restrict__ D, const double* __restrict__ sq,
                                                       const int* __restrict__ idx,
                                                       int k, int ld, double* __restrict__ S, const int* stop) {
    extern __shared__ double acc_all[];
    if (stop && *stop) return;
    const int r = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* acc = acc_all + size_t(w) * ld;
    for (int c = threadIdx.x; c < NW * ld; c += NW * 64) acc_all[c] = 0.0;
    __syncthreads();
    if (r < k) {
        const int i = idx[r];
        const int a0 = Ap[i], len = Ap[i + 1] - a0;
        const int per = (len + NW - 1) / NW;
        const int e0 = a0 + min(len, w * per), e1 = a0 + min(len, (w + 1) * per);
        // Batches of 8 nonzeros: every load of a batch (column ids, weights,
        // the first 64 strong entries of each column, compacted by
        // k_fold_weak: ranks and values) is issued before the adds, which then
        // run in the original order.
        constexpr int B = 8;
        for (int e = e0; e < e1; e += B) {
            int jv[B], f0[B], f1[B], q[B];
            double c[B], av[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int ee = min(e + u, e1 - 1);
                jv[u] = Ac[ee];
                c[u] = (e + u < e1) ? Av[ee] / D[jv[u]] : 0.0;
                f0[u] = Atp[jv[u]];
                f1[u] = (e + u < e1) ? f0[u] + scnt[jv[u]] : f0[u];
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int f = f0[u] + lane;
                const bool in = f < f1[u];
                const int ff = in ? f : 0;   // a valid index when idle (A has nonzeros when k > 0)
                av[u] = in ? scv[ff] : 0.0;
                q[u] = in ? scr[ff] : -1;
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                if (q[u] >= 0) acc[q[u]] += c[u] * av[u];
                for (int f = f0[u] + 64 + lane; f < f1[u]; f += 64) acc[scr[f]] += c[u] * scv[f];   // columns with > 64
            }
        }
    }
    __syncthreads();
    // sqrt(Sigma) of the strong rows from the per-row table (k_strong_rows,
    // the same sqrt of the same value)
    const double si = (r < k) ? sq[r] : 0.0;
    for (int c = threadIdx.x; c < ld; c += NW * 64) {
        double t = acc_all[c];
#pragma unroll
        for (int w2 = 1; w2 < NW; ++w2) t += acc_all[size_t(w2) * ld + c];
        double v = (r < k && c < k) ? si * sq[c] * t : 0.0;
        if (c == r) v += 1.0;
        S[size_t(r) * ld + c] = v;
    }
}

// ---- inverse by a block Gauss-Jordan sweep --------------------------------------
//
// For each pivot tile b (TS x TS):  P = S_bb^{-1};  S_bj <- P S_bj;
// S_ij <- S_ij - S_ib (P S_bj);  S_ib <- -S_ib P;  S_bb <- P  (i, j != b).
// After the last pivot S holds S^{-1}.  Every pivot is a Schur complement of
// S, and S has eigenvalues >= 1, so every pivot tile has eigenvalues >= 1: no
// pivoting is needed.
//
// One launch per pivot (k_gj_step), reading the matrix of the previous step
// and writing the next one (two buffers, so no tile waits for another): a
// wavefront per 32 x 32 tile forms Q_j = P S_bj and its update on FP64 MFMA
// 16x16x4, and the workgroup holding tile (b+1, b+1) -- dispatched first --
// inverts that tile once it is final, so P for the next step is ready when
// the launch ends.  The step is latency-bound at these sizes (~10^9 flops per
// inversion); one launch per pivot keeps the serial chain at T launches.

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
// Row / column of element r of 16 x 16 block (ra, cb) in lane l.
__device__ __forceinline__ int res_row(int ra, int l, int r) { return 16 * ra + (l >> 4) + 4 * r; }
__device__ __forceinline__ int res_col(int cb, int l) { return 16 * cb + (l & 15); }

// 1/v for v >= 1 (pivots of S): hardware reciprocal estimate refined by two
// Newton steps (r <- r + r(1 - v r)), accurate to about one ulp; a pivot that
// is not a finite number >= some tiny positive value maps to 1 so a rounding
// accident cannot spread NaN through the preconditioner.
__device__ __forceinline__ double pivot_recip(double v) {
    if (!(v > 0.0 && __builtin_isfinite(v))) return 1.0;
    double r = __builtin_amdgcn_rcp(v);
    r = fma(r, fma(-v, r, 1.0), r);
    r = fma(r, fma(-v, r, 1.0), r);
    return r;
}

// Gauss-Jordan inversion of a TS x TS tile in LDS by the whole workgroup
// (256 threads).  Thread t keeps entries (t/TS + 8q, t%TS), q < 4, in
// registers; each elimination step needs only the current pivot row and
// pivot column, which their owners publish in double-buffered LDS arrays, so
// a step is one barrier.  The step is branch-free: all its LDS reads are
// issued together and selects replace the special cases (pivot row, pivot
// column).
__device__ __forceinline__ void lds_gj_invert(double (*a)[TS + 1]) {
    __shared__ double rowbuf[2][TS], colbuf[2][TS];
    const int c = threadIdx.x % TS, r0 = threadIdx.x / TS;
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = a[r0 + 8 * q][c];
    if (r0 == 0) rowbuf[0][c] = v[0];
    if (c == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) colbuf[0][r0 + 8 * q] = v[q];
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < TS; ++jj) {
        const int cur = jj & 1, nxt = cur ^ 1;
        const double pv = rowbuf[cur][jj];
        const double rc = rowbuf[cur][c];
        double f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) f[q] = colbuf[cur][r0 + 8 * q];
        const double pinv = pivot_recip(pv);
        const double rowj = (c == jj) ? pinv : rc * pinv;
        // new entry: rowj on the pivot row; -f*pinv on the pivot column;
        // v - f*rowj elsewhere
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double base = (c == jj) ? 0.0 : v[q];
            const double nv = fma(-f[q], rowj, base);
            v[q] = (r0 + 8 * q == jj) ? rowj : nv;
        }
        if (jj + 1 < TS) {   // publish row and column jj+1 of the updated tile
            if (r0 == ((jj + 1) & 7)) rowbuf[nxt][c] = v[(jj + 1) >> 3];
            if (c == jj + 1)
#pragma unroll
                for (int q = 0; q < 4; ++q) colbuf[nxt][r0 + 8 * q] = v[q];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) a[r0 + 8 * q][c] = v[q];
    __syncthreads();
}

// P (in LDS) to both operand layouts: P[0..1024) left, P[1024..2048) right.
__device__ __forceinline__ void store_pivot(const double (*a)[TS + 1], double* P) {
    for (int e = threadIdx.x; e < TS * TS; e += 256) {
        const int r = e / TS, c = e % TS;
        P[frag_left(r, c)] = a[r][c];
        P[TS * TS + frag_right(r, c)] = a[r][c];
    }
}

// Inverse of the first pivot tile S_00 into P (one workgroup).
__global__ __launch_bounds__(256) void k_gj_pivot0(const double* S, int ld, double* P, const int* stop) {
    __shared__ double a[TS][TS + 1];
    if (stop && *stop) return;
    for (int e = threadIdx.x; e < TS * TS; e += 256) a[e / TS][e % TS] = S[size_t(e / TS) * ld + e % TS];
    __syncthreads();
    lds_gj_invert(a);
    store_pivot(a, P);
}

// New value of tile (i, j) at pivot step b, in the result layout (o[ra][cb]
// element r is entry (res_row(ra, l, r), res_col(cb, l))); x: this
// wavefront's LDS exchange buffer (TS*TS doubles).
__device__ __forceinline__ void tile_step(const double* __restrict__ So, int ld, int b, int i, int j,
                                          const double* __restrict__ Pin, double* x, int l, f64x4 (&o)[2][2]) {
    const double* P_left = Pin;
    const double* P_right = Pin + TS * TS;
    if (i == b && j == b) {          // S_bb <- P
#pragma unroll
        for (int ra = 0; ra < 2; ++ra)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) o[ra][cb][r] = P_left[frag_left(res_row(ra, l, r), res_col(cb, l))];
        return;
    }
    f64x4 acc[2][2];
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[ra][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
    const double* c = So + size_t(i) * TS * ld + size_t(b) * TS;   // C_i = S_ib (left operand)
    if (j == b) {                    // S_ib <- -C_i P
#pragma unroll
        for (int s = 0; s < TS / 4; ++s) {
            const double a0 = c[size_t(l & 15) * ld + 4 * s + (l >> 4)];
            const double a1 = c[size_t(16 + (l & 15)) * ld + 4 * s + (l >> 4)];
            const double b0 = P_right[(0 * 8 + s) * 64 + l], b1 = P_right[(1 * 8 + s) * 64 + l];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
#pragma unroll
        for (int ra = 0; ra < 2; ++ra)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) o[ra][cb] = -acc[ra][cb];
        return;
    }
    // Q_j = P S_bj
    const double* sbj = So + size_t(b) * TS * ld + size_t(j) * TS;
#pragma unroll
    for (int s = 0; s < TS / 4; ++s) {
        const double a0 = P_left[(0 * 8 + s) * 64 + l], a1 = P_left[(1 * 8 + s) * 64 + l];
        const double b0 = sbj[size_t(4 * s + (l >> 4)) * ld + (l & 15)];
        const double b1 = sbj[size_t(4 * s + (l >> 4)) * ld + 16 + (l & 15)];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (i == b) {                    // S_bj <- Q_j
#pragma unroll
        for (int ra = 0; ra < 2; ++ra)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) o[ra][cb] = acc[ra][cb];
        return;
    }
    // S_ij <- S_ij - C_i Q_j, Q_j to right-operand order through LDS (the
    // wavefront's own LDS writes precede its reads in order)
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) x[res_row(ra, l, r) * TS + res_col(cb, l)] = acc[ra][cb][r];
    f64x4 u[2][2];
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) u[ra][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < TS / 4; ++s) {
        const double a0 = c[size_t(l & 15) * ld + 4 * s + (l >> 4)];
        const double a1 = c[size_t(16 + (l & 15)) * ld + 4 * s + (l >> 4)];
        const double b0 = x[(4 * s + (l >> 4)) * TS + (l & 15)];
        const double b1 = x[(4 * s + (l >> 4)) * TS + 16 + (l & 15)];
        u[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, u[0][0], 0, 0, 0);
        u[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, u[0][1], 0, 0, 0);
        u[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, u[1][0], 0, 0, 0);
        u[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, u[1][1], 0, 0, 0);
    }
    const double* sij = So + size_t(i) * TS * ld + size_t(j) * TS;
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                o[ra][cb][r] = sij[size_t(res_row(ra, l, r)) * ld + res_col(cb, l)] - u[ra][cb][r];
}

// Pivot step b: So (matrix after step b-1) -> Sn; Pin = S_bb^{-1} in both
// operand layouts.  When b+1 < T, workgroup 0 (dispatched first) recomputes
// only tile (b+1, b+1) and writes its inverse to Pout; workgroups 1.. each
// update a 2 x 2 group of tiles of the lower triangle (and its mirror), a
// wavefront per tile.  Grid: 1 + gx(gx+1)/2 workgroups, gx = (T+1)/2.
__global__ __launch_bounds__(256) void k_gj_step(const double* __restrict__ So, double* __restrict__ Sn, int ld,
                                                 int T, int b, const double* __restrict__ Pin,
                                                 double* __restrict__ Pout, const int* stop) {
    __shared__ double xch[4][TS * TS];    // per wavefront: Q_j from result to right-operand order
    __shared__ double piv[TS][TS + 1];
    if (stop && *stop) return;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int nb = b + 1;
    const int lead = nb < T ? 1 : 0;
    if (lead && blockIdx.x == 0) {   // next pivot: tile (nb, nb) after this step, inverted
        if (w == 0) {
            f64x4 o[2][2];
            tile_step(So, ld, b, nb, nb, Pin, xch[0], l, o);
#pragma unroll
            for (int ra = 0; ra < 2; ++ra)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) piv[res_row(ra, l, r)][res_col(cb, l)] = o[ra][cb][r];
        }
        __syncthreads();
        lds_gj_invert(piv);
        store_pivot(piv, Pout);
        return;
    }
    // Groups of the lower triangle only (by >= bx, L = by(by+1)/2 + bx): the
    // sweep keeps S symmetric up to sign -- with K the blocks swept so far
    // (0..b after this step), S_ji = -S_ij^T when exactly one of i, j is in K,
    // else S_ji = S_ij^T -- so a group below the diagonal computes its four
    // tiles (all with i > j) and writes each also transposed, with that sign,
    // to (j, i); groups on the diagonal compute all four tiles.
    const int L = int(blockIdx.x) - lead;
    int by = int((sqrt(8.0 * L + 1.0) - 1.0) * 0.5);
    while ((by + 1) * (by + 2) / 2 <= L) ++by;
    while (by * (by + 1) / 2 > L) --by;
    const int bx = L - by * (by + 1) / 2;
    const int i = 2 * by + (w >> 1), j = 2 * bx + (w & 1);
    if (i >= T || j >= T) return;    // whole wavefronts; no barrier follows
    f64x4 o[2][2];
    tile_step(So, ld, b, i, j, Pin, xch[w], l, o);
    double* dst = Sn + size_t(i) * TS * ld + size_t(j) * TS;
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[size_t(res_row(ra, l, r)) * ld + res_col(cb, l)] = o[ra][cb][r];
    if (by != bx) {
        const double sg = (j <= b && b < i) ? -1.0 : 1.0;
        double* dtr = Sn + size_t(j) * TS * ld + size_t(i) * TS;
#pragma unroll
        for (int ra = 0; ra < 2; ++ra)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    dtr[size_t(res_col(cb, l)) * ld + res_row(ra, l, r)] = sg * o[ra][cb][r];
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
