// Kernels of one IPM iteration (Algorithm 1 of the paper, all on the device).
//
// Constraint groups (bounds kept apart from the rows of A, Section 4):
//   lx: x_j >= lo_j        ux: -x_j >= -hi_j
//   lA: (Ax)_i >= lo_i     uA: -(Ax)_i >= -hi_i
// Each present side has a slack s > 0 and a multiplier lambda > 0; an absent
// side (infinite bound) is stored as s = 1, lambda = 0 and is skipped by every
// norm, ratio test and sum.  Residuals follow eq. (perturbed_KKT) with the
// s_u sign of eq. (qp_barrier):
//   r_H = H x + p - sum_g G_g^T lambda_g,  r_g = G_g x - s_g - c_g,
//   r_c = lambda_g s_g - mu.
// The direction solves the condensed form of eq. (newton_system):
//   (H + Sigma_x + A^T Sigma_A A) dx
//       = -(H x + p) + sum_g G_g^T (mu/s_g - Sigma_g r_g),   Sigma_g = lambda_g/s_g,
// then ds_g = G_g dx + r_g and dlambda_g = -lambda_g + mu/s_g - Sigma_g ds_g.
#pragma once

#include "device_common.hpp"

namespace qpg {

__device__ __forceinline__ bool finite_d(double v) { return __builtin_isfinite(v); }

__device__ __forceinline__ bool pcg_stopped_raw(const Flags* fl) {
    return fl && (fl->pcg_converged | fl->pcg_breakdown | fl->pcg_capped | fl->ipm_done);
}

// Stop test that every thread of the block answers the same way: thread 0
// reads the flags once and broadcasts through LDS.  (Block 0 of a kernel may
// set a flag while other blocks start, so per-thread reads could disagree
// inside one block and split it around a barrier.)
__device__ __forceinline__ bool block_flag(bool v_thread0) {
    __shared__ int s_flag;
    if (threadIdx.x == 0) s_flag = v_thread0 ? 1 : 0;
    __syncthreads();
    const bool r = s_flag != 0;
    __syncthreads();
    return r;
}
__device__ __forceinline__ bool pcg_stopped(const Flags* fl) {
    return block_flag(threadIdx.x == 0 && pcg_stopped_raw(fl));
}
__device__ __forceinline__ bool ipm_finished(const Flags* fl) {
    return block_flag(threadIdx.x == 0 && fl->ipm_done);
}
// Stop test for kernels that never write the flags: they cannot change while
// such a kernel runs, so every thread reads them directly (one uniform load,
// no barrier), and the read overlaps the kernel's first index loads.
__device__ __forceinline__ bool pcg_stopped_ro(const Flags* fl) { return pcg_stopped_raw(fl); }

// ==========================================================================
// Operator kernels (one PCG product q = K p)
// ==========================================================================

// The doubly augmented system of eq. (2x2_augmented), with B = [A_L; -A_U]
// (rows of A with a finite lower / upper side) and D = diag(s/lambda) of those
// rows, acts on N = n + 2m vectors (x part, then one entry per row and side;
// an absent side has a zero row of B, D = 1 and stays zero):
//   y_x = (Q + 2 B^T D^-1 B) p_x + B^T p_lambda
//       = H p_x + Sigma_x p_x + A^T (2 Sigma_A (A p_x) + p_l - p_u),
//   y_l = (A p_x) + D_l p_l,   y_u = -(A p_x) + D_u p_u,
// Sigma_A = Sigma_lA + Sigma_uA.  The rows of A carry the lambda block: given
// (A p_x)_i they form u_i (the vector A^T multiplies) and y_l, y_u.
struct AugRows {
    const double* dlu;     // D_l (m) then D_u (m); 0 marks an absent side; null: condensed system
    double* q;             // output of the product (N): the lambda block at q + n
    double* part;          // PCG product: one p^T q partial per row (its lambda block), may be null
    int n;
};

// Row i of the lambda block: a = (A p_x)_i, g the product's gathered vector
// (N entries; p2 non-null in a PCG product, where the new direction's lambda
// entries are stored back).  Returns u_i.
template <typename GV>
__device__ __forceinline__ double aug_row(const AugRows& a, int m, int i, double a_i, double sig, const GV& g,
                                          double* p2) {
    const double pl = g(a.n + i), pu = g(a.n + m + i);
    const double Dl = a.dlu[i], Du = a.dlu[m + i];
    if (p2) {
        p2[a.n + i] = pl;
        p2[a.n + m + i] = pu;
    }
    const double ql = Dl > 0.0 ? a_i + Dl * pl : 0.0;
    const double qu = Du > 0.0 ? -a_i + Du * pu : 0.0;
    a.q[a.n + i] = ql;
    a.q[a.n + m + i] = qu;
    if (a.part) a.part[i] = pl * ql + pu * qu;
    return 2.0 * sig * a_i + (Dl > 0.0 ? pl : 0.0) - (Du > 0.0 ? pu : 0.0);
}

template <typename VT>
struct FwdArgs {
    const int* Jp; const int* Jc; const VT* Jv; const double* W; int nJ;
    const int* Ap; const int* Ac; const double* Av; int m;
    const double* x;       // gathered vector (n)
    const double* p2;      // PCG: the gathered vector is x + beta*p2 (beta in sc); null: x
    const PcgScal* sc;
    double* t;             // W .* (J x)        (nJ)
    double* u;             // sigA .* (A x)     (m), or A x when sigA is null
    const double* sigA;
    int nbJ;               // blocks of the grid that work on rows of J
    const Flags* fl;
    AugRows aug;           // doubly augmented system: the lambda block (aug.dlu null: condensed)
};

__device__ __forceinline__ Gather make_gather(const double* x, const double* p2, const PcgScal* sc) {
    return Gather{x, p2, p2 ? sc->beta : 0.0};
}

// Rows of A in the forward pass: a full wavefront per row, four rows per
// block ab.
template <typename VT>
__device__ __forceinline__ void fwd_a_rows(const FwdArgs<VT>& a, const Gather& g, int ab) {
    const int row = ab * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row < a.m) {
        double s = row_dot_lane_g<64, double, double>(a.Ap, a.Ac, a.Av, g, row, lane);
        s = group_sum<double, 64>(s);
        if (lane == 0) {
            if (a.aug.dlu) a.u[row] = aug_row(a.aug, a.m, row, s, a.sigA[row], g, const_cast<double*>(a.p2));
            else a.u[row] = a.sigA ? a.sigA[row] * s : s;
        }
    }
}

// t = W .* (J x) and u = Sigma_A .* (A x).  Rows of J: G lanes per row; rows
// of A: a full wavefront per row.
template <int G, typename VT, typename AT>
__global__ __launch_bounds__(kBlock) void k_op_fwd(FwdArgs<VT> a) {
    if (pcg_stopped_ro(a.fl)) return;
    const Gather g = make_gather(a.x, a.p2, a.sc);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    if (b < a.nbJ) {
        constexpr int RPB = kBlock / G;
        const int row = b * RPB + threadIdx.x / G;
        const int lane = threadIdx.x % G;
        if (row < a.nJ) {   // whole groups are uniform: inactive groups skip together
            const AT s = canon_sum<G, AT>(a.Jp[row], a.Jp[row + 1], lane,
                                          [&](int e) { return mul_nc(cvt<AT>(a.Jv[e]), AT(g(a.Jc[e]))); });
            if (lane == 0) a.t[row] = a.W[row] * double(s);
        }
    } else {
        fwd_a_rows(a, g, b - a.nbJ);
    }
}

// The forward pass over nonzero-balanced blocks of rows of J, for rows short
// against the 64 x 8 terms a wavefront pass of canon_sum spans (where most of
// a G-lane group's clamped loads would repeat an address).  Block b takes the
// rows rb[b].x .. rb[b+1].x - 1, whose nonzeros rb[b].y .. rb[b+1].y - 1 are
// at most kStreamNnz (and the rows at most kStreamRows), or a single longer
// row.  Its threads load the nonzeros contiguously (every load useful and
// coalesced) and store the products in LDS; then a wavefront per row adds
// them in the order canon_sum defines (virtual lane v adds the row's terms
// v, v+64, ... in order, then the butterfly), so t has the same bits as with
// any lane count.  A longer row is staged in chunks of kStreamNnz terms
// (multiples of 64, so each lane keeps its virtual lane across chunks).
constexpr int kStreamNnz = 2048;
constexpr int kStreamRows = 256;
template <bool NT, typename VT, typename AT>
__device__ __forceinline__ void stream_stage(const FwdArgs<VT>& a, const Gather& g, int e0, int e1, AT* prod) {
    constexpr int PER = kStreamNnz / kBlock;
    if (e1 <= e0) return;
    int c[PER];
    AT v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = min(e0 + int(threadIdx.x) + u * kBlock, e1 - 1);   // clamped: a valid address
        c[u] = load_val<NT>(a.Jc + e);
        v[u] = cvt<AT>(load_val<NT>(a.Jv + e));
    }
    double xv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) xv[u] = g(c[u]);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int k = int(threadIdx.x) + u * kBlock;
        if (e0 + k < e1) prod[k] = mul_nc(v[u], AT(xv[u]));
    }
}
template <typename VT, typename AT, bool NT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_op_fwd_stream(FwdArgs<VT> a, const int2* rb) {
    __shared__ AT prod[kStreamNnz];
    __shared__ int rp[kStreamRows + 1];
    __shared__ double wl[kStreamRows];
    if (pcg_stopped_ro(a.fl)) return;
    const Gather g = make_gather(a.x, a.p2, a.sc);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    if (b >= a.nbJ) {
        fwd_a_rows(a, g, b - a.nbJ);
        return;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int2 lo = rb[b], hi = rb[b + 1];
    const int r0 = lo.x, nr = hi.x - lo.x, e0 = lo.y, e1 = hi.y;
    if (e1 - e0 > kStreamNnz) {   // one long row (nr == 1)
        AT s = AT(0);
        for (int ch = e0; ch < e1; ch += kStreamNnz) {
            const int ce = min(e1, ch + kStreamNnz);
            stream_stage<NT>(a, g, ch, ce, prod);
            __syncthreads();
            if (w == 0)
                for (int k = lane; k < ce - ch; k += 64) s += prod[k];
            __syncthreads();
        }
        if (w == 0) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
            if (lane == 0) a.t[r0] = a.W[r0] * double(s);
        }
        return;
    }
    // the rows' extents (relative to e0) and weights, loaded beside the nonzeros
    for (int i = threadIdx.x; i <= nr; i += kBlock) {
        rp[i] = a.Jp[r0 + i] - e0;
        if (i < nr) wl[i] = a.W[r0 + i];
    }
    stream_stage<NT>(a, g, e0, e1, prod);
    __syncthreads();
    for (int i = w; i < nr; i += kBlock / 64) {
        const int k0 = rp[i], k1 = rp[i + 1];
        AT s = AT(0);
        for (int k = k0 + lane; k < k1; k += 64) s += prod[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) a.t[r0 + i] = wl[i] * double(s);
    }
}

// PCG bookkeeping of an operator product: where the search direction and
// beta live.
struct PcgLink {
    double* p2;            // previous direction p; overwritten with p = x + beta*p
    const PcgScal* sc;
};

template <typename VT>
struct BwdArgs {
    const int* Jtp; const int* Jtc; const VT* Jtv; int n;
    const int* Atp; const int* Atc; const double* Atv; int hasA;
    const double* t; const double* u;
    const double* x;       // gathered vector (its own entries only)
    const double* sigx;    // may be null
    double hs, gamma;
    double* q;
    double* part;          // per-block partial p^T q (may be null)
    const Flags* fl;       // stop flags (null: always run)
    PcgLink pcg;           // pcg.p2 null: plain product
    const double* U;       // n x lr_k column-major low-rank factor (lr_k = 0: none)
    const double* lr_v;    // w .* (U^T p), lr_k entries
    int lr_k;
};

// Low-rank part of row j: sum_c U_jc v_c, split over the group's lanes (lane l
// takes c = l, l+G, ...) so it joins the group sum of the SpMV.
template <int G>
__device__ __forceinline__ double lowrank_lane(const double* U, const double* v, int k, int n, int j, int lane) {
    double s = 0.0;
    for (int c = lane; c < k; c += G) s += U[j + size_t(n) * c] * v[c];
    return s;
}

// Entry j of the product's output.  In a PCG product the direction entry
// p_j = x_j + beta*p_j is formed here and stored back (each entry is read and
// written by the group owning row j only).
__device__ __forceinline__ double direction_entry(const double* x, const PcgLink& pl, double beta, int j) {
    if (!pl.p2) return x[j];
    const double pj = x[j] + beta * pl.p2[j];
    pl.p2[j] = pj;
    return pj;
}

// End of a product: block partials of p^T q (k_pcg_xr reduces them).
__device__ __forceinline__ void product_tail(double dot, double* part, int b, double* sh) {
    if (!part) return;
    const double tot = block_sum(dot, sh);
    if (threadIdx.x == 0) part[b] = tot;
}

// q_j = hs*(J^T t + gamma p + U(w .* U^T p))_j + Sigma_x,j p_j + (A^T u)_j and per-block
// partials of p^T q.  Grid-stride over row groups with a capped grid so the
// partial count stays small.
template <int G, typename VT, typename AT, bool NT>
__global__ __launch_bounds__(kBlock) void k_op_bwd(BwdArgs<VT> a) {
    __shared__ double rowv[kBlock / 4];   // per row of one pass (RPB <= 64)
    if (pcg_stopped_ro(a.fl)) return;
    constexpr int RPB = kBlock / G;
    static_assert(RPB % kChunkRows == 0, "whole chunks per pass");
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x % G;
    const int rib = threadIdx.x / G;
    const double beta = a.pcg.p2 ? a.pcg.sc->beta : 0.0;
    for (int base = b * RPB; base < a.n; base += gridDim.x * RPB) {
        const int row = base + rib;
        double dv = 0.0;
        if (row < a.n) {
            // each part summed in the schedule-independent order, then added
            const AT sj = canon_sum<G, AT>(a.Jtp[row], a.Jtp[row + 1], lane,
                                           [&](int e) {
                                               return cvt<AT>(load_val<NT>(a.Jtv + e)) * AT(a.t[load_val<NT>(a.Jtc + e)]);
                                           });
            double s = a.hs * double(sj);
            if (a.lr_k)
                s += a.hs * canon_sum<G, double>(0, a.lr_k, lane, [&](int c) {
                    return a.U[row + size_t(a.n) * c] * a.lr_v[c];
                });
            if (a.hasA)
                s += canon_sum<G, double>(a.Atp[row], a.Atp[row + 1], lane,
                                          [&](int e) { return a.Atv[e] * a.u[a.Atc[e]]; });
            if (lane == 0) {
                const double pj = direction_entry(a.x, a.pcg, beta, row);
                double y = s + a.hs * a.gamma * pj;
                if (a.sigx) y += a.sigx[row] * pj;
                a.q[row] = y;
                dv = pj * y;
            }
        }
        if (a.part) {   // partials of p^T q per chunk of four rows
            if (lane == 0) rowv[rib] = dv;
            __syncthreads();
            chunk_partials<RPB, 1>(rowv, RPB, base, a.n, a.part);
            __syncthreads();
        }
    }
}

// ==========================================================================
// PCG vector updates
// ==========================================================================
// One iteration: the product kernels form p = z + beta p on the fly and
// q = K p with partials of p^T q; k_pcg_xr reduces them (every block, in the
// same fixed order) into alpha, updates x and r and applies the diagonal part
// of the preconditioner; with the constraint block, k_pcg_xr also runs step 1
// of z = P^{-1} r (on r - alpha q, before r is stored), and k_prec_symv and
// k_prec_at finish z and store r; k_pcg_scalars (one block) reduces r^T r and
// r^T z into the stop test, beta and rho.  Reductions are finished by the
// consumer: kernel boundaries make the partials visible without device-wide
// fences.
// Preconditioner z = P^{-1} r.  Jacobi (the paper, Section 4.1.2): z = r ./ d
// with d = diag(K).  Constraint block (woodbury = 1): y = r ./ D with
// D = diag(Hs + Sigma_x), then z = y - D^{-1} A^T Sigma^{1/2} S^{-1}
// Sigma^{1/2} A y.

// Constraint-block preconditioner, step 1: w_r = sqrt(Sigma_i) (A y)_i for the
// strong rows i = idx[r] (a wavefront per row; padding rows k..ld-1 get 0),
// and vm = 0 on all m rows (step 2 fills the strong ones).  k (strong rows)
// is read from the device, ld = k rounded up to TS_PREC; grids cover the
// largest possible ld, so launch shapes do not depend on the current k.  The
// row's range in A and sqrt(Sigma_i) come from one load of the per-row table
// (k_strong_rows), which holds empty ranges past k.
struct PrecRows {
    const int* Ac; const double* Av;
    const int* ext; const double* sq;   // per strong row: range in A, sqrt(Sigma)
    const int* kdev; int m;
    double* w; double* vm;
};
constexpr int TS_PREC = 32;   // tile edge of the dense block (schur_kernels.hpp: TS)
template <typename GV>
__device__ __forceinline__ void prec_rows(const PrecRows& a, const GV& y, int blk) {
    const int row = blk * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int k = *a.kdev;
    const int ld = ((k + TS_PREC - 1) / TS_PREC) * TS_PREC;
    for (int q = row * 64 + lane; q < a.m && q < (row + 1) * 64; q += 64) a.vm[q] = 0.0;
    if (row >= ld) return;
    const double sq = a.sq[row];
    double s = row_dot_lane_g<64, double, double, 8>(a.ext + 2 * row, a.Ac, a.Av, y, 0, lane);
    s = group_sum<double, 64>(s);
    if (lane == 0) a.w[row] = sq * s;
}

// Step 1 at the start of a solve: y = r ./ D is held in z.
struct PrecAArgs {
    PrecRows pa; const double* y; const Flags* fl;
};
__device__ __forceinline__ void prec_a_body(const PrecAArgs& a, int b) {
    if (pcg_stopped_ro(a.fl)) return;
    prec_rows(a.pa, Gather{a.y, nullptr, 0.0}, b);
}
__global__ __launch_bounds__(kBlock) void k_prec_a(PrecAArgs a) { prec_a_body(a, int(blockIdx.x)); }

struct PcgArgs {
    int n;
    double* x; double* r; double* z; const double* p; const double* q; const double* d;
    const double* part_pq; int n_pq;     // partials of p^T q from the product
    double* part_rz;                     // partials of r^T z (Jacobi)
    double* part_rr;                     // partials of r^T r
    int woodbury;
    PcgScal* sc;
    Flags* fl;
    PrecRows pa;                         // constraint block: step 1 of z = P^{-1} r
    int nbA;                             // blocks of the grid (the first ones) working on pa
};

// y_c = (r_c - alpha q_c) / D_c: the preconditioner's first vector, read from
// the residual before it is updated (the update is stored by k_prec_at).
struct ScaledResidual {
    const double* r; const double* q; const double* D; double alpha;
    __device__ __forceinline__ double operator()(int c) const { return fma(-alpha, q[c], r[c]) / D[c]; }
};

// alpha = rho / p^T q; x += alpha p; partials of r^T r for r - alpha q.
// Jacobi: r -= alpha q and z = r ./ d stored, with partials of r^T z.
// Constraint block: the first nbA blocks run step 1 of the preconditioner on
// y = (r - alpha q) ./ D, so r is left for k_prec_at to update.
// What does not depend on alpha is loaded before the p^T q reduction, so the
// two overlap: a strong row's range, scale and first pass of entries (column
// ids, values and the gathered r, q and D), an element block's first entries.
__device__ __forceinline__ void pcg_xr_body(const PcgArgs& a, int bid, int nb) {
    constexpr int U = 8;
    __shared__ double sh[kBlock / 64];
    if (pcg_stopped(a.fl)) return;
    const int lane = threadIdx.x & 63;
    const bool arow = bid < a.nbA;
    // strong-row blocks: a wavefront per row
    const int row = bid * (kBlock / 64) + (threadIdx.x >> 6);
    int e0 = 0, e1 = 0, ld = 0;
    double sqr = 0.0;
    double av[U], rv[U], qv[U], dv[U];
    // element blocks: the first entry of the grid-stride loop
    const int eb = bid - a.nbA;
    const int ne = nb - a.nbA;
    const int j0 = eb * kBlock + threadIdx.x;
    double x0 = 0.0, p0 = 0.0, q0 = 0.0, r0 = 0.0, d0 = 1.0;
    if (arow) {
        const int k = *a.pa.kdev;
        ld = ((k + TS_PREC - 1) / TS_PREC) * TS_PREC;
        for (int t = row * 64 + lane; t < a.pa.m && t < (row + 1) * 64; t += 64) a.pa.vm[t] = 0.0;
        if (row < ld) {
            e0 = a.pa.ext[2 * row];
            e1 = a.pa.ext[2 * row + 1];
            sqr = a.pa.sq[row];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            av[u] = 0.0; rv[u] = 0.0; qv[u] = 0.0; dv[u] = 1.0;
        }
        if (e1 > e0) {   // wavefront-uniform; indices past the row end clamped, zeroed below
            int c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = min(e0 + lane + 64 * u, e1 - 1);
                c[u] = a.pa.Ac[kk];
                av[u] = (e0 + lane + 64 * u < e1) ? a.pa.Av[kk] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                rv[u] = a.r[c[u]];
                qv[u] = a.q[c[u]];
                dv[u] = a.d[c[u]];
            }
        }
    } else if (j0 < a.n) {
        x0 = a.x[j0]; p0 = a.p[j0]; q0 = a.q[j0]; r0 = a.r[j0]; d0 = a.d[j0];
    }
    const double pq = reduce_partials_sum(a.part_pq, a.n_pq, 1, sh);
    const double alpha = a.sc->rho / pq;
    const bool bad = !(pq > 0.0) || !finite_d(alpha);
    if (bid == 0 && threadIdx.x == 0) {
        a.sc->pq = pq;
        a.sc->alpha = alpha;
        if (bad) a.fl->pcg_breakdown = 1;
    }
    if (bad) return;
    if (arow) {
        if (row >= ld) return;
        double acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = av[u] * (fma(-alpha, qv[u], rv[u]) / dv[u]);
        double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        // rows longer than U*64 entries: the rest, one gather round per pass
        const ScaledResidual y{a.r, a.q, a.d, alpha};
        for (int kk = e0 + U * 64 + lane; kk < e1; kk += 64) s += a.pa.Av[kk] * y(a.pa.Ac[kk]);
        s = group_sum<double, 64>(s);
        if (lane == 0) a.pa.w[row] = sqr * s;
        return;
    }
    double rz = 0.0, rr = 0.0;
    for (int j = j0; j < a.n; j += ne * kBlock) {
        double xj = x0, pj = p0, qj = q0, rj0 = r0, dj = d0;
        if (j != j0) {
            xj = a.x[j]; pj = a.p[j]; qj = a.q[j]; rj0 = a.r[j]; dj = a.d[j];
        }
        a.x[j] = xj + alpha * pj;
        const double rj = fma(-alpha, qj, rj0);
        if (!a.woodbury) {
            const double zj = rj / dj;
            a.r[j] = rj;
            a.z[j] = zj;
            rz += rj * zj;
        }
        rr += rj * rj;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        if (!a.woodbury) a.part_rz[eb] = rz;
        a.part_rr[eb] = rr;
    }
}
__global__ __launch_bounds__(kBlock) void k_pcg_xr(PcgArgs a) { pcg_xr_body(a, int(blockIdx.x), int(gridDim.x)); }

// A z for the line-format PCG product, which forms A p of the new direction
// p = z + beta p as A z + beta (A p) (k_line_pass): the rows of A, a
// wavefront per row.
struct AzArgs {
    const int* Ap; const int* Ac; const double* Av; const double* z; int m;
    double* az;
};

// Block 0.  mode 0: ||r||^2, iteration count, convergence / cap flags,
// beta = r^T z / rho, rho = r^T z.  Start of a solve (p was zeroed, so the
// first direction is z; beta = 0): mode 1 stops at rel_tol * ||rhs|| and
// records ||rhs||^2 as the outer norm; mode 2 (a refinement solve) stops at
// max(rel_tol * ||rhs||, tol * outer norm), and at once when rhs already
// meets tol * outer norm.  Blocks 1.. (when az.m > 0): A z, four rows each.
struct ScalArgs {
    const double* part_rz; int n_rz; const double* part_rr; int n_rr;
    int mode; double rel_tol; double tol; int max_iter;
    PcgScal* sc; Flags* fl; AzArgs az;
};
__device__ __forceinline__ void pcg_scalars_body(const ScalArgs& s_, int bid) {
    const double* part_rz = s_.part_rz; const int n_rz = s_.n_rz;
    const double* part_rr = s_.part_rr; const int n_rr = s_.n_rr;
    const int mode = s_.mode; const double rel_tol = s_.rel_tol, tol = s_.tol;
    const int max_iter = s_.max_iter;
    PcgScal* sc = s_.sc; Flags* fl = s_.fl; const AzArgs& az = s_.az;
    __shared__ double sh[kBlock / 64];
    if (bid > 0) {
        // A z needs no block barrier: each wavefront reads the flags with one
        // uniform load beside its first index load (block 0 may set a flag
        // meanwhile; either reading leaves a valid state, since later kernels
        // test the flags themselves)
        if (mode ? fl->ipm_done : pcg_stopped_raw(fl)) return;
        const int row = (bid - 1) * (kBlock / 64) + (threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        if (row >= az.m) return;
        double s = row_dot_lane<64, double, double, 8>(az.Ap, az.Ac, az.Av, az.z, row, lane);
        s = group_sum<double, 64>(s);
        if (lane == 0) az.az[row] = s;
        return;
    }
    if (mode ? ipm_finished(fl) : pcg_stopped(fl)) return;
    const double rz = reduce_partials_sum(part_rz, n_rz, 1, sh);
    const double rr = reduce_partials_sum(part_rr, n_rr, 1, sh);
    if (threadIdx.x != 0) return;
    if (mode) {
        if (mode == 1) sc->bnorm2_outer = rr;
        const double floor2 = tol * tol * sc->bnorm2_outer;
        sc->rho = rz;
        sc->beta = 0.0;
        sc->alpha = 0.0;
        sc->pq = 0.0;
        sc->bnorm2 = rr;
        sc->rr = rr;
        sc->tol2 = fmax(rel_tol * rel_tol * rr, mode == 2 ? floor2 : 0.0);
        sc->iters = 0;
        sc->max_iter = max_iter;
        fl->pcg_iters = 0;
        const bool conv = rr == 0.0 || (mode == 2 && rr <= floor2);
        fl->pcg_converged = conv ? 1 : 0;
        // a preconditioner that is not positive definite on r (r^T z <= 0,
        // or non-finite) cannot drive CG: stop at once
        if (!conv && !(rz > 0.0 && finite_d(rz))) fl->pcg_breakdown = 1;
        return;
    }
    sc->rr = rr;
    const int it = sc->iters + 1;
    sc->iters = it;
    fl->pcg_iters = it;
    if (rr <= sc->tol2) fl->pcg_converged = 1;
    else if (!(rz > 0.0 && finite_d(rz))) fl->pcg_breakdown = 1;   // as at the start
    else if (it >= sc->max_iter) fl->pcg_capped = 1;
    sc->beta = rz / sc->rho;
    sc->rho = rz;
}
__global__ __launch_bounds__(kBlock) void k_pcg_scalars(ScalArgs a) { pcg_scalars_body(a, int(blockIdx.x)); }

struct PcgInitArgs {
    int n;
    const double* rhs_a;   // may be null: rhs = rhs_b
    const double* rhs_b;
    const IpmScal* ipm;    // mu for rhs = mu*rhs_a + rhs_b (null: mu = 0)
    double* x; double* r; double* z; double* p; const double* d;
    double* part_rz; double* part_rr;
    int woodbury;
    Flags* fl;
    double* apv; int m;    // A p of the line-format product (may be null): zeroed with p
};

// x = 0; r = rhs; z = r ./ d; p = 0; partials.  Clears the PCG flags of the
// previous solve (no other block of this kernel reads them; later kernels of
// this solve see them cleared).
__device__ __forceinline__ void pcg_init0_body(const PcgInitArgs& a, int bid, int nb) {
    __shared__ double sh[kBlock / 64];
    if (ipm_finished(a.fl)) return;
    if (bid == 0 && threadIdx.x == 0) {
        a.fl->pcg_converged = 0;
        a.fl->pcg_breakdown = 0;
        a.fl->pcg_capped = 0;
    }
    const double mu = a.ipm ? a.ipm->mu : 0.0;
    double rz = 0.0, rr = 0.0;
    for (int j = bid * kBlock + threadIdx.x; j < a.n; j += nb * kBlock) {
        const double rj = a.rhs_a ? mu * a.rhs_a[j] + a.rhs_b[j] : a.rhs_b[j];
        const double zj = rj / a.d[j];
        a.x[j] = 0.0;
        a.r[j] = rj;
        a.z[j] = zj;
        a.p[j] = 0.0;
        rz += rj * zj;
        rr += rj * rj;
    }
    if (a.apv)
        for (int i = bid * kBlock + threadIdx.x; i < a.m; i += nb * kBlock) a.apv[i] = 0.0;
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        if (!a.woodbury) a.part_rz[bid] = rz;
        a.part_rr[bid] = rr;
    }
}
__global__ __launch_bounds__(kBlock) void k_pcg_init0(PcgInitArgs a) {
    pcg_init0_body(a, int(blockIdx.x), int(gridDim.x));
}

// Step 2: vm[idx[r]] = sqrt(Sigma) (S^{-1} w)_r, a wavefront per row of the
// dense symmetric inverse (row-major, leading dimension ld); k from the device.
struct SymvArgs {
    const double* Sinv; const double* w; const double* sq; const int* idx; const int* kdev; double* vm;
    const Flags* fl;
};
__device__ __forceinline__ void prec_symv_body(const SymvArgs& a, int bid) {
    const double* Sinv = a.Sinv; const double* w = a.w; const double* sq = a.sq; const int* idx = a.idx;
    double* vm = a.vm;
    if (pcg_stopped_ro(a.fl)) return;
    const int k = *a.kdev;
    const int ld = ((k + TS_PREC - 1) / TS_PREC) * TS_PREC;
    const int row = bid * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= k) return;
    const int i = idx[row];       // the output's place and scale, loaded beside the row
    const double sqi = sq[row];
    const double* srow = Sinv + size_t(row) * ld;
    // passes of 8 loads per lane in flight (indices past ld clamped, zeroed)
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    for (int c = lane; c < ld; c += 512) {
        double sv[8], wv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int cc = min(c + 64 * u, ld - 1);
            sv[u] = srow[cc];
            wv[u] = w[cc];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += (c + 64 * u < ld) ? sv[u] * wv[u] : 0.0;
    }
    double s = group_sum<double, 64>(((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])));
    if (lane == 0) vm[i] = sqi * s;
}
__global__ __launch_bounds__(kBlock) void k_prec_symv(SymvArgs a) { prec_symv_body(a, int(blockIdx.x)); }

// Step 3: z_j = y_j - (A^T v)_j / D_j and partials of r^T z.  Start of a
// solve (q null): y is held in z and r is final.  In an iteration: r_j -=
// alpha q_j is stored here and y_j = r_j / D_j.  G lanes per row of A^T,
// grid-stride with a capped grid.
struct PrecAtArgs {
    const int* Atp; const int* Atc; const double* Atv; const double* v; const double* D;
    double* r; const double* q; const PcgScal* sc; double* z; int n; double* part_rz; const Flags* fl;
};
template <int G>
__device__ __forceinline__ void prec_at_body(const PrecAtArgs& a, int bid, int nb) {
    const int* Atp = a.Atp; const int* Atc = a.Atc; const double* Atv = a.Atv; const double* v = a.v;
    const double* D = a.D; double* r = a.r; const double* q = a.q; double* z = a.z; const int n = a.n;
    __shared__ double sh[kBlock / 64];
    if (pcg_stopped_ro(a.fl)) return;
    constexpr int RPB = kBlock / G;
    const int lane = threadIdx.x % G;
    const double alpha = q ? a.sc->alpha : 0.0;
    double rz = 0.0;
    for (int base = bid * RPB; base < n; base += nb * RPB) {
        const int j = base + threadIdx.x / G;
        if (j < n) {
            // the column's own entries are loaded first, beside the sum's loads
            const double r0 = r[j], dj = D[j];
            const double q0 = q ? q[j] : 0.0;
            const double z0 = q ? 0.0 : z[j];
            double s = row_dot_lane<G, double, double>(Atp, Atc, Atv, v, j, lane);
            s = group_sum<double, G>(s);
            if (lane == 0) {
                double rj, yj;
                if (q) {
                    rj = fma(-alpha, q0, r0);
                    yj = rj / dj;
                    r[j] = rj;
                } else {
                    rj = r0;
                    yj = z0;
                }
                const double zj = yj - s / dj;
                z[j] = zj;
                rz += rj * zj;
            }
        }
    }
    rz = block_sum(rz, sh);
    if (threadIdx.x == 0) a.part_rz[bid] = rz;
}
template <int G>
__global__ __launch_bounds__(kBlock) void k_prec_at(PrecAtArgs a) {
    prec_at_body<G>(a, int(blockIdx.x), int(gridDim.x));
}

// ==========================================================================
// IPM state, residuals and the right-hand side
// ==========================================================================
struct IpmVec {
    int n, m;
    const double* xlo; const double* xhi; const double* alo; const double* ahi;
    const double* p;          // unscaled linear term
    const double* diagH;      // unscaled diag(H)
    double* x;
    double* s_lx; double* s_ux; double* l_lx; double* l_ux;
    double* s_lA; double* s_uA; double* l_lA; double* l_uA;
    double* ax;               // A x
    double* r_lx; double* r_ux; double* r_lA; double* r_uA;
    double* sigx; double* sigA;
    double* va; double* vb; double* ya;       // m-vectors feeding A^T
    double* hx;               // scaled H x
    double* d;                // Jacobi diagonal of K
    double* dh;               // diag(Hs + Sigma_x), the H part of the constraint-block preconditioner
    double* rhs_a; double* rhs_b;
    double* dx;
    double* ds_lx; double* ds_ux; double* dl_lx; double* dl_ux;
    double* ds_lA; double* ds_uA; double* dl_lA; double* dl_uA;
};

// Start point: x0 = bound midpoint, or a finite bound +- 1, or 0; slacks of
// the bounds max(x0 - lo, 1) / max(hi - x0, 1); multipliers 1.  Partials of
// the slack sum (for mu0) over present sides.
__global__ __launch_bounds__(kBlock) void k_ipm_init_x(IpmVec v, double* part) {
    __shared__ double sh[kBlock / 64];
    double ssum = 0.0;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < v.n; j += gridDim.x * kBlock) {
        const double lo = v.xlo[j], hi = v.xhi[j];
        const bool hl = finite_d(lo), hu = finite_d(hi);
        double x0 = 0.0;
        if (hl && hu) x0 = 0.5 * (lo + hi);
        else if (hl) x0 = lo + 1.0;
        else if (hu) x0 = hi - 1.0;
        v.x[j] = x0;
        v.s_lx[j] = hl ? fmax(x0 - lo, 1.0) : 1.0;
        v.l_lx[j] = hl ? 1.0 : 0.0;
        v.s_ux[j] = hu ? fmax(hi - x0, 1.0) : 1.0;
        v.l_ux[j] = hu ? 1.0 : 0.0;
        ssum += (hl ? v.s_lx[j] : 0.0) + (hu ? v.s_ux[j] : 0.0);
    }
    ssum = block_sum(ssum, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = ssum;
}

// Slacks of the rows of A at x0: max(ax - lo, 1), max(hi - ax, 1).
__global__ __launch_bounds__(kBlock) void k_ipm_init_A(IpmVec v, const int* Ap, const int* Ac,
                                                       const double* Av, double* part) {
    __shared__ double sh[kBlock / 64];
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double ssum = 0.0;
    if (row < v.m) {
        double s = row_dot_lane<64, double, double>(Ap, Ac, Av, v.x, row, lane);
        s = group_sum<double, 64>(s);
        if (lane == 0) {
            const double lo = v.alo[row], hi = v.ahi[row];
            const bool hl = finite_d(lo), hu = finite_d(hi);
            v.s_lA[row] = hl ? fmax(s - lo, 1.0) : 1.0;
            v.l_lA[row] = hl ? 1.0 : 0.0;
            v.s_uA[row] = hu ? fmax(hi - s, 1.0) : 1.0;
            v.l_uA[row] = hu ? 1.0 : 0.0;
            ssum = (hl ? v.s_lA[row] : 0.0) + (hu ? v.s_uA[row] : 0.0);
        }
    }
    ssum = block_sum(ssum, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = ssum;
}

// zeta = max(1, ||H x0 + p||_inf) (q holds H x0), hs = 1/zeta, pmax, and
// mu0 = sum of start slacks / m_tot (multipliers are all 1).
__global__ __launch_bounds__(kBlock) void k_ipm_scale(const double* q, const double* p, int n,
                                                      const double* part_s, int n_s, double mtot,
                                                      int scale, double mu0_user, IpmScal* sc) {
    __shared__ double sh[kBlock / 64];
    double g = 0.0, pm = 0.0;
    for (int j = threadIdx.x; j < n; j += kBlock) {
        g = fmax(g, fabs(q[j] + p[j]));
        pm = fmax(pm, fabs(p[j]));
    }
    g = block_max(g, sh);
    pm = block_max(pm, sh);
    const double ssum = reduce_partials_sum(part_s, n_s, 1, sh);
    if (threadIdx.x == 0) {
        const double zeta = scale ? fmax(1.0, g) : 1.0;
        sc->zeta = zeta;
        sc->hs = 1.0 / zeta;
        sc->pmax = pm / zeta;
        sc->mtot = mtot;
        sc->mu = mu0_user > 0.0 ? mu0_user : (mtot > 0.0 ? ssum / mtot : sc->mu_tol);
        sc->done = 0;
        sc->iter = 0;
        sc->rnorm = 0.0;
        sc->alpha_p = sc->alpha_d = 0.0;
    }
}

// Residual pass, part 1: t = W .* (J x) for rows of J; for rows of A: A x,
// the group residuals, Sigma_A, and the m-vectors va (mu coefficient of the
// rhs), vb (mu-free part) and ya = lambda_uA - lambda_lA that the next kernel
// multiplies by A^T.  Per-block partial maxima of |r_g| and |lambda s - mu|.
template <int G>
__global__ __launch_bounds__(kBlock) void k_ipm_fwd(FwdArgs<double> a, IpmVec v, const IpmScal* sc,
                                                    double* part, const Flags* fl) {
    __shared__ double sh[kBlock / 64];
    if (ipm_finished(fl)) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    if (b < a.nbJ) {
        constexpr int RPB = kBlock / G;
        const int row = b * RPB + threadIdx.x / G;
        const int lane = threadIdx.x % G;
        if (row < a.nJ) {
            const double s = canon_sum<G, double>(a.Jp[row], a.Jp[row + 1], lane,
                                                  [&](int e) { return a.Jv[e] * a.x[a.Jc[e]]; });
            if (lane == 0) a.t[row] = a.W[row] * s;
        }
        return;
    }
    const int ab = b - a.nbJ;
    const int row = ab * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double rg = 0.0, rc = 0.0;
    if (row < a.m) {
        double s = row_dot_lane<64, double, double>(a.Ap, a.Ac, a.Av, a.x, row, lane);
        s = group_sum<double, 64>(s);
        if (lane == 0) {
            const double mu = sc->mu;
            const double lo = v.alo[row], hi = v.ahi[row];
            const bool hl = finite_d(lo), hu = finite_d(hi);
            const double sl = v.s_lA[row], su = v.s_uA[row], ll = v.l_lA[row], lu = v.l_uA[row];
            const double rl = hl ? s - sl - lo : 0.0;
            const double ru = hu ? -s - su + hi : 0.0;
            const double gl = hl ? ll / sl : 0.0, gu = hu ? lu / su : 0.0;
            v.ax[row] = s;
            v.r_lA[row] = rl;
            v.r_uA[row] = ru;
            v.sigA[row] = gl + gu;
            v.va[row] = (hl ? 1.0 / sl : 0.0) - (hu ? 1.0 / su : 0.0);
            v.vb[row] = -gl * rl + gu * ru;
            v.ya[row] = lu - ll;
            rg = fmax(fabs(rl), fabs(ru));
            rc = fmax(hl ? fabs(ll * sl - mu) : 0.0, hu ? fabs(lu * su - mu) : 0.0);
        }
    }
    rg = block_max(rg, sh);
    rc = block_max(rc, sh);
    if (threadIdx.x == 0) {
        part[2 * ab] = rg;
        part[2 * ab + 1] = rc;
    }
}

struct IpmBwdArgs {
    const int* Jtp; const int* Jtc; const double* Jtv;
    const int* sptr; const int* sslot; const double* lc;   // line format: per-spot slot ids, per-slot J^T W J x shares
    const int* Atp; const int* Atc; const double* Atv; int hasA;
    const double* t;
    double gamma;
    const double* U; const double* lr_v; int lr_k;   // low-rank part of H (lr_v = w .* U^T x)
    int aug;               // 1: right-hand side and Jacobi diagonal of the doubly augmented system
};

// Residual pass, part 2, per variable j: H x (scaled), the A^T products of
// ya, va, vb and of the squared values with Sigma_A (Jacobi diagonal of
// A^T Sigma_A A), then r_H, the bound residuals, Sigma_x, the Jacobi diagonal
// d, and the two rhs parts.  Partials (6 per chunk of four variables):
// max|r_H|, max|Hx|, max|r_g| and max|r_c| of the bounds, sum x.Hx, sum p.x.
template <int G>
__global__ __launch_bounds__(kBlock) void k_ipm_bwd(IpmBwdArgs a, IpmVec v, const IpmScal* sc,
                                                    double* part, const Flags* fl) {
    __shared__ double rowv[6][kBlock / 4];   // per row of one pass (RPB <= 64)
    if (ipm_finished(fl)) return;
    constexpr int RPB = kBlock / G;
    static_assert(RPB % kChunkRows == 0, "whole chunks per pass");
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x % G;
    const int rib = threadIdx.x / G;
    const double hs = sc->hs, mu = sc->mu;
    for (int base = b * RPB; base < v.n; base += gridDim.x * RPB) {
        const int j = base + rib;
        double mrH = 0.0, mHx = 0.0, mrg = 0.0, mrc = 0.0, sxh = 0.0, spx = 0.0;
        if (j < v.n) {
            // every sum in the schedule-independent order
            double hj = hs * (a.lc ? canon_sum<G, double>(a.sptr[j], a.sptr[j + 1], lane,
                                                          [&](int e) { return a.lc[a.sslot[e]]; })
                                   : canon_sum<G, double>(a.Jtp[j], a.Jtp[j + 1], lane,
                                                          [&](int e) { return a.Jtv[e] * a.t[a.Jtc[e]]; }));
            if (a.lr_k)
                hj += hs * canon_sum<G, double>(0, a.lr_k, lane,
                                                [&](int c) { return a.U[j + size_t(v.n) * c] * a.lr_v[c]; });
            double aty = 0.0, ava = 0.0, avb = 0.0, a2s = 0.0;
            if (a.hasA) {
                const int s0 = a.Atp[j], s1 = a.Atp[j + 1];
                aty = canon_sum<G, double>(s0, s1, lane, [&](int e) { return a.Atv[e] * v.ya[a.Atc[e]]; });
                ava = canon_sum<G, double>(s0, s1, lane, [&](int e) { return a.Atv[e] * v.va[a.Atc[e]]; });
                avb = canon_sum<G, double>(s0, s1, lane, [&](int e) { return a.Atv[e] * v.vb[a.Atc[e]]; });
                a2s = canon_sum<G, double>(s0, s1, lane,
                                           [&](int e) { return a.Atv[e] * a.Atv[e] * v.sigA[a.Atc[e]]; });
            }
            if (lane == 0) {
                const double xj = v.x[j];
                const double hx = hj + hs * a.gamma * xj;
                const double pj = v.p[j] * hs;
                const double lo = v.xlo[j], hi = v.xhi[j];
                const bool hl = finite_d(lo), hu = finite_d(hi);
                const double sl = v.s_lx[j], su = v.s_ux[j], ll = v.l_lx[j], lu = v.l_ux[j];
                const double rl = hl ? xj - sl - lo : 0.0;
                const double ru = hu ? -xj - su + hi : 0.0;
                const double gl = hl ? ll / sl : 0.0, gu = hu ? lu / su : 0.0;
                const double rH = hx + pj + (lu - ll) + aty;
                v.hx[j] = hx;
                v.r_lx[j] = rl;
                v.r_ux[j] = ru;
                v.sigx[j] = gl + gu;
                v.dh[j] = hs * v.diagH[j] + gl + gu;
                // doubly augmented (eq. (2x2_augmented)): the top-left block
                // holds 2 A^T Sigma_A A, and its right-hand side r_1 + 2 B^T
                // D^-1 r_2 is the condensed one plus A^T(mu va + vb + ya)
                v.d[j] = v.dh[j] + (a.aug ? 2.0 : 1.0) * a2s;
                v.rhs_a[j] = (hl ? 1.0 / sl : 0.0) - (hu ? 1.0 / su : 0.0) + (a.aug ? 2.0 : 1.0) * ava;
                v.rhs_b[j] = -(hx + pj) - gl * rl + gu * ru + (a.aug ? 2.0 * avb + aty : avb);
                mrH = fabs(rH);
                mHx = fabs(hx);
                mrg = fmax(fabs(rl), fabs(ru));
                mrc = fmax(hl ? fabs(ll * sl - mu) : 0.0, hu ? fabs(lu * su - mu) : 0.0);
                sxh = xj * hx;
                spx = pj * xj;
            }
        }
        // partials per chunk of four rows: four maxima, two sums
        if (lane == 0) {
            rowv[0][rib] = mrH; rowv[1][rib] = mHx; rowv[2][rib] = mrg;
            rowv[3][rib] = mrc; rowv[4][rib] = sxh; rowv[5][rib] = spx;
        }
        __syncthreads();
        chunk_partials<RPB, 6>(&rowv[0][0], kBlock / 4, base, v.n, part);
        __syncthreads();
    }
}

// Residual norm and the barrier rule of Algorithm 1:
//   if ||r|| < mu: if mu <= mu_tol: done; else mu <- mu/10.
// ||r|| = max(||r_H||/(1 + max(||p||, ||Hx||)), ||r_g||/cscale, ||r_c||), all
// infinity norms in scaled units.  apply = 0 evaluates without the rule (the
// start point).
__global__ __launch_bounds__(kBlock) void k_ipm_check(const double* partA, int nA, const double* partX,
                                                      int nX, int apply, IpmScal* sc, Flags* fl,
                                                      double* log) {
    __shared__ double sh[kBlock / 64];
    if (ipm_finished(fl)) return;
    const double rgA = nA ? reduce_partials_max(partA, nA, 2, sh) : 0.0;
    const double rcA = nA ? reduce_partials_max(partA + 1, nA, 2, sh) : 0.0;
    const double rH = reduce_partials_max(partX, nX, 6, sh);
    const double Hx = reduce_partials_max(partX + 1, nX, 6, sh);
    const double rgx = reduce_partials_max(partX + 2, nX, 6, sh);
    const double rcx = reduce_partials_max(partX + 3, nX, 6, sh);
    const double xHx = reduce_partials_sum(partX + 4, nX, 6, sh);
    const double px = reduce_partials_sum(partX + 5, nX, 6, sh);
    if (threadIdx.x == 0) {
        const double dscale = 1.0 + fmax(sc->pmax, Hx);
        const double rn = fmax(rH / dscale, fmax(fmax(rgA, rgx) / sc->cscale, fmax(rcA, rcx)));
        sc->rnorm = rn;
        sc->xHx = xHx;
        sc->px = px;
        if (apply) {
            const int it = sc->iter + 1;
            sc->iter = it;
            fl->ipm_iter = it;
            if (log) {
                double* e = log + 4 * size_t(it - 1);
                e[0] = sc->mu; e[1] = rn; e[2] = sc->alpha_p; e[3] = sc->alpha_d;
            }
            if (rn < sc->mu) {
                if (sc->mu <= sc->mu_tol) {
                    sc->done = 1;
                    fl->ipm_done = 1;
                } else {
                    sc->mu = sc->mu / 10.0;
                }
            }
        }
    }
}

// Direction recovery and ratio test.  Blocks [0, nbA) handle rows of A
// (A dx by a wavefront per row), the rest handle the bounds of x.  Per-block
// partial minima of -s/ds over ds < 0 and of -lambda/dl over dl < 0.
__global__ __launch_bounds__(kBlock) void k_ipm_recover(IpmVec v, const int* Ap, const int* Ac,
                                                        const double* Av, int nbA, const IpmScal* sc,
                                                        double* part, const Flags* fl) {
    __shared__ double sh[kBlock / 64];
    if (ipm_finished(fl)) return;
    const double mu = sc->mu;
    double mp = 1.0e300, md = 1.0e300;
    if ((int)blockIdx.x < nbA) {
        const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        if (row < v.m) {
            double s = row_dot_lane<64, double, double>(Ap, Ac, Av, v.dx, row, lane);
            s = group_sum<double, 64>(s);
            if (lane == 0) {
                const bool hl = finite_d(v.alo[row]), hu = finite_d(v.ahi[row]);
                const double sl = v.s_lA[row], su = v.s_uA[row], ll = v.l_lA[row], lu = v.l_uA[row];
                const double dsl = hl ? s + v.r_lA[row] : 0.0;
                const double dsu = hu ? -s + v.r_uA[row] : 0.0;
                const double dll = hl ? -ll + mu / sl - (ll / sl) * dsl : 0.0;
                const double dlu = hu ? -lu + mu / su - (lu / su) * dsu : 0.0;
                v.ds_lA[row] = dsl; v.ds_uA[row] = dsu;
                v.dl_lA[row] = dll; v.dl_uA[row] = dlu;
                if (dsl < 0.0) mp = fmin(mp, -sl / dsl);
                if (dsu < 0.0) mp = fmin(mp, -su / dsu);
                if (dll < 0.0) md = fmin(md, -ll / dll);
                if (dlu < 0.0) md = fmin(md, -lu / dlu);
            }
        }
    } else {
        const int nbx = gridDim.x - nbA;
        for (int j = (blockIdx.x - nbA) * kBlock + threadIdx.x; j < v.n; j += nbx * kBlock) {
            const bool hl = finite_d(v.xlo[j]), hu = finite_d(v.xhi[j]);
            const double dxj = v.dx[j];
            const double sl = v.s_lx[j], su = v.s_ux[j], ll = v.l_lx[j], lu = v.l_ux[j];
            const double dsl = hl ? dxj + v.r_lx[j] : 0.0;
            const double dsu = hu ? -dxj + v.r_ux[j] : 0.0;
            const double dll = hl ? -ll + mu / sl - (ll / sl) * dsl : 0.0;
            const double dlu = hu ? -lu + mu / su - (lu / su) * dsu : 0.0;
            v.ds_lx[j] = dsl; v.ds_ux[j] = dsu;
            v.dl_lx[j] = dll; v.dl_ux[j] = dlu;
            if (dsl < 0.0) mp = fmin(mp, -sl / dsl);
            if (dsu < 0.0) mp = fmin(mp, -su / dsu);
            if (dll < 0.0) md = fmin(md, -ll / dll);
            if (dlu < 0.0) md = fmin(md, -lu / dlu);
        }
    }
    mp = block_min(mp, sh);
    md = block_min(md, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = mp;
        part[2 * blockIdx.x + 1] = md;
    }
}

// Step lengths alpha_P = min(1, tau*min ratio) and alpha_D likewise (equal
// when step_mode = 1), then x += alpha_P dx, s += alpha_P ds,
// lambda += alpha_D dl.  Every block reduces the same partials.
__global__ __launch_bounds__(kBlock) void k_ipm_update(IpmVec v, const double* part, int np,
                                                       IpmScal* sc, const Flags* fl) {
    __shared__ double sh[kBlock / 64];
    if (ipm_finished(fl)) return;
    const double mp = reduce_partials_min(part, np, 2, sh);
    const double md = reduce_partials_min(part + 1, np, 2, sh);
    double ap = fmin(1.0, sc->tau * mp);
    double ad = fmin(1.0, sc->tau * md);
    if (sc->step_mode == 1) ap = ad = fmin(ap, ad);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->alpha_p = ap;
        sc->alpha_d = ad;
    }
    const int tot = v.n + v.m;
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < tot; k += gridDim.x * kBlock) {
        if (k < v.n) {
            const int j = k;
            v.x[j] += ap * v.dx[j];
            if (finite_d(v.xlo[j])) { v.s_lx[j] += ap * v.ds_lx[j]; v.l_lx[j] += ad * v.dl_lx[j]; }
            if (finite_d(v.xhi[j])) { v.s_ux[j] += ap * v.ds_ux[j]; v.l_ux[j] += ad * v.dl_ux[j]; }
        } else {
            const int i = k - v.n;
            if (finite_d(v.alo[i])) { v.s_lA[i] += ap * v.ds_lA[i]; v.l_lA[i] += ad * v.dl_lA[i]; }
            if (finite_d(v.ahi[i])) { v.s_uA[i] += ap * v.ds_uA[i]; v.l_uA[i] += ad * v.dl_uA[i]; }
        }
    }
}

// Multipliers in original units: lam_x = zeta(lambda_ux - lambda_lx),
// lam_A = zeta(lambda_uA - lambda_lA).
__global__ __launch_bounds__(kBlock) void k_ipm_output(IpmVec v, const IpmScal* sc, double* lam_x,
                                                       double* lam_A) {
    const double z = sc->zeta;
    const int tot = v.n + v.m;
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < tot; k += gridDim.x * kBlock) {
        if (k < v.n) lam_x[k] = z * (v.l_ux[k] - v.l_lx[k]);
        else lam_A[k - v.n] = z * (v.l_uA[k - v.n] - v.l_lA[k - v.n]);
    }
}

// ==========================================================================
// KKT certificate of the returned point (original units)
// ==========================================================================
// The optimality conditions of eq. (qp) (eq. (perturbed_KKT) with mu = 0),
// measured at the returned x and combined multipliers y_x = zeta(lambda_ux -
// lambda_lx), y_A = zeta(lambda_uA - lambda_lA), with lambda_l = max(-y, 0),
// lambda_u = max(y, 0) per side.  H x and A x come from the residual pass at
// that x (hx is H x / zeta).  Per-block partials, reduced by k_cert_final in
// a fixed order.
constexpr int kCertBlocks = 512;
constexpr int kCertX = 10;   // partials per block of k_cert_x
constexpr int kCertA = 3;    // partials per block of k_cert_a

// Per variable j (G lanes per row of A^T for (A^T y_A)_j): maxima of |r_H|,
// |H x|, |p|, |y_x|, |A^T y_A|, bound violation, lambda*slack; sums of
// x^T H x, p^T x and the bounds' dual term lambda_l lo - lambda_u hi.
template <int G>
__global__ __launch_bounds__(kBlock) void k_cert_x(IpmVec v, const int* Atp, const int* Atc, const double* Atv,
                                                   int hasA, const IpmScal* sc, double* part) {
    __shared__ double sh[kBlock / 64];
    constexpr int RPB = kBlock / G;
    const int lane = threadIdx.x % G;
    const double z = sc->zeta;
    double mx[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double xhx = 0.0, px = 0.0, dual = 0.0;
    for (int base = blockIdx.x * RPB; base < v.n; base += gridDim.x * RPB) {
        const int j = base + threadIdx.x / G;
        if (j >= v.n) continue;   // whole groups
        double aty = 0.0;
        if (hasA) {
            for (int e = Atp[j] + lane; e < Atp[j + 1]; e += G) aty += Atv[e] * (v.l_uA[Atc[e]] - v.l_lA[Atc[e]]);
            aty = z * group_sum<double, G>(aty);
        }
        if (lane != 0) continue;
        const double xj = v.x[j], hx = z * v.hx[j], pj = v.p[j];
        const double lo = v.xlo[j], hi = v.xhi[j];
        const bool hl = finite_d(lo), hu = finite_d(hi);
        const double yx = z * (v.l_ux[j] - v.l_lx[j]);
        const double ll = fmax(-yx, 0.0), lu = fmax(yx, 0.0);
        const double rH = hx + pj + yx + aty;
        mx[0] = fmax(mx[0], fabs(rH));
        mx[1] = fmax(mx[1], fabs(hx));
        mx[2] = fmax(mx[2], fabs(pj));
        mx[3] = fmax(mx[3], fabs(yx));
        mx[4] = fmax(mx[4], fabs(aty));
        if (hl) mx[5] = fmax(mx[5], lo - xj);
        if (hu) mx[5] = fmax(mx[5], xj - hi);
        if (hl && ll > 0.0) { mx[6] = fmax(mx[6], fabs(ll * (xj - lo))); dual += ll * lo; }
        if (hu && lu > 0.0) { mx[6] = fmax(mx[6], fabs(lu * (hi - xj))); dual -= lu * hi; }
        xhx += xj * hx;
        px += pj * xj;
    }
    double out[kCertX];
#pragma unroll
    for (int k = 0; k < 7; ++k) out[k] = block_max(mx[k], sh);
    out[7] = block_sum(xhx, sh);
    out[8] = block_sum(px, sh);
    out[9] = block_sum(dual, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < kCertX; ++k) part[size_t(blockIdx.x) * kCertX + k] = out[k];
}

// Per row i of A: row violation, lambda*slack maximum, dual term sum (A x
// from the residual pass).
__global__ __launch_bounds__(kBlock) void k_cert_a(IpmVec v, const IpmScal* sc, double* part) {
    __shared__ double sh[kBlock / 64];
    const double z = sc->zeta;
    double viol = 0.0, comp = 0.0, dual = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < v.m; i += gridDim.x * kBlock) {
        const double ax = v.ax[i], lo = v.alo[i], hi = v.ahi[i];
        const bool hl = finite_d(lo), hu = finite_d(hi);
        const double y = z * (v.l_uA[i] - v.l_lA[i]);
        const double ll = fmax(-y, 0.0), lu = fmax(y, 0.0);
        if (hl) viol = fmax(viol, lo - ax);
        if (hu) viol = fmax(viol, ax - hi);
        if (hl && ll > 0.0) { comp = fmax(comp, fabs(ll * (ax - lo))); dual += ll * lo; }
        if (hu && lu > 0.0) { comp = fmax(comp, fabs(lu * (hi - ax))); dual -= lu * hi; }
    }
    viol = block_max(viol, sh);
    comp = block_max(comp, sh);
    dual = block_sum(dual, sh);
    if (threadIdx.x == 0) {
        part[size_t(blockIdx.x) * kCertA] = viol;
        part[size_t(blockIdx.x) * kCertA + 1] = comp;
        part[size_t(blockIdx.x) * kCertA + 2] = dual;
    }
}

struct CertOut {
    double eps_d, eps_p, eps_c, gap;
};

// One block: the certificate from the partials of k_cert_x (nx blocks) and
// k_cert_a (na blocks, 0 when there are no rows of A).
__global__ __launch_bounds__(kBlock) void k_cert_final(const double* px, int nx, const double* pa, int na,
                                                       const IpmScal* sc, CertOut* out) {
    __shared__ double sh[kBlock / 64];
    double mx[7];
    for (int k = 0; k < 7; ++k) mx[k] = reduce_partials_max(px + k, nx, kCertX, sh);
    const double xhx = reduce_partials_sum(px + 7, nx, kCertX, sh);
    const double ptx = reduce_partials_sum(px + 8, nx, kCertX, sh);
    double dual = reduce_partials_sum(px + 9, nx, kCertX, sh);
    double viol = mx[5], comp = mx[6];
    if (na > 0) {
        viol = fmax(viol, reduce_partials_max(pa, na, kCertA, sh));
        comp = fmax(comp, reduce_partials_max(pa + 1, na, kCertA, sh));
        dual += reduce_partials_sum(pa + 2, na, kCertA, sh);
    }
    if (threadIdx.x == 0) {
        const double dscale = 1.0 + fmax(fmax(mx[1], mx[2]), fmax(mx[3], mx[4]));
        const double oscale = 1.0 + 0.5 * fabs(xhx) + fabs(ptx);
        const double f = 0.5 * xhx + ptx;
        out->eps_d = mx[0] / dscale;
        out->eps_p = viol / sc->cscale;
        out->eps_c = comp / oscale;
        out->gap = fabs(f - (-0.5 * xhx + dual)) / oscale;
    }
}

// ==========================================================================
// Setup kernels
// ==========================================================================

// diag(H)_j = gamma + sum_i W_i J_ij^2 (+ sum_c w_c U_jc^2), from the rows of J^T.
template <int G>
__global__ __launch_bounds__(kBlock) void k_diag_h(const int* Jtp, const int* Jtc, const double* Jtv,
                                                   const double* W, int n, double gamma,
                                                   const double* U, const double* w, int k,
                                                   double* diagH) {
    constexpr int RPB = kBlock / G;
    const int j = blockIdx.x * RPB + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (j >= n) return;
    double s = 0.0;
    for (int e = Jtp[j] + lane; e < Jtp[j + 1]; e += G) {
        const double v = Jtv[e];
        s += W[Jtc[e]] * v * v;
    }
    s = group_sum<double, G>(s);
    if (lane == 0) {
        double dj = gamma + s;
        for (int c = 0; c < k; ++c) {
            const double u = U[j + size_t(n) * c];
            dj += w[c] * u * u;
        }
        diagH[j] = dj;
    }
}

// diag(H) on the line format of J, in two steps: k_line_diag gives every
// slot s of a line the weighted squares sum_r W_r J_(r,s)^2 over the line's
// 64 rows (a wavefront per slot, lane = row, fixed butterfly), and
// k_spot_diag sums them over each spot's slots: diag(H)_j = gamma +
// sum_slots + sum_c w_c U_jc^2.  A block per line; slot values contiguous per
// slot (64 rows).
__global__ __launch_bounds__(kBlock) void k_line_diag(const int* lptr, const double* lval, const double* W, int L,
                                                      double* d) {
    const int l = blockIdx.x;
    if (l >= L) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int off = lptr[l], end = lptr[l + 1];
    const double wr = W[size_t(l) * 64 + lane];
    for (int k = off + w; k < end; k += kBlock / 64) {
        const double v = lval[size_t(k) * 64 + lane];
        const double s = group_sum<double, 64>(wr * v * v);
        if (lane == 0) d[k] = s;
    }
}
template <int G>
__global__ __launch_bounds__(kBlock) void k_spot_diag(const int* sptr, const int* sslot, const double* d, int n,
                                                      double gamma, const double* U, const double* w, int k,
                                                      double* diagH) {
    constexpr int RPB = kBlock / G;
    const int j = blockIdx.x * RPB + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (j >= n) return;   // whole groups leave together
    double s = canon_sum<G, double>(sptr[j], sptr[j + 1], lane, [&](int e) { return d[sslot[e]]; });
    if (lane == 0) {
        double dj = gamma + s;
        for (int c = 0; c < k; ++c) {
            const double u = U[j + size_t(n) * c];
            dj += w[c] * u * u;
        }
        diagH[j] = dj;
    }
}

// Low-precision copies of FP64 values, rounded on the device exactly as the
// host does it (host_prep.cpp): FP32 by the conversion's round to nearest
// even; BF16 by rounding to odd onto binary32 first, then to nearest even
// (the two-step rounding that is exact, Boldo and Melquiond), values outside
// the binary32 normal range through the plain conversion.
__device__ __forceinline__ uint32_t d2f_bits(double v) { return __float_as_uint(float(v)); }
__device__ __forceinline__ uint16_t d2bf16_bits(double v) {
    const uint64_t d = uint64_t(__double_as_longlong(v));
    const uint64_t sign = d >> 63;
    const int64_t e = int64_t((d >> 52) & 0x7FF) - 1023 + 127;
    const uint64_t m = d & ((uint64_t(1) << 52) - 1);
    uint32_t b;
    if (e >= 1 && e <= 254) {
        b = uint32_t(sign << 31) | uint32_t(uint64_t(e) << 23) | uint32_t(m >> 29);
        if (m & ((uint64_t(1) << 29) - 1)) b |= 1u;
    } else {
        b = d2f_bits(v);
    }
    b += 0x7FFFu + ((b >> 16) & 1u);
    return uint16_t(b >> 16);
}
__global__ __launch_bounds__(kBlock) void k_round_f32(const double* src, size_t count, uint32_t* dst) {
    for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += size_t(gridDim.x) * kBlock)
        dst[i] = d2f_bits(src[i]);
}
__global__ __launch_bounds__(kBlock) void k_round_bf16(const double* src, size_t count, uint16_t* dst) {
    for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += size_t(gridDim.x) * kBlock)
        dst[i] = d2bf16_bits(src[i]);
}

// Jacobi diagonals for a given Sigma: dh_j = diagH_j + sigx_j and
// d_j = dh_j + sum_i (A^T)_ji^2 sigA_i.
__global__ __launch_bounds__(kBlock) void k_jacobi(const int* Atp, const double* Atv, const int* Atc,
                                                   int hasA, const double* sigA, const double* sigx,
                                                   const double* diagH, int n, double* d, double* dh, int aug) {
    const int j = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= n) return;
    double s = 0.0;
    if (hasA)
        for (int e = Atp[j] + lane; e < Atp[j + 1]; e += 64) {
            const double v = Atv[e];
            s += v * v * sigA[Atc[e]];
        }
    s = group_sum<double, 64>(s);
    if (lane == 0) {
        dh[j] = diagH[j] + sigx[j];
        d[j] = dh[j] + (aug ? 2.0 * s : s);
    }
}

// Lambda block of the doubly augmented system at an IPM iterate, per row i of
// A and side: D = s/lambda (0 in dlu for an absent side), the Jacobi diagonal
// (D, or 1 for an absent side) and r_2 = -(r_g + r_c/lambda) = mu/lambda -
// r_g - s split into its mu coefficient (rhs_a) and the rest (rhs_b), at
// offsets n (lower side) and n + m (upper side).
__global__ __launch_bounds__(kBlock) void k_aug_rows(IpmVec v, double* dlu, const Flags* fl) {
    if (ipm_finished(fl)) return;
    const int n = v.n, m = v.m;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
        const bool hl = finite_d(v.alo[i]), hu = finite_d(v.ahi[i]);
        const double sl = v.s_lA[i], su = v.s_uA[i], ll = v.l_lA[i], lu = v.l_uA[i];
        const double Dl = hl ? sl / ll : 0.0, Du = hu ? su / lu : 0.0;
        dlu[i] = Dl;
        dlu[m + i] = Du;
        v.d[n + i] = hl ? Dl : 1.0;
        v.d[n + m + i] = hu ? Du : 1.0;
        v.rhs_a[n + i] = hl ? 1.0 / ll : 0.0;
        v.rhs_b[n + i] = hl ? -v.r_lA[i] - sl : 0.0;
        v.rhs_a[n + m + i] = hu ? 1.0 / lu : 0.0;
        v.rhs_b[n + m + i] = hu ? -v.r_uA[i] - su : 0.0;
    }
}

// Lambda block of the doubly augmented system for a Newton step of the
// condensed system (H + Sigma_x + A^T diag(sigA) A) dx = rhs: each row with
// sigA_i > 0 is one side with D = 1/sigA_i and r_2 = 0, so the x part of the
// solution is that dx (the Schur complement of eq. (2x2_augmented)).
__global__ __launch_bounds__(kBlock) void k_aug_newton_rows(const double* sigA, int n, int m, double* dlu,
                                                            double* d, double* rhs) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
        const double s = sigA[i];
        const double Du = s > 0.0 ? 1.0 / s : 0.0;
        dlu[i] = 0.0;
        dlu[m + i] = Du;
        d[n + i] = 1.0;
        d[n + m + i] = Du > 0.0 ? Du : 1.0;
        rhs[n + i] = 0.0;
        rhs[n + m + i] = 0.0;
    }
}

// Low-rank factor product v = w .* (U^T p) (eq. (bfgs_hessian) applied
// matrix-free), p the gathered vector: per-block partials of up to 32 columns
// (grid.y walks column groups), then a one-block fixed-order reduction.
// Partial layout part[b * k + c] for x-block b and column c.
__global__ __launch_bounds__(kBlock) void k_lr_partial(const double* U, int n, int k, const double* x,
                                                       const double* p2, const PcgScal* sc, double* part,
                                                       const Flags* fl) {
    __shared__ double sh[kBlock / 64];
    if (pcg_stopped_ro(fl)) return;
    const Gather g = make_gather(x, p2, sc);
    const int c0 = blockIdx.y * 32;
    const int kc = min(32, k - c0);
    double acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = 0.0;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
        const double pj = g(j);
#pragma unroll
        for (int c = 0; c < 32; ++c)
            if (c < kc) acc[c] += U[j + size_t(n) * (c0 + c)] * pj;
    }
#pragma unroll
    for (int c = 0; c < 32; ++c) {   // static indices keep acc in registers
        if (c < kc) {                 // kc is uniform over the block
            const double t = block_sum(acc[c], sh);
            if (threadIdx.x == 0) part[size_t(blockIdx.x) * k + c0 + c] = t;
        }
    }
}

// v_c = w_c * sum_b part[b][c]: thread (s, c) adds x-blocks s, s+8, ... of
// column c of a 32-column group, then the 8 sums are added in order.
__global__ __launch_bounds__(kBlock) void k_lr_reduce(const double* part, int nb, int k, const double* w,
                                                      double* v, const Flags* fl) {
    __shared__ double sub[kBlock / 32][32];
    if (pcg_stopped_ro(fl)) return;
    const int c = threadIdx.x & 31, s8 = threadIdx.x >> 5;
    constexpr int S = kBlock / 32;
    for (int cg = 0; cg < k; cg += 32) {
        const int col = min(cg + c, k - 1);
        double a = 0.0;
        for (int bx = s8; bx < nb; bx += 8 * S) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = part[size_t(min(bx + u * S, nb - 1)) * k + col];
#pragma unroll
            for (int u = 0; u < 8; ++u) a += (bx + u * S < nb) ? t[u] : 0.0;
        }
        sub[s8][c] = a;
        __syncthreads();
        if (threadIdx.x < 32 && cg + c < k) {
            double tot = 0.0;
#pragma unroll
            for (int i = 0; i < S; ++i) tot += sub[i][c];
            v[cg + c] = w[cg + c] * tot;
        }
        __syncthreads();
    }
}

// Mixed-precision refinement helpers (skipped once the IPM has finished).
// rhs = mu*rhs_a + rhs_b with mu read on the device.
__global__ __launch_bounds__(kBlock) void k_rhs_combine(int n, const double* rhs_a, const double* rhs_b,
                                                        const IpmScal* sc, double* out, const Flags* fl) {
    if (ipm_finished(fl)) return;
    const double mu = sc->mu;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock)
        out[j] = mu * rhs_a[j] + rhs_b[j];
}

// out = rhs - q (the FP64 residual of the current direction).
__global__ __launch_bounds__(kBlock) void k_sub(int n, const double* rhs, const double* q, double* out,
                                                const Flags* fl) {
    if (ipm_finished(fl)) return;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) out[j] = rhs[j] - q[j];
}

// acc = px (init) or acc += px.
__global__ __launch_bounds__(kBlock) void k_acc(int n, double* acc, const double* px, int init, const Flags* fl) {
    if (ipm_finished(fl)) return;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock)
        acc[j] = init ? px[j] : acc[j] + px[j];
}

__global__ __launch_bounds__(kBlock) void k_fill(double* a, double v, int n) {
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) a[j] = v;
}

}  // namespace qpg
