// Batched PCG over many QPs of uneven size (qp_solve_batch).
//
// Every kernel of a PCG solve exists as a body that serves one block of one
// QP's grid (line_kernels.hpp, ipm_kernels.hpp).  A batched solve runs each
// kind of work as ONE persistent launch over a global work list: the items
// of a kind are the blocks of every QP taking part, concatenated; the
// launch's workgroups walk the list (each XCD one contiguous range of it, so
// neighbouring lines of one QP share that XCD's L2), look up the QP of an
// item and call the body with the QP's arguments and the item's block
// number within that QP's grid.  The lists live in device memory and are
// rebuilt on the device by k_batch_plan after every PCG iteration from the
// QPs' own stop flags: a QP whose solve has converged (or whose IPM has
// finished) drops out of every list and costs nothing afterwards, while
// launch shapes stay fixed, so the iterations can be captured once as a HIP
// graph and replayed.  Each QP keeps its own device state (vectors, PCG
// scalars, flags) in its handle, so a batched iteration computes for every
// QP exactly what that QP's own launches compute, bit for bit.
#pragma once

#include "line_kernels.hpp"

namespace qpg {

constexpr int kMaxBatch = 256;   // QPs of one batched launch (one planning thread each)

// Kinds of work.  PCG products use the BK_LINE (or, with FP64 values in a
// low-precision batch, BK_LINE64) and BK_SPOT lists; plain FP64 products
// (the refinement residual) BK_LINE_PLAIN and BK_SPOT.
enum BatchKind : int {
    BK_INIT = 0,     // k_pcg_init0
    BK_PRECA,        // constraint-block step 1 at a solve's start (k_prec_a)
    BK_SYMV,         // step 2 (k_prec_symv)
    BK_AT,           // step 3 (k_prec_at)
    BK_SCAL,         // k_pcg_scalars (block 0 the scalars, then the rows of A z)
    BK_LINE,         // line pass of a PCG product in the batch's precision
    BK_LINE64,       // line pass of an FP64 PCG product (sized from the FP64 line arguments)
    BK_LINE_PLAIN,   // line pass of a plain product (rows of A in the grid)
    BK_SPOT,         // spot pass
    BK_XR,           // k_pcg_xr
    BK_VEC,          // elementwise steps of the refinement
    BK_COUNT
};

// Work list of one kind.
struct BatchList {
    int nq;                    // QPs on the list
    int total;                 // items
    int qid[kMaxBatch];        // their indices in the batch
    int off[kMaxBatch + 1];    // first item of each
};

// Per QP: its stop flags, whether it takes part in the current phase, and
// its item count for each kind (0: the kind has no work for it).
struct BatchQp {
    const Flags* fl;
    int nblk[BK_COUNT];
};

// What the host reads after each chunk of iterations: the QPs still active
// and every QP's flags.
struct BatchStatus {
    int active;
    int pad[3];
};

// Planning modes of k_batch_plan.
enum : int {
    BP_START = 0,   // a QP takes part when it is in the phase and its IPM has not finished
    BP_ITER = 1     // ... and its PCG solve has not stopped
};

// One block of kMaxBatch threads: thread q decides whether QP q is active,
// then an inclusive scan of the active flags (list positions) and, per kind,
// of the item counts (offsets) builds every list; flags of all QPs are
// copied to one array for the host.
__global__ __launch_bounds__(kMaxBatch) void k_batch_plan(const BatchQp* qs, const int* in_phase, int nq, int mode,
                                                          BatchList* lists, BatchStatus* status, Flags* flags_out) {
    __shared__ int sa[kMaxBatch], sc[kMaxBatch];
    const int q = threadIdx.x;
    bool act = false;
    int nblk[BK_COUNT];
#pragma unroll
    for (int k = 0; k < BK_COUNT; ++k) nblk[k] = 0;
    if (q < nq) {
        const Flags f = *qs[q].fl;
        flags_out[q] = f;
        act = in_phase[q] != 0 && !f.ipm_done;
        if (mode == BP_ITER) act = act && !(f.pcg_converged | f.pcg_breakdown | f.pcg_capped);
        if (act)
#pragma unroll
            for (int k = 0; k < BK_COUNT; ++k) nblk[k] = qs[q].nblk[k];
    }
    // active count (for the host's stop test)
    sa[q] = act ? 1 : 0;
    __syncthreads();
    for (int d = 1; d < kMaxBatch; d <<= 1) {
        const int v = q >= d ? sa[q - d] : 0;
        __syncthreads();
        sa[q] += v;
        __syncthreads();
    }
    if (q == kMaxBatch - 1) status->active = sa[q];
    for (int k = 0; k < BK_COUNT; ++k) {
        const bool on = nblk[k] > 0;
        sa[q] = on ? 1 : 0;
        sc[q] = nblk[k];
        __syncthreads();
        for (int d = 1; d < kMaxBatch; d <<= 1) {
            const int va = q >= d ? sa[q - d] : 0;
            const int vc = q >= d ? sc[q - d] : 0;
            __syncthreads();
            sa[q] += va;
            sc[q] += vc;
            __syncthreads();
        }
        BatchList& L = lists[k];
        if (on) {
            const int pos = sa[q] - 1;
            L.qid[pos] = q;
            L.off[pos] = sc[q] - nblk[k];
        }
        if (q == kMaxBatch - 1) {
            L.nq = sa[q];
            L.total = sc[q];
            L.off[sa[q]] = sc[q];
        }
        __syncthreads();
    }
}

// The persistent walk: workgroup b serves XCD b % 8, whose share of the
// items is one contiguous range, taken in steps of the XCD's workgroup
// count.  body(qp, item within the QP's grid, the QP's grid size).  Bodies
// synchronise the whole workgroup in the same places for every item (their
// early returns are workgroup-uniform before any barrier), and a barrier
// after each item keeps the next item's LDS use behind the last reads.
template <typename F>
__device__ __forceinline__ void batch_walk(const BatchList* L, F&& body) {
    const int total = L->total;
    const int nq = L->nq;
    const int x = int(blockIdx.x) & 7, lb = int(blockIdx.x) >> 3, nbx = int(gridDim.x) >> 3;
    const int start = int((int64_t(total) * x) >> 3), end = int((int64_t(total) * (x + 1)) >> 3);
    for (int g = start + lb; g < end; g += nbx) {
        int lo = 0, hi = nq - 1;   // the last QP whose first item is <= g
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L->off[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const int o = L->off[lo];
        body(L->qid[lo], g - o, L->off[lo + 1] - o);
        __syncthreads();
    }
}

// The walk around the line pass takes a few registers more than the single
// QP's kernel: with FP64 values the budget of six (or five) wavefronts per
// SIMD would spill, so that one runs four.
template <typename VT>
constexpr int kb_line_waves() { return sizeof(VT) == 8 ? 4 : 6; }
template <typename VT, typename AT, bool NT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kb_line_waves<VT>()))) void kb_line(
    const LineArgs<VT>* tab, const BatchList* L) {
    batch_walk(L, [&](int q, int b, int nb) { line_pass_body<VT, AT, NT>(tab[q], b, nb, false); });
}

template <int G>
__global__ __launch_bounds__(kBlock) void kb_spot(const SpotArgs* tab, const BatchList* L) {
    batch_walk(L, [&](int q, int b, int nb) { spot_pass_body<G>(tab[q], b, nb); });
}

__global__ __launch_bounds__(kBlock) void kb_xr(const PcgArgs* tab, const BatchList* L) {
    batch_walk(L, [&](int q, int b, int nb) { pcg_xr_body(tab[q], b, nb); });
}

__global__ __launch_bounds__(kBlock) void kb_symv(const SymvArgs* tab, const BatchList* L) {
    batch_walk(L, [&](int q, int b, int) { prec_symv_body(tab[q], b); });
}

template <int G>
__global__ __launch_bounds__(kBlock) void kb_at(const PrecAtArgs* tab, const BatchList* L) {
    batch_walk(L, [&](int q, int b, int nb) { prec_at_body<G>(tab[q], b, nb); });
}

__global__ __launch_bounds__(kBlock) void kb_scal(const ScalArgs* tab, const BatchList* L) {
    batch_walk(L, [&](int q, int b, int) { pcg_scalars_body(tab[q], b); });
}

__global__ __launch_bounds__(kBlock) void kb_init0(const PcgInitArgs* tab, const BatchList* L) {
    batch_walk(L, [&](int q, int b, int nb) { pcg_init0_body(tab[q], b, nb); });
}

__global__ __launch_bounds__(kBlock) void kb_preca(const PrecAArgs* tab, const BatchList* L) {
    batch_walk(L, [&](int q, int b, int) { prec_a_body(tab[q], b); });
}

// Elementwise steps of the refinement of a low-precision direction, one
// table per step (the k_rhs_combine, k_sub and k_acc of a single solve):
//   VEC_RHS   out = mu*a + b (mu of the QP's IPM)
//   VEC_SUB   out = a - b
//   VEC_SET   out = a
//   VEC_ADD   out += a
enum : int { VEC_RHS = 0, VEC_SUB, VEC_SET, VEC_ADD };
struct VecArgs {
    int op, n;
    const double* a; const double* b; const IpmScal* isc; double* out;
};
__device__ __forceinline__ void vec_body(const VecArgs& v, int bid, int nb) {
    const double mu = v.op == VEC_RHS ? v.isc->mu : 0.0;
    for (int j = bid * kBlock + threadIdx.x; j < v.n; j += nb * kBlock) {
        switch (v.op) {
            case VEC_RHS: v.out[j] = mu * v.a[j] + v.b[j]; break;
            case VEC_SUB: v.out[j] = v.a[j] - v.b[j]; break;
            case VEC_SET: v.out[j] = v.a[j]; break;
            default: v.out[j] = v.out[j] + v.a[j]; break;
        }
    }
}
__global__ __launch_bounds__(kBlock) void kb_vec(const VecArgs* tab, const BatchList* L) {
    batch_walk(L, [&](int q, int b, int nb) { vec_body(tab[q], b, nb); });
}

}  // namespace qpg
