// Batched PCG over many QPs of uneven size (qp_solve_batch).
//
// Every kernel of a PCG solve exists as a body that serves one block of one
// QP's grid (line_kernels.hpp, ipm_kernels.hpp).  A batched solve runs each
// kind of work as ONE launch over a global work list: the items of a kind
// are the blocks of every QP taking part, concatenated; workgroup i takes
// item i (remapped so each XCD serves one contiguous range of the list, and
// neighbouring lines of one QP share that XCD's L2), looks up the QP of the
// item and calls the body with the QP's arguments and the item's block
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

// A QP's arguments come from a table in memory, so the compiler cannot tell
// that their pointers address global memory (as it can for a kernel's own
// arguments) and would use generic (flat) loads and stores, which take more
// registers and wait on both memory counters.  Each pointer is rebuilt as a
// global-address-space pointer (device memory and pinned host memory both
// are global addresses), which lets the compiler use global instructions.
template <typename T>
__device__ __forceinline__ T* gptr(T* p) {
    typedef __attribute__((address_space(1))) T GT;
    return (T*)(GT*)(uintptr_t)p;
}

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
// then one inclusive scan over the QPs, carrying for every kind at once the
// count of QPs on its list (list positions) and of their items (offsets),
// builds every list; flags of all QPs are copied to one array for the host.
__global__ __launch_bounds__(kMaxBatch) void k_batch_plan(const BatchQp* qs, const int* in_phase, int nq, int mode,
                                                          BatchList* lists, BatchStatus* status, Flags* flags_out) {
    constexpr int NV = 2 * BK_COUNT + 1;   // per kind: on the list, items; then: active
    __shared__ int sv[NV][kMaxBatch];
    const int q = threadIdx.x;
    bool act = false;
    int nblk[BK_COUNT];
#pragma unroll
    for (int k = 0; k < BK_COUNT; ++k) nblk[k] = 0;
    if (q < nq) {
        const Flags f = *gptr(qs[q].fl);
        flags_out[q] = f;
        act = in_phase[q] != 0 && !f.ipm_done;
        if (mode == BP_ITER) act = act && !(f.pcg_converged | f.pcg_breakdown | f.pcg_capped);
        if (act)
#pragma unroll
            for (int k = 0; k < BK_COUNT; ++k) nblk[k] = qs[q].nblk[k];
    }
    int v[NV];
#pragma unroll
    for (int k = 0; k < BK_COUNT; ++k) {
        v[2 * k] = nblk[k] > 0 ? 1 : 0;
        v[2 * k + 1] = nblk[k];
    }
    v[NV - 1] = act ? 1 : 0;
    for (int d = 1; d < kMaxBatch; d <<= 1) {
#pragma unroll
        for (int k = 0; k < NV; ++k) sv[k][q] = v[k];
        __syncthreads();
        if (q >= d)
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] += sv[k][q - d];
        __syncthreads();
    }
    if (q == kMaxBatch - 1) status->active = v[NV - 1];
#pragma unroll
    for (int k = 0; k < BK_COUNT; ++k) {
        BatchList& L = lists[k];
        if (nblk[k] > 0) {
            const int pos = v[2 * k] - 1;
            L.qid[pos] = q;
            L.off[pos] = v[2 * k + 1] - nblk[k];
        }
        if (q == kMaxBatch - 1) {
            L.nq = v[2 * k];
            L.total = v[2 * k + 1];
            L.off[v[2 * k]] = v[2 * k + 1];
        }
    }
}

// One item per workgroup: a kind's grid covers the longest list the batch
// can have, and workgroups past the current list's length return at once.  Item order is
// remapped so that each XCD takes one contiguous range of the list (its
// lines stay neighbours in its L2); the QP of an item is found in a copy of
// the list's offsets in LDS.  Unlike the walk, the hardware dispatcher keeps
// starting workgroups as others finish, so one item's chain of dependent
// loads overlaps the next ones' as in a single QP's launch (a persistent
// grid walking the list, measured first, left each workgroup's items in
// sequence and ran the 16-QP FP64 batch's line passes at about half the
// single-QP rate).
template <typename F>
__device__ __forceinline__ void batch_item(const BatchList* L, F&& body) {
    __shared__ int s_off[kMaxBatch + 1];
    __shared__ int s_qid[kMaxBatch];
    const int total = L->total;
    const int b = int(blockIdx.x);
    if (b >= total) return;   // workgroup-uniform, before any barrier
    const int nq = L->nq;
    for (int i = threadIdx.x; i <= nq; i += kBlock) {
        s_off[i] = L->off[i];
        if (i < nq) s_qid[i] = L->qid[i];
    }
    __syncthreads();
    const int g = xcd_remap(b, total);
    int lo = 0, hi = nq - 1;   // the last QP whose first item is <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    // uniform across the workgroup: made scalar, so the QP's arguments are
    // read with scalar loads into scalar registers, as kernel arguments are
    const int o = __builtin_amdgcn_readfirstlane(s_off[lo]);
    const int q = __builtin_amdgcn_readfirstlane(s_qid[lo]);
    const int e = __builtin_amdgcn_readfirstlane(s_off[lo + 1]);
    body(q, __builtin_amdgcn_readfirstlane(g) - o, e - o);
}

#define QPG_G(f) a.f = gptr(a.f)
template <typename VT>
__device__ __forceinline__ LineArgs<VT> global_args(LineArgs<VT> a) {
    QPG_G(lptr); QPG_G(lcol); QPG_G(lval); QPG_G(W); QPG_G(Ap); QPG_G(Ac); QPG_G(Av); QPG_G(x); QPG_G(p2);
    QPG_G(sc); QPG_G(c); QPG_G(u); QPG_G(sigA); QPG_G(az); QPG_G(apv); QPG_G(fl); QPG_G(fl_ipm);
    QPG_G(aug.dlu); QPG_G(aug.q); QPG_G(aug.part);
    return a;
}
__device__ __forceinline__ SpotArgs global_args(SpotArgs a) {
    QPG_G(sptr); QPG_G(sslot); QPG_G(c); QPG_G(Atp); QPG_G(Atc); QPG_G(Atv); QPG_G(u); QPG_G(x); QPG_G(sigx);
    QPG_G(q); QPG_G(part); QPG_G(fl); QPG_G(pcg.p2); QPG_G(pcg.sc); QPG_G(U); QPG_G(lr_v);
    return a;
}
__device__ __forceinline__ PrecRows global_rows(PrecRows a) {
    QPG_G(Ac); QPG_G(Av); QPG_G(ext); QPG_G(sq); QPG_G(kdev); QPG_G(w); QPG_G(vm);
    return a;
}
__device__ __forceinline__ PcgArgs global_args(PcgArgs a) {
    QPG_G(x); QPG_G(r); QPG_G(z); QPG_G(p); QPG_G(q); QPG_G(d); QPG_G(part_pq); QPG_G(part_rz); QPG_G(part_rr);
    QPG_G(sc); QPG_G(fl);
    a.pa = global_rows(a.pa);
    return a;
}
__device__ __forceinline__ SymvArgs global_args(SymvArgs a) {
    QPG_G(Sinv); QPG_G(w); QPG_G(sq); QPG_G(idx); QPG_G(kdev); QPG_G(vm); QPG_G(fl);
    return a;
}
__device__ __forceinline__ PrecAtArgs global_args(PrecAtArgs a) {
    QPG_G(Atp); QPG_G(Atc); QPG_G(Atv); QPG_G(v); QPG_G(D); QPG_G(r); QPG_G(q); QPG_G(sc); QPG_G(z);
    QPG_G(part_rz); QPG_G(fl);
    return a;
}
__device__ __forceinline__ ScalArgs global_args(ScalArgs a) {
    QPG_G(part_rz); QPG_G(part_rr); QPG_G(sc); QPG_G(fl);
    QPG_G(az.Ap); QPG_G(az.Ac); QPG_G(az.Av); QPG_G(az.z); QPG_G(az.az);
    return a;
}
__device__ __forceinline__ PcgInitArgs global_args(PcgInitArgs a) {
    QPG_G(rhs_a); QPG_G(rhs_b); QPG_G(ipm); QPG_G(x); QPG_G(r); QPG_G(z); QPG_G(p); QPG_G(d);
    QPG_G(part_rz); QPG_G(part_rr); QPG_G(fl); QPG_G(apv);
    return a;
}
__device__ __forceinline__ PrecAArgs global_args(PrecAArgs a) {
    a.pa = global_rows(a.pa);
    QPG_G(y); QPG_G(fl);
    return a;
}
#undef QPG_G

template <typename VT, typename AT, bool NT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void kb_line(const LineArgs<VT>* tab,
                                                                                          const BatchList* L) {
    batch_item(L, [&](int q, int b, int nb) { line_pass_body<VT, AT, NT>(global_args(tab[q]), b, nb, false); });
}

template <int G>
__global__ __launch_bounds__(kBlock) void kb_spot(const SpotArgs* tab, const BatchList* L) {
    batch_item(L, [&](int q, int b, int nb) { spot_pass_body<G>(global_args(tab[q]), b, nb); });
}

__global__ __launch_bounds__(kBlock) void kb_xr(const PcgArgs* tab, const BatchList* L) {
    batch_item(L, [&](int q, int b, int nb) { pcg_xr_body(global_args(tab[q]), b, nb); });
}

__global__ __launch_bounds__(kBlock) void kb_symv(const SymvArgs* tab, const BatchList* L) {
    batch_item(L, [&](int q, int b, int) { prec_symv_body(global_args(tab[q]), b); });
}

template <int G>
__global__ __launch_bounds__(kBlock) void kb_at(const PrecAtArgs* tab, const BatchList* L) {
    batch_item(L, [&](int q, int b, int nb) { prec_at_body<G>(global_args(tab[q]), b, nb); });
}

__global__ __launch_bounds__(kBlock) void kb_scal(const ScalArgs* tab, const BatchList* L) {
    batch_item(L, [&](int q, int b, int) { pcg_scalars_body(global_args(tab[q]), b); });
}

__global__ __launch_bounds__(kBlock) void kb_init0(const PcgInitArgs* tab, const BatchList* L) {
    batch_item(L, [&](int q, int b, int nb) { pcg_init0_body(global_args(tab[q]), b, nb); });
}

__global__ __launch_bounds__(kBlock) void kb_preca(const PrecAArgs* tab, const BatchList* L) {
    batch_item(L, [&](int q, int b, int) { prec_a_body(global_args(tab[q]), b); });
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
    batch_item(L, [&](int q, int b, int nb) {
        VecArgs v = tab[q];
        v.a = gptr(v.a); v.b = gptr(v.b); v.isc = gptr(v.isc); v.out = gptr(v.out);
        vec_body(v, b, nb);
    });
}

}  // namespace qpg
