// Host side of the C ABI declared in include/qpgpu.h: handle lifecycle, device
// memory, kernel launch schedule, and the Algorithm 1 loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_prep.h"
#include "ipm_kernels.hpp"
#include "schur_kernels.hpp"
#include "line_kernels.hpp"
#include "sequence_kernels.hpp"
#include "batch_kernels.hpp"
#include "qpgpu.h"

using namespace qpg;

static_assert(kLineSlotAlign == kLineGroup, "line slot counts hold whole packed groups");

namespace {

thread_local std::string g_create_error;



struct HipError {
    hipError_t e;
    const char* what;
};

#define HIPCHK(call)                                             \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) throw HipError{e_, #call};         \
    } while (0)

int pick_lanes(int64_t nnz, int64_t rows) {
    const double L = rows > 0 ? double(nnz) / double(rows) : 0.0;
    if (L <= 12) return 4;
    if (L <= 24) return 8;
    if (L <= 96) return 16;
    if (L <= 320) return 32;
    return 64;
}

}  // namespace

struct qp_handle {
    std::string err;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    qp_settings set{};

    int32_t n = 0, m = 0, nJ = 0, k = 0;
    int64_t nnzJ = 0, nnzA = 0;
    int64_t nvals = 0;          // J values the PCG operator stores: line slots * 64 (zeros included), or nnzJ
    double gamma = 0.0, cscale = 1.0, mtot = 0.0;
    int k_cap = 0;              // columns U, w, lr_part, lr_v have room for
    int wb_attempt_cap = 0;     // > 0: the attempt cap of constraint-block-preconditioned solves is on
    int wb_seen = 0;            // longest converged constraint-block solve of the current run
    int wb_cap_used = 0;        // iteration cap the last constraint-block solve set up with
    int wb_cap_dir = 0;         // attempt cap of the current direction's constraint-block solves
    double* x0d = nullptr;      // caller's start point (qp_solve_from), allocated on first use
    int GJ = 16, GJt = 64;   // lanes per row of J and of J^T (and A^T)
    bool fwd_stream = false;  // CSR forward pass over nonzero-balanced row blocks (k_op_fwd_stream)
    int2* jrb = nullptr;      // those blocks (first row, first nonzero), nbs + 1 pairs
    int nbs = 0;

    std::vector<void*> allocs;

    // matrices
    int *Jp = nullptr, *Jc = nullptr, *Jtp = nullptr, *Jtc = nullptr;
    double *Jv = nullptr, *Jtv = nullptr;
    float *Jv32 = nullptr, *Jtv32 = nullptr;
    bf16_t *Jv16 = nullptr, *Jtv16 = nullptr;
    double* W = nullptr;
    int *Ap = nullptr, *Ac = nullptr, *Atp = nullptr, *Atc = nullptr;
    double *Av = nullptr, *Atv = nullptr;
    // iterations of the two previous PCG solves of each kind (first solve of
    // a direction, refinement solve), for the chunk sizes
    int last_pcg_iters[2][2] = {{0, 0}, {0, 0}};
    // line format of J (64-row lines sharing a column list), used by the PCG operator
    bool line = false;
    int L = 0;
    int64_t nslots = 0;   // line slots (entries of lc)
    // doubly augmented system (kkt_system = 1): D of each row and side, and
    // whether the current operator products use it
    double* dlu = nullptr;
    bool aug = false;
    int *lptr = nullptr, *lcol = nullptr, *sptr = nullptr, *sslot = nullptr;
    double* lval = nullptr;
    double* lc = nullptr;   // per-slot J^T contributions of the line pass
    float* lval32 = nullptr;
    bf16_t* lval16 = nullptr;
    double *xlo = nullptr, *xhi = nullptr, *alo = nullptr, *ahi = nullptr;
    double *p = nullptr, *diagH = nullptr, *U = nullptr, *w = nullptr;

    // work
    IpmVec iv{};
    double *t = nullptr, *u = nullptr;
    double *az = nullptr, *apv = nullptr;   // A z and A p of the line-format PCG product
    double *px = nullptr, *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr;
    double *zero_n = nullptr, *zero_m = nullptr, *tmp_n = nullptr, *tmp_n2 = nullptr, *tmp_m = nullptr;
    double *rhs_full = nullptr, *rho = nullptr, *dxacc = nullptr;   // refinement of low-precision directions
    double *part = nullptr, *part2 = nullptr, *partA = nullptr, *part_rz = nullptr, *part_rr = nullptr;
    // constraint-block preconditioner (dense m x m, leading dimension ld)
    int woodbury = 0, ld = 0, T = 0;            // allocation sizes (all m rows)
    int kcur = 0, ldcur = 0, Tcur = 0;           // strong rows of the current build
    double *Sm = nullptr, *Sm2 = nullptr, *Sinv = nullptr, *Pbuf = nullptr, *wpre = nullptr, *vpre = nullptr;
    double* Dw = nullptr;                        // D plus the weak rows' diagonal
    double *lr_part = nullptr, *lr_v = nullptr;  // low-rank term: U^T p partials and w .* U^T p
    int *rflag = nullptr, *rpos = nullptr, *ridx = nullptr, *kdev = nullptr;
    double* rmii = nullptr;     // M_ii of every row of A (k_row_strength)
    int* sext = nullptr;        // per strong row: range in A (k_strong_rows)
    int *scr = nullptr, *scnt = nullptr;   // per column of A: strong entries' ranks, count (k_fold_weak)
    double* scv = nullptr;                 // and their values
    double* ssq = nullptr;      // per strong row: sqrt(Sigma)
    int srows = 0;              // rows of that table (covers every step-1 grid)
    size_t part_len = 0;
    double* log = nullptr;
    IpmScal* isc = nullptr;
    PcgScal* psc = nullptr;
    CertOut* cert = nullptr;
    Flags* fl = nullptr;
    Flags* fl_host = nullptr;   // pinned, 2 slots
    int* k_host = nullptr;      // pinned: the strong-row count read back by build_precond
    hipEvent_t ev_k = nullptr;

    // captured PCG iteration graphs, one per operator (precision, preconditioner, operands)
    struct PcgGraph {
        int prec = 0, wb = 0, n_rz = 0;
        bool aug = false;
        const void* ops[4] = {nullptr, nullptr, nullptr, nullptr};   // sigx, sigA, d, dh
        double hs = 0.0;
        hipGraph_t graph = nullptr;   // kept with its executable until both are dropped
        hipGraphExec_t exec = nullptr;
    };
    std::vector<PcgGraph> graphs;
    bool graphs_failed = false;

    std::vector<hipEvent_t> tev;  // timing events, pairs
    hipEvent_t ev_chunk[2] = {nullptr, nullptr};
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
    hipEvent_t ev_p0[2] = {nullptr, nullptr}, ev_p1[2] = {nullptr, nullptr};   // PCG time, two IPM iterations in flight

    template <typename T>
    T* dalloc(size_t count) {
        if (count == 0) count = 1;
        void* ptr = nullptr;
        hipError_t e = hipMalloc(&ptr, count * sizeof(T));
        if (e != hipSuccess) throw HipError{e, "hipMalloc"};
        allocs.push_back(ptr);
        return static_cast<T*>(ptr);
    }
    void dfree(void* ptr) {
        if (!ptr) return;
        for (auto it = allocs.begin(); it != allocs.end(); ++it)
            if (*it == ptr) {
                allocs.erase(it);
                (void)hipFree(ptr);
                return;
            }
    }
    template <typename T>
    T* upload(const T* src, size_t count) {
        T* d = dalloc<T>(count);
        if (count) HIPCHK(hipMemcpyAsync(d, src, count * sizeof(T), hipMemcpyHostToDevice, stream));
        return d;
    }
    ~qp_handle() {
        // teardown: errors here have no caller to go to
        if (stream) (void)hipStreamSynchronize(stream);
        for (void* a : allocs) (void)hipFree(a);
        if (fl_host) (void)hipHostFree(fl_host);
        if (k_host) (void)hipHostFree(k_host);
        if (ev_k) (void)hipEventDestroy(ev_k);
        for (auto& g : graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
        }
        for (auto e : tev) (void)hipEventDestroy(e);
        for (auto e : {ev_chunk[0], ev_chunk[1], ev_t0, ev_t1, ev_p0[0], ev_p0[1], ev_p1[0], ev_p1[1]})
            if (e) (void)hipEventDestroy(e);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

// ==========================================================================
// launch helpers
// ==========================================================================
namespace {

constexpr int kLrBlocks = 256;   // blocks of the U^T p partial pass
// Attempt cap of a constraint-block-preconditioned solve: the larger of
// kPrecAttemptIters and kPrecAttemptGrowth times the longest converged
// constraint-block solve of the run so far.  Its solves take tens of
// iterations when the preconditioner is sound and the H part well
// conditioned; with an ill-conditioned H part their counts grow steadily
// over the IPM (hundreds, then thousands), which is no reason to leave the
// block, while a block that has lost definiteness (below) usually shows it
// at once through r^T z <= 0 (a breakdown) and otherwise stops converging.
constexpr int kPrecAttemptIters = 2000;
constexpr int kPrecAttemptGrowth = 4;

// The constraint-block preconditioner subtracts from D^-1 a Woodbury
// correction that nearly cancels it in the row space of the active rows of
// A; late in the IPM (Sigma_A -> infinity, cond(S) beyond about 1e8) its
// rounding can make the computed preconditioner indefinite, and PCG then
// cannot converge.  While an entry point holds this guard its
// constraint-block solves stop at the attempt cap; the caller repeats a
// solve that hits the cap (or breaks down) with the next preconditioner tier.
struct PrecAttemptCap {
    qp_handle* h;
    explicit PrecAttemptCap(qp_handle* hh) : h(hh) {
        h->wb_attempt_cap = kPrecAttemptIters;
        h->wb_seen = 0;
    }
    ~PrecAttemptCap() { h->wb_attempt_cap = 0; }
};
int wb_attempt_cap(const qp_handle* h) {
    return std::max(h->wb_attempt_cap, kPrecAttemptGrowth * h->wb_seen);
}
// A constraint-block solve ended in a way that calls for the next tier (a
// cap of pcg_max_iter itself, when not above the attempt cap, is final).
bool prec_stalled(const qp_handle* h, const Flags& f) {
    return f.pcg_breakdown || (f.pcg_capped && h->wb_cap_used < h->set.pcg_max_iter);
}
// Record a finished constraint-block solve for the attempt cap.
void note_wb_solve(qp_handle* h, const Flags& f) {
    if (f.pcg_converged && !f.ipm_done) h->wb_seen = std::max(h->wb_seen, int(f.pcg_iters));
}
// Preconditioner tiers of a QP: the constraint block; the capped block
// (Sigma of the dense block limited so that S_ii <= 1 + kPrecCapTau), used
// once the exact block has stalled or broken down; the Jacobi diagonal, once
// the capped block has too.  A QP moves down the tiers only, and keeps its
// tier for the rest of its run.
constexpr double kPrecCapTau = 1e4;
enum { TIER_BLOCK = 0, TIER_CAPPED = 1, TIER_JACOBI = 2 };
double tier_tau(int tier) { return tier == TIER_CAPPED ? kPrecCapTau : 0.0; }
constexpr int kGraphIters = 4;   // PCG iterations per captured graph (and per trailing chunk)

// Where an operator product keeps its intermediates, and the stream it is
// enqueued on: the handle's own buffers, or (qp_operator_apply_noalloc) the
// library's static scratch array and the caller's stream.
struct OpWork {
    hipStream_t st;
    double* t;         // W .* (J p), CSR format (nJ)
    double* c;         // per-slot J^T contributions, line format (nslots)
    double* u;         // Sigma_A .* (A p) (m)
    double* lr_part;   // U^T p partials (kLrBlocks * k)
    double* lr_v;      // w .* (U^T p) (k)
};
OpWork handle_work(qp_handle* h) { return OpWork{h->stream, h->t, h->lc, h->u, h->lr_part, h->lr_v}; }

// v = w .* (U^T p) for the low-rank part of H (no-op when k = 0); p is x, or
// x + beta*p2 in a PCG product.
void lowrank_prepare(qp_handle* h, const OpWork& wk, const double* x, const double* p2, const Flags* fl) {
    if (h->k == 0) return;
    const int gy = (h->k + 31) / 32;
    hipLaunchKernelGGL(k_lr_partial, dim3(kLrBlocks, gy), dim3(kBlock), 0, wk.st, (const double*)h->U, h->n,
                       h->k, x, p2, (const PcgScal*)h->psc, wk.lr_part, fl);
    hipLaunchKernelGGL(k_lr_reduce, dim3(1), dim3(kBlock), 0, wk.st, (const double*)wk.lr_part, kLrBlocks,
                       h->k, (const double*)h->w, wk.lr_v, fl);
    HIPCHK(hipGetLastError());
}
void lowrank_prepare(qp_handle* h, const double* x, const double* p2, const Flags* fl) {
    lowrank_prepare(h, handle_work(h), x, p2, fl);
}

int grid_elems(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    return int(std::max<int64_t>(1, std::min<int64_t>(g, kMaxElemGrid)));
}
int grid_rows(int64_t rows, int G) {
    const int rpb = kBlock / G;
    return int(std::max<int64_t>(1, (rows + rpb - 1) / rpb));
}
int grid_rows_capped(int64_t rows, int G) { return std::min(grid_rows(rows, G), kMaxPartials); }

// rb non-null: the rows of J in the nbs blocks of rb (k_op_fwd_stream), else
// G lanes per row (k_op_fwd).  nt (csr_streamed): the row-block pass reads
// J's values and column ids with non-temporal loads; its blocks read whole
// contiguous runs of them.  The G-lane pass keeps cacheable loads: its
// groups read a row in runs of G entries per load, and a run that ends
// inside a cache line leaves the rest of that line to the next load, which
// a non-temporal load would have evicted (measured: slower).
template <typename VT, typename AT>
void launch_fwd(hipStream_t st, int G, const FwdArgs<VT>& a0, int nbA, bool nt, const int2* rb = nullptr,
                int nbs = 0) {
    FwdArgs<VT> a = a0;
    a.nbJ = (a.nJ > 0) ? (rb ? nbs : grid_rows(a.nJ, G)) : 0;
    const int grid = a.nbJ + nbA;
    if (grid == 0) return;
    if (rb) {
        if (nt) hipLaunchKernelGGL((k_op_fwd_stream<VT, AT, true>), dim3(grid), dim3(kBlock), 0, st, a, rb);
        else hipLaunchKernelGGL((k_op_fwd_stream<VT, AT, false>), dim3(grid), dim3(kBlock), 0, st, a, rb);
        HIPCHK(hipGetLastError());
        return;
    }
    switch (G) {
        case 4: hipLaunchKernelGGL((k_op_fwd<4, VT, AT>), dim3(grid), dim3(kBlock), 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_op_fwd<8, VT, AT>), dim3(grid), dim3(kBlock), 0, st, a); break;
        case 16: hipLaunchKernelGGL((k_op_fwd<16, VT, AT>), dim3(grid), dim3(kBlock), 0, st, a); break;
        case 32: hipLaunchKernelGGL((k_op_fwd<32, VT, AT>), dim3(grid), dim3(kBlock), 0, st, a); break;
        default: hipLaunchKernelGGL((k_op_fwd<64, VT, AT>), dim3(grid), dim3(kBlock), 0, st, a); break;
    }
    HIPCHK(hipGetLastError());
}

// nt (csr_streamed): with 64 lanes per row, whose groups read whole runs of
// 64 entries per load, J^T's values and row ids are read with non-temporal
// loads; fewer lanes keep cacheable loads, as in the forward pass.
template <typename VT, typename AT>
int launch_bwd(hipStream_t st, int G, const BwdArgs<VT>& a, bool nt) {
    const int grid = grid_rows_capped(a.n, G);
    switch (G) {
        case 4: hipLaunchKernelGGL((k_op_bwd<4, VT, AT, false>), dim3(grid), dim3(kBlock), 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_op_bwd<8, VT, AT, false>), dim3(grid), dim3(kBlock), 0, st, a); break;
        case 16: hipLaunchKernelGGL((k_op_bwd<16, VT, AT, false>), dim3(grid), dim3(kBlock), 0, st, a); break;
        case 32: hipLaunchKernelGGL((k_op_bwd<32, VT, AT, false>), dim3(grid), dim3(kBlock), 0, st, a); break;
        default:
            if (nt) hipLaunchKernelGGL((k_op_bwd<64, VT, AT, true>), dim3(grid), dim3(kBlock), 0, st, a);
            else hipLaunchKernelGGL((k_op_bwd<64, VT, AT, false>), dim3(grid), dim3(kBlock), 0, st, a);
            break;
    }
    HIPCHK(hipGetLastError());
    return (a.n + kChunkRows - 1) / kChunkRows;   // p^T q partials: one per chunk of rows
}

template <typename VT>
void mat_ptrs(qp_handle* h, const VT*& jv, const VT*& jtv);
template <>
void mat_ptrs<double>(qp_handle* h, const double*& jv, const double*& jtv) { jv = h->Jv; jtv = h->Jtv; }
template <>
void mat_ptrs<float>(qp_handle* h, const float*& jv, const float*& jtv) { jv = h->Jv32; jtv = h->Jtv32; }
template <>
void mat_ptrs<bf16_t>(qp_handle* h, const bf16_t*& jv, const bf16_t*& jtv) { jv = h->Jv16; jtv = h->Jtv16; }

template <typename VT>
const VT* line_vals(qp_handle* h);
template <>
const double* line_vals<double>(qp_handle* h) { return h->lval; }
template <>
const float* line_vals<float>(qp_handle* h) { return h->lval32; }
template <>
const bf16_t* line_vals<bf16_t>(qp_handle* h) { return h->lval16; }

// Value arrays above this size are read with non-temporal loads
// (line_kernels.hpp: load_val): three quarters of the 256 MB last-level cache.
constexpr size_t kStreamedValueBytes = size_t(192) << 20;
template <typename VT>
bool line_vals_streamed(const qp_handle* h) {
    return size_t(h->nvals) * sizeof(VT) > kStreamedValueBytes;
}
// The CSR operator reads J's values and column ids once in each of its two
// passes (J, then the stored J^T): non-temporal when one pass's arrays
// exceed the same threshold.
template <typename VT>
bool csr_streamed(const qp_handle* h) {
    return size_t(h->nnzJ) * (sizeof(VT) + sizeof(int)) > kStreamedValueBytes;
}

// PCG link of a product: in a PCG product (pcg = true) the gathered vector is
// z + beta*p and p is written back.
PcgLink pcg_link(qp_handle* h, bool pcg) {
    PcgLink l{};
    if (pcg) {
        l.p2 = h->pp;
        l.sc = h->psc;
    }
    return l;
}

// q = K p on the line format of J (same contract as apply_op): the line pass
// (J and the per-slot J^T contributions, A) and the spot pass.
constexpr int kSpotLanes = 16;

// Arguments of the two kernels of a line-format product (shared by single
// solves and batched ones).
template <typename VT>
LineArgs<VT> line_args(qp_handle* h, const OpWork& wk, const double* x, double* q, const double* sigA, bool pcg) {
    const PcgLink pl = pcg_link(h, pcg);
    double* part = pcg ? h->part : nullptr;
    LineArgs<VT> f{};
    f.lptr = h->lptr; f.lcol = h->lcol; f.lval = line_vals<VT>(h); f.L = h->L; f.W = h->W;
    f.Ap = h->Ap; f.Ac = h->Ac; f.Av = h->Av; f.m = sigA ? h->m : 0;
    f.x = x; f.p2 = pl.p2; f.sc = h->psc; f.c = wk.c; f.u = wk.u; f.sigA = sigA; f.fl = pcg ? h->fl : nullptr;
    f.nbL = h->L;
    const int grid_spot = grid_rows_capped(h->n, kSpotLanes);
    const bool aug = h->aug && f.m > 0;
    if (aug) {   // lambda block on the rows of A, one per workgroup
        f.nbA = f.m;
        f.aug.dlu = h->dlu; f.aug.q = q; f.aug.n = h->n; f.aug.part = part ? part + grid_spot : nullptr;
    } else if (pcg && f.m > 0) {   // A p from A z (k_pcg_scalars) and the previous A p
        f.az = h->az;
        f.apv = h->apv;
        f.nbU = std::min((f.m + kBlock - 1) / kBlock, 64);
    } else {
        f.nbA = f.m;
    }
    return f;
}
template <typename VT>
int line_blocks(const LineArgs<VT>& f) { return std::max(1, f.nbL + f.nbA + f.nbU); }

SpotArgs spot_args(qp_handle* h, const OpWork& wk, const double* x, double* q, const double* sigx,
                   const double* sigA, double hs, bool pcg) {
    SpotArgs b{};
    b.sptr = h->sptr; b.sslot = h->sslot; b.c = wk.c; b.n = h->n;
    b.Atp = h->Atp; b.Atc = h->Atc; b.Atv = h->Atv; b.hasA = (sigA && h->m > 0) ? 1 : 0;
    b.u = wk.u; b.x = x; b.sigx = sigx; b.hs = hs; b.gamma = h->gamma;
    b.q = q; b.part = pcg ? h->part : nullptr; b.fl = pcg ? h->fl : nullptr; b.pcg = pcg_link(h, pcg);
    b.U = h->U; b.lr_v = wk.lr_v; b.lr_k = h->k;
    return b;
}
int spot_blocks(const qp_handle* h) { return grid_rows_capped(h->n, kSpotLanes); }
// p^T q partials of a PCG product on the line format
int line_pq_partials(const qp_handle* h, const double* sigA) {
    return spot_blocks(h) + ((h->aug && sigA && h->m > 0) ? h->m : 0);
}

template <typename VT, typename AT>
int apply_op_line(qp_handle* h, const OpWork& wk, const double* x, double* q, const double* sigx,
                  const double* sigA, double hs, bool pcg, bool timed, int tslot) {
    const LineArgs<VT> f = line_args<VT>(h, wk, x, q, sigA, pcg);
    if (timed) HIPCHK(hipEventRecord(h->tev[4 * tslot], wk.st));
    const dim3 lgrid(line_blocks(f));
    if (line_vals_streamed<VT>(h))
        hipLaunchKernelGGL((k_line_pass<VT, AT, true>), lgrid, dim3(kBlock), 0, wk.st, f);
    else
        hipLaunchKernelGGL((k_line_pass<VT, AT, false>), lgrid, dim3(kBlock), 0, wk.st, f);
    HIPCHK(hipGetLastError());
    if (timed) HIPCHK(hipEventRecord(h->tev[4 * tslot + 1], wk.st));
    lowrank_prepare(h, wk, x, f.p2, f.fl);
    const SpotArgs b = spot_args(h, wk, x, q, sigx, sigA, hs, pcg);
    if (timed) HIPCHK(hipEventRecord(h->tev[4 * tslot + 2], wk.st));
    hipLaunchKernelGGL(k_spot_pass<kSpotLanes>, dim3(spot_blocks(h)), dim3(kBlock), 0, wk.st, b);
    HIPCHK(hipGetLastError());
    if (timed) HIPCHK(hipEventRecord(h->tev[4 * tslot + 3], wk.st));
    return pcg ? line_pq_partials(h, sigA) : 0;
}

// q = K p with K = hs*H + diag(sigx) + A^T diag(sigA) A.  pcg = false: p = x,
// run unconditionally; pcg = true: p = z + beta*p of the PCG iteration
// (x = z), skipped once the solve has stopped.  Returns the number of p^T q
// partials (0 when pcg is false).
template <typename VT, typename AT>
int apply_op(qp_handle* h, const OpWork& wk, const double* x, double* q, const double* sigx, const double* sigA,
             double hs, bool pcg, bool timed, int tslot) {
    const PcgLink pl = pcg_link(h, pcg);
    const Flags* fl = pcg ? h->fl : nullptr;
    double* part = pcg ? h->part : nullptr;
    FwdArgs<VT> f{};
    const VT *jv = nullptr, *jtv = nullptr;
    mat_ptrs<VT>(h, jv, jtv);
    f.Jp = h->Jp; f.Jc = h->Jc; f.Jv = jv; f.W = h->W; f.nJ = h->nJ;
    f.Ap = h->Ap; f.Ac = h->Ac; f.Av = h->Av; f.m = sigA ? h->m : 0;
    f.x = x; f.p2 = pl.p2; f.sc = h->psc; f.t = wk.t; f.u = wk.u; f.sigA = sigA; f.fl = fl;
    const int nbA = f.m > 0 ? grid_rows(f.m, 64) : 0;
    const int n_pq_x = (h->n + kChunkRows - 1) / kChunkRows;   // k_op_bwd's p^T q partials
    const bool aug = h->aug && f.m > 0;
    if (aug) {
        f.aug.dlu = h->dlu; f.aug.q = q; f.aug.n = h->n; f.aug.part = part ? part + n_pq_x : nullptr;
    }
    if (timed) HIPCHK(hipEventRecord(h->tev[4 * tslot], wk.st));
    launch_fwd<VT, AT>(wk.st, h->GJ, f, nbA, csr_streamed<VT>(h), h->fwd_stream ? h->jrb : nullptr, h->nbs);
    if (timed) HIPCHK(hipEventRecord(h->tev[4 * tslot + 1], wk.st));
    lowrank_prepare(h, wk, x, pl.p2, fl);
    BwdArgs<VT> b{};
    b.Jtp = h->Jtp; b.Jtc = h->Jtc; b.Jtv = jtv; b.n = h->n;
    b.Atp = h->Atp; b.Atc = h->Atc; b.Atv = h->Atv; b.hasA = f.m > 0;
    b.t = wk.t; b.u = wk.u; b.x = x; b.sigx = sigx; b.hs = hs; b.gamma = h->gamma;
    b.q = q; b.part = part; b.fl = fl; b.pcg = pl;
    b.U = h->U; b.lr_v = wk.lr_v; b.lr_k = h->k;
    if (timed) HIPCHK(hipEventRecord(h->tev[4 * tslot + 2], wk.st));
    const int g = launch_bwd<VT, AT>(wk.st, h->GJt, b, csr_streamed<VT>(h));
    if (timed) HIPCHK(hipEventRecord(h->tev[4 * tslot + 3], wk.st));
    return part ? g + (aug ? f.m : 0) : 0;
}

int apply_op_prec(qp_handle* h, const OpWork& wk, int prec, const double* x, double* q, const double* sigx,
                  const double* sigA, double hs, bool pcg, bool timed, int tslot) {
    if (h->line) {
        switch (prec) {
            case QP_FP32: return apply_op_line<float, float>(h, wk, x, q, sigx, sigA, hs, pcg, timed, tslot);
            case QP_BF16: return apply_op_line<bf16_t, float>(h, wk, x, q, sigx, sigA, hs, pcg, timed, tslot);
            default: return apply_op_line<double, double>(h, wk, x, q, sigx, sigA, hs, pcg, timed, tslot);
        }
    }
    switch (prec) {
        case QP_FP32: return apply_op<float, float>(h, wk, x, q, sigx, sigA, hs, pcg, timed, tslot);
        case QP_BF16: return apply_op<bf16_t, float>(h, wk, x, q, sigx, sigA, hs, pcg, timed, tslot);
        default: return apply_op<double, double>(h, wk, x, q, sigx, sigA, hs, pcg, timed, tslot);
    }
}
int apply_op_prec(qp_handle* h, int prec, const double* x, double* q, const double* sigx, const double* sigA,
                  double hs, bool pcg, bool timed, int tslot) {
    return apply_op_prec(h, handle_work(h), prec, x, q, sigx, sigA, hs, pcg, timed, tslot);
}

// The operator's format and (CSR) schedule, as qp_info reports them.
void set_format_info(const qp_handle* h, qp_info* info) {
    info->spmv_format = h->line ? 1 : 0;
    info->spmv_schedule = h->line ? 0 : (h->fwd_stream ? 1 : h->GJ);
}

// SpMV schedule autotuner for CSR matrices: time each lane-group size for the
// J pass and the J^T pass, and the J pass over nonzero-balanced row blocks (a
// few launches each, HIP events), and keep the fastest; results are cached
// per (rows, cols, nnz) for the process.  Every schedule gives the same bits.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int64_t, int, int>, std::tuple<int, int, int>> g_tune_cache;

void autotune_schedule(qp_handle* h);

// Low-precision copies of J's values for the PCG operator, made on first use
// by rounding the resident FP64 values on the device: the line format's
// values when J has it (the CSR copies are then never read), else J's and
// J^T's CSR values.
void ensure_lowp(qp_handle* h, int prec) {
    if (prec != QP_FP32 && prec != QP_BF16) return;
    auto round = [&](const double* src, size_t count, void* dst) {
        const int g = int(std::max<size_t>(1, std::min<size_t>((count + kBlock - 1) / kBlock, 8192)));
        if (prec == QP_FP32)
            hipLaunchKernelGGL(k_round_f32, dim3(g), dim3(kBlock), 0, h->stream, src, count,
                               static_cast<uint32_t*>(dst));
        else
            hipLaunchKernelGGL(k_round_bf16, dim3(g), dim3(kBlock), 0, h->stream, src, count,
                               static_cast<uint16_t*>(dst));
        HIPCHK(hipGetLastError());
    };
    const size_t nz = size_t(h->nvals);
    if (h->line) {
        // packed slot groups (line_kernels.hpp: k_pack_line)
        auto pack = [&](auto* dst, auto tag) {
            using VT = decltype(tag);
            const size_t groups = size_t(h->nslots) / SlotPack<VT>::P;
            const int g = int(std::max<size_t>(1, std::min<size_t>((groups * 64 + kBlock - 1) / kBlock, 8192)));
            hipLaunchKernelGGL(k_pack_line<VT>, dim3(g), dim3(kBlock), 0, h->stream, (const double*)h->lval, groups,
                               reinterpret_cast<uint64_t*>(dst));
            HIPCHK(hipGetLastError());
        };
        if (prec == QP_FP32 && !h->lval32) {
            h->lval32 = h->dalloc<float>(nz);
            pack(h->lval32, float{});
        }
        if (prec == QP_BF16 && !h->lval16) {
            h->lval16 = h->dalloc<bf16_t>(nz);
            pack(h->lval16, bf16_t{});
        }
    } else {
        if (prec == QP_FP32 && !h->Jv32) {
            h->Jv32 = h->dalloc<float>(nz);
            h->Jtv32 = h->dalloc<float>(nz);
            round(h->Jv, nz, h->Jv32);
            round(h->Jtv, nz, h->Jtv32);
        }
        if (prec == QP_BF16 && !h->Jv16) {
            h->Jv16 = h->dalloc<bf16_t>(nz);
            h->Jtv16 = h->dalloc<bf16_t>(nz);
            round(h->Jv, nz, h->Jv16);
            round(h->Jtv, nz, h->Jtv16);
        }
    }
    HIPCHK(hipStreamSynchronize(h->stream));
}

struct TimingAcc {
    int pairs = 0;              // event pairs handed out
    std::vector<char> valid;    // slot ran real work (not a no-op launch after convergence)
};

// Constraint-block preconditioner for the current D = diag(Hs + Sigma_x) and
// Sigma_A: select the strong rows, fold the weak ones into Dw, form S over the
// strong rows, factor it and build S^{-1} (schur_kernels.hpp).  `stop`
// (device int, may be null) turns every launch into a no-op once set.
// Returns true when the dense block is non-empty (else Jacobi with d applies).
// tau > 0: the capped block (k_strong_rows).
bool build_precond(qp_handle* h, const double* D, const double* sigA, const int* stop, double tau = 0.0) {
    if (!h->woodbury) return false;
    const int m = h->m, n = h->n;
    hipLaunchKernelGGL(k_row_strength, dim3((m + 3) / 4), dim3(256), 0, h->stream, (const int*)h->Ap,
                       (const int*)h->Ac, (const double*)h->Av, D, sigA, m, h->rflag, h->rmii, stop);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, h->stream, (const int*)h->rflag, m, h->rpos, h->ridx,
                       h->kdev, stop);
    // k goes to the host as soon as it is known; the two kernels below keep
    // the device busy while the host waits for it
    HIPCHK(hipMemcpyAsync(h->k_host, h->kdev, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipEventRecord(h->ev_k, h->stream));
    hipLaunchKernelGGL(k_strong_rows, dim3((h->srows + 255) / 256), dim3(256), 0, h->stream, (const int*)h->Ap,
                       (const int*)h->ridx, sigA, (const double*)h->rmii, tau, (const int*)h->kdev, h->srows,
                       h->sext, h->ssq, stop);
    hipLaunchKernelGGL(k_fold_weak, dim3((n + 15) / 16), dim3(256), 0, h->stream, (const int*)h->Atp,
                       (const int*)h->Atc, (const double*)h->Atv, sigA, (const int*)h->rpos, D, n, h->Dw, h->scr,
                       h->scv, h->scnt, stop);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(h->ev_k));
    int k = *h->k_host;
    if (k < 0 || k > m) k = 0;   // never happens; keeps launch shapes in range
    h->kcur = k;
    h->ldcur = ((k + TS - 1) / TS) * TS;
    h->Tcur = h->ldcur / TS;
    if (k == 0) return false;
    const int ld = h->ldcur, T = h->Tcur;
    {   // wavefronts per row: as many as fit their LDS row copies in 64 KiB, at most 8
        const size_t row_bytes = size_t(ld) * sizeof(double);
        const int nw = row_bytes * 8 <= 64 * 1024   ? 8
                       : row_bytes * 4 <= 64 * 1024 ? 4
                       : row_bytes * 2 <= 64 * 1024 ? 2
                                                    : 1;
        auto kern = nw == 8   ? k_schur_form<8>
                    : nw == 4 ? k_schur_form<4>
                    : nw == 2 ? k_schur_form<2>
                              : k_schur_form<1>;
        hipLaunchKernelGGL(kern, dim3(ld), dim3(64 * nw), row_bytes * nw, h->stream, (const int*)h->Ap,
                           (const int*)h->Ac, (const double*)h->Av, (const int*)h->Atp, (const int*)h->scr,
                           (const double*)h->scv, (const int*)h->scnt, (const double*)h->Dw,
                           (const double*)h->ssq, (const int*)h->ridx, k, ld, h->Sm, stop);
    }
    HIPCHK(hipGetLastError());
    // sweep: S alternates between Sm and Sm2; P between the two halves of Pbuf
    double* Sb[2] = {h->Sm, h->Sm2};
    double* Pb[2] = {h->Pbuf, h->Pbuf + 2 * TS * TS};
    hipLaunchKernelGGL(k_gj_pivot0, dim3(1), dim3(256), 0, h->stream, (const double*)h->Sm, ld, Pb[0], stop);
    const int gx = (T + 1) / 2;
    for (int b = 0; b < T; ++b)
        hipLaunchKernelGGL(k_gj_step, dim3(gx * (gx + 1) / 2 + (b + 1 < T ? 1 : 0)), dim3(256), 0, h->stream,
                           (const double*)Sb[b & 1],
                           Sb[(b + 1) & 1], ld, T, b, (const double*)Pb[b & 1], Pb[(b + 1) & 1], stop);
    const double* Sfin = Sb[T & 1];
    HIPCHK(hipGetLastError());
    {
        const size_t N = size_t(ld) * ld;
        const int g = int(std::min<size_t>((N + 255) / 256, 4096));
        hipLaunchKernelGGL(k_symmetrize, dim3(g), dim3(256), 0, h->stream, Sfin, ld, h->Sinv, stop);
    }
    HIPCHK(hipGetLastError());
    return true;
}

// Step 1 of the constraint-block preconditioner on the strong rows of A; the
// grid covers the largest dense block (all m rows strong), kernels read the
// current k.
PrecRows prec_rows_args(qp_handle* h) {
    PrecRows pa{};
    pa.Ac = h->Ac; pa.Av = h->Av; pa.ext = h->sext; pa.sq = h->ssq;
    pa.kdev = h->kdev; pa.m = h->m;
    pa.w = h->wpre; pa.vm = h->vpre;
    return pa;
}
int prec_rows_blocks(const qp_handle* h) {
    const int rows_a = std::max(h->ld, (h->m + 63) / 64);
    return (rows_a + 3) / 4;
}

// Steps 2 and 3 of z = P^{-1} r for the constraint-block preconditioner
// (step 1 runs before: k_prec_a at the start of a solve, k_pcg_xr in an
// iteration, where q != null makes step 3 store r -= alpha q).  Step 3's
// blocks each leave one r^T z partial.
constexpr int kPrecAtLanes = 16;
SymvArgs symv_args(qp_handle* h) {
    SymvArgs a{};
    a.Sinv = h->Sinv; a.w = h->wpre; a.sq = h->ssq; a.idx = h->ridx; a.kdev = h->kdev; a.vm = h->vpre;
    a.fl = h->fl;
    return a;
}
PrecAtArgs prec_at_args(qp_handle* h, const double* D, const double* q) {
    PrecAtArgs a{};
    a.Atp = h->Atp; a.Atc = h->Atc; a.Atv = h->Atv; a.v = h->vpre; a.D = D; a.r = h->pr; a.q = q;
    a.sc = h->psc; a.z = h->pz; a.n = h->n; a.part_rz = h->part_rz; a.fl = h->fl;
    return a;
}

void autotune_schedule(qp_handle* h) {
    if (h->line || h->set.schedule != 0) return;
    const auto key = std::make_tuple(h->nJ, h->n, h->nnzJ, h->m, int(h->nnzA > 0));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            h->GJ = std::get<0>(it->second);
            h->GJt = std::get<1>(it->second);
            h->fwd_stream = std::get<2>(it->second) != 0;
            return;
        }
    }
    // lane counts (both passes), then the forward pass over row blocks (0)
    const int cand[] = {8, 16, 32, 64, 0};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best_f = 1e30f, best_b = 1e30f, t_stream = 1e30f;
    int gf = h->GJ, gb = h->GJt;
    auto timed = [&](auto&& launch) {
        HIPCHK(hipEventRecord(e0, h->stream));
        launch();
        HIPCHK(hipEventRecord(e1, h->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        return ms;
    };
    const bool nt = csr_streamed<double>(h);
    for (int g : cand) {
        if (g == 0 && !h->jrb) continue;
        float tf = 0.f, tb = 0.f;
        for (int rep = 0; rep < 4; ++rep) {   // first repetition warms up
            FwdArgs<double> f{};
            f.Jp = h->Jp; f.Jc = h->Jc; f.Jv = h->Jv; f.W = h->W; f.nJ = h->nJ;
            f.x = h->zero_n; f.t = h->t; f.u = h->u;
            const float mf = timed([&] { launch_fwd<double, double>(h->stream, g ? g : 64, f, 0, nt,
                                                                     g ? nullptr : h->jrb, h->nbs); });
            if (rep) tf += mf;
            if (g == 0) continue;
            BwdArgs<double> b{};
            b.Jtp = h->Jtp; b.Jtc = h->Jtc; b.Jtv = h->Jtv; b.n = h->n;
            b.Atp = h->Atp; b.Atc = h->Atc; b.Atv = h->Atv; b.hasA = h->m > 0;
            b.t = h->t; b.u = h->zero_m; b.x = h->zero_n; b.hs = 1.0; b.q = h->tmp_n;
            const float mb = timed([&] { launch_bwd<double, double>(h->stream, g, b, nt); });
            if (rep) tb += mb;
        }
        if (g == 0) {
            t_stream = tf;
            continue;
        }
        if (tf < best_f) { best_f = tf; gf = g; }
        if (tb < best_b) { best_b = tb; gb = g; }
    }
    h->GJ = gf;   // also the lane count of the residual pass's rows of J
    h->GJt = gb;
    h->fwd_stream = t_stream < best_f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = std::make_tuple(gf, gb, int(h->fwd_stream));
}

// One PCG solve of K dx = rhs (rhs = mu*rhs_a + rhs_b when rhs_a is given, mu
// read on the device).  Preconditioner: Jacobi with d, or (h->woodbury and
// sigA given) the constraint block with D = dh.  dx is written to h->px.
// Returns the flags after the solve.
// Launch arguments of one PCG solve of a QP (shared by run_pcg and the
// batched solves): the start (k_pcg_init0, the preconditioner's first
// application, k_pcg_scalars in mode 1 or 2) and the iterations (k_pcg_xr,
// steps 2 and 3 of the preconditioner, k_pcg_scalars in mode 0), with the
// grid of each.
struct PcgSetup {
    int n = 0, ge = 0, wb = 0, n_rz = 0, gs = 0;
    PcgInitArgs ia{};
    PrecAArgs prea{};      // wb: step 1 at the start
    SymvArgs sy{};         // wb: step 2
    PrecAtArgs at0{}, at{};   // wb: step 3 at the start / in an iteration
    ScalArgs sa{}, si{};   // start / iteration
    PcgArgs pa{};          // pa.n_pq is the product's to fill
    int nb_preca = 0, nb_symv = 0, nb_at = 0, nb_xr = 0;
};

PcgSetup pcg_setup(qp_handle* h, const double* rhs_a, const double* rhs_b, const double* sigA, const double* d,
                   const double* dh, bool ipm_mode, double rel_tol, bool refine) {
    PcgSetup S;
    // vector length of the system: n, or n + 2m for the doubly augmented one
    const int n = h->aug ? h->n + 2 * h->m : h->n;
    S.n = n;
    S.ge = grid_elems(n);
    // dh != null selects the constraint-block preconditioner (built for this Sigma)
    S.wb = (h->woodbury && sigA && dh) ? 1 : 0;
    const double* dd = S.wb ? dh : d;
    PcgInitArgs& ia = S.ia;
    ia.n = n; ia.rhs_a = rhs_a; ia.rhs_b = rhs_b; ia.ipm = ipm_mode ? h->isc : nullptr;
    ia.x = h->px; ia.r = h->pr; ia.z = h->pz; ia.p = h->pp; ia.d = dd;
    ia.part_rz = h->part_rz; ia.part_rr = h->part_rr; ia.woodbury = S.wb; ia.fl = h->fl;
    // line format: the product forms A p = A z + beta A p, with A z from the
    // scalar kernel's other blocks
    AzArgs az{};
    if (h->line && sigA && h->m > 0 && !h->aug) {
        az.Ap = h->Ap; az.Ac = h->Ac; az.Av = h->Av; az.z = h->pz; az.m = h->m; az.az = h->az;
        ia.apv = h->apv; ia.m = h->m;
    }
    S.gs = 1 + (az.m + kBlock / 64 - 1) / (kBlock / 64);
    if (S.wb) {
        S.prea.pa = prec_rows_args(h); S.prea.y = h->pz; S.prea.fl = h->fl;
        S.nb_preca = prec_rows_blocks(h);
        S.sy = symv_args(h);
        S.nb_symv = (h->m + 3) / 4;
        S.at0 = prec_at_args(h, dh, nullptr);
        S.at = prec_at_args(h, dh, h->pq);
        S.nb_at = grid_rows_capped(h->n, kPrecAtLanes);
    }
    S.n_rz = S.wb ? S.nb_at : S.ge;
    const int cap = (S.wb && h->wb_attempt_cap > 0) ? std::min(h->set.pcg_max_iter, h->wb_cap_dir)
                                                    : h->set.pcg_max_iter;
    if (S.wb) h->wb_cap_used = cap;
    ScalArgs& sa = S.sa;
    sa.part_rz = h->part_rz; sa.n_rz = S.n_rz; sa.part_rr = h->part_rr; sa.n_rr = S.ge;
    sa.mode = refine ? 2 : 1; sa.rel_tol = rel_tol; sa.tol = h->set.pcg_tol; sa.max_iter = cap;
    sa.sc = h->psc; sa.fl = h->fl; sa.az = az;
    S.si = sa;   // the iterations' update
    S.si.mode = 0; S.si.rel_tol = 0.0; S.si.tol = 0.0; S.si.max_iter = 0;
    PcgArgs& pa = S.pa;
    pa.n = n; pa.x = h->px; pa.r = h->pr; pa.z = h->pz; pa.p = h->pp; pa.q = h->pq; pa.d = dd;
    pa.part_pq = h->part; pa.part_rz = h->part_rz; pa.part_rr = h->part_rr;
    pa.woodbury = S.wb; pa.sc = h->psc; pa.fl = h->fl;
    if (S.wb) {
        pa.pa = prec_rows_args(h);
        pa.nbA = prec_rows_blocks(h);
    }
    S.nb_xr = pa.nbA + S.ge;
    return S;
}

// One PCG solve of K dx = rhs (rhs = mu*rhs_a + rhs_b when rhs_a is given, mu
// read on the device).  Preconditioner: Jacobi with d, or (h->woodbury and
// sigA given) the constraint block with D = dh.  dx is written to h->px.
// Returns the flags after the solve.
Flags run_pcg(qp_handle* h, int prec, const double* rhs_a, const double* rhs_b, const double* sigx,
              const double* sigA, const double* d, const double* dh, double hs, bool ipm_mode, TimingAcc* tacc,
              double rel_tol, bool refine, bool check_only = false) {
    PcgSetup S = pcg_setup(h, rhs_a, rhs_b, sigA, d, dh, ipm_mode, rel_tol, refine);
    const int wb = S.wb, n_rz = S.n_rz, ge = S.ge, gs = S.gs;
    hipLaunchKernelGGL(k_pcg_init0, dim3(ge), dim3(kBlock), 0, h->stream, S.ia);
    HIPCHK(hipGetLastError());
    if (wb) {
        hipLaunchKernelGGL(k_prec_a, dim3(S.nb_preca), dim3(kBlock), 0, h->stream, S.prea);
        hipLaunchKernelGGL(k_prec_symv, dim3(S.nb_symv), dim3(kBlock), 0, h->stream, S.sy);
        hipLaunchKernelGGL(k_prec_at<kPrecAtLanes>, dim3(S.nb_at), dim3(kBlock), 0, h->stream, S.at0);
        HIPCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_pcg_scalars, dim3(gs), dim3(kBlock), 0, h->stream, S.sa);
    HIPCHK(hipGetLastError());
    const ScalArgs si = S.si;

    if (refine) {
        // A refinement solve is often converged at its start (the FP64
        // residual already meets pcg_tol): find out before queuing iterations.
        HIPCHK(hipMemcpyAsync(&h->fl_host[0], h->fl, sizeof(Flags), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        const Flags f0 = h->fl_host[0];
        if (f0.pcg_converged || f0.pcg_breakdown || f0.pcg_capped || f0.ipm_done || check_only) return f0;
    }

    PcgArgs pa = S.pa;

    const bool timing = h->set.timing != 0 && tacc != nullptr;
    const int slot_begin = tacc ? tacc->pairs : 0;
    auto one_iter = [&]() {
        bool timed = false;
        int slot = 0;
        if (timing && tacc->pairs < int(h->tev.size() / 4)) {
            timed = true;
            slot = tacc->pairs++;
            tacc->valid.push_back(1);
        }
        pa.n_pq = apply_op_prec(h, prec, h->pz, h->pq, sigx, sigA, hs, true, timed, slot);
        hipLaunchKernelGGL(k_pcg_xr, dim3(S.nb_xr), dim3(kBlock), 0, h->stream, pa);
        if (wb) {
            hipLaunchKernelGGL(k_prec_symv, dim3(S.nb_symv), dim3(kBlock), 0, h->stream, S.sy);
            hipLaunchKernelGGL(k_prec_at<kPrecAtLanes>, dim3(S.nb_at), dim3(kBlock), 0, h->stream, S.at);
        }
        hipLaunchKernelGGL(k_pcg_scalars, dim3(gs), dim3(kBlock), 0, h->stream, si);
    };
    // Graph mode: the iterations of this operator are captured once as a graph
    // of kGraphIters iterations and replayed (one launch call per kGraphIters
    // iterations instead of one per kernel).  Every dynamic quantity of an
    // iteration lives in device memory, so replays are exact repeats of the
    // direct launches.
    hipGraphExec_t gexec = nullptr;
    if (h->set.graphs && !timing && !h->graphs_failed) {
        const void* ops[4] = {sigx, sigA, d, dh};
        for (auto& g : h->graphs)
            if (g.prec == prec && g.wb == wb && g.n_rz == n_rz && g.hs == hs && g.aug == h->aug && g.ops[0] == ops[0] &&
                g.ops[1] == ops[1] && g.ops[2] == ops[2] && g.ops[3] == ops[3])
                gexec = g.exec;
        if (!gexec) {
            hipGraph_t graph = nullptr;
            bool ok = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                try {
                    for (int i = 0; i < kGraphIters; ++i) one_iter();
                } catch (...) {
                    (void)hipStreamEndCapture(h->stream, &graph);
                    if (graph) (void)hipGraphDestroy(graph);
                    throw;
                }
                ok = hipStreamEndCapture(h->stream, &graph) == hipSuccess && graph != nullptr;
                if (ok) ok = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) == hipSuccess;
                if (!ok && graph) {
                    (void)hipGraphDestroy(graph);
                    graph = nullptr;
                }
            }
            if (ok) {
                if (h->graphs.size() >= 8) {   // keep a few operators per handle
                    // the evicted graph may still be queued on the stream
                    HIPCHK(hipStreamSynchronize(h->stream));
                    (void)hipGraphExecDestroy(h->graphs.front().exec);
                    (void)hipGraphDestroy(h->graphs.front().graph);
                    h->graphs.erase(h->graphs.begin());
                }
                qp_handle::PcgGraph g;
                g.prec = prec; g.wb = wb; g.n_rz = n_rz; g.hs = hs; g.aug = h->aug;
                for (int i = 0; i < 4; ++i) g.ops[i] = ops[i];
                g.graph = graph;
                g.exec = gexec;
                h->graphs.push_back(g);
            } else {
                (void)hipGetLastError();   // capture unsupported here: launch directly from now on
                h->graphs_failed = true;
                gexec = nullptr;
            }
        }
    }
    auto queue = [&](int iters) {   // iters is a multiple of kGraphIters in graph mode
        if (gexec)
            for (int i = 0; i < iters; i += kGraphIters) HIPCHK(hipGraphLaunch(gexec, h->stream));
        else
            for (int i = 0; i < iters; ++i) one_iter();
    };
    auto snapshot = [&](int slot) {
        HIPCHK(hipMemcpyAsync(&h->fl_host[slot], h->fl, sizeof(Flags), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipEventRecord(h->ev_chunk[slot], h->stream));
    };
    auto stop = [&](const Flags& f) {
        return f.pcg_converged || f.pcg_breakdown || f.pcg_capped || f.ipm_done;
    };
    // Chunks of iterations are queued ahead of the host check: kernels of a
    // finished solve return at once, so the GPU never waits on the host.  The
    // first chunk covers most of the smaller of the two previous solves'
    // iteration counts of the same kind (consecutive IPM directions alternate
    // between short and long solves; refinement solves are shorter than
    // first solves); later chunks are kGraphIters iterations, so few no-op
    // launches trail the converged iteration.
    int* hist = h->last_pcg_iters[refine ? 1 : 0];
    const int pred = std::min(hist[0], hist[1]);
    int chunk = std::max(kGraphIters, std::min(512, (pred * 3) / 4));
    chunk = ((chunk + kGraphIters - 1) / kGraphIters) * kGraphIters;
    int64_t launched = 0;
    const int64_t guard = int64_t(h->set.pcg_max_iter) + 4096;
    int cur = 0;
    queue(chunk);
    launched += chunk;
    snapshot(cur);
    Flags f{};
    while (true) {
        chunk = kGraphIters;
        queue(chunk);
        launched += chunk;
        snapshot(cur ^ 1);
        HIPCHK(hipEventSynchronize(h->ev_chunk[cur]));
        f = h->fl_host[cur];
        // A stopped solve's flags no longer change: the chunk queued behind
        // this snapshot runs as no-ops while the host queues what follows.
        if (stop(f)) break;
        if (launched > guard) {
            HIPCHK(hipEventSynchronize(h->ev_chunk[cur ^ 1]));
            f = h->fl_host[cur ^ 1];
            break;
        }
        cur ^= 1;
    }
    if (!f.ipm_done) {
        hist[1] = hist[0];
        hist[0] = f.pcg_iters;
    }
    if (wb) note_wb_solve(h, f);
    if (timing) {
        // launches past the last executed iteration returned at once: drop them
        for (int sl = slot_begin + std::max(f.pcg_iters, 0); sl < tacc->pairs; ++sl) tacc->valid[sl] = 0;
        if (f.ipm_done)
            for (int sl = slot_begin; sl < tacc->pairs; ++sl) tacc->valid[sl] = 0;
    }
    return f;
}

// One Newton direction into h->px.  FP64: one PCG solve to pcg_tol.
// FP32/BF16: PCG on the low-precision operator to refine_tol, then up to
// `refine_steps` passes of rho = rhs - K_64 dx (FP64 operator),
// delta = PCG_lo(rho) (to refine_tol of rho, but never below pcg_tol of the
// original rhs), dx += delta; a pass whose rho already meets pcg_tol * ||rhs||
// takes no iteration and ends the refinement.  rhs = mu*rhs_a + rhs_b
// (ipm_mode) or rhs_b.  The returned flags carry the PCG iteration count
// summed over the solves; `solves` counts them.
Flags newton_direction(qp_handle* h, int prec, const double* rhs_a, const double* rhs_b, const double* sigx,
                       const double* sigA, const double* d, const double* dh, double hs, bool ipm_mode,
                       TimingAcc* tacc, int* solves) {
    const double tol = h->set.pcg_tol;
    h->wb_cap_dir = wb_attempt_cap(h);   // one attempt cap for all solves of this direction
    if (prec == QP_FP64) {
        *solves = 1;
        return run_pcg(h, QP_FP64, rhs_a, rhs_b, sigx, sigA, d, dh, hs, ipm_mode, tacc, tol, false);
    }
    const int n = h->aug ? h->n + 2 * h->m : h->n;
    const int ge = grid_elems(n);
    const double* rhs = rhs_b;
    if (rhs_a) {
        hipLaunchKernelGGL(k_rhs_combine, dim3(ge), dim3(kBlock), 0, h->stream, n, rhs_a, rhs_b,
                           (const IpmScal*)h->isc, h->rhs_full, (const Flags*)h->fl);
        HIPCHK(hipGetLastError());
        rhs = h->rhs_full;
    }
    const double inner = h->set.refine_steps > 0 ? std::max(h->set.refine_tol, tol) : tol;
    Flags f = run_pcg(h, prec, nullptr, rhs, sigx, sigA, d, dh, hs, false, tacc, inner, false);
    *solves = 1;
    int total = f.pcg_iters;
    if (f.ipm_done || f.pcg_breakdown || h->set.refine_steps == 0) return f;   // 0: no refinement
    hipLaunchKernelGGL(k_acc, dim3(ge), dim3(kBlock), 0, h->stream, n, h->dxacc, (const double*)h->px, 1,
                       (const Flags*)h->fl);
    // Passes k < refine_steps correct dx; the pass after the last correction
    // only checks its FP64 residual.
    bool met = false;
    for (int k = 0; k <= h->set.refine_steps; ++k) {
        apply_op_prec(h, QP_FP64, h->dxacc, h->pq, sigx, sigA, hs, false, false, 0);
        hipLaunchKernelGGL(k_sub, dim3(ge), dim3(kBlock), 0, h->stream, n, rhs, (const double*)h->pq, h->rho,
                           (const Flags*)h->fl);
        const bool check = k == h->set.refine_steps;
        Flags f2 = run_pcg(h, prec, nullptr, h->rho, sigx, sigA, d, dh, hs, false, tacc, inner, true, check);
        if (f2.ipm_done) return f2;
        met = f2.pcg_iters == 0 && f2.pcg_converged;   // the FP64 residual already meets pcg_tol
        if (check) break;
        *solves += 1;
        total += f2.pcg_iters;
        f.pcg_capped |= f2.pcg_capped;
        f.pcg_converged = f2.pcg_converged;
        if (f2.pcg_breakdown) {
            // a zero residual (exact direction) is not a breakdown; rr == 0 stops at init
            f.pcg_breakdown = 1;
            break;
        }
        if (met) break;
        hipLaunchKernelGGL(k_acc, dim3(ge), dim3(kBlock), 0, h->stream, n, h->dxacc, (const double*)h->px, 0,
                           (const Flags*)h->fl);
    }
    if (!met && !f.pcg_breakdown) {
        // Refinement converges only while the low-precision operator is close
        // enough to K (spectral radius of I - K_lo^-1 K below 1).  Where it is
        // not -- e.g. J without full column rank and a small gamma, where
        // rounding J moves the eigenvalues near gamma by far more than
        // gamma -- the direction is solved in FP64 instead.
        Flags f3 = run_pcg(h, QP_FP64, nullptr, rhs, sigx, sigA, d, dh, hs, false, tacc, tol, false);
        *solves += 1;
        f3.pcg_iters += total;
        f3.pcg_capped |= f.pcg_capped;
        return f3;
    }
    HIPCHK(hipMemcpyAsync(h->px, h->dxacc, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipGetLastError());
    f.pcg_iters = total;
    return f;
}

void reset_flags(qp_handle* h) {
    Flags z{};
    HIPCHK(hipMemcpyAsync(h->fl, &z, sizeof(Flags), hipMemcpyHostToDevice, h->stream));
}

void harvest_timing(qp_handle* h, const TimingAcc& ta, qp_info* info) {
    if (!info) return;
    double f = 0.0, b = 0.0;
    int64_t cnt = 0;
    for (int i = 0; i < ta.pairs; ++i) {
        if (i < int(ta.valid.size()) && !ta.valid[i]) continue;
        ++cnt;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->tev[4 * i], h->tev[4 * i + 1]));
        f += ms;
        HIPCHK(hipEventElapsedTime(&ms, h->tev[4 * i + 2], h->tev[4 * i + 3]));
        b += ms;
    }
    info->t_spmv_fwd_ms += f;
    info->t_spmv_bwd_ms += b;
    info->n_spmv_fwd += cnt;
    info->n_spmv_bwd += cnt;
}

void ensure_timing_events(qp_handle* h) {
    if (h->set.timing && h->tev.empty()) {
        h->tev.resize(4 * 1024);
        for (auto& e : h->tev) HIPCHK(hipEventCreate(&e));
    }
}

// diag(H) = gamma + sum_i W_i J_ij^2 + sum_c w_c U_jc^2 into h->diagH: from
// the line format (per-slot weighted squares in h->lc, then per spot), or
// from the CSR rows of J^T.
void compute_diag_h(qp_handle* h) {
    if (h->line) {
        if (h->L > 0)
            hipLaunchKernelGGL(k_line_diag, dim3(h->L), dim3(kBlock), 0, h->stream, (const int*)h->lptr,
                               (const double*)h->lval, (const double*)h->W, h->L, h->lc);
        hipLaunchKernelGGL(k_spot_diag<kSpotLanes>, dim3(grid_rows(h->n, kSpotLanes)), dim3(kBlock), 0, h->stream,
                           (const int*)h->sptr, (const int*)h->sslot, (const double*)h->lc, h->n, h->gamma,
                           (const double*)h->U, (const double*)h->w, h->k, h->diagH);
        HIPCHK(hipGetLastError());
        return;
    }
    const int G = 64;
    hipLaunchKernelGGL(k_diag_h<G>, dim3(grid_rows(h->n, G)), dim3(kBlock), 0, h->stream, (const int*)h->Jtp,
                       (const int*)h->Jtc, (const double*)h->Jtv, (const double*)h->W, h->n, h->gamma,
                       (const double*)h->U, (const double*)h->w, h->k, h->diagH);
    HIPCHK(hipGetLastError());
}

// Captured PCG graphs hold gamma, U and k by value: a new objective drops them.
void drop_graphs(qp_handle* h) {
    if (!h->graphs.empty()) HIPCHK(hipStreamSynchronize(h->stream));
    for (auto& g : h->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    h->graphs.clear();
}

qp_status fail(qp_handle* h, qp_status st, const std::string& msg) {
    if (h) h->err = msg;
    return st;
}

// --------------------------------------------------------------------------
// Scratch of qp_operator_apply_noalloc: one array per GPU, part of the
// library's code object (loaded with it, held until the process ends).  In
// host code its name is only a stand-in for the symbol; the device address
// comes from hipGetSymbolAddress, resolved once per device by
// resolve_scratch (qp_create, with the handle's device current) and kept
// per device.
// --------------------------------------------------------------------------
constexpr size_t kScratchDoubles = size_t(4) << 20;   // 32 MiB
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Device address of `scratch` on device dev (current), resolved on the first
// call for that device.
hipError_t resolve_scratch(int dev, double** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Layout of the scratch for one operator product of h: the per-slot sums
// (line format) or W .* (J p) (CSR), then Sigma_A .* (A p), then the low-rank
// partials and w .* (U^T p); each part starts on a 256-byte boundary.  Returns
// the doubles needed.
size_t scratch_layout(const qp_handle* h, size_t off[4]) {
    auto up = [](size_t v) { return (v + 31) / 32 * 32; };
    const size_t first = h->line ? size_t(h->nslots) : size_t(std::max(h->nJ, 1));
    off[0] = 0;
    off[1] = up(first);
    off[2] = off[1] + up(size_t(std::max(h->m, 1)));
    off[3] = off[2] + up(size_t(kLrBlocks) * size_t(h->k));
    return off[3] + up(size_t(h->k));
}


// ==========================================================================
// Algorithm 1 in phases: start, direction, step, finish.  qp_solve runs the
// phases of one QP in turn; qp_solve_batch interleaves the phases of many
// QPs around batched PCG solves.
// ==========================================================================

// State of one QP's run, kept between its phases.
struct IpmRun {
    qp_handle* h = nullptr;
    double hs = 1.0;              // objective scale 1/zeta
    bool wbp = false;             // constraint-block preconditioner built for the current iterate
    int tier = TIER_BLOCK;        // preconditioner tier (a stalled solve moves the QP down)
    int fallbacks = 0;
    int64_t pcg_total = 0;
    int pcg_solves = 0, capped = 0;
    float pcg_ms = 0.f;
    bool pcg_timed[2] = {false, false};
    int it = 0;                   // IPM iterations whose direction was computed
    bool done = false;            // the IPM has finished or stopped on an error
    qp_status st = QP_OK;
    TimingAcc ta;
};

// Residual pass at the current iterate (Algorithm 1, the residuals before
// the barrier rule): H x, A x, r_H, r_g, Sigma, the Jacobi diagonals, the
// right-hand side, and the barrier rule on the device (k_ipm_check; apply = 0
// at the start point).
void ipm_residuals(qp_handle* h, int apply) {
    const int n = h->n, m = h->m;
    IpmVec& v = h->iv;
    const int G = h->GJ, Gt = h->GJt;
    FwdArgs<double> f{};
    f.Jp = h->Jp; f.Jc = h->Jc; f.Jv = h->Jv; f.W = h->W; f.nJ = h->nJ;
    f.Ap = h->Ap; f.Ac = h->Ac; f.Av = h->Av; f.m = m;
    f.x = v.x; f.t = h->t; f.u = h->u; f.sigA = nullptr; f.fl = nullptr;
    // line format: J x and the per-slot shares of J^T W J x come from
    // one read of J in the line pass; k_ipm_fwd keeps the rows of A
    f.nbJ = (h->nJ > 0 && !h->line) ? grid_rows(h->nJ, G) : 0;
    const int nbA = m > 0 ? grid_rows(m, 64) : 0;
    if (h->line) {
        LineArgs<double> la{};
        la.lptr = h->lptr; la.lcol = h->lcol; la.lval = h->lval; la.L = h->L; la.W = h->W;
        la.x = v.x; la.c = h->lc; la.u = h->u; la.nbL = h->L; la.nbA = 0; la.fl_ipm = h->fl;
        if (line_vals_streamed<double>(h))
            hipLaunchKernelGGL((k_line_pass<double, double, true>), dim3(std::max(1, h->L)), dim3(kBlock), 0,
                               h->stream, la);
        else
            hipLaunchKernelGGL((k_line_pass<double, double, false>), dim3(std::max(1, h->L)), dim3(kBlock), 0,
                               h->stream, la);
        HIPCHK(hipGetLastError());
    }
    const int grid = std::max(1, f.nbJ + nbA);
    const IpmScal* isc = h->isc;
    const Flags* fl = h->fl;
    switch (G) {
        case 4: hipLaunchKernelGGL(k_ipm_fwd<4>, dim3(grid), dim3(kBlock), 0, h->stream, f, v, isc, h->partA, fl); break;
        case 8: hipLaunchKernelGGL(k_ipm_fwd<8>, dim3(grid), dim3(kBlock), 0, h->stream, f, v, isc, h->partA, fl); break;
        case 16: hipLaunchKernelGGL(k_ipm_fwd<16>, dim3(grid), dim3(kBlock), 0, h->stream, f, v, isc, h->partA, fl); break;
        case 32: hipLaunchKernelGGL(k_ipm_fwd<32>, dim3(grid), dim3(kBlock), 0, h->stream, f, v, isc, h->partA, fl); break;
        default: hipLaunchKernelGGL(k_ipm_fwd<64>, dim3(grid), dim3(kBlock), 0, h->stream, f, v, isc, h->partA, fl); break;
    }
    HIPCHK(hipGetLastError());
    IpmBwdArgs ba{};
    ba.Jtp = h->Jtp; ba.Jtc = h->Jtc; ba.Jtv = h->Jtv;
    if (h->line) { ba.sptr = h->sptr; ba.sslot = h->sslot; ba.lc = h->lc; }
    ba.Atp = h->Atp; ba.Atc = h->Atc; ba.Atv = h->Atv; ba.hasA = m > 0;
    ba.t = h->t; ba.gamma = h->gamma;
    ba.U = h->U; ba.lr_v = h->lr_v; ba.lr_k = h->k;
    ba.aug = h->aug ? 1 : 0;
    lowrank_prepare(h, v.x, nullptr, nullptr);
    // lanes per variable: with the line format a variable sums one
    // double per slot of its spot, not one term per nonzero of J
    const int Gb = h->line ? pick_lanes(h->nslots + h->nnzA, n) : Gt;
    const int gb = grid_rows_capped(n, Gb);
    switch (Gb) {
        case 4: hipLaunchKernelGGL(k_ipm_bwd<4>, dim3(gb), dim3(kBlock), 0, h->stream, ba, v, isc, h->part, fl); break;
        case 8: hipLaunchKernelGGL(k_ipm_bwd<8>, dim3(gb), dim3(kBlock), 0, h->stream, ba, v, isc, h->part, fl); break;
        case 16: hipLaunchKernelGGL(k_ipm_bwd<16>, dim3(gb), dim3(kBlock), 0, h->stream, ba, v, isc, h->part, fl); break;
        case 32: hipLaunchKernelGGL(k_ipm_bwd<32>, dim3(gb), dim3(kBlock), 0, h->stream, ba, v, isc, h->part, fl); break;
        default: hipLaunchKernelGGL(k_ipm_bwd<64>, dim3(gb), dim3(kBlock), 0, h->stream, ba, v, isc, h->part, fl); break;
    }
    HIPCHK(hipGetLastError());
    if (h->aug)   // lambda block of eq. (2x2_augmented): D, its Jacobi entries, r_2
        hipLaunchKernelGGL(k_aug_rows, dim3(grid_elems(m)), dim3(kBlock), 0, h->stream, v, h->dlu, fl);
    hipLaunchKernelGGL(k_ipm_check, dim3(1), dim3(kBlock), 0, h->stream, (const double*)h->partA, nbA,
                       (const double*)h->part, (n + kChunkRows - 1) / kChunkRows, apply, h->isc, h->fl, h->log);
    HIPCHK(hipGetLastError());
}

const int* ipm_stop_flag(qp_handle* h) { return reinterpret_cast<const int*>(&h->fl->ipm_done); }

// Start point (R6 reading of Section 3.1), objective scale, mu0, the first
// residual pass and the first preconditioner.
void ipm_start(IpmRun& r, const double* x0) {
    qp_handle* h = r.h;
    ensure_timing_events(h);
    const int n = h->n, m = h->m;
    IpmVec& v = h->iv;
    h->aug = h->set.kkt_system == 1 && m > 0;
    reset_flags(h);
    {
        IpmScal s0{};
        s0.mu_tol = h->set.mu_tol;
        s0.tau = h->set.tau;
        s0.cscale = h->cscale;
        s0.step_mode = h->set.step_mode;
        HIPCHK(hipMemcpyAsync(h->isc, &s0, sizeof(IpmScal), hipMemcpyHostToDevice, h->stream));
    }
    HIPCHK(hipEventRecord(h->ev_t0, h->stream));
    const int gx = grid_elems(n);
    if (x0) {
        if (!h->x0d) h->x0d = h->dalloc<double>(n);
        HIPCHK(hipMemcpyAsync(h->x0d, x0, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
        hipLaunchKernelGGL(k_ipm_init_x_from, dim3(gx), dim3(kBlock), 0, h->stream, v, (const double*)h->x0d,
                           h->partA);
    } else {
        hipLaunchKernelGGL(k_ipm_init_x, dim3(gx), dim3(kBlock), 0, h->stream, v, h->partA);
    }
    HIPCHK(hipGetLastError());
    int nps = gx;
    if (m > 0) {
        const int ga = grid_rows(m, 64);
        hipLaunchKernelGGL(k_ipm_init_A, dim3(ga), dim3(kBlock), 0, h->stream, v, (const int*)h->Ap,
                           (const int*)h->Ac, (const double*)h->Av, h->partA + gx);
        HIPCHK(hipGetLastError());
        nps += ga;
    }
    apply_op_prec(h, QP_FP64, v.x, h->tmp_n, nullptr, nullptr, 1.0, false, false, 0);
    hipLaunchKernelGGL(k_ipm_scale, dim3(1), dim3(kBlock), 0, h->stream, (const double*)h->tmp_n,
                       (const double*)h->p, n, (const double*)h->partA, nps, h->mtot, h->set.scale_objective,
                       h->set.mu0, h->isc);
    HIPCHK(hipGetLastError());
    IpmScal sc{};
    HIPCHK(hipMemcpyAsync(&sc, h->isc, sizeof(IpmScal), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    r.hs = sc.hs;
    ipm_residuals(h, 0);
    r.wbp = (m > 0) && build_precond(h, v.dh, v.sigA, ipm_stop_flag(h));
}

// The PCG time of an IPM iteration is read two iterations later (its events
// are long complete by then), so the host never waits for the device just
// to time it.
void harvest_pcg_ms(IpmRun& r, int slot) {
    if (!r.pcg_timed[slot]) return;
    qp_handle* h = r.h;
    HIPCHK(hipEventSynchronize(h->ev_p1[slot]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev_p0[slot], h->ev_p1[slot]));
    r.pcg_ms += ms;
    r.pcg_timed[slot] = false;
}

// The Newton direction of the current iterate (the PCG solve of Algorithm 1) into
// h->px, repeated with the Jacobi diagonal when a constraint-block solve
// stalls.
Flags ipm_direction(IpmRun& r, int* nsolves) {
    qp_handle* h = r.h;
    IpmVec& v = h->iv;
    const int m = h->m;
    const int ps = r.it & 1;
    harvest_pcg_ms(r, ps);
    HIPCHK(hipEventRecord(h->ev_p0[ps], h->stream));
    *nsolves = 0;
    Flags f = newton_direction(h, h->set.precision, v.rhs_a, v.rhs_b, v.sigx, m > 0 ? v.sigA : nullptr, v.d,
                               r.wbp ? h->Dw : nullptr, r.hs, true, &r.ta, nsolves);
    while (!f.ipm_done && r.wbp && prec_stalled(h, f)) {
        r.pcg_total += f.pcg_iters;
        r.pcg_solves += *nsolves;
        ++r.fallbacks;
        ++r.tier;
        if (h->set.log_level > 0)
            std::fprintf(stderr, "[qpgpu] constraint-block PCG stopped after %d iterations: %s from here\n",
                         f.pcg_iters, r.tier == TIER_CAPPED ? "capped block" : "Jacobi");
        r.wbp = r.tier == TIER_CAPPED && build_precond(h, v.dh, v.sigA, ipm_stop_flag(h), kPrecCapTau);
        f = newton_direction(h, h->set.precision, v.rhs_a, v.rhs_b, v.sigx, m > 0 ? v.sigA : nullptr, v.d,
                             r.wbp ? h->Dw : nullptr, r.hs, true, &r.ta, nsolves);
    }
    HIPCHK(hipEventRecord(h->ev_p1[ps], h->stream));
    if (!f.ipm_done) r.pcg_timed[ps] = true;
    return f;
}

// Accounting after a direction; false when the run ends here (the IPM had
// finished, or PCG broke down).
bool ipm_after_direction(IpmRun& r, const Flags& f, int nsolves) {
    qp_handle* h = r.h;
    if (f.ipm_done) {
        r.done = true;
        return false;
    }
    ++r.it;
    r.pcg_total += f.pcg_iters;
    r.pcg_solves += nsolves;
    r.capped += f.pcg_capped;
    if (h->set.log_level > 0) {
        IpmScal cur{};
        HIPCHK(hipMemcpyAsync(&cur, h->isc, sizeof(IpmScal), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        std::fprintf(stderr, "[qpgpu] ipm %3d mu %.3e rnorm %.3e pcg %6d%s alpha %.3f/%.3f\n", cur.iter, cur.mu,
                     cur.rnorm, f.pcg_iters, f.pcg_capped ? " (cap)" : "", cur.alpha_p, cur.alpha_d);
        std::fflush(stderr);
    }
    if (f.pcg_breakdown) {
        r.st = QP_ERR_NUMERIC;
        r.done = true;
        return false;
    }
    if (r.it >= h->set.max_ipm_iter) r.done = true;   // the step below is the last
    return true;
}

// Recovery of ds and dlambda, the ratio test and the update of Algorithm 1,
// then the residual pass, the barrier rule and the next preconditioner.
void ipm_step(IpmRun& r) {
    qp_handle* h = r.h;
    IpmVec& v = h->iv;
    const int n = h->n, m = h->m;
    const int nbA = m > 0 ? grid_rows(m, 64) : 0;
    const int nbx = grid_elems(n);
    hipLaunchKernelGGL(k_ipm_recover, dim3(nbA + nbx), dim3(kBlock), 0, h->stream, v, (const int*)h->Ap,
                       (const int*)h->Ac, (const double*)h->Av, nbA, (const IpmScal*)h->isc, h->part2,
                       (const Flags*)h->fl);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_ipm_update, dim3(grid_elems(int64_t(n) + m)), dim3(kBlock), 0, h->stream, v,
                       (const double*)h->part2, nbA + nbx, h->isc, (const Flags*)h->fl);
    HIPCHK(hipGetLastError());
    ipm_residuals(h, 1);
    r.wbp = r.tier < TIER_JACOBI && (m > 0) && build_precond(h, v.dh, v.sigA, ipm_stop_flag(h), tier_tau(r.tier));
}

// Outputs: the KKT certificate of the returned point (H x and A x of the
// last residual pass are at that point), the multipliers, x, and the info.
void ipm_finish(IpmRun& r, double* x, double* lam_A, double* lam_x, qp_info* info) {
    qp_handle* h = r.h;
    IpmVec& v = h->iv;
    const int n = h->n, m = h->m;
    HIPCHK(hipEventRecord(h->ev_t1, h->stream));
    {
        const int gc = std::min(kCertBlocks, grid_rows(n, 16));
        hipLaunchKernelGGL(k_cert_x<16>, dim3(gc), dim3(kBlock), 0, h->stream, v, (const int*)h->Atp,
                           (const int*)h->Atc, (const double*)h->Atv, m > 0 ? 1 : 0, (const IpmScal*)h->isc,
                           h->part2);
        const int ga = m > 0 ? std::min(kCertBlocks, (m + kBlock - 1) / kBlock) : 0;
        if (ga > 0)
            hipLaunchKernelGGL(k_cert_a, dim3(ga), dim3(kBlock), 0, h->stream, v, (const IpmScal*)h->isc,
                               h->partA);
        hipLaunchKernelGGL(k_cert_final, dim3(1), dim3(kBlock), 0, h->stream, (const double*)h->part2, gc,
                           (const double*)h->partA, ga, (const IpmScal*)h->isc, h->cert);
        HIPCHK(hipGetLastError());
    }
    double* lx = h->tmp_n;
    double* lA = h->tmp_m;
    hipLaunchKernelGGL(k_ipm_output, dim3(grid_elems(int64_t(n) + m)), dim3(kBlock), 0, h->stream, v,
                       (const IpmScal*)h->isc, lx, lA);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(x, v.x, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
    if (lam_x) HIPCHK(hipMemcpyAsync(lam_x, lx, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
    if (lam_A && m > 0) HIPCHK(hipMemcpyAsync(lam_A, lA, sizeof(double) * m, hipMemcpyDeviceToHost, h->stream));
    IpmScal sc{};
    HIPCHK(hipMemcpyAsync(&sc, h->isc, sizeof(IpmScal), hipMemcpyDeviceToHost, h->stream));
    PcgScal ps{};
    HIPCHK(hipMemcpyAsync(&ps, h->psc, sizeof(PcgScal), hipMemcpyDeviceToHost, h->stream));
    CertOut co{};
    HIPCHK(hipMemcpyAsync(&co, h->cert, sizeof(CertOut), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    harvest_pcg_ms(r, 0);
    harvest_pcg_ms(r, 1);
    if (r.st == QP_OK && !sc.done) r.st = QP_ERR_NOT_CONVERGED;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->status = r.st;
        info->ipm_iters = sc.iter;
        info->pcg_iters = r.pcg_total;
        info->pcg_solves = r.pcg_solves;
        info->pcg_capped = r.capped;
        info->mu = sc.mu;
        info->rnorm = sc.rnorm;
        info->zeta = sc.zeta;
        info->objective = sc.zeta * (0.5 * sc.xHx + sc.px);
        info->pcg_relres = ps.bnorm2 > 0 ? std::sqrt(ps.rr / ps.bnorm2) : 0.0;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev_t0, h->ev_t1));
        info->t_solve_ms = ms;
        info->t_pcg_ms = r.pcg_ms;
        set_format_info(h, info);
        info->prec_fallbacks = r.fallbacks;
        info->prec_tier = (h->woodbury && h->m > 0) ? r.tier : TIER_JACOBI;
        info->eps_d = co.eps_d;
        info->eps_p = co.eps_p;
        info->eps_c = co.eps_c;
        info->gap = co.gap;
        harvest_timing(h, r.ta, info);
    }
    if (r.st == QP_ERR_NUMERIC) h->err = "PCG breakdown";
    else if (r.st == QP_ERR_NOT_CONVERGED) h->err = "IPM reached max_ipm_iter";
}


// ==========================================================================
// Batched solves: many QPs, one persistent launch per kind of PCG work
// (batch_kernels.hpp).  Every QP keeps its own handle state and runs the
// phases of Algorithm 1 (start, step, finish) on its own stream, driven by
// host workers; the search directions of all QPs still iterating are
// computed together on the batch stream by batched PCG solves whose
// iterations are captured once as a HIP graph.  A QP whose PCG solve has
// stopped leaves the work lists on the device; a QP whose IPM has finished
// leaves the batch.
// ==========================================================================


struct BatchRun {
    std::vector<qp_handle*> hs;
    std::vector<IpmRun> runs;
    int nq = 0;
    int prec = QP_FP64;
    bool nt_lo = false, nt_64 = false;   // value arrays above the cache: non-temporal loads
    int items[BK_COUNT] = {};   // grid of each kind: its longest list (every QP of the batch on it)
    hipStream_t st = nullptr;
    hipEvent_t ev_dir = nullptr;         // end of the last direction phase
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
    hipEvent_t ev_snap[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> ev_q;        // per QP: end of its last step
    // device memory (one allocation)
    void* dmem = nullptr;
    BatchQp* d_qs = nullptr;
    int* d_phase = nullptr;
    BatchList* d_lists = nullptr;
    BatchStatus* d_status = nullptr;
    Flags* d_flags = nullptr;
    void* d_line_lo = nullptr;           // LineArgs<VT> of the batch precision, PCG products
    LineArgs<double>* d_line_64 = nullptr;     // FP64 PCG products
    LineArgs<double>* d_line_plain = nullptr;  // FP64 plain products
    SpotArgs* d_spot = nullptr;
    SpotArgs* d_spot_plain = nullptr;
    PcgInitArgs* d_init[3] = {nullptr, nullptr, nullptr};   // IPM right-hand side, rhs_full, rho
    ScalArgs* d_scal0[3] = {nullptr, nullptr, nullptr};     // mode 1 at pcg_tol, mode 1 at refine_tol, mode 2
    ScalArgs* d_scal = nullptr;
    PrecAArgs* d_preca = nullptr;
    SymvArgs* d_symv = nullptr;
    PrecAtArgs* d_at0 = nullptr;
    PrecAtArgs* d_at = nullptr;
    PcgArgs* d_xr = nullptr;
    VecArgs* d_vec[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // pinned host memory: the table image, the phase mask, two snapshots
    char* h_tab = nullptr;
    size_t tab_bytes = 0;
    int* h_phase = nullptr;
    char* h_snap = nullptr;
    size_t snap_bytes = 0;
    hipEvent_t ev_stage = nullptr;       // last copy out of the pinned table image / mask
    bool staged = false;
    // graphs of kGraphIters batched iterations: low-precision and FP64 products
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int hist[2][2] = {{0, 0}, {0, 0}};   // longest solves of the previous two phases of each kind
    float pcg_ms = 0.f;

    ~BatchRun() {
        if (st) (void)hipStreamSynchronize(st);
        for (int i = 0; i < 2; ++i) {
            if (gexec[i]) (void)hipGraphExecDestroy(gexec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
        }
        if (dmem) (void)hipFree(dmem);
        if (h_tab) (void)hipHostFree(h_tab);
        if (h_phase) (void)hipHostFree(h_phase);
        if (h_snap) (void)hipHostFree(h_snap);
        for (hipEvent_t e : {ev_dir, ev_t0, ev_t1, ev_snap[0], ev_snap[1], ev_stage})
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : ev_q)
            if (e) (void)hipEventDestroy(e);
        if (st) (void)hipStreamDestroy(st);
    }
    const BatchList* list(int k) const { return d_lists + k; }
    const BatchStatus& snap_status(int slot) const {
        return *reinterpret_cast<const BatchStatus*>(h_snap + slot * snap_bytes);
    }
    const Flags* snap_flags(int slot) const {
        return reinterpret_cast<const Flags*>(h_snap + slot * snap_bytes + sizeof(BatchStatus));
    }
};

// The persistent path serves handles that ask for it (batch_mode = 1) on the
// line format with the condensed system, no low-rank term, one precision and
// graph setting, no event timing, on one device; other batches run each QP's
// own solve on host workers.  Host workers are the default: with every QP on
// its own stream the GPU overlaps one QP's latency-bound kernels with other
// QPs' line passes, while the persistent path advances all QPs' IPM
// iterations together, so each batched PCG solve lasts as long as its
// slowest QP's and its last iterations carry few QPs (measured on the 16
// uneven QPs: FP64 1078 ms persistent against 937 ms on host workers).
bool batch_persistent_ok(qp_handle* const* hs, int count) {
    if (count < 2 || count > kMaxBatch) return false;
    for (int i = 0; i < count; ++i) {
        const qp_handle* h = hs[i];
        if (h->set.batch_mode != 1) return false;
        if (!h->line || h->k > 0 || h->set.kkt_system != 0 || h->set.timing) return false;
        if (h->set.precision != hs[0]->set.precision || h->set.refine_steps != hs[0]->set.refine_steps ||
            h->set.graphs != hs[0]->set.graphs || h->device != hs[0]->device)
            return false;
    }
    return true;
}

// Offsets of the tables in the table image (each 256-byte aligned).
struct TabLayout {
    size_t qs, line_lo, line_64, line_plain, spot, spot_plain, init[3], scal0[3], scal, preca, symv, at0, at, xr,
        vec[5], total;
};
TabLayout tab_layout(int nq, size_t line_lo_size) {
    TabLayout t{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    t.qs = take(sizeof(BatchQp) * nq);
    t.line_lo = take(line_lo_size * nq);
    t.line_64 = take(sizeof(LineArgs<double>) * nq);
    t.line_plain = take(sizeof(LineArgs<double>) * nq);
    t.spot = take(sizeof(SpotArgs) * nq);
    t.spot_plain = take(sizeof(SpotArgs) * nq);
    for (auto& v : t.init) v = take(sizeof(PcgInitArgs) * nq);
    for (auto& v : t.scal0) v = take(sizeof(ScalArgs) * nq);
    t.scal = take(sizeof(ScalArgs) * nq);
    t.preca = take(sizeof(PrecAArgs) * nq);
    t.symv = take(sizeof(SymvArgs) * nq);
    t.at0 = take(sizeof(PrecAtArgs) * nq);
    t.at = take(sizeof(PrecAtArgs) * nq);
    t.xr = take(sizeof(PcgArgs) * nq);
    for (auto& v : t.vec) v = take(sizeof(VecArgs) * nq);
    t.total = o;
    return t;
}

size_t line_args_size(int prec) {
    return prec == QP_FP32 ? sizeof(LineArgs<float>) : prec == QP_BF16 ? sizeof(LineArgs<bf16_t>)
                                                                       : sizeof(LineArgs<double>);
}

void batch_alloc(BatchRun& B) {
    const int nq = B.nq;
    const TabLayout t = tab_layout(nq, line_args_size(B.prec));
    B.tab_bytes = t.total;
    size_t o = t.total;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t o_phase = take(sizeof(int) * kMaxBatch);
    const size_t o_lists = take(sizeof(BatchList) * BK_COUNT);
    const size_t o_status = take(sizeof(BatchStatus));
    const size_t o_flags = take(sizeof(Flags) * kMaxBatch);
    HIPCHK(hipMalloc(&B.dmem, o));
    char* d = static_cast<char*>(B.dmem);
    B.d_qs = reinterpret_cast<BatchQp*>(d + t.qs);
    B.d_line_lo = d + t.line_lo;
    B.d_line_64 = reinterpret_cast<LineArgs<double>*>(d + t.line_64);
    B.d_line_plain = reinterpret_cast<LineArgs<double>*>(d + t.line_plain);
    B.d_spot = reinterpret_cast<SpotArgs*>(d + t.spot);
    B.d_spot_plain = reinterpret_cast<SpotArgs*>(d + t.spot_plain);
    for (int i = 0; i < 3; ++i) {
        B.d_init[i] = reinterpret_cast<PcgInitArgs*>(d + t.init[i]);
        B.d_scal0[i] = reinterpret_cast<ScalArgs*>(d + t.scal0[i]);
    }
    B.d_scal = reinterpret_cast<ScalArgs*>(d + t.scal);
    B.d_preca = reinterpret_cast<PrecAArgs*>(d + t.preca);
    B.d_symv = reinterpret_cast<SymvArgs*>(d + t.symv);
    B.d_at0 = reinterpret_cast<PrecAtArgs*>(d + t.at0);
    B.d_at = reinterpret_cast<PrecAtArgs*>(d + t.at);
    B.d_xr = reinterpret_cast<PcgArgs*>(d + t.xr);
    for (int i = 0; i < 5; ++i) B.d_vec[i] = reinterpret_cast<VecArgs*>(d + t.vec[i]);
    B.d_phase = reinterpret_cast<int*>(d + o_phase);
    B.d_lists = reinterpret_cast<BatchList*>(d + o_lists);
    B.d_status = reinterpret_cast<BatchStatus*>(d + o_status);
    B.d_flags = reinterpret_cast<Flags*>(d + o_flags);
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&B.h_tab), B.tab_bytes, hipHostMallocDefault));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&B.h_phase), sizeof(int) * kMaxBatch, hipHostMallocDefault));
    B.snap_bytes = (sizeof(BatchStatus) + sizeof(Flags) * kMaxBatch + 255) / 256 * 256;
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&B.h_snap), 2 * B.snap_bytes, hipHostMallocDefault));
    std::memset(B.h_phase, 0, sizeof(int) * kMaxBatch);
}

// The host rewrites the pinned table image or mask only after the copy that
// last read it has finished.
void batch_stage_wait(BatchRun& B) {
    if (B.staged) HIPCHK(hipEventSynchronize(B.ev_stage));
    B.staged = false;
}
void batch_stage_done(BatchRun& B) {
    HIPCHK(hipEventRecord(B.ev_stage, B.st));
    B.staged = true;
}

// Fill and upload every QP's tables for the current iterate: the arguments
// its own solve would launch with (pcg_setup, line_args, spot_args), with the
// constraint-block preconditioner (exact or capped) where the QP's run has
// one built.
template <typename VT>
void batch_tables_t(BatchRun& B) {
    const int nq = B.nq;
    const TabLayout t = tab_layout(nq, sizeof(LineArgs<VT>));
    batch_stage_wait(B);
    char* img = B.h_tab;
    std::memset(img, 0, B.tab_bytes);
    for (int q = 0; q < nq; ++q) {
        qp_handle* h = B.hs[q];
        const IpmRun& r = B.runs[q];
        IpmVec& v = h->iv;
        const int m = h->m;
        const double* sigA = m > 0 ? v.sigA : nullptr;
        const double* dh = r.wbp ? h->Dw : nullptr;
        const double tol = h->set.pcg_tol;
        const double inner = h->set.refine_steps > 0 ? std::max(h->set.refine_tol, tol) : tol;
        h->wb_cap_dir = wb_attempt_cap(h);   // as newton_direction: one cap per direction
        const PcgSetup S_ipm = pcg_setup(h, v.rhs_a, v.rhs_b, sigA, v.d, dh, true, tol, false);
        const PcgSetup S_lo = pcg_setup(h, nullptr, h->rhs_full, sigA, v.d, dh, false, inner, false);
        const PcgSetup S_rho = pcg_setup(h, nullptr, h->rho, sigA, v.d, dh, false, inner, true);
        const OpWork wk = handle_work(h);
        const LineArgs<VT> lo = line_args<VT>(h, wk, h->pz, h->pq, sigA, true);
        const LineArgs<double> l64 = line_args<double>(h, wk, h->pz, h->pq, sigA, true);
        const LineArgs<double> lpl = line_args<double>(h, wk, h->dxacc, h->pq, sigA, false);
        BatchQp bq{};
        bq.fl = h->fl;
        bq.nblk[BK_INIT] = S_ipm.ge;
        bq.nblk[BK_PRECA] = S_ipm.wb ? S_ipm.nb_preca : 0;
        bq.nblk[BK_SYMV] = S_ipm.wb ? S_ipm.nb_symv : 0;
        bq.nblk[BK_AT] = S_ipm.wb ? S_ipm.nb_at : 0;
        bq.nblk[BK_SCAL] = S_ipm.gs;
        bq.nblk[BK_LINE] = line_blocks(lo);
        bq.nblk[BK_LINE64] = line_blocks(l64);
        bq.nblk[BK_LINE_PLAIN] = line_blocks(lpl);
        bq.nblk[BK_SPOT] = spot_blocks(h);
        bq.nblk[BK_XR] = S_ipm.nb_xr;
        bq.nblk[BK_VEC] = grid_elems(h->n);
        auto put = [&](size_t off, const auto& val) {
            std::memcpy(img + off + sizeof(val) * size_t(q), &val, sizeof(val));
        };
        put(t.qs, bq);
        put(t.line_lo, lo);
        put(t.line_64, l64);
        put(t.line_plain, lpl);
        put(t.spot, spot_args(h, wk, h->pz, h->pq, v.sigx, sigA, r.hs, true));
        put(t.spot_plain, spot_args(h, wk, h->dxacc, h->pq, v.sigx, sigA, r.hs, false));
        put(t.init[0], S_ipm.ia);
        put(t.init[1], S_lo.ia);
        put(t.init[2], S_rho.ia);
        put(t.scal0[0], S_ipm.sa);   // mode 1 at pcg_tol (FP64 solves and the FP64 fallback)
        put(t.scal0[1], S_lo.sa);    // mode 1 at refine_tol
        put(t.scal0[2], S_rho.sa);   // mode 2
        put(t.scal, S_ipm.si);
        put(t.preca, S_ipm.prea);
        put(t.symv, S_ipm.sy);
        put(t.at0, S_ipm.at0);
        put(t.at, S_ipm.at);
        PcgArgs pa = S_ipm.pa;
        pa.n_pq = line_pq_partials(h, sigA);
        put(t.xr, pa);
        const int n = h->n;
        put(t.vec[0], VecArgs{VEC_RHS, n, v.rhs_a, v.rhs_b, h->isc, h->rhs_full});
        put(t.vec[1], VecArgs{VEC_SET, n, h->px, nullptr, nullptr, h->dxacc});
        put(t.vec[2], VecArgs{VEC_ADD, n, h->px, nullptr, nullptr, h->dxacc});
        put(t.vec[3], VecArgs{VEC_SUB, n, h->rhs_full, h->pq, nullptr, h->rho});
        put(t.vec[4], VecArgs{VEC_SET, n, h->dxacc, nullptr, nullptr, h->px});
    }
    // grid of each kind: every QP of the batch on its list (the line kinds
    // share one grid, the largest)
    int64_t tot[BK_COUNT] = {};
    for (int q = 0; q < nq; ++q) {
        const BatchQp* bq = reinterpret_cast<const BatchQp*>(img + t.qs) + q;
        for (int k = 0; k < BK_COUNT; ++k) tot[k] += bq->nblk[k];
    }
    tot[BK_LINE] = std::max({tot[BK_LINE], tot[BK_LINE64], tot[BK_LINE_PLAIN]});
    for (int k = 0; k < BK_COUNT; ++k) B.items[k] = int(std::max<int64_t>(1, std::min<int64_t>(tot[k], INT32_MAX)));
    HIPCHK(hipMemcpyAsync(B.d_qs, img, B.tab_bytes, hipMemcpyHostToDevice, B.st));
    batch_stage_done(B);
}
void batch_tables(BatchRun& B) {
    switch (B.prec) {
        case QP_FP32: batch_tables_t<float>(B); break;
        case QP_BF16: batch_tables_t<bf16_t>(B); break;
        default: batch_tables_t<double>(B); break;
    }
}

// Plan the work lists for the QPs in `mask` (mode BP_START or BP_ITER).
void batch_plan(BatchRun& B, int mode) {
    hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(kMaxBatch), 0, B.st, (const BatchQp*)B.d_qs,
                       (const int*)B.d_phase, B.nq, mode, B.d_lists, B.d_status, B.d_flags);
}
void batch_set_phase(BatchRun& B, const std::vector<char>& mask) {
    batch_stage_wait(B);
    for (int q = 0; q < B.nq; ++q) B.h_phase[q] = mask[q] ? 1 : 0;
    HIPCHK(hipMemcpyAsync(B.d_phase, B.h_phase, sizeof(int) * B.nq, hipMemcpyHostToDevice, B.st));
    batch_stage_done(B);
}
void batch_snapshot(BatchRun& B, int slot) {
    HIPCHK(hipMemcpyAsync(B.h_snap + slot * B.snap_bytes, B.d_status, sizeof(BatchStatus), hipMemcpyDeviceToHost,
                          B.st));
    HIPCHK(hipMemcpyAsync(B.h_snap + slot * B.snap_bytes + sizeof(BatchStatus), B.d_flags, sizeof(Flags) * B.nq,
                          hipMemcpyDeviceToHost, B.st));
    HIPCHK(hipEventRecord(B.ev_snap[slot], B.st));
}

template <typename VT, typename AT>
void batch_line_launch(BatchRun& B, const void* tab, const BatchList* L, bool nt) {
    const LineArgs<VT>* tb = static_cast<const LineArgs<VT>*>(tab);
    if (nt) hipLaunchKernelGGL((kb_line<VT, AT, true>), dim3(B.items[BK_LINE]), dim3(kBlock), 0, B.st, tb, L);
    else hipLaunchKernelGGL((kb_line<VT, AT, false>), dim3(B.items[BK_LINE]), dim3(kBlock), 0, B.st, tb, L);
}
// Line pass of a PCG product, in the batch precision (lo) or FP64.
void batch_line(BatchRun& B, bool lo) {
    if (lo && B.prec == QP_FP32) batch_line_launch<float, float>(B, B.d_line_lo, B.list(BK_LINE), B.nt_lo);
    else if (lo && B.prec == QP_BF16) batch_line_launch<bf16_t, float>(B, B.d_line_lo, B.list(BK_LINE), B.nt_lo);
    else batch_line_launch<double, double>(B, lo ? B.d_line_lo : B.d_line_64, B.list(lo ? BK_LINE : BK_LINE64),
                                           B.nt_64);
}

// One batched PCG iteration (kernels in the order of run_pcg's).
void batch_iter(BatchRun& B, bool lo) {
    batch_line(B, lo);
    hipLaunchKernelGGL(kb_spot<kSpotLanes>, dim3(B.items[BK_SPOT]), dim3(kBlock), 0, B.st, (const SpotArgs*)B.d_spot,
                       B.list(BK_SPOT));
    hipLaunchKernelGGL(kb_xr, dim3(B.items[BK_XR]), dim3(kBlock), 0, B.st, (const PcgArgs*)B.d_xr, B.list(BK_XR));
    hipLaunchKernelGGL(kb_symv, dim3(B.items[BK_SYMV]), dim3(kBlock), 0, B.st, (const SymvArgs*)B.d_symv, B.list(BK_SYMV));
    hipLaunchKernelGGL(kb_at<kPrecAtLanes>, dim3(B.items[BK_AT]), dim3(kBlock), 0, B.st, (const PrecAtArgs*)B.d_at,
                       B.list(BK_AT));
    hipLaunchKernelGGL(kb_scal, dim3(B.items[BK_SCAL]), dim3(kBlock), 0, B.st, (const ScalArgs*)B.d_scal, B.list(BK_SCAL));
    batch_plan(B, BP_ITER);
    HIPCHK(hipGetLastError());
}

// Graph of kGraphIters batched iterations (its launches read the tables and
// lists through fixed pointers, so one capture serves every later solve).
hipGraphExec_t batch_graph(BatchRun& B, bool lo) {
    const int g = lo ? 0 : 1;
    if (B.gexec[g]) return B.gexec[g];
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(B.st, hipStreamCaptureModeThreadLocal));
    try {
        for (int i = 0; i < kGraphIters; ++i) batch_iter(B, lo);
    } catch (...) {
        (void)hipStreamEndCapture(B.st, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    HIPCHK(hipStreamEndCapture(B.st, &graph));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        throw HipError{e, "hipGraphInstantiate (batch)"};
    }
    B.graph[g] = graph;
    B.gexec[g] = ex;
    return ex;
}

// Start variants of a batched solve.
enum { BS_IPM = 0, BS_LO = 1, BS_RHO = 2, BS_FULL64 = 3 };

// One batched PCG solve for the QPs in `mask` (start variant sv; products in
// the batch precision when lo, else FP64).  check_only: stop after the start
// (a refinement pass that only measures its residual).  Returns every QP's
// flags after the solve.
std::vector<Flags> batch_pcg(BatchRun& B, const std::vector<char>& mask, int sv, bool lo, bool check_only) {
    const int init_tab = sv == BS_IPM ? 0 : sv == BS_RHO ? 2 : 1;
    const int scal_tab = (sv == BS_IPM || sv == BS_FULL64) ? 0 : sv == BS_LO ? 1 : 2;
    const bool refine = sv == BS_RHO;
    batch_set_phase(B, mask);
    batch_plan(B, BP_START);
    hipLaunchKernelGGL(kb_init0, dim3(B.items[BK_INIT]), dim3(kBlock), 0, B.st, (const PcgInitArgs*)B.d_init[init_tab],
                       B.list(BK_INIT));
    hipLaunchKernelGGL(kb_preca, dim3(B.items[BK_PRECA]), dim3(kBlock), 0, B.st, (const PrecAArgs*)B.d_preca,
                       B.list(BK_PRECA));
    hipLaunchKernelGGL(kb_symv, dim3(B.items[BK_SYMV]), dim3(kBlock), 0, B.st, (const SymvArgs*)B.d_symv, B.list(BK_SYMV));
    hipLaunchKernelGGL(kb_at<kPrecAtLanes>, dim3(B.items[BK_AT]), dim3(kBlock), 0, B.st, (const PrecAtArgs*)B.d_at0,
                       B.list(BK_AT));
    hipLaunchKernelGGL(kb_scal, dim3(B.items[BK_SCAL]), dim3(kBlock), 0, B.st, (const ScalArgs*)B.d_scal0[scal_tab],
                       B.list(BK_SCAL));
    batch_plan(B, BP_ITER);
    HIPCHK(hipGetLastError());
    std::vector<Flags> out(B.nq);
    auto harvest = [&](int slot) {
        const Flags* f = B.snap_flags(slot);
        std::copy(f, f + B.nq, out.begin());
    };
    if (refine || check_only) {
        // often every QP's refinement residual already meets pcg_tol
        batch_snapshot(B, 0);
        HIPCHK(hipEventSynchronize(B.ev_snap[0]));
        harvest(0);
        if (check_only || B.snap_status(0).active == 0) return out;
    }
    // graphs = 0 (the handles' setting): the same iterations launched directly
    const hipGraphExec_t gx = B.hs[0]->set.graphs ? batch_graph(B, lo) : nullptr;
    int* hist = B.hist[refine ? 1 : 0];
    const int pred = std::min(hist[0], hist[1]);
    int chunk = std::max(kGraphIters, std::min(512, (pred * 3) / 4));
    chunk = ((chunk + kGraphIters - 1) / kGraphIters) * kGraphIters;
    auto queue = [&](int iters) {
        for (int i = 0; i < iters; i += kGraphIters) {
            if (gx) HIPCHK(hipGraphLaunch(gx, B.st));
            else
                for (int j = 0; j < kGraphIters; ++j) batch_iter(B, lo);
        }
    };
    int64_t launched = 0;
    int64_t guard = 4096;
    for (int q = 0; q < B.nq; ++q)
        if (mask[q]) guard = std::max<int64_t>(guard, int64_t(B.hs[q]->set.pcg_max_iter) + 4096);
    int cur = 0;
    queue(chunk);
    launched += chunk;
    batch_snapshot(B, cur);
    while (true) {
        queue(kGraphIters);
        launched += kGraphIters;
        batch_snapshot(B, cur ^ 1);
        HIPCHK(hipEventSynchronize(B.ev_snap[cur]));
        if (B.snap_status(cur).active == 0) {
            harvest(cur);
            break;
        }
        if (launched > guard) {
            HIPCHK(hipEventSynchronize(B.ev_snap[cur ^ 1]));
            harvest(cur ^ 1);
            break;
        }
        cur ^= 1;
    }
    int longest = 0;
    for (int q = 0; q < B.nq; ++q) {
        if (!mask[q]) continue;
        if (!out[q].ipm_done) longest = std::max(longest, out[q].pcg_iters);
        if (B.runs[q].wbp) note_wb_solve(B.hs[q], out[q]);
    }
    hist[1] = hist[0];
    hist[0] = longest;
    return out;
}

// A batched elementwise step (table i of d_vec) or the plain FP64 product
// (dxacc -> pq) for the QPs in mask.
void batch_vec(BatchRun& B, const std::vector<char>& mask, int i) {
    batch_set_phase(B, mask);
    batch_plan(B, BP_START);
    hipLaunchKernelGGL(kb_vec, dim3(B.items[BK_VEC]), dim3(kBlock), 0, B.st, (const VecArgs*)B.d_vec[i], B.list(BK_VEC));
    HIPCHK(hipGetLastError());
}
void batch_plain_product(BatchRun& B, const std::vector<char>& mask) {
    batch_set_phase(B, mask);
    batch_plan(B, BP_START);
    batch_line_launch<double, double>(B, B.d_line_plain, B.list(BK_LINE_PLAIN), B.nt_64);
    hipLaunchKernelGGL(kb_spot<kSpotLanes>, dim3(B.items[BK_SPOT]), dim3(kBlock), 0, B.st,
                       (const SpotArgs*)B.d_spot_plain, B.list(BK_SPOT));
    HIPCHK(hipGetLastError());
}

bool any_of(const std::vector<char>& v) {
    for (char c : v)
        if (c) return true;
    return false;
}

// The Newton directions of the QPs in mask, as newton_direction computes
// each (FP64: one solve; FP32/BF16: the low-precision solve, refinement
// passes against the FP64 product, the FP64 fallback), batched step by
// step.  Fills f (flags with the PCG iterations summed) and solves per QP.
void batch_direction(BatchRun& B, const std::vector<char>& mask, std::vector<Flags>& f, std::vector<int>& solves) {
    const int nq = B.nq;
    f.assign(nq, Flags{});
    solves.assign(nq, 0);
    if (B.prec == QP_FP64) {
        const std::vector<Flags> r = batch_pcg(B, mask, BS_IPM, true, false);
        for (int q = 0; q < nq; ++q)
            if (mask[q]) {
                f[q] = r[q];
                solves[q] = 1;
            }
        return;
    }
    batch_vec(B, mask, 0);   // rhs_full = mu rhs_a + rhs_b
    const std::vector<Flags> r0 = batch_pcg(B, mask, BS_LO, true, false);
    std::vector<int> total(nq, 0);
    std::vector<char> refining(nq, 0), met(nq, 0), fixed(nq, 0);   // fixed: direction final
    for (int q = 0; q < nq; ++q) {
        if (!mask[q]) continue;
        f[q] = r0[q];
        solves[q] = 1;
        total[q] = r0[q].pcg_iters;
        const qp_handle* h = B.hs[q];
        if (r0[q].ipm_done || r0[q].pcg_breakdown || h->set.refine_steps == 0) fixed[q] = 1;
        else refining[q] = 1;
    }
    batch_vec(B, refining, 1);   // dxacc = px
    std::vector<char> live = refining;   // passes still to run
    const int steps = B.hs[0]->set.refine_steps;
    for (int k = 0; k <= steps && any_of(live); ++k) {
        batch_plain_product(B, live);
        batch_vec(B, live, 3);   // rho = rhs_full - K dxacc
        const bool check = k == steps;
        const std::vector<Flags> r2 = batch_pcg(B, live, BS_RHO, true, check);
        std::vector<char> add(nq, 0);
        for (int q = 0; q < nq; ++q) {
            if (!live[q]) continue;
            const Flags& g = r2[q];
            if (g.ipm_done) {
                f[q] = g;
                fixed[q] = 1;
                refining[q] = 0;
                live[q] = 0;
                continue;
            }
            met[q] = (g.pcg_iters == 0 && g.pcg_converged) ? 1 : 0;
            if (check) {
                live[q] = 0;
                continue;
            }
            solves[q] += 1;
            total[q] += g.pcg_iters;
            f[q].pcg_capped |= g.pcg_capped;
            f[q].pcg_converged = g.pcg_converged;
            if (g.pcg_breakdown) {
                f[q].pcg_breakdown = 1;
                live[q] = 0;
                continue;
            }
            if (met[q]) {
                live[q] = 0;
                continue;
            }
            add[q] = 1;
        }
        batch_vec(B, add, 2);   // dxacc += px
    }
    std::vector<char> fb(nq, 0), keep(nq, 0);
    for (int q = 0; q < nq; ++q) {
        if (!refining[q]) continue;
        if (!met[q] && !f[q].pcg_breakdown) fb[q] = 1;
        else keep[q] = 1;
    }
    if (any_of(fb)) {
        const std::vector<Flags> r3 = batch_pcg(B, fb, BS_FULL64, false, false);
        for (int q = 0; q < nq; ++q)
            if (fb[q]) {
                Flags g = r3[q];
                solves[q] += 1;
                g.pcg_iters += total[q];
                g.pcg_capped |= f[q].pcg_capped;
                f[q] = g;
            }
    }
    batch_vec(B, keep, 4);   // px = dxacc
    for (int q = 0; q < nq; ++q)
        if (keep[q]) f[q].pcg_iters = total[q];
}

// Per-QP phases on host workers, each QP on its own stream.
template <typename F>
void batch_each(BatchRun& B, const std::vector<char>& mask, int workers, F&& fn, std::vector<qp_status>& st) {
    std::atomic<int> next{0};
    auto work = [&]() {
        (void)hipSetDevice(B.hs[0]->device);
        while (true) {
            const int q = next.fetch_add(1);
            if (q >= B.nq) break;
            if (!mask[q] || st[q] != QP_OK) continue;
            try {
                fn(q);
            } catch (const HipError& he) {
                B.hs[q]->err = std::string("HIP error in ") + he.what + ": " + hipGetErrorString(he.e);
                st[q] = QP_ERR_DEVICE;
                B.runs[q].done = true;
            }
        }
    };
    std::vector<std::thread> pool;
    for (int w = 1; w < workers; ++w) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
}

// The whole batch on the persistent path.  Returns per-QP statuses.
std::vector<qp_status> batch_solve(qp_handle* const* hs, int count, double* const* xs, qp_info* infos) {
    BatchRun B;
    B.nq = count;
    B.hs.assign(hs, hs + count);
    B.runs.resize(count);
    B.prec = hs[0]->set.precision;
    std::vector<qp_status> st(count, QP_OK);
    HIPCHK(hipSetDevice(hs[0]->device));
    HIPCHK(hipStreamCreateWithFlags(&B.st, hipStreamNonBlocking));
    for (hipEvent_t* e : {&B.ev_dir, &B.ev_snap[0], &B.ev_snap[1], &B.ev_stage})
        HIPCHK(hipEventCreateWithFlags(e, hipEventDisableTiming));
    HIPCHK(hipEventCreate(&B.ev_t0));
    HIPCHK(hipEventCreate(&B.ev_t1));
    B.ev_q.assign(count, nullptr);
    for (auto& e : B.ev_q) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    size_t bytes_lo = 0, bytes_64 = 0;
    for (int q = 0; q < count; ++q) {
        B.runs[q].h = hs[q];
        ensure_lowp(hs[q], B.prec);
        bytes_lo += size_t(hs[q]->nvals) * (B.prec == QP_FP32 ? 4 : B.prec == QP_BF16 ? 2 : 8);
        bytes_64 += size_t(hs[q]->nvals) * 8;
    }
    B.nt_lo = bytes_lo > kStreamedValueBytes;
    B.nt_64 = bytes_64 > kStreamedValueBytes;
    batch_alloc(B);
    int workers = 6;
    if (const char* e = std::getenv("QPGPU_BATCH_WORKERS")) workers = std::max(1, std::atoi(e));
    workers = std::min(workers, count);
    std::vector<char> all(count, 1);

    // start every QP on its own stream; then the tables and the schedule
    std::vector<std::unique_ptr<PrecAttemptCap>> caps;
    for (auto* h : B.hs) caps.emplace_back(new PrecAttemptCap(h));
    batch_each(B, all, workers, [&](int q) {
        ipm_start(B.runs[q], nullptr);
        HIPCHK(hipEventRecord(B.ev_q[q], B.hs[q]->stream));
    }, st);
    for (int q = 0; q < count; ++q) HIPCHK(hipStreamWaitEvent(B.st, B.ev_q[q], 0));
    batch_tables(B);
    while (true) {
        std::vector<char> live(count, 0);
        for (int q = 0; q < count; ++q) live[q] = (st[q] == QP_OK && !B.runs[q].done) ? 1 : 0;
        if (!any_of(live)) break;
        // the directions of every live QP (their steps ended before: events)
        for (int q = 0; q < count; ++q)
            if (live[q]) HIPCHK(hipStreamWaitEvent(B.st, B.ev_q[q], 0));
        batch_tables(B);
        HIPCHK(hipEventRecord(B.ev_t0, B.st));
        std::vector<Flags> f;
        std::vector<int> ns;
        batch_direction(B, live, f, ns);
        // a stalled constraint-block solve: that QP's direction again with
        // the next preconditioner tier, which then serves the rest of its run
        for (int round = 0; round < 2; ++round) {
            std::vector<char> redo(count, 0);
            for (int q = 0; q < count; ++q) {
                IpmRun& r = B.runs[q];
                if (live[q] && !f[q].ipm_done && r.wbp && prec_stalled(B.hs[q], f[q])) {
                    r.pcg_total += f[q].pcg_iters;
                    r.pcg_solves += ns[q];
                    ++r.fallbacks;
                    ++r.tier;
                    r.wbp = false;
                    redo[q] = 1;
                }
            }
            if (!any_of(redo)) break;
            // the capped block is built on the QP's own stream, after the
            // batched solve that read the exact one
            HIPCHK(hipEventRecord(B.ev_dir, B.st));
            batch_each(B, redo, workers, [&](int q) {
                IpmRun& r = B.runs[q];
                qp_handle* h = B.hs[q];
                if (r.tier == TIER_CAPPED) {
                    HIPCHK(hipStreamWaitEvent(h->stream, B.ev_dir, 0));
                    r.wbp = build_precond(h, h->iv.dh, h->iv.sigA, ipm_stop_flag(h), kPrecCapTau);
                }
                HIPCHK(hipEventRecord(B.ev_q[q], h->stream));
            }, st);
            for (int q = 0; q < count; ++q)
                if (redo[q]) HIPCHK(hipStreamWaitEvent(B.st, B.ev_q[q], 0));
            batch_tables(B);
            std::vector<Flags> f2;
            std::vector<int> ns2;
            batch_direction(B, redo, f2, ns2);
            for (int q = 0; q < count; ++q)
                if (redo[q]) {
                    f[q] = f2[q];
                    ns[q] = ns2[q];
                }
        }
        HIPCHK(hipEventRecord(B.ev_t1, B.st));
        HIPCHK(hipEventRecord(B.ev_dir, B.st));
        HIPCHK(hipEventSynchronize(B.ev_t1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, B.ev_t0, B.ev_t1));
        B.pcg_ms += ms;
        // accounting, then each QP's step on its own stream after the directions
        std::vector<char> step(count, 0);
        for (int q = 0; q < count; ++q) {
            if (!live[q]) continue;
            IpmRun& r = B.runs[q];
            r.pcg_ms += ms;
            if (ipm_after_direction(r, f[q], ns[q])) step[q] = 1;
        }
        batch_each(B, step, workers, [&](int q) {
            qp_handle* h = B.hs[q];
            HIPCHK(hipStreamWaitEvent(h->stream, B.ev_dir, 0));
            ipm_step(B.runs[q]);
            HIPCHK(hipEventRecord(B.ev_q[q], h->stream));
        }, st);
    }
    caps.clear();
    batch_each(B, all, workers, [&](int q) {
        qp_info inf{};
        HIPCHK(hipStreamWaitEvent(B.hs[q]->stream, B.ev_dir, 0));
        ipm_finish(B.runs[q], xs[q], nullptr, nullptr, &inf);
        st[q] = B.runs[q].st;
        if (infos) infos[q] = inf;
    }, st);
    return st;
}
}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

void qp_default_settings(qp_settings* s) {
    if (!s) return;
    std::memset(s, 0, sizeof(*s));
    s->precision = QP_FP64;
    s->refine_steps = 6;
    s->pcg_tol = 1e-8;
    s->pcg_max_iter = 20000;
    s->mu0 = -1.0;
    s->mu_tol = 1e-10;
    s->tau = 0.995;
    s->max_ipm_iter = 200;
    s->step_mode = 0;
    s->scale_objective = 1;
    s->schedule = 0;
    s->timing = 0;
    s->log_level = 0;
    s->precond = 1;
    s->spmv_format = 0;
    s->refine_tol = 1e-3;
    s->graphs = 1;
}

const char* qp_last_error(const qp_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

void qp_destroy(qp_handle* h) { delete h; }

void qp_sizes(const qp_handle* h, int32_t* n, int32_t* m, int32_t* nJ, int64_t* nnzJ, int64_t* nnzA) {
    if (!h) return;
    if (n) *n = h->n;
    if (m) *m = h->m;
    if (nJ) *nJ = h->nJ;
    if (nnzJ) *nnzJ = h->nnzJ;
    if (nnzA) *nnzA = h->nnzA;
}

qp_status qp_create(qp_handle** out, const qp_hessian* H, const qp_csr* J, const double* W,
                    const qp_csr* A, const qp_range* b, const qp_range* bounds, const qp_settings* s,
                    void* hip_stream) {
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is NULL";
        return QP_ERR_INVALID;
    }
    *out = nullptr;
    std::string e = validate_problem(H, J, W, A, b, bounds, s);
    if (!e.empty()) {
        g_create_error = e;
        return QP_ERR_INVALID;
    }
    (void)hipGetLastError();  // drop an error left by an earlier, unrelated call
    qp_handle* h = new (std::nothrow) qp_handle();
    if (!h) {
        g_create_error = "host allocation failed";
        return QP_ERR_NOMEM;
    }
    try {
        if (s) h->set = *s;
        else qp_default_settings(&h->set);
        h->n = J->cols;
        h->nJ = J->rows;
        h->m = A ? A->rows : 0;
        h->k = H->k;
        h->gamma = H->gamma;
        const int n = h->n, m = h->m, nJ = h->nJ;

        // host preparation (no device calls yet)
        HostCsr hJ = to_host_csr(J);
        LineFormat lf;
        const bool use_line = (h->set.spmv_format != 1) && build_line_format(hJ, 64, lf);
        // the CSR J and its stored transpose serve matrices without the line structure
        HostCsr hJt;
        if (!use_line) hJt = transpose(hJ);
        HostCsr hA, hAt;
        if (m > 0) {
            hA = to_host_csr(A);
            hAt = transpose(hA);
        }
        h->nnzJ = hJ.nnz();
        h->nnzA = m > 0 ? hA.nnz() : 0;
        // m = 0 keeps one padding entry so every device array has a valid source
        std::vector<double> xlo(n, -INFINITY), xhi(n, INFINITY), alo(std::max(m, 1), -INFINITY),
            ahi(std::max(m, 1), INFINITY);
        if (bounds) {
            if (bounds->lo) std::copy(bounds->lo, bounds->lo + n, xlo.begin());
            if (bounds->hi) std::copy(bounds->hi, bounds->hi + n, xhi.begin());
        }
        if (m > 0) {
            if (b->lo) std::copy(b->lo, b->lo + m, alo.begin());
            if (b->hi) std::copy(b->hi, b->hi + m, ahi.begin());
        }
        double cmax = 0.0, mt = 0.0;
        for (int j = 0; j < n; ++j) {
            if (std::isfinite(xlo[j])) { cmax = std::max(cmax, std::fabs(xlo[j])); mt += 1; }
            if (std::isfinite(xhi[j])) { cmax = std::max(cmax, std::fabs(xhi[j])); mt += 1; }
        }
        for (int i = 0; i < m; ++i) {
            if (std::isfinite(alo[i])) { cmax = std::max(cmax, std::fabs(alo[i])); mt += 1; }
            if (std::isfinite(ahi[i])) { cmax = std::max(cmax, std::fabs(ahi[i])); mt += 1; }
        }
        h->cscale = 1.0 + cmax;
        h->mtot = mt;
        if (h->set.schedule == 1) {   // the J pass over row blocks, lane counts as by default
            h->fwd_stream = true;
            h->GJ = pick_lanes(h->nnzJ, nJ);
            h->GJt = pick_lanes(h->nnzJ + h->nnzA, n);
        } else if (h->set.schedule != 0) {
            h->GJ = h->GJt = h->set.schedule;
        } else {
            h->GJ = pick_lanes(h->nnzJ, nJ);
            const int64_t col_nnz = h->nnzJ + h->nnzA;
            h->GJt = pick_lanes(col_nnz, n);
        }

        // device
        HIPCHK(hipGetDevice(&h->device));
        {   // once per device: the scratch of qp_operator_apply_noalloc (a failure
            // here is reported by that entry point, which retries)
            double* sp = nullptr;
            if (resolve_scratch(h->device, &sp) != hipSuccess) (void)hipGetLastError();
        }
        if (hip_stream) {
            h->stream = static_cast<hipStream_t>(hip_stream);
        } else {
            HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
            h->own_stream = true;
        }
        if (!use_line) {
            h->Jp = h->upload(hJ.ptr.data(), hJ.ptr.size());
            h->Jc = h->upload(hJ.col.data(), hJ.col.size());
            h->Jv = h->upload(hJ.val.data(), hJ.val.size());
            h->Jtp = h->upload(hJt.ptr.data(), hJt.ptr.size());
            h->Jtc = h->upload(hJt.col.data(), hJt.col.size());
            h->Jtv = h->upload(hJt.val.data(), hJt.val.size());
            std::vector<int32_t> rb;
            build_row_blocks(hJ.ptr, nJ, kStreamNnz, kStreamRows, rb);
            h->nbs = int(rb.size() / 2) - 1;
            if (h->nbs > 0) h->jrb = reinterpret_cast<int2*>(h->upload(rb.data(), rb.size()));
            else h->fwd_stream = false;
        }
        if (use_line) {
            h->line = true;
            h->L = lf.lines;
            h->lptr = h->upload(lf.ptr.data(), lf.ptr.size());
            h->lcol = h->upload(lf.col.data(), lf.col.size());
            h->lval = h->upload(lf.val.data(), lf.val.size());
            h->sptr = h->upload(lf.sptr.data(), lf.sptr.size());
            h->sslot = h->upload(lf.sslot.data(), lf.sslot.size());
            h->lc = h->dalloc<double>(lf.col.size());
            h->nslots = int64_t(lf.col.size());
        }
        h->nvals = use_line ? h->nslots * 64 : h->nnzJ;
        if (use_line && size_t(h->L) * 64 > size_t(nJ)) {
            // the last line's padding rows weigh nothing
            h->W = h->dalloc<double>(size_t(h->L) * 64);
            HIPCHK(hipMemsetAsync(h->W, 0, sizeof(double) * size_t(h->L) * 64, h->stream));
            if (nJ > 0) HIPCHK(hipMemcpyAsync(h->W, W, sizeof(double) * size_t(nJ), hipMemcpyHostToDevice, h->stream));
        } else {
            h->W = nJ > 0 ? h->upload(W, size_t(nJ)) : h->dalloc<double>(1);
        }
        if (m > 0) {
            h->Ap = h->upload(hA.ptr.data(), hA.ptr.size());
            h->Ac = h->upload(hA.col.data(), hA.col.size());
            h->Av = h->upload(hA.val.data(), hA.val.size());
            h->Atp = h->upload(hAt.ptr.data(), hAt.ptr.size());
            h->Atc = h->upload(hAt.col.data(), hAt.col.size());
            h->Atv = h->upload(hAt.val.data(), hAt.val.size());
        }
        h->xlo = h->upload(xlo.data(), n);
        h->xhi = h->upload(xhi.data(), n);
        h->alo = h->upload(alo.data(), std::max(m, 1));
        h->ahi = h->upload(ahi.data(), std::max(m, 1));
        h->p = h->upload(H->p, n);
        if (h->k > 0) {
            h->U = h->upload(H->U, size_t(n) * h->k);
            h->w = h->upload(H->w, size_t(h->k));
            h->k_cap = h->k;
        }
        h->diagH = h->dalloc<double>(n);

        // work vectors
        IpmVec& v = h->iv;
        v.n = n; v.m = m;
        v.xlo = h->xlo; v.xhi = h->xhi; v.alo = h->alo; v.ahi = h->ahi; v.p = h->p; v.diagH = h->diagH;
        double** nvec[] = {&v.x, &v.s_lx, &v.s_ux, &v.l_lx, &v.l_ux, &v.r_lx, &v.r_ux, &v.sigx, &v.hx,
                           &v.ds_lx, &v.ds_ux, &v.dl_lx, &v.dl_ux};
        for (double** pv : nvec) *pv = h->dalloc<double>(n);
        // vectors of the PCG system: n entries, n + 2m for the doubly augmented one
        const size_t N = size_t(n) + (h->set.kkt_system == 1 ? 2 * size_t(m) : 0);
        double** Nvec[] = {&v.d, &v.rhs_a, &v.rhs_b};
        for (double** pv : Nvec) *pv = h->dalloc<double>(N);
        if (h->set.kkt_system == 1 && m > 0) h->dlu = h->dalloc<double>(2 * size_t(m));
        double** mvec[] = {&v.s_lA, &v.s_uA, &v.l_lA, &v.l_uA, &v.ax, &v.r_lA, &v.r_uA, &v.sigA,
                           &v.va, &v.vb, &v.ya, &v.ds_lA, &v.ds_uA, &v.dl_lA, &v.dl_uA};
        for (double** pv : mvec) *pv = h->dalloc<double>(std::max(m, 1));
        h->t = h->dalloc<double>(std::max(nJ, 1));
        h->u = h->dalloc<double>(std::max(m, 1));
        h->az = h->dalloc<double>(std::max(m, 1));
        h->apv = h->dalloc<double>(std::max(m, 1));
        h->px = h->dalloc<double>(N);
        h->pr = h->dalloc<double>(N);
        h->pz = h->dalloc<double>(N);
        h->pp = h->dalloc<double>(N);
        h->pq = h->dalloc<double>(N);
        v.dx = h->px;
        h->zero_n = h->dalloc<double>(n);
        h->zero_m = h->dalloc<double>(std::max(m, 1));
        h->tmp_n = h->dalloc<double>(n);
        h->tmp_n2 = h->dalloc<double>(n);
        h->tmp_m = h->dalloc<double>(std::max(m, 1));
        h->rhs_full = h->dalloc<double>(N);
        if (h->k > 0) {
            h->lr_part = h->dalloc<double>(size_t(kLrBlocks) * h->k);
            h->lr_v = h->dalloc<double>(h->k);
        }
        h->rho = h->dalloc<double>(N);
        h->dxacc = h->dalloc<double>(N);
        const size_t nbA = size_t((m + 3) / 4) + 1;
        // per-block partials, and six per chunk of four variables (residual pass)
        h->part_len = std::max(8 * (size_t(kMaxPartials) + nbA + 64),
                               6 * (size_t(n) / kChunkRows + 1) + 64) + size_t(m);
        h->part = h->dalloc<double>(h->part_len);
        h->part2 = h->dalloc<double>(h->part_len);
        h->partA = h->dalloc<double>(h->part_len);
        h->part_rz = h->dalloc<double>(h->part_len);
        h->part_rr = h->dalloc<double>(h->part_len);
        v.dh = h->dalloc<double>(n);
        // the doubly augmented system runs with the Jacobi diagonal (Section 4.1.2)
        h->woodbury = (h->set.precond == 1 && m > 0 && h->set.kkt_system == 0) ? 1 : 0;
        if (h->woodbury) {
            h->ld = ((m + TS - 1) / TS) * TS;
            h->T = h->ld / TS;
            if (size_t(h->ld) * sizeof(double) > 64 * 1024) {
                // the dense block would not fit one workgroup's LDS row buffer
                h->woodbury = 0;
            } else {
                const size_t mm = size_t(h->ld) * h->ld;
                h->Sm = h->dalloc<double>(mm);
                h->Sinv = h->dalloc<double>(mm);
                h->Sm2 = h->dalloc<double>(mm);                       // second matrix of the sweep
                h->Pbuf = h->dalloc<double>(4 * size_t(TS) * TS);      // two pivot inverses, both layouts
                h->wpre = h->dalloc<double>(h->ld);
                h->vpre = h->dalloc<double>(std::max(h->ld, m));
                h->Dw = h->dalloc<double>(n);
                h->scr = h->dalloc<int>(std::max<int64_t>(h->nnzA, 1));
                h->scv = h->dalloc<double>(std::max<int64_t>(h->nnzA, 1));
                h->scnt = h->dalloc<int>(n);
                h->rflag = h->dalloc<int>(m);
                h->rmii = h->dalloc<double>(m);
                h->rpos = h->dalloc<int>(m);
                h->ridx = h->dalloc<int>(m);
                h->kdev = h->dalloc<int>(1);
                HIPCHK(hipMemsetAsync(h->kdev, 0, sizeof(int), h->stream));
                h->srows = 4 * prec_rows_blocks(h);
                h->sext = h->dalloc<int>(2 * size_t(h->srows));
                h->ssq = h->dalloc<double>(h->srows);
            }
        }
        h->log = h->dalloc<double>(4 * size_t(h->set.max_ipm_iter + 1));
        h->isc = h->dalloc<IpmScal>(1);
        h->psc = h->dalloc<PcgScal>(1);
        HIPCHK(hipMemsetAsync(h->psc, 0, sizeof(PcgScal), h->stream));
        h->cert = h->dalloc<CertOut>(1);
        h->fl = h->dalloc<Flags>(1);
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&h->fl_host), 2 * sizeof(Flags), hipHostMallocDefault));
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&h->k_host), sizeof(int), hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&h->ev_k, hipEventDisableTiming));
        for (auto& ev : h->ev_chunk) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventCreate(&h->ev_t0));
        HIPCHK(hipEventCreate(&h->ev_t1));
        for (int i = 0; i < 2; ++i) {
            HIPCHK(hipEventCreate(&h->ev_p0[i]));
            HIPCHK(hipEventCreate(&h->ev_p1[i]));
        }
        HIPCHK(hipMemsetAsync(h->zero_n, 0, sizeof(double) * n, h->stream));
        HIPCHK(hipMemsetAsync(h->zero_m, 0, sizeof(double) * std::max(m, 1), h->stream));

        // cached diag(H) (Section 4.1.2: computed once per objective)
        compute_diag_h(h);
        if (h->set.precision != QP_FP64) ensure_lowp(h, h->set.precision);
        HIPCHK(hipStreamSynchronize(h->stream));
        autotune_schedule(h);
    } catch (const HipError& he) {
        g_create_error = std::string("HIP error in ") + he.what + ": " + hipGetErrorString(he.e);
        delete h;
        return he.e == hipErrorOutOfMemory ? QP_ERR_NOMEM : QP_ERR_DEVICE;
    } catch (const std::bad_alloc&) {
        g_create_error = "host allocation failed";
        delete h;
        return QP_ERR_NOMEM;
    }
    *out = h;
    return QP_OK;
}

qp_status qp_create_device(qp_handle** out, const qp_hessian* H, const qp_csr* J, const double* W,
                           const qp_csr* A, const qp_range* b, const qp_range* bounds, const qp_settings* s,
                           void* hip_stream) {
    g_create_error.clear();
    if (!out || !H || !J) {
        g_create_error = "out, H or J is NULL";
        return QP_ERR_INVALID;
    }
    *out = nullptr;
    if (J->rows < 0 || J->cols < 1 || J->nnz < 0 || (A && (A->rows < 0 || A->nnz < 0)) || H->k < 0) {
        g_create_error = "negative size (or no columns)";
        return QP_ERR_INVALID;
    }
    const size_t n = size_t(J->cols), nJ = size_t(J->rows);
    const size_t m = A ? size_t(A->rows) : 0;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // Host copies of every device array (NULL stays NULL and is judged by
    // qp_create's validation).
    try {
        (void)hipGetLastError();
        hipError_t err = hipSuccess;
        auto fetch = [&](const void* d, size_t count, auto& vec) {
            vec.clear();
            if (!d || count == 0 || err != hipSuccess) return;
            vec.resize(count);
            err = hipMemcpyAsync(vec.data(), d, count * sizeof(vec[0]), hipMemcpyDeviceToHost, st);
        };
        std::vector<double> p, U, w, Wv, Jv, Av, blo, bhi, xlo, xhi;
        std::vector<int64_t> Jp, Ap;
        std::vector<int32_t> Jc, Ac;
        fetch(H->p, n, p);
        fetch(H->U, n * size_t(H->k), U);
        fetch(H->w, size_t(H->k), w);
        fetch(W, nJ, Wv);
        fetch(J->row_ptr, nJ + 1, Jp);
        fetch(J->col_idx, size_t(J->nnz), Jc);
        fetch(J->val, size_t(J->nnz), Jv);
        if (A) {
            fetch(A->row_ptr, m + 1, Ap);
            fetch(A->col_idx, size_t(A->nnz), Ac);
            fetch(A->val, size_t(A->nnz), Av);
        }
        if (b) {
            fetch(b->lo, m, blo);
            fetch(b->hi, m, bhi);
        }
        if (bounds) {
            fetch(bounds->lo, n, xlo);
            fetch(bounds->hi, n, xhi);
        }
        if (err == hipSuccess) err = hipStreamSynchronize(st);
        if (err != hipSuccess) {
            g_create_error = std::string("reading the device arrays: ") + hipGetErrorString(err);
            return QP_ERR_DEVICE;
        }
        auto ptr = [](const auto& vec, const void* orig) { return orig ? vec.data() : nullptr; };
        qp_hessian hH = *H;
        hH.p = ptr(p, H->p);
        hH.U = ptr(U, H->U);
        hH.w = ptr(w, H->w);
        qp_csr hJ = *J;
        hJ.row_ptr = ptr(Jp, J->row_ptr);
        hJ.col_idx = ptr(Jc, J->col_idx);
        hJ.val = ptr(Jv, J->val);
        qp_csr hA{};
        if (A) {
            hA = *A;
            hA.row_ptr = ptr(Ap, A->row_ptr);
            hA.col_idx = ptr(Ac, A->col_idx);
            hA.val = ptr(Av, A->val);
        }
        qp_range hb{}, hx{};
        if (b) {
            hb.lo = ptr(blo, b->lo);
            hb.hi = ptr(bhi, b->hi);
        }
        if (bounds) {
            hx.lo = ptr(xlo, bounds->lo);
            hx.hi = ptr(xhi, bounds->hi);
        }
        return qp_create(out, &hH, &hJ, ptr(Wv, W), A ? &hA : nullptr, b ? &hb : nullptr,
                         bounds ? &hx : nullptr, s, hip_stream);
    } catch (const std::bad_alloc&) {
        g_create_error = "host allocation failed";
        return QP_ERR_NOMEM;
    }
}

qp_status qp_operator_apply(qp_handle* h, const double* sigma_x, const double* sigma_A, const double* v,
                            double* y, int32_t precision, int32_t reps, qp_info* info) {
    if (!h) return QP_ERR_INVALID;
    (void)hipGetLastError();  // drop an error left by an earlier, unrelated call
    if (!sigma_x || !v || !y || (h->m > 0 && !sigma_A)) return fail(h, QP_ERR_INVALID, "NULL argument");
    if (precision < QP_FP64 || precision > QP_BF16) return fail(h, QP_ERR_INVALID, "precision out of range");
    if (reps < 1) reps = 1;
    for (int j = 0; j < h->n; ++j)
        if (!(sigma_x[j] >= 0.0) || !std::isfinite(sigma_x[j]) || !std::isfinite(v[j]))
            return fail(h, QP_ERR_INVALID, "sigma_x must be finite >= 0 and v finite");
    for (int i = 0; i < h->m; ++i)
        if (!(sigma_A[i] >= 0.0) || !std::isfinite(sigma_A[i]))
            return fail(h, QP_ERR_INVALID, "sigma_A must be finite and >= 0");
    try {
        h->aug = false;   // the condensed operator
        ensure_lowp(h, precision);
        ensure_timing_events(h);
        HIPCHK(hipMemcpyAsync(h->tmp_n, sigma_x, sizeof(double) * h->n, hipMemcpyHostToDevice, h->stream));
        if (h->m > 0)
            HIPCHK(hipMemcpyAsync(h->tmp_m, sigma_A, sizeof(double) * h->m, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->tmp_n2, v, sizeof(double) * h->n, hipMemcpyHostToDevice, h->stream));
        TimingAcc ta;
        HIPCHK(hipEventRecord(h->ev_t0, h->stream));
        for (int r = 0; r < reps; ++r) {
            const bool timed = h->set.timing && ta.pairs < int(h->tev.size() / 4);
            const int slot = timed ? ta.pairs++ : 0;
            if (timed) ta.valid.push_back(1);
            apply_op_prec(h, precision, h->tmp_n2, h->pq, h->tmp_n, h->m > 0 ? h->tmp_m : nullptr, 1.0,
                          false, timed, slot);
        }
        HIPCHK(hipEventRecord(h->ev_t1, h->stream));
        HIPCHK(hipMemcpyAsync(y, h->pq, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (info) {
            std::memset(info, 0, sizeof(*info));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, h->ev_t0, h->ev_t1));
            info->t_solve_ms = ms;
            set_format_info(h, info);
            harvest_timing(h, ta, info);
        }
    } catch (const HipError& he) {
        return fail(h, QP_ERR_DEVICE, std::string("HIP error in ") + he.what + ": " + hipGetErrorString(he.e));
    }
    return QP_OK;
}

qp_status qp_operator_apply_noalloc(qp_handle* h, const double* sigma_x, const double* sigma_A, const double* v,
                                    double* y, int32_t precision, void* hip_stream) {
    if (!h) return QP_ERR_INVALID;
    if (!sigma_x || !v || !y || (h->m > 0 && !sigma_A)) return fail(h, QP_ERR_INVALID, "NULL argument");
    if (precision < QP_FP64 || precision > QP_BF16) return fail(h, QP_ERR_INVALID, "precision out of range");
    const bool resident = precision == QP_FP64 ||
                          (h->line ? (precision == QP_FP32 ? h->lval32 != nullptr : h->lval16 != nullptr)
                                   : (precision == QP_FP32 ? h->Jv32 != nullptr : h->Jv16 != nullptr));
    if (!resident)
        return fail(h, QP_ERR_INVALID,
                    "the J values of this precision are not resident (create the handle with that precision, or "
                    "call qp_operator_apply with it once)");
    size_t off[4];
    const size_t need = scratch_layout(h, off);
    if (need > kScratchDoubles)
        return fail(h, QP_ERR_INVALID,
                    "problem too large for the static scratch: needs " + std::to_string(need) +
                        " doubles, the maximum is " + std::to_string(kScratchDoubles) +
                        " (32 MiB); use qp_operator_apply");
    double* sp = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        sp = (h->device >= 0 && h->device < kMaxDevices) ? g_scratch_ptr[h->device] : nullptr;
    }
    if (!sp) {   // not resolved by qp_create on this device: resolve now
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
            return fail(h, QP_ERR_DEVICE, "scratch address unresolved and the handle's device is not current");
        const hipError_t e = resolve_scratch(h->device, &sp);
        if (e != hipSuccess)
            return fail(h, QP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    const OpWork wk{hip_stream ? static_cast<hipStream_t>(hip_stream) : h->stream, sp + off[0], sp + off[0],
                    sp + off[1], sp + off[2], sp + off[3]};
    const bool aug = h->aug;
    h->aug = false;   // the condensed operator
    try {
        (void)hipGetLastError();   // drop an error left by an earlier, unrelated call
        apply_op_prec(h, wk, precision, v, y, sigma_x, h->m > 0 ? sigma_A : nullptr, 1.0, false, false, 0);
    } catch (const HipError& he) {
        h->aug = aug;
        return fail(h, QP_ERR_DEVICE, std::string("HIP error in ") + he.what + ": " + hipGetErrorString(he.e));
    }
    h->aug = aug;
    return QP_OK;
}

qp_status qp_newton_step(qp_handle* h, const double* sigma_x, const double* sigma_A, const double* rhs,
                         double* dx, qp_info* info) {
    if (!h) return QP_ERR_INVALID;
    (void)hipGetLastError();  // drop an error left by an earlier, unrelated call
    if (!sigma_x || !rhs || !dx || (h->m > 0 && !sigma_A)) return fail(h, QP_ERR_INVALID, "NULL argument");
    for (int j = 0; j < h->n; ++j)
        if (!(sigma_x[j] >= 0.0) || !std::isfinite(sigma_x[j]))
            return fail(h, QP_ERR_INVALID, "sigma_x must be finite and >= 0");
    for (int i = 0; i < h->m; ++i)
        if (!(sigma_A[i] >= 0.0) || !std::isfinite(sigma_A[i]))
            return fail(h, QP_ERR_INVALID, "sigma_A must be finite and >= 0");
    qp_status st = QP_OK;
    try {
        ensure_timing_events(h);
        const int n = h->n, m = h->m;
        double* sigx = h->iv.sigx;
        double* sigA = h->iv.sigA;
        double* d = h->iv.d;
        double* b = h->iv.rhs_b;
        HIPCHK(hipMemcpyAsync(sigx, sigma_x, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
        if (m > 0) HIPCHK(hipMemcpyAsync(sigA, sigma_A, sizeof(double) * m, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(b, rhs, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
        reset_flags(h);
        double* dh = h->iv.dh;
        h->aug = h->set.kkt_system == 1 && m > 0;
        hipLaunchKernelGGL(k_jacobi, dim3(grid_rows(n, 64)), dim3(kBlock), 0, h->stream, (const int*)h->Atp,
                           (const double*)h->Atv, (const int*)h->Atc, m > 0 ? 1 : 0, (const double*)sigA,
                           (const double*)sigx, (const double*)h->diagH, n, d, dh, h->aug ? 1 : 0);
        if (h->aug)
            hipLaunchKernelGGL(k_aug_newton_rows, dim3(grid_elems(m)), dim3(kBlock), 0, h->stream,
                               (const double*)sigA, n, m, h->dlu, d, b);
        HIPCHK(hipGetLastError());
        TimingAcc ta;
        HIPCHK(hipEventRecord(h->ev_t0, h->stream));
        bool wbp = (m > 0) && build_precond(h, dh, sigA, nullptr);
        int nsolves = 0;
        PrecAttemptCap cap_guard(h);
        Flags f = newton_direction(h, h->set.precision, nullptr, b, sigx, m > 0 ? sigA : nullptr, d,
                                   wbp ? h->Dw : nullptr, 1.0, false, &ta, &nsolves);
        int fallbacks = 0, tier = TIER_BLOCK;
        while (wbp && prec_stalled(h, f)) {
            // a stalled constraint-block solve: again with the next tier
            // (the capped block, then the Jacobi diagonal)
            ++fallbacks;
            ++tier;
            wbp = tier == TIER_CAPPED && build_precond(h, dh, sigA, nullptr, kPrecCapTau);
            int more = 0;
            const int spent = f.pcg_iters;
            f = newton_direction(h, h->set.precision, nullptr, b, sigx, m > 0 ? sigA : nullptr, d,
                                 wbp ? h->Dw : nullptr, 1.0, false, &ta, &more);
            f.pcg_iters += spent;
            nsolves += more;
        }
        HIPCHK(hipEventRecord(h->ev_t1, h->stream));
        HIPCHK(hipMemcpyAsync(dx, h->px, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
        PcgScal ps{};
        HIPCHK(hipMemcpyAsync(&ps, h->psc, sizeof(PcgScal), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (f.pcg_breakdown) st = QP_ERR_NUMERIC;
        else if (!f.pcg_converged) st = QP_ERR_NOT_CONVERGED;
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->status = st;
            info->pcg_iters = f.pcg_iters;
            info->pcg_solves = nsolves;
            info->pcg_capped = f.pcg_capped;
            info->pcg_relres = ps.bnorm2 > 0 ? std::sqrt(ps.rr / ps.bnorm2) : 0.0;
            info->prec_fallbacks = fallbacks;
            info->prec_tier = (h->woodbury && m > 0) ? tier : TIER_JACOBI;
            set_format_info(h, info);
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, h->ev_t0, h->ev_t1));
            info->t_solve_ms = info->t_pcg_ms = ms;
            harvest_timing(h, ta, info);
        }
    } catch (const HipError& he) {
        return fail(h, QP_ERR_DEVICE, std::string("HIP error in ") + he.what + ": " + hipGetErrorString(he.e));
    }
    if (st == QP_ERR_NUMERIC) h->err = "PCG breakdown";
    else if (st == QP_ERR_NOT_CONVERGED) h->err = "PCG reached pcg_max_iter";
    return st;
}

qp_status qp_solve_from(qp_handle* h, const double* x0, double* x, double* lam_A, double* lam_x,
                        qp_info* info) {
    if (!h) return QP_ERR_INVALID;
    (void)hipGetLastError();  // drop an error left by an earlier, unrelated call
    if (!x) return fail(h, QP_ERR_INVALID, "x is NULL");
    if (x0)
        for (int j = 0; j < h->n; ++j)
            if (!std::isfinite(x0[j])) return fail(h, QP_ERR_INVALID, "x0 has a non-finite entry");
    IpmRun r;
    r.h = h;
    try {
        // a stalled constraint-block solve is repeated with the Jacobi
        // diagonal, which then serves the rest of this QP
        PrecAttemptCap cap_guard(h);
        ipm_start(r, x0);
        while (!r.done) {
            int nsolves = 0;
            const Flags f = ipm_direction(r, &nsolves);
            if (!ipm_after_direction(r, f, nsolves)) break;
            ipm_step(r);
        }
        ipm_finish(r, x, lam_A, lam_x, info);
    } catch (const HipError& he) {
        return fail(h, QP_ERR_DEVICE, std::string("HIP error in ") + he.what + ": " + hipGetErrorString(he.e));
    }
    return r.st;
}

qp_status qp_solve(qp_handle* h, double* x, double* lam_A, double* lam_x, qp_info* info) {
    return qp_solve_from(h, nullptr, x, lam_A, lam_x, info);
}

qp_status qp_update_hessian(qp_handle* h, const qp_hessian* H) {
    if (!h) return QP_ERR_INVALID;
    (void)hipGetLastError();  // drop an error left by an earlier, unrelated call
    const std::string e = validate_hessian(H, h->n);
    if (!e.empty()) return fail(h, QP_ERR_INVALID, e);
    try {
        const int n = h->n, k = H->k;
        // queued work may still read the old objective
        HIPCHK(hipStreamSynchronize(h->stream));
        drop_graphs(h);
        if (k > h->k_cap) {
            h->dfree(h->U); h->dfree(h->w); h->dfree(h->lr_part); h->dfree(h->lr_v);
            const int cap = std::max(k, 2 * h->k_cap);   // a growing term reallocates rarely
            h->U = h->w = h->lr_part = h->lr_v = nullptr;
            h->k = 0;
            h->k_cap = 0;
            h->U = h->dalloc<double>(size_t(n) * cap);
            h->w = h->dalloc<double>(size_t(cap));
            h->lr_part = h->dalloc<double>(size_t(kLrBlocks) * cap);
            h->lr_v = h->dalloc<double>(size_t(cap));
            h->k_cap = cap;
        }
        HIPCHK(hipMemcpyAsync(h->p, H->p, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
        if (k > 0) {
            HIPCHK(hipMemcpyAsync(h->U, H->U, sizeof(double) * size_t(n) * k, hipMemcpyHostToDevice, h->stream));
            HIPCHK(hipMemcpyAsync(h->w, H->w, sizeof(double) * size_t(k), hipMemcpyHostToDevice, h->stream));
        }
        h->k = k;
        h->gamma = H->gamma;
        compute_diag_h(h);
        // the caller may free H's arrays on return
        HIPCHK(hipStreamSynchronize(h->stream));
    } catch (const HipError& he) {
        // the objective is left unspecified (k = 0 if the larger U could not be allocated)
        return fail(h, he.e == hipErrorOutOfMemory ? QP_ERR_NOMEM : QP_ERR_DEVICE,
                    std::string("HIP error in ") + he.what + ": " + hipGetErrorString(he.e));
    }
    return QP_OK;
}

qp_status qp_solve_batch(qp_handle* const* hs, int32_t count, double* const* xs, qp_info* infos) {
    g_create_error.clear();
    if (count < 0 || (count > 0 && (!hs || !xs))) {
        g_create_error = "qp_solve_batch: NULL array or negative count";
        return QP_ERR_INVALID;
    }
    for (int i = 0; i < count; ++i) {
        if (!hs[i] || !xs[i]) {
            g_create_error = "qp_solve_batch: NULL handle or output at index " + std::to_string(i);
            return QP_ERR_INVALID;
        }
        for (int j = 0; j < i; ++j) {
            if (hs[j] == hs[i]) {
                g_create_error = "qp_solve_batch: a handle appears twice";
                return QP_ERR_INVALID;
            }
            // concurrent workers capture and launch on their handles' streams
            if (hs[j]->stream == hs[i]->stream) {
                g_create_error = "qp_solve_batch: two handles share a stream";
                return QP_ERR_INVALID;
            }
        }
    }
    if (count == 0) return QP_OK;
    if (batch_persistent_ok(hs, count)) {
        std::vector<qp_status> st;
        try {
            st = batch_solve(hs, count, xs, infos);
        } catch (const HipError& he) {
            g_create_error = std::string("qp_solve_batch: HIP error in ") + he.what + ": " + hipGetErrorString(he.e);
            return he.e == hipErrorOutOfMemory ? QP_ERR_NOMEM : QP_ERR_DEVICE;
        }
        qp_status worst = QP_OK;
        for (int i = 0; i < count; ++i) {
            if (infos && st[i] != QP_OK) infos[i].status = st[i];
            if (st[i] != QP_OK && (worst == QP_OK || st[i] == QP_ERR_DEVICE)) worst = st[i];
        }
        return worst;
    }
    // largest problems first, so the tail of the batch is short
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return hs[a]->nnzJ + hs[a]->nnzA > hs[b]->nnzJ + hs[b]->nnzA;
    });
    // host workers (each drives its handles' streams): six by default, the
    // fastest of 2/4/6/8 on the 16-QP uneven batch (FP64: 1029, 986, 935,
    // 944 ms); the host's waits on one handle's flags leave other workers'
    // launches in flight
    int workers = 6;
    if (const char* e = std::getenv("QPGPU_BATCH_WORKERS")) workers = std::max(1, std::atoi(e));
    workers = std::min(workers, count);
    std::vector<qp_status> st(count, QP_OK);
    std::atomic<int> next{0};
    auto work = [&]() {
        while (true) {
            const int q = next.fetch_add(1);
            if (q >= count) break;
            const int i = order[q];
            (void)hipSetDevice(hs[i]->device);
            qp_info inf{};
            st[i] = qp_solve(hs[i], xs[i], nullptr, nullptr, &inf);
            if (infos) infos[i] = inf;
        }
    };
    std::vector<std::thread> pool;
    for (int w = 1; w < workers; ++w) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    qp_status worst = QP_OK;
    for (int i = 0; i < count; ++i)
        if (st[i] != QP_OK && (worst == QP_OK || st[i] == QP_ERR_DEVICE)) worst = st[i];
    return worst;
}

}  // extern "C"
