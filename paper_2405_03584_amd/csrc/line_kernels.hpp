// Operator kernels for the line format of J (host_prep.h: LineFormat).
//
// A dose matrix whose rows come in lines of 64 voxels sharing one column list
// (the 64-voxel bands of every spot) is stored once: column ids per line and
// values slot-major with the 64 rows of a slot contiguous.
//
// The product J^T W J p takes two kernels and reads the values of J once:
//
//  k_line_pass   a block per line: lane r of each wavefront owns row r, the
//                four wavefronts take contiguous quarters of the line's
//                slots and keep their values in registers.  Pass 1 forms
//                t_r = W_r (J p)_r (the quarters' partial sums combined in a
//                fixed order through LDS); pass 2 multiplies the held values
//                by t_r and reduces over the 64 rows of every slot, giving
//                c[slot] = sum_r J_(r,slot) t_r, the line's contribution to
//                (J^T t)_col(slot).  Other blocks: u = Sigma_A .* (A p), by
//                rows of A, or in a PCG product from A z (left by the
//                previous iteration's k_pcg_scalars) as A p = A z + beta A p.
//  k_spot_pass   spot j sums c over the slots it covers (its (line, slot)
//                list), adds gamma p_j, the low-rank term, Sigma_x p_j and
//                (A^T u)_j, and in a PCG product stores p and the p^T q
//                partials.
//
// Against two SpMV passes (J, then J^T reading the values again) this halves
// the HBM traffic of J; c is one double per slot (1/64 per nonzero).
#pragma once

#include <type_traits>

#include "ipm_kernels.hpp"

namespace qpg {

// Slots of a line kept in registers per wavefront; a line with more than
// 4*kLineHeld slots streams the rest from memory in both passes.
constexpr int kLineHeld = 32;

// Slot groups of the low-precision copies: the P values of one row in P
// consecutive slots of a line sit together (8 bytes), so a lane loads its
// row's group in one load and a wavefront moves 512 bytes per load, as with
// FP64 values.  Group g of a line (slots gP .. gP+P-1) occupies 64 lanes x 8
// bytes at the line's values + g*64*P; lines hold whole groups (their slot
// counts are multiples of kLineGroup).  FP64 values keep one slot per load.
constexpr int kLineGroup = 4;
template <typename VT> struct SlotPack { static constexpr int P = 8 / int(sizeof(VT)); };
template <> struct SlotPack<double> { static constexpr int P = 1; };

// A lane's base pointer into a line's values: its row's first value (P = 1)
// or its row's 8-byte word of the first slot group (P > 1); group gi is 64
// words further per group.
template <typename VT>
using LaneWord = typename std::conditional<SlotPack<VT>::P == 1, VT, uint64_t>::type;
template <typename VT>
__device__ __forceinline__ const LaneWord<VT>* lane_base(const VT* lval, int off, int lane) {
    return reinterpret_cast<const LaneWord<VT>*>(lval + size_t(off) * 64) + lane;
}

// The P values of slot group gi (slots gi*P ...) of the lane's row.
template <typename VT, typename AT, bool NT>
__device__ __forceinline__ void load_group(const LaneWord<VT>* v, int gi, AT* out) {
    constexpr int P = SlotPack<VT>::P;
    if constexpr (P == 1) {
        out[0] = cvt<AT>(load_val<NT>(&v[size_t(gi) * 64]));
    } else {
        const uint64_t* pb = &v[size_t(gi) * 64];
        const uint64_t wv = NT ? __builtin_nontemporal_load(pb) : *pb;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            if constexpr (P == 4)
                out[s] = cvt<AT>(bf16_t{uint16_t(wv >> (16 * s))});
            else
                out[s] = AT(__uint_as_float(uint32_t(wv >> (32 * s))));
        }
    }
}

// The packed low-precision copy of a line format's values (FP64, slot-major,
// nslots * 64): thread (g, r) writes the 8-byte group of row r in slot group g,
// each value rounded as d2f_bits / d2bf16_bits round.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_pack_line(const double* src, size_t groups, uint64_t* dst) {
    constexpr int P = SlotPack<VT>::P;
    static_assert(P == 2 || P == 4, "packed copies hold 2- or 4-byte values");
    for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < groups * 64; i += size_t(gridDim.x) * kBlock) {
        const size_t g = i >> 6, r = i & 63;
        uint64_t wv = 0;
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const double x = src[(g * P + s) * 64 + r];
            const uint64_t bits = P == 4 ? uint64_t(d2bf16_bits(x)) : uint64_t(d2f_bits(x));
            wv |= bits << ((64 / P) * s);
        }
        dst[i] = wv;
    }
}

template <typename VT>
struct LineArgs {
    const int* lptr; const int* lcol; const VT* lval; int L; const double* W;
    const int* Ap; const int* Ac; const double* Av; int m;
    const double* x; const double* p2; const PcgScal* sc;   // gathered vector, as in FwdArgs
    double* c;             // per slot (lptr[L] entries)
    double* u; const double* sigA;
    const double* az;      // A z of the new direction's z (nbU > 0)
    double* apv;           // A p: the previous direction's on entry, the new one's on exit (nbU > 0)
    int nbL;               // blocks working on lines (one line per block)
    int nbA;               // blocks working on rows of A (after the nbU blocks, one row each)
    int nbU;               // blocks forming u from A z and A p (first in the grid)
    const Flags* fl;       // PCG product: skipped once the PCG solve has stopped
    const Flags* fl_ipm;   // residual pass: skipped once the IPM has finished
    AugRows aug;           // doubly augmented system: the lambda block (aug.dlu null: condensed)
};

// Body of the line pass for block bi of a grid of nb blocks (the blocks of one
// QP; a batched launch hands each QP its own range).  remap: spread the line
// blocks over the XCDs here (a batched launch remaps its whole grid instead).
template <typename VT, typename AT, bool NT>
__device__ __forceinline__ void line_pass_body(const LineArgs<VT>& a, int bi, int nb, bool remap) {
    constexpr int NW = kBlock / 64;
    constexpr int RH = kLineHeld;
    static_assert(NW == 4, "the pass-1 combine adds four wavefront partials");
    __shared__ AT part[NW][64];
    // The u blocks and the rows of A come first in the grid, so their longer
    // dependent chains run beside the line blocks instead of trailing them;
    // the line blocks are remapped so each XCD streams one contiguous range
    // of lines.
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int first = a.nbU + a.nbA;
    const bool side = bi < first;   // a u block or an A-row block
    const int b = side ? a.nbL : (remap ? xcd_remap(bi - first, nb - first) : bi - first);
    // the line's extent is loaded before the stop test so both loads overlap
    // (blocks past the lines read the last line's extent, unused; L = 0 reads
    // nothing).  With 2- and 4-byte values, where a line is short work and
    // the block's chain of dependent loads sets its time, the rows' weights
    // are loaded here too; with doubles they are loaded after pass 1, where
    // no register is free for them earlier.
    constexpr bool kEarlyW = sizeof(VT) < 8;
    const int lb = max(0, min(b, a.L - 1));
    const int off = a.L > 0 ? a.lptr[lb] : 0;
    const int end = a.L > 0 ? a.lptr[lb + 1] : 0;
    const double wrow = (kEarlyW && a.L > 0) ? a.W[size_t(lb) * 64 + lane] : 0.0;
    if (pcg_stopped_ro(a.fl) || (a.fl_ipm && a.fl_ipm->ipm_done)) return;
    const Gather g = make_gather(a.x, a.p2, a.sc);
    if (bi < a.nbU) {
        // A p of the new direction p = z + beta p from the two m-vectors
        for (int i = bi * kBlock + threadIdx.x; i < a.m; i += a.nbU * kBlock) {
            const double v = fma(g.beta, a.apv[i], a.az[i]);
            a.apv[i] = v;
            a.u[i] = a.sigA ? a.sigA[i] * v : v;
        }
        return;
    }
    if (b < a.nbL) {
        constexpr int P = SlotPack<VT>::P;
        static_assert(kLineGroup % P == 0 && RH % P == 0 && 8 % P == 0, "whole slot groups");
        const int l = b;
        const int len = end - off;   // a multiple of kLineGroup
        // each wavefront's range holds whole slot groups
        const int q = (((len + NW - 1) / NW) + P - 1) / P * P;
        const int k0 = __builtin_amdgcn_readfirstlane(min(len, w * q));
        const int k1 = __builtin_amdgcn_readfirstlane(min(len, k0 + q));
        // held slots [kh, k1): the last RH of the wavefront's range; the
        // slots before them (only in lines longer than NW*RH slots) are
        // streamed first, so their registers are free before the held loads
        const int kh = max(k0, k1 - RH);
        const LaneWord<VT>* v = lane_base(a.lval, off, lane);
        const int* col = a.lcol + off;
        AT acc = AT(0);
        for (int k = k0; k < kh; k += 4) {
            AT s4 = AT(0);
#pragma unroll
            for (int j = 0; j < 4 / P; ++j) {
                AT gv[P];
                load_group<VT, AT, NT>(v, min((k + j * P) / P, kh / P - 1), gv);
#pragma unroll
                for (int t = 0; t < P; ++t) {
                    const int kk = min(k + j * P + t, kh - 1);
                    const AT prod = gv[t] * AT(g(col[kk]));
                    s4 += (k + j * P + t < kh) ? prod : AT(0);
                }
            }
            acc += s4;
        }
        // pass 1: partial (J p)_r over this wavefront's held slots.  Lane i
        // gathers p at the column of held slot kh+i (one coalesced index load
        // and one gather per lane instead of RH wave-uniform ones), and the
        // product loop reads it back with readlane.  Value loads past k1 are
        // clamped to k1-1 (a valid address) and zeroed, so every load is
        // issued at once, without branches between them.
        AT hv[RH];
        if (kh < k1) {
            const double pl = g(col[min(kh + (lane & (RH - 1)), k1 - 1)]);
            // FP32 accumulation: each lane rounds its gathered value to float
            // once, so a slot costs one 32-bit broadcast and no conversion
            // (the same float as converting the broadcast double)
            constexpr bool kF = sizeof(AT) == 4;
            const int plo = kF ? __float_as_int(float(pl)) : __double2loint(pl);
            const int phi = kF ? 0 : __double2hiint(pl);
#pragma unroll
            for (int j = 0; j < RH / P; ++j) {
                AT gv[P];
                load_group<VT, AT, NT>(v, min(kh / P + j, k1 / P - 1), gv);
#pragma unroll
                for (int t = 0; t < P; ++t) hv[j * P + t] = (kh + j * P < k1) ? gv[t] : AT(0);
            }
            AT a2[2] = {AT(0), AT(0)};   // two chains, no product array
#pragma unroll
            for (int i = 0; i < RH; ++i) {
                AT xv;
                if constexpr (kF) {
                    xv = __int_as_float(__builtin_amdgcn_readlane(plo, i));
                } else {
                    xv = AT(__hiloint2double(__builtin_amdgcn_readlane(phi, i), __builtin_amdgcn_readlane(plo, i)));
                }
                a2[i & 1] = fma(hv[i], xv, a2[i & 1]);
            }
            acc += a2[0] + a2[1];
        } else {
#pragma unroll
            for (int i = 0; i < RH; ++i) hv[i] = AT(0);
        }
        part[w][lane] = acc;
        __syncthreads();
        const AT s = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
        const AT t = AT((kEarlyW ? wrow : a.W[size_t(l) * 64 + lane]) * double(s));
        // pass 2: c[slot] = sum_r J_(r,slot) t_r, RH slots per reduce-scatter
        constexpr int SHIFT = RH == 32 ? 1 : RH == 16 ? 2 : RH == 8 ? 3 : RH == 4 ? 4 : RH == 2 ? 5 : 6;
        const int slot = lane >> SHIFT;
        const bool writer = (lane & ((1 << SHIFT) - 1)) == 0;
        if (kh < k1) {   // held slots (hv is dead afterwards)
#pragma unroll
            for (int i = 0; i < RH; ++i) hv[i] *= t;
            const AT cs = wave_reduce_scatter<RH>(hv, lane);
            if (writer && kh + slot < k1) a.c[off + kh + slot] = double(cs);
        }
        for (int kg = k0; kg < kh; kg += 8) {   // streamed slots of long lines, 8 at a time
            AT pv[8];
#pragma unroll
            for (int j = 0; j < 8 / P; ++j) {
                AT gv[P];
                load_group<VT, AT, NT>(v, min(kg / P + j, kh / P - 1), gv);
#pragma unroll
                for (int u = 0; u < P; ++u) pv[j * P + u] = (kg + j * P < kh) ? gv[u] * t : AT(0);
            }
            const AT cs = wave_reduce_scatter<8>(pv, lane);
            if ((lane & 7) == 0 && kg + (lane >> 3) < kh) a.c[off + kg + (lane >> 3)] = double(cs);
        }
    } else {
        // a row of A per workgroup: 256 lanes with two loads each cover up to
        // 512 nonzeros in one round of gathers; wavefront sums combined in
        // a fixed order through LDS
        const int row = bi - a.nbU;
        double s = 0.0;
        if (row < a.m) s = row_dot_lane_g<kBlock, double, double, 2>(a.Ap, a.Ac, a.Av, g, row, threadIdx.x);
        s = group_sum<double, 64>(s);
        __shared__ double rs[NW];
        if (lane == 0) rs[w] = s;
        __syncthreads();
        if (threadIdx.x == 0 && row < a.m) {
            const double tot = (rs[0] + rs[1]) + (rs[2] + rs[3]);
            if (a.aug.dlu) a.u[row] = aug_row(a.aug, a.m, row, tot, a.sigA[row], g, const_cast<double*>(a.p2));
            else a.u[row] = a.sigA ? a.sigA[row] * tot : tot;
        }
    }
}

template <typename VT, typename AT, bool NT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_line_pass(LineArgs<VT> a) {
    line_pass_body<VT, AT, NT>(a, int(blockIdx.x), int(gridDim.x), true);
}

struct SpotArgs {
    const int* sptr; const int* sslot; const double* c; int n;
    const int* Atp; const int* Atc; const double* Atv; int hasA;
    const double* u;
    const double* x;       // gathered vector (its own entries only)
    const double* sigx;
    double hs, gamma;
    double* q;
    double* part;
    const Flags* fl;
    PcgLink pcg;           // as in BwdArgs
    const double* U; const double* lr_v; int lr_k;
};

// q_j = hs*((J^T W J p)_j + gamma p_j + (U(w .* U^T p))_j) + Sigma_x,j p_j + (A^T u)_j
// with G lanes per spot, per-block partials of p^T q and, in a PCG product,
// p stored back.
// Body for block b (already placed on its XCD) of a grid of nb blocks.
template <int G>
__device__ __forceinline__ void spot_pass_body(const SpotArgs& a, int b, int nb) {
    __shared__ double sh[kBlock / 64];
    if (pcg_stopped_ro(a.fl)) return;
    constexpr int RPB = kBlock / G;
    const int lane = threadIdx.x % G;
    const double beta = a.pcg.p2 ? a.pcg.sc->beta : 0.0;
    double dot = 0.0;
    for (int base = b * RPB; base < a.n; base += nb * RPB) {
        const int j = base + threadIdx.x / G;
        if (j < a.n) {
            // the spot's own entries are loaded first, beside the sums' loads
            const double xj = a.x[j];
            const double p2j = a.pcg.p2 ? a.pcg.p2[j] : 0.0;
            const double sxj = a.sigx ? a.sigx[j] : 0.0;
            double s = index_sum_plus_row_dot<G>(a.sptr, a.sslot, a.c, a.hasA ? a.Atp : nullptr, a.Atc, a.Atv,
                                                 a.u, a.hs, j, lane);
            if (a.lr_k) s += a.hs * lowrank_lane<G>(a.U, a.lr_v, a.lr_k, a.n, j, lane);
            s = group_sum<double, G>(s);
            if (lane == 0) {
                // direction entry p_j = z_j + beta p_j, stored back in a PCG product
                const double pj = a.pcg.p2 ? xj + beta * p2j : xj;
                if (a.pcg.p2) a.pcg.p2[j] = pj;
                double y = s + a.hs * a.gamma * pj;
                if (a.sigx) y += sxj * pj;
                a.q[j] = y;
                dot += pj * y;
            }
        }
    }
    product_tail(dot, a.part, b, sh);
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_spot_pass(SpotArgs a) {
    spot_pass_body<G>(a, xcd_remap(int(blockIdx.x), int(gridDim.x)), int(gridDim.x));
}

}  // namespace qpg
