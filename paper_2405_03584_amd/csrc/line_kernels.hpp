// Operator kernels for the line format of J (host_prep.h: LineFormat).
//
// A dose matrix whose rows come in lines of 64 voxels sharing one column list
// (the 64-voxel bands of every spot) is stored once: column ids per line and
// values slot-major with the 64 rows of a slot contiguous.  J p then needs no
// per-entry index: a wavefront owns a line, lane r owns row r, the column id
// and p[col] of each slot are wave-uniform (scalar loads) and each slot's 64
// values are one coalesced load.  J^T t reads the same values: spot j visits
// the (line, slot) pairs it covers, and both lval[slot*64 + r] and
// t[line*64 + r] are contiguous in r.  Index traffic falls from 4 bytes per
// nonzero (CSR) to 4 bytes per (line, slot) pair, 1/64 per nonzero.
#pragma once

#include "ipm_kernels.hpp"

namespace qpg {

template <typename VT>
struct LineFwdArgs {
    const int* lptr; const int* lcol; const VT* lval; int L; const double* W;
    const int* Ap; const int* Ac; const double* Av; int m;
    const double* x; double* t; double* u; const double* sigA;
    int nbL;               // blocks working on lines (one line per block)
    const Flags* fl;
};

// t = W .* (J x): a block per line, lane = row; the 4 wavefronts of the block
// take contiguous quarters of the line's slots and their partial row sums are
// added in a fixed order through LDS.  u = Sigma_A .* (A x): a wavefront per
// row of A in the remaining blocks.
template <typename VT, typename AT>
__global__ __launch_bounds__(kBlock) void k_op_fwd_line(LineFwdArgs<VT> a) {
    __shared__ AT part[kBlock / 64][64];
    if (pcg_stopped(a.fl)) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    if (b < a.nbL) {
        const int l = b;
        const int off = a.lptr[l];
        const int len = a.lptr[l + 1] - off;
        const int q = (len + 3) >> 2;
        const int k0 = __builtin_amdgcn_readfirstlane(min(len, w * q));
        const int k1 = __builtin_amdgcn_readfirstlane(min(len, k0 + q));
        const VT* v = a.lval + size_t(off) * 64 + lane;
        const int* c = a.lcol + off;
        AT acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = AT(0);
        // passes of 8 slots; slots past k1 are clamped to k1-1 (valid address)
        // and contribute 0, so each pass issues all its loads without branches
        for (int k = k0; k < k1; k += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kk = min(k + u, k1 - 1);
                const AT prod = cvt<AT>(v[size_t(kk) * 64]) * AT(a.x[c[kk]]);
                acc[u] += (k + u < k1) ? prod : AT(0);
            }
        }
        part[w][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        __syncthreads();
        if (w == 0) {
            const AT s = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
            const int row = l * 64 + lane;
            a.t[row] = a.W[row] * double(s);
        }
    } else {
        const int row = (b - a.nbL) * (kBlock / 64) + w;
        if (row < a.m) {
            double s = row_dot_lane<64, double, double>(a.Ap, a.Ac, a.Av, a.x, row, lane);
            s = group_sum<double, 64>(s);
            if (lane == 0) a.u[row] = a.sigA ? a.sigA[row] * s : s;
        }
    }
}

template <typename VT>
struct LineBwdArgs {
    const int* sptr; const int* sline; const int* sslot; const VT* lval; int n;
    const int* Atp; const int* Atc; const double* Atv; int hasA;
    const double* t; const double* u; const double* p;
    const double* sigx;
    double hs, gamma;
    double* q;
    double* part;
    const Flags* fl;
    const double* U; const double* lr_v; int lr_k;
};

// q_j = hs*(J^T t + gamma p + U(w .* U^T p))_j + Sigma_x,j p_j + (A^T u)_j with
// a wavefront per spot j, and per-block partials of p^T q.
template <typename VT, typename AT>
__global__ __launch_bounds__(kBlock) void k_op_bwd_line(LineBwdArgs<VT> a) {
    __shared__ double sh[kBlock / 64];
    if (pcg_stopped(a.fl)) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    constexpr int WPB = kBlock / 64;
    double dot = 0.0;
    for (int base = b * WPB; base < a.n; base += gridDim.x * WPB) {
        const int j = __builtin_amdgcn_readfirstlane(base + (threadIdx.x >> 6));
        if (j < a.n) {
            const int e0 = a.sptr[j], e1 = a.sptr[j + 1];
            AT acc[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = AT(0);
            // passes of 16 pairs, tail clamped to the last pair and zeroed
            for (int e = e0; e < e1; e += 16) {
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int ee = min(e + u, e1 - 1);
                    const int l = a.sline[ee], s = a.sslot[ee];
                    const AT prod = cvt<AT>(a.lval[size_t(s) * 64 + lane]) * AT(a.t[size_t(l) * 64 + lane]);
                    acc[u] += (e + u < e1) ? prod : AT(0);
                }
            }
            AT sj = AT(0);
#pragma unroll
            for (int u = 0; u < 16; u += 2) sj += acc[u] + acc[u + 1];
            double s = a.hs * double(sj);
            if (a.hasA) s += row_dot_lane<64, double, double>(a.Atp, a.Atc, a.Atv, a.u, j, lane);
            if (a.lr_k) s += a.hs * lowrank_lane<64>(a.U, a.lr_v, a.lr_k, a.n, j, lane);
            s = group_sum<double, 64>(s);
            if (lane == 0) {
                const double pj = a.p[j];
                double y = s + a.hs * a.gamma * pj;
                if (a.sigx) y += a.sigx[j] * pj;
                a.q[j] = y;
                dot += pj * y;
            }
        }
    }
    if (a.part) {
        const double tot = block_sum(dot, sh);
        if (threadIdx.x == 0) a.part[b] = tot;
    }
}

}  // namespace qpg
