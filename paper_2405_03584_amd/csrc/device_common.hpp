// Device kernels of the IPM search-direction path for gfx950 (wave64).
//
// Operator of every PCG iteration (condensed Newton system, Section 4 of the
// paper, in the matrix-free style of Section 4.1.1):
//
//     q = hs*(gamma*p + J^T (W .* (J p)) [+ U(w .* (U^T p))]) + Sigma_x .* p
//         + A^T (Sigma_A .* (A p))
//
// with hs = 1/zeta the objective scale.  J and its stored transpose J^T (the
// paper stores transposes so every SpMV is transpose-free, Section 4.1.1) are
// CSR; each row is handled by a group of G lanes of one wavefront (G picked
// per matrix from its row lengths).  No atomics: every sum has a fixed order,
// reductions across blocks are two-stage (per-block partials reduced by the
// consumer in a fixed order), so results are bitwise reproducible run to run
// (the reproducibility requirement the paper meets with a deterministic
// sparse library mode, Section 6.1.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qpg {

constexpr int kBlock = 256;         // 4 wavefronts
constexpr int kMaxPartials = 8192;  // cap on blocks that emit reduction partials
constexpr int kMaxElemGrid = 2048;  // cap on grid-stride elementwise grids

// --------------------------------------------------------------------------
// scalar state shared by kernels (device memory)
// --------------------------------------------------------------------------
// PCG scalars.  Each field is written by one thread of one kernel and read
// only by later kernels (kernel boundaries order the accesses).
struct PcgScal {
    double rho;        // r^T z of the current z
    double beta;       // p <- z + beta p, applied on the fly by the next product
    double alpha;      // rho / p^T q
    double pq;         // p^T q
    double bnorm2;     // ||rhs||^2
    double tol2;       // pcg_tol^2 * ||rhs||^2
    double rr;         // ||r||^2 after the last update
    double bnorm2_outer;   // ||rhs||^2 of the first solve of a refined direction
    int32_t iters;
    int32_t max_iter;
};

struct IpmScal {
    double mu;
    double mu_tol;
    double hs;         // 1/zeta
    double zeta;
    double pmax;       // ||p/zeta||_inf
    double cscale;     // 1 + ||c||_inf over finite bounds
    double rnorm;
    double alpha_p, alpha_d;
    double tau;
    double xHx, px;    // scaled x^T H x, p^T x at the last residual pass
    double mtot;
    int32_t done;
    int32_t iter;
    int32_t step_mode;
    int32_t pad;
};

// flags the host polls (one small struct copied to pinned memory)
struct Flags {
    int32_t pcg_converged, pcg_breakdown, pcg_capped, ipm_done;
    int32_t pcg_iters, ipm_iter, pad0, pad1;
};

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------
struct bf16_t { uint16_t b; };

__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(bf16_t v) { return __uint_as_float(uint32_t(v.b) << 16); }
__device__ __forceinline__ double to_f64(float v) { return double(v); }
__device__ __forceinline__ double to_f64(bf16_t v) { return double(__uint_as_float(uint32_t(v.b) << 16)); }

template <typename AT, typename VT> __device__ __forceinline__ AT cvt(VT v);
template <> __device__ __forceinline__ double cvt<double, double>(double v) { return v; }
template <> __device__ __forceinline__ double cvt<double, float>(float v) { return double(v); }
template <> __device__ __forceinline__ double cvt<double, bf16_t>(bf16_t v) { return to_f64(v); }
template <> __device__ __forceinline__ float cvt<float, float>(float v) { return v; }
template <> __device__ __forceinline__ float cvt<float, bf16_t>(bf16_t v) { return to_f32(v); }

// Loads of matrix values and column ids that are read once per product.
// When the arrays streamed by one product are larger than the last-level
// cache (MI355X: 256 MB Infinity Cache), cycling them through the caches
// only evicts what is reused (the gathered vectors, W, the per-row or
// per-slot sums), so such arrays are read with non-temporal loads
// (NT = true); smaller arrays stay cacheable, and then stay resident between
// products.
template <bool NT, typename T>
__device__ __forceinline__ T load_val(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ bf16_t load_val(const bf16_t* p) {
    if constexpr (NT) return bf16_t{__builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p))};
    else return *p;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Remap so that each XCD works on one contiguous range of logical
// blocks: neighbouring rows gather neighbouring vector entries, which then
// share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    // XCD x owns q (+1 if x < r) consecutive logical blocks
    const int start = x * q + (x < r ? x : r);
    const int cnt = q + (x < r ? 1 : 0);
    return (i < cnt) ? start + i : b;  // i < cnt always holds; keep b as a guard
}

template <typename T, int W>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
}

// Sum over the block in a fixed order; result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = group_sum<double, 64>(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) s += sh[i];
    return s;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) s = fmax(s, sh[i]);
    return s;
}

__device__ __forceinline__ double block_min(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
#pragma unroll
    for (int i = 1; i < kBlock / 64; ++i) s = fmin(s, sh[i]);
    return s;
}

// Gathered vector of a product: x, or (PCG) the search direction z + beta p
// formed on the fly from the last z and the previous p.
// A product that is never fused into a later addition: sums whose terms are
// formed in different kernels (a term kept in registers, or staged in LDS)
// then round every term the same way.
template <typename T>
__device__ __forceinline__ T mul_nc(T a, T b) {
#pragma clang fp contract(off)
    return a * b;
}

struct Gather {
    const double* x;
    const double* p2;   // null: plain x
    double beta;
    __device__ __forceinline__ double operator()(int c) const { return p2 ? x[c] + beta * p2[c] : x[c]; }
};

// Reduce `count` per-block partials (stride `stride` between them) in a fixed
// order; every block that calls this gets the identical value.  Thread t adds
// partials t, t+B, t+2B, ... in increasing order; each pass issues 8 loads at
// once (indices past the end clamped and their values dropped) so a long
// list costs one memory latency per 8B partials.
__device__ __forceinline__ double reduce_partials_sum(const double* part, int count, int stride, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < count; i += 8 * kBlock) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = part[size_t(min(i + u * kBlock, count - 1)) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += (i + u * kBlock < count) ? t[u] : 0.0;
    }
    return block_sum(v, sh);
}
__device__ __forceinline__ double reduce_partials_max(const double* part, int count, int stride, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) v = fmax(v, part[size_t(i) * stride]);
    return block_max(v, sh);
}
__device__ __forceinline__ double reduce_partials_min(const double* part, int count, int stride, double* sh) {
    double v = 1.0e300;
    for (int i = threadIdx.x; i < count; i += kBlock) v = fmin(v, part[size_t(i) * stride]);
    return block_min(v, sh);
}

// Dot product of CSR row `row` with a gathered vector by a group of G lanes (lane in [0,G)).
// Each pass lets every lane issue U index/value loads at once (clamped
// past the row end), then U gathers, so a row costs about one index latency
// plus one gather latency per U*G entries instead of one per entry; U
// independent accumulators are combined in a fixed order.  The group sum is
// done by the caller.
template <int G, typename VT, typename AT, int U = 4, typename GV>
__device__ __forceinline__ AT row_dot_lane_g(const int* __restrict__ ptr, const int* __restrict__ col,
                                             const VT* __restrict__ val, const GV& x, int row, int lane) {
    const int a = ptr[row], b = ptr[row + 1];
    AT acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = AT(0);
    if (b <= a) return AT(0);
    // Indices past the row end are clamped to its last entry (a valid
    // address) and their products zeroed, so every load of a pass is issued
    // unconditionally, without branches between them.
    for (int k = a + lane; k < b; k += U * G) {
        int c[U];
        AT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kk = min(k + u * G, b - 1);
            c[u] = col[kk];
            v[u] = cvt<AT>(val[kk]);
        }
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x(c[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] += (k + u * G < b) ? v[u] * AT(xv[u]) : AT(0);
    }
    AT s = acc[0];
#pragma unroll
    for (int u = 1; u < U; ++u) s += acc[u];
    return s;
}

// Sum of term(e) over e in [a, b) by a group of G lanes (G divides 64) with
// the same bits for every G: it is the sum 64 virtual lanes would form, where
// virtual lane v adds the terms e = a + v, a + v + 64, ... in order and the 64
// partial sums are combined by the butterfly with offsets 32, 16, ..., 1.
// Lane p of the group keeps virtual lanes p + G*j (j < 64/G); butterfly
// offsets >= G combine them inside the lane, smaller ones across lanes.  Each
// pass issues about 8 term loads per lane before adding (indices past b
// clamped to b-1 and not added).  Every lane of the group returns the sum.
// Used where the lane count is a tunable schedule, so that the schedule
// never changes results.
template <int G, typename AT, typename Term>
__device__ __forceinline__ AT canon_sum(int a, int b, int lane, const Term& term) {
    static_assert(G >= 1 && G <= 64 && 64 % G == 0, "G must divide 64");
    constexpr int NJ = 64 / G;
    constexpr int UT = NJ >= 8 ? 1 : 8 / NJ;
    AT vs[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) vs[j] = AT(0);
    for (int base = a; base < b; base += 64 * UT) {
        AT tv[UT][NJ];
#pragma unroll
        for (int u = 0; u < UT; ++u)
#pragma unroll
            for (int j = 0; j < NJ; ++j) tv[u][j] = term(min(base + 64 * u + lane + G * j, b - 1));
#pragma unroll
        for (int u = 0; u < UT; ++u)
#pragma unroll
            for (int j = 0; j < NJ; ++j) vs[j] = (base + 64 * u + lane + G * j < b) ? vs[j] + tv[u][j] : vs[j];
    }
#pragma unroll
    for (int off = 32; off >= G; off >>= 1) {
        AT nv[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) nv[j] = vs[j] + vs[j ^ (off / G)];
#pragma unroll
        for (int j = 0; j < NJ; ++j) vs[j] = nv[j];
    }
    AT s = vs[0];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
    return s;
}

// Partials of per-row values over fixed chunks of kChunkRows consecutive rows
// (chunk c = rows 4c..4c+3): the chunk structure follows the row numbers
// only, not the rows per workgroup, so sums built from these partials do not
// depend on the lane count per row.  vals[k * ld + r] holds value k of row
// base + r of the pass (r < RPB, rows past n hold 0); values k < NV - 2 are
// maxima (when NV > 1), the last two (or the only one) sums in row order.
// One thread per chunk writes out[NV * chunk + k].
constexpr int kChunkRows = 4;
template <int RPB, int NV>
__device__ __forceinline__ void chunk_partials(const double* vals, int ld, int base, int n, double* out) {
    const int c = threadIdx.x;
    if (c >= RPB / kChunkRows || base + kChunkRows * c >= n) return;
    const size_t chunk = size_t(base / kChunkRows + c);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double* r = vals + size_t(k) * ld + kChunkRows * c;
        const bool is_max = NV > 1 && k < NV - 2;
        out[NV * chunk + k] = is_max ? fmax(fmax(r[0], r[1]), fmax(r[2], r[3])) : ((r[0] + r[1]) + r[2]) + r[3];
    }
}

template <int G, typename VT, typename AT, int U = 4>
__device__ __forceinline__ AT row_dot_lane(const int* __restrict__ ptr, const int* __restrict__ col,
                                           const VT* __restrict__ val, const double* __restrict__ x,
                                           int row, int lane) {
    const Gather g{x, nullptr, 0.0};
    return row_dot_lane_g<G, VT, AT, U>(ptr, col, val, g, row, lane);
}

// Sum of val[idx[e]] over e in [ptr[row], ptr[row+1]) by a group of G lanes,
// U loads per lane in flight per pass (clamped past the end, as above).
template <int G, int U = 4>
__device__ __forceinline__ double index_sum_lane(const int* __restrict__ ptr, const int* __restrict__ idx,
                                                 const double* __restrict__ val, int row, int lane) {
    const int a = ptr[row], b = ptr[row + 1];
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0;
    if (b <= a) return 0.0;
    for (int k = a + lane; k < b; k += U * G) {
        int c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = idx[min(k + u * G, b - 1)];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = val[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] += (k + u * G < b) ? v[u] : 0.0;
    }
    double s = acc[0];
#pragma unroll
    for (int u = 1; u < U; ++u) s += acc[u];
    return s;
}

// Cross-lane half swaps of CDNA4: permlane32_swap exchanges lanes 32..63 of
// x with lanes 0..31 of y; permlane16_swap exchanges the odd 16-lane rows of x
// with the even rows of y.  Doubles move as two 32-bit halves.
template <int M>
__device__ __forceinline__ void lane_swap(float& x, float& y) {
    static_assert(M == 32 || M == 16, "half swaps exist for masks 32 and 16");
    const auto r = (M == 32) ? __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false)
                             : __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    x = __uint_as_float(r[0]);
    y = __uint_as_float(r[1]);
}
template <int M>
__device__ __forceinline__ void lane_swap(double& x, double& y) {
    float xl = __int_as_float(__double2loint(x)), xh = __int_as_float(__double2hiint(x));
    float yl = __int_as_float(__double2loint(y)), yh = __int_as_float(__double2hiint(y));
    lane_swap<M>(xl, yl);
    lane_swap<M>(xh, yh);
    x = __hiloint2double(__float_as_int(xh), __float_as_int(xl));
    y = __hiloint2double(__float_as_int(yh), __float_as_int(yl));
}

// h1 * index_sum_lane (ptr/idx/val) plus row_dot_lane (ptr2/col2/val2
// against x2; ptr2 null: none) for the same row, by a group of G lanes with U
// loads per lane and term: the
// loads of both sums are issued level by level together (row bounds, then
// indices and values, then the gathers), so the two three-level chains
// overlap.  Each covers up to U*G entries in one pass; longer rows loop.
template <int G, int U = 4>
__device__ __forceinline__ double index_sum_plus_row_dot(const int* __restrict__ ptr, const int* __restrict__ idx,
                                                         const double* __restrict__ val,
                                                         const int* __restrict__ ptr2, const int* __restrict__ col2,
                                                         const double* __restrict__ val2,
                                                         const double* __restrict__ x2, double h1, int row,
                                                         int lane) {
    const int a = ptr[row], b = ptr[row + 1];
    const int a2 = ptr2 ? ptr2[row] : 0, b2 = ptr2 ? ptr2[row + 1] : 0;
    const bool has1 = b > a, has2 = b2 > a2;   // uniform over the group
    double s1 = 0.0, s2 = 0.0;
    int k = a + lane, k2 = a2 + lane;
    while (k < b || k2 < b2) {
        int c[U], c2[U];
        double w2[U], g1[U], g2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = 0;
            c2[u] = 0;
            w2[u] = 0.0;
        }
        if (has1) {
#pragma unroll
            for (int u = 0; u < U; ++u) c[u] = idx[min(k + u * G, b - 1)];
        }
        if (has2) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c2[u] = col2[min(k2 + u * G, b2 - 1)];
                w2[u] = val2[min(k2 + u * G, b2 - 1)];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            g1[u] = 0.0;
            g2[u] = 0.0;
        }
        if (has1) {
#pragma unroll
            for (int u = 0; u < U; ++u) g1[u] = val[c[u]];
        }
        if (has2) {
#pragma unroll
            for (int u = 0; u < U; ++u) g2[u] = x2[c2[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s1 += (k + u * G < b) ? g1[u] : 0.0;
            s2 += (k2 + u * G < b2) ? w2[u] * g2[u] : 0.0;
        }
        k += U * G;
        k2 += U * G;
    }
    return h1 * s1 + s2;
}

// Reduce-scatter over the 64 lanes of a wavefront: each lane holds N values
// v[0..N) (N a power of two, N <= 32); on return every lane holds, in the
// value returned, the sum over all 64 lanes of value index
// slot(lane) = lane >> (6 - log2 N).  Level by level, lane pairs (L, L^M)
// split the remaining values in halves and each keeps the sum of one half,
// so N values cost N-1 exchanges plus 6 - log2 N for the final group sum,
// instead of 6 per value.  For masks 32 and 16 one half swap of (v[i],
// v[i+N/2]) leaves each lane its own and its partner's copy of the half it
// keeps.  The order of additions is fixed.
template <int N, int M, typename T>
struct ReduceScatter {
    template <int NV>
    static __device__ __forceinline__ void run(T (&v)[NV], int lane) {
        if constexpr (M == 32 || M == 16) {
#pragma unroll
            for (int i = 0; i < N / 2; ++i) {
                T x = v[i], y = v[i + N / 2];
                lane_swap<M>(x, y);
                v[i] = x + y;
            }
        } else {
            const bool hi = (lane & M) != 0;
#pragma unroll
            for (int i = 0; i < N / 2; ++i) {
                const T send = hi ? v[i] : v[i + N / 2];
                const T keep = hi ? v[i + N / 2] : v[i];
                v[i] = keep + __shfl_xor(send, M, 64);
            }
        }
        ReduceScatter<N / 2, M / 2, T>::run(v, lane);
    }
};
template <int M, typename T>
struct ReduceScatter<1, M, T> {
    template <int NV>
    static __device__ __forceinline__ void run(T (&)[NV], int) {}
};

template <int N, typename T>
__device__ __forceinline__ T wave_reduce_scatter(T (&v)[N], int lane) {
    static_assert(N >= 1 && N <= 32 && (N & (N - 1)) == 0, "N must be a power of two <= 32");
    ReduceScatter<N, 32, T>::run(v, lane);
    T s = v[0];
#pragma unroll
    for (int M = 32 / N; M >= 1; M >>= 1) s += __shfl_xor(s, M, 64);
    return s;
}

}  // namespace qpg
