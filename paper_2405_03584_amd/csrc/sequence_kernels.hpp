// Kernels for sequences of related QPs.
//
// In SQP (Section 3.2) consecutive QP sub-problems share J, A and the bounds
// and differ in the objective: the quasi-Newton term U w U^T of
// eq. (bfgs_hessian) (Section 4) gains two columns per SQP iteration
// (Section 5.2) and p changes.  A handle keeps the constraint data resident; a
// new objective only replaces gamma, p, U, w and the cached diag(H), and a
// solve may start from the previous QP's minimiser.  The paper gives no warm-start rule:
// here the given x0 replaces the default start point and every other part of
// the start (slacks, multipliers, mu0) follows the default rule.
#pragma once

#include "ipm_kernels.hpp"

namespace qpg {

// Start point x0 given by the caller; slacks of the bounds max(x0 - lo, 1) /
// max(hi - x0, 1) and multipliers 1 as in the default start; partials of the
// slack sum over present sides.
__global__ __launch_bounds__(kBlock) void k_ipm_init_x_from(IpmVec v, const double* x0, double* part) {
    __shared__ double sh[kBlock / 64];
    double ssum = 0.0;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < v.n; j += gridDim.x * kBlock) {
        const double lo = v.xlo[j], hi = v.xhi[j];
        const bool hl = finite_d(lo), hu = finite_d(hi);
        const double xj = x0[j];
        v.x[j] = xj;
        v.s_lx[j] = hl ? fmax(xj - lo, 1.0) : 1.0;
        v.l_lx[j] = hl ? 1.0 : 0.0;
        v.s_ux[j] = hu ? fmax(hi - xj, 1.0) : 1.0;
        v.l_ux[j] = hu ? 1.0 : 0.0;
        ssum += (hl ? v.s_lx[j] : 0.0) + (hu ? v.s_ux[j] : 0.0);
    }
    ssum = block_sum(ssum, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = ssum;
}

}  // namespace qpg
