// Device-side pieces of the Metropolis loop with drift (Sec. II: sampling
// |Psi|^2 by single-electron moves, with grad_i ln Psi evaluated at R for
// the drift of the proposal and at R' for the reverse move, twice per step).
// Proposal r' = r + tau g(R) + sqrt(tau) chi, chi ~ N(0, 1) given by the
// caller; acceptance probability
//   min(1, |Psi(R')/Psi(R)|^2 G(r <- r') / G(r' <- r)),
//   G(b <- a) = exp(-|b - a - tau g(a)|^2 / (2 tau)),
// decided against a uniform number u given by the caller (accept if u < p).
#include "mde_internal.h"

namespace mde {

__global__ void k_vmc_drift(int W, int n_tot, int e, double tau, const double *__restrict__ pos,
                            const double *__restrict__ g0, const double *__restrict__ chi,
                            double *__restrict__ cur, double *__restrict__ newp, int phase) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    const double st = sqrt(tau);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double r = pos[((size_t)w * n_tot + e) * 3 + d];
        if (phase == 0) cur[(size_t)w * 3 + d] = r;
        else newp[(size_t)w * 3 + d] = r + tau * g0[(size_t)w * 3 + d] + st * chi[(size_t)w * 3 + d];
    }
}

__global__ void k_vmc_decide(int W, int n_tot, int e, double tau, double *__restrict__ pos,
                             const double *__restrict__ cur, const double *__restrict__ newp,
                             const double *__restrict__ g0, const double *__restrict__ g1,
                             const double *__restrict__ ratio, const double *__restrict__ u,
                             uint8_t *__restrict__ mask, int32_t *__restrict__ accepted) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    double fwd = 0.0, rev = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double a = cur[(size_t)w * 3 + d], b = newp[(size_t)w * 3 + d];
        const double f = b - a - tau * g0[(size_t)w * 3 + d];
        const double r = a - b - tau * g1[(size_t)w * 3 + d];
        fwd = fma(f, f, fwd);
        rev = fma(r, r, rev);
    }
    const double q = ratio[w];
    const double p = q * q * exp((fwd - rev) / (2.0 * tau));
    const bool acc = u[w] < p;     // false for a NaN probability
    mask[w] = acc ? 1 : 0;
    if (acc) {
#pragma unroll
        for (int d = 0; d < 3; ++d) pos[((size_t)w * n_tot + e) * 3 + d] = newp[(size_t)w * 3 + d];
        accepted[w] += 1;
    }
}

hipError_t launch_vmc_drift(hipStream_t st, int W, int n_tot, int e, double tau, const double *pos,
                            const double *g0, const double *chi, double *cur, double *newp, int phase) {
    hipLaunchKernelGGL(k_vmc_drift, dim3((W + 255) / 256), dim3(256), 0, st, W, n_tot, e, tau, pos, g0,
                       chi, cur, newp, phase);
    return hipGetLastError();
}

hipError_t launch_vmc_decide(hipStream_t st, int W, int n_tot, int e, double tau, double *pos,
                             const double *cur, const double *newp, const double *g0, const double *g1,
                             const double *ratio, const double *u, uint8_t *mask, int32_t *accepted) {
    hipLaunchKernelGGL(k_vmc_decide, dim3((W + 255) / 256), dim3(256), 0, st, W, n_tot, e, tau, pos, cur,
                       newp, g0, g1, ratio, u, mask, accepted);
    return hipGetLastError();
}

}  // namespace mde
