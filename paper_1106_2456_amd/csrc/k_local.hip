// All-electron derivatives at fixed positions: grad_i ln Psi and
// lap_i Psi / Psi for every electron i (Sec. IV: the laplacian of every
// particle, once per sweep, for the kinetic energy).
//
// For electron i of spin sigma, each excited determinant's derivative over
// the reference is the bordered determinant of Sec. IV-A read at R:
//   grad^a_i D_u / D_0 = rho^a_i det S_u + g^a_i[p]^T adj(S_u) c_i[h],
// with c_i = A^-1 e_i, rho^a_i = d^a_i,O . c_i and
// g^a_i = d^a_i,V - d^a_i,O^T T_V (d^a_i = grad^a of electron i's orbital
// row).  Weighted with the CI weights C_u and summed over the excitations,
// the adjugate terms regroup by table entry (h, p):
//   sum_u C_u g^a_i[p]^T adj(S_u) c_i[h] = sum_{h,p} A^-1[h][i] g^a_i[p] Y[h][p],
//   Y[h][p] = sum_u C_u cof(S_u)[j][l] over the (u, j, l) with h_j = h, p_l = p
// = dN/dT_V[h][p], the table gradient of the adjoint.  With Z = A^-T Y / N
// and T_V the table, all four derivatives of every electron are one contraction
// of its orbital row with the same matrix:
//   grad^a_i Psi / Psi = sum_q d^a_i[q] M[i][q],   M = [A^-T - Z T_V^T | Z]
// (occupied columns, then virtual).  Per walker and spin this is two dense
// products of n x n x m, run on v_mfma_f64_16x16x4f64, and four row
// contractions; the per-excitation work is the cofactor gather of Y.
#include <mutex>

#include "mde_internal.h"

namespace mde {

typedef double doublex4 __attribute__((ext_vector_type(4)));

__global__ void k_inv_nold(const InstDev *__restrict__ insts) {
    const InstDev &I = insts[0];
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < I.W) I.Lnew[w] = 1.0 / I.Nold[w];
}

// One block per walker, ceil(n / 16) waves; wave v owns rows i in
// [16v, 16v + 16) of M.  v_mfma_f64_16x16x4f64 lanes: A[l % 16][l / 16],
// B[l / 16][l % 16], and element j of the result D[l / 16 + 4 j][l % 16].
__global__ void __launch_bounds__(256)
k_local_derivs(const InstDev *__restrict__ insts, int spin, const double *__restrict__ orb,
               const double *__restrict__ Yn, double *__restrict__ grad, double *__restrict__ lap,
               int32_t *__restrict__ status, int e0, int n_tot) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[spin];
    const int n = S.n, m = S.m, no = S.no, WT = S.WT;
    const int w = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int mp = (m + 15) & ~15, np = (n + 15) & ~15;
    const int zs = mp + 1, ks = np + 1;
    extern __shared__ double lds[];
    double *Z = lds + (size_t)wave * 16 * (zs + ks);   // [16][mp + 1]
    double *K = Z + 16 * zs;                           // [16][np + 1]
    const int i0 = wave * 16;
    const int lr = lane & 15, lk = lane >> 4;
    const auto Bw = MDE_G(double, S.B) + (size_t)w * n * n;          // A^-1[h][i]
    const auto Yw = MDE_G(double, Yn) + (size_t)w * n * m;           // Y / N
    const auto Tt = MDE_G(double, S.T) + (size_t)(w / WT) * n * m * WT + (w % WT);
    // Z[i][p] = sum_h A^-1[h][i] Y[h][p] / N  (rows of this wave)
    for (int pt = 0; pt < mp; pt += 16) {
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
        const int i = i0 + lr, p = pt + lr;
        for (int h0 = 0; h0 < n; h0 += 4) {
            const int h = h0 + lk;
            const double a = (i < n && h < n) ? Bw[h * n + i] : 0.0;
            const double b = (h < n && p < m) ? Yw[h * m + p] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) Z[(lk + 4 * j) * zs + pt + lr] = acc[j];
    }
    __syncthreads();
    // K[i][r] = sum_p Z[i][p] T_V[r][p]
    for (int rt = 0; rt < np; rt += 16) {
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
        const int r = rt + lr;
        for (int p0 = 0; p0 < mp; p0 += 4) {
            const int p = p0 + lk;
            const double a = Z[lr * zs + p];
            const double b = (r < n && p < m) ? Tt[(size_t)(r * m + p) * WT] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) K[(lk + 4 * j) * ks + rt + lr] = acc[j];
    }
    __syncthreads();
    // lane (row i = i0 + l % 16, component a = l / 16): the row contraction
    const int i = i0 + lr, a = lk;
    if (i >= n) return;
    const auto d = MDE_G(double, orb) + (((size_t)w * n + i) * 5 + 1 + a) * no;
    double occ = 0.0, vir = 0.0;
    for (int r = 0; r < n; ++r) occ = fma(d[r], Bw[r * n + i] - K[lr * ks + r], occ);
    for (int p = 0; p < m; ++p) vir = fma(d[n + p], Z[lr * zs + p], vir);
    const double v = occ + vir;
    const size_t e = (size_t)w * n_tot + e0 + i;
    if (a < 3) grad[e * 3 + a] = v;
    else lap[e] = v;
    if (!isfinite(v) && status) atomicOr(&status[w], 4);
}

size_t local_derivs_lds(int n, int m) {
    const int mp = (m + 15) & ~15, np = (n + 15) & ~15;
    return sizeof(double) * (size_t)(np / 16) * 16 * (mp + 1 + np + 1);
}

hipError_t launch_local_derivs(hipStream_t st, const InstDev *d_inst, const InstDev &h, int spin,
                               const double *orb, const double *Yn, double *grad, double *lap,
                               int32_t *status) {
    const SpinDev &S = h.s[spin];
    const int waves = (S.n + 15) / 16;
    const size_t lds = local_derivs_lds(S.n, S.m);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_local_derivs,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int n_tot = h.s[0].n + h.s[1].n;
    hipLaunchKernelGGL(k_local_derivs, dim3(h.W), dim3(64 * waves), lds, st, d_inst, spin, orb,
                       Yn, grad, lap, status, spin == 0 ? 0 : h.s[0].n, n_tot);
    return hipGetLastError();
}

// Scratch of the allocation-free variant of the all-electron derivatives: the
// table gradient dN/dT / N of one spin ([W][n][m] doubles), held in a
// file-scope device array that every GPU the library runs on keeps until the
// process ends.  Host code never passes the array's name to a kernel: the
// per-device address comes from hipGetSymbolAddress, taken once per device
// with that device current.
static __device__ __align__(256) double scratch[LOCAL_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
double *scratch_addr[MAX_DEVICES] = {};
}  // namespace

hipError_t local_scratch(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_addr[dev] = static_cast<double *>(p);
    }
    *out = scratch_addr[dev];
    return hipSuccess;
}

hipError_t launch_inv_nold(hipStream_t st, const InstDev *d_inst, const InstDev &h) {
    hipLaunchKernelGGL(k_inv_nold, dim3((h.W + 255) / 256), dim3(256), 0, st, d_inst);
    return hipGetLastError();
}

}  // namespace mde
