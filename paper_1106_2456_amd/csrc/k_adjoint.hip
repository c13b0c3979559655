// Adjoint of the multi-determinant sum written in table form,
//   N = sum_I c_I det S_up,I det S_dn,I,  S[j][l] = T[h_j][p_l]  (Sec. III).
//   dlog|N|/dc_I            = det S_up,I det S_dn,I / N
//   dlog|N|/dT_sigma[h][p]  = sum over excitations u of sigma holding hole h
//                             at position j and particle p at position l of
//                             C_u cof(S_u)[j][l] / N,
// with C_u the CI weight of u (sum of c_I det S_other over the terms using
// u) and cof(S)[j][l] = d det S / d S[j][l].  The table-entry gradient is
// gathered through an inverted index (entry -> (u, j, l)), so every output
// element is one fixed-order sum: no atomics, bitwise-reproducible.
#include <algorithm>

#include "mde_internal.h"
#include "smalldet.h"

namespace mde {

__device__ __forceinline__ int exc_byte_a(const uint4 &x, int i) {
    uint32_t word = (i >> 2) == 0 ? x.x : (i >> 2) == 1 ? x.y : (i >> 2) == 2 ? x.z : x.w;
    return (int)((word >> ((i & 3) * 8)) & 0xffu);
}

__global__ void k_gw(const InstDev *__restrict__ insts, const double *__restrict__ go) {
    const InstDev &I = insts[0];
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < I.W) I.Lnew[w] = go[w] / I.Nold[w];
}

// grad_c[I] = sum_w gw[w] R_up[w][u(I)] R_dn[w][d(I)]; one wave per CI term
// k (terms are stored grouped by their up excitation: u(k) is found by
// bisection of the segment offsets), lanes over walkers, fixed butterfly
// reduction.  A wave per term keeps the work even: the terms of one
// excitation (the reference's above all) are spread over many waves.
__global__ void k_grad_coef(const InstDev *__restrict__ insts, double *__restrict__ grad_coef) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[0];
    const SpinDev &O = I.s[1];
    const int lane = threadIdx.x & 63;
    const int k = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int32_t *seg = S.ci_seg;
    if (k >= seg[S.U]) return;
    // largest u with seg[u] <= k: its segment [seg[u], seg[u + 1]) holds k
    int lo = 0, hi = S.U;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= k) lo = mid;
        else hi = mid;
    }
    const int u = lo;
    const int d = S.ci_other[k];
    const int WT = S.WT, W = I.W;
    double s = 0.0;
    for (int w0 = 0; w0 < W; w0 += 64) {
        const int w = w0 + lane;
        if (w < W) {
            const int t = w / WT, wl = w - t * WT;
            const double ru = S.R[((size_t)t * S.U + u) * WT + wl];
            const double rd = O.R[((size_t)t * O.U + d) * WT + wl];
            s = fma(I.Lnew[w] * ru, rd, s);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) grad_coef[S.ci_idx[k]] = s;
}

template <int K>
__device__ __forceinline__ double cof_entry(const double *tabs, const uint4 &ex, int m, int WTP,
                                            int wl, int j, int l) {
    double col[K][K], c[K], y[K];
#pragma unroll
    for (int jj = 0; jj < K; ++jj) {
        const int p = exc_byte_a(ex, 8 + jj);
#pragma unroll
        for (int r = 0; r < K; ++r) col[jj][r] = tabs[(exc_byte_a(ex, r) * m + p) * WTP + wl];
    }
#pragma unroll
    for (int r = 0; r < K; ++r) c[r] = (r == j) ? 1.0 : 0.0;
    (void)SmallDet<K, double>::run(col, c, y);
    // y[l] = det(S with column l -> e_j) = cof(S)[j][l]
    double out = 0.0;
#pragma unroll
    for (int jj = 0; jj < K; ++jj) out = (jj == l) ? y[jj] : out;
    return out;
}

__device__ double cof_entry_generic(const double *tabs, const uint4 &ex, int k, int m, int WTP,
                                    int wl, int j, int l) {
    double col[8][8], c[8], y[8];
    for (int jj = 0; jj < k; ++jj) {
        const int p = exc_byte_a(ex, 8 + jj);
        for (int r = 0; r < k; ++r) col[jj][r] = tabs[(exc_byte_a(ex, r) * m + p) * WTP + wl];
    }
    for (int r = 0; r < k; ++r) c[r] = (r == j) ? 1.0 : 0.0;
    (void)small_det_generic<double>(k, col, c, y);
    return y[l];
}

// table-gradient launch shape: GT_MAX_THREADS threads per block; with the
// lists split over a block's slots, GT_SPLIT_ENTRIES consecutive entries per
// block (the tile's table staged once for all of them)
constexpr int GT_MAX_THREADS = 512;
constexpr int GT_SPLIT_ENTRIES = 2;

// grad_T_sigma: block (walker tile, part) stages the tile's table in LDS once
// and takes the part's contiguous range of table entries.  In the split form
// (wide tiles: few tiles, short tables; a few entries per part) each entry's
// inverted list is split over the block's slots (lanes of a slot are the
// tile's walkers) and the slot sums are added in slot order; otherwise each
// entry's list is summed by one lane of one slot in list order.  Either way
// every output element is one fixed-order sum.
__global__ void __launch_bounds__(GT_MAX_THREADS)
k_grad_T(const InstDev *__restrict__ insts, int spin, const double *__restrict__ Tin,
         double *__restrict__ grad_T, int parts, int split) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[spin];
    const int n = S.n, m = S.m, WT = S.WT, WTP = S.WTP, W = I.W;
    const int t = blockIdx.x, part = blockIdx.y;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wl = tid % WT, slot = tid / WT, nslot = nthr / WT;
    extern __shared__ double tabs[];
    const int nm = n * m;
    if (Tin) {
        for (int idx = tid; idx < nm * WT; idx += nthr) {
            const int ee = idx % nm, l = idx / nm, w = t * WT + l;
            tabs[ee * WTP + l] = (w < W) ? Tin[(size_t)w * nm + ee] : 0.0;
        }
    } else {
        // the context's own table, walker-tiled [tile][entry][WT]
        const auto Tt = MDE_G(double, S.T) + (size_t)t * nm * WT;
        for (int idx = tid; idx < nm * WT; idx += nthr) {
            const int ee = idx / WT, l = idx % WT, w = t * WT + l;
            tabs[ee * WTP + l] = (w < W) ? Tt[idx] : 0.0;
        }
    }
    __syncthreads();
    const int w = t * WT + wl;
    // (walkers past W compute on zero tables and store nothing: every
    // thread reaches the block barrier of the split form)
    const bool live = w < W;
    const double gw = live ? I.Lnew[w] : 0.0;
    const auto Cb = MDE_G(double, S.C) + (size_t)t * S.U * WT + wl;
    const auto inv_off = MDE_G(int32_t, S.inv_off);
    const auto inv_ent = MDE_G(int32_t, S.inv_ent);
    const uint4 *__restrict__ exs = S.ex;
    const int per = (nm + parts - 1) / parts;
    const int e_begin = part * per, e_end = min(nm, e_begin + per);
    for (int e = e_begin + (split ? 0 : slot); e < e_end; e += (split ? 1 : nslot)) {
        int a = inv_off[e], b = inv_off[e + 1];
        if (split) {
            const int pl = (b - a + nslot - 1) / nslot;
            a = min(b, a + slot * pl);
            b = min(b, a + pl);
        }
        double acc = 0.0;
        // software pipeline over the list: the entry codes run four entries
        // ahead, the records and CI weights they index two entries ahead, so
        // no load waits on another load issued in the same iteration
        auto code_at = [&](int i) { return i < b ? inv_ent[i] : 0; };
        int cq0 = code_at(a), cq1 = code_at(a + 1), cq2 = code_at(a + 2), cq3 = code_at(a + 3),
            cq4 = code_at(a + 4);
        uint4 ex0 = make_uint4(0, 0, 0, 0), ex1 = ex0;
        double cw0 = 0.0, cw1 = 0.0;
        if (a < b) {
            ex0 = exs[cq0 >> 10];
            cw0 = Cb[(size_t)(cq0 >> 10) * WT];
        }
        if (a + 1 < b) {
            ex1 = exs[cq1 >> 10];
            cw1 = Cb[(size_t)(cq1 >> 10) * WT];
        }
        for (int q = a; q < b; ++q) {
            uint4 ex2 = make_uint4(0, 0, 0, 0);
            double cw2 = 0.0;
            if (q + 2 < b) {
                ex2 = exs[cq2 >> 10];
                cw2 = Cb[(size_t)(cq2 >> 10) * WT];
            }
            const int cq5 = code_at(q + 5);
            const int code = cq0;
            const int k = (code >> 6) & 15, j = (code >> 3) & 7, l = code & 7;
            double cf;
            switch (k) {
                case 1: cf = 1.0; break;
                case 2: cf = cof_entry<2>(tabs, ex0, m, WTP, wl, j, l); break;
                case 3: cf = cof_entry<3>(tabs, ex0, m, WTP, wl, j, l); break;
                case 4: cf = cof_entry<4>(tabs, ex0, m, WTP, wl, j, l); break;
                default: cf = cof_entry_generic(tabs, ex0, k, m, WTP, wl, j, l); break;
            }
            acc = fma(cw0, cf, acc);
            cq0 = cq1; cq1 = cq2; cq2 = cq3; cq3 = cq4; cq4 = cq5;
            ex0 = ex1; ex1 = ex2;
            cw0 = cw1; cw1 = cw2;
        }
        if (!split) {
            if (live) grad_T[(size_t)w * nm + e] = gw * acc;
            continue;
        }
        __shared__ double red[GT_MAX_THREADS];
        red[slot * WT + wl] = acc;
        __syncthreads();
        if (slot == 0 && live) {
            double sum = 0.0;
            for (int v = 0; v < nslot; ++v) sum += red[v * WT + wl];
            grad_T[(size_t)w * nm + e] = gw * sum;
        }
        __syncthreads();   // red is rewritten for the block's next entry
    }
}

hipError_t launch_backward(hipStream_t st, const InstDev *d_inst, const InstDev &h,
                           const double *go, const double *Nw, const double *coef,
                           double *grad_coef, double *grad_T_up, double *grad_T_dn,
                           const double *T_up, const double *T_dn) {
    (void)Nw; (void)coef;
    hipLaunchKernelGGL(k_gw, dim3((h.W + 255) / 256), dim3(256), 0, st, d_inst, go);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (grad_coef) {
        const int wpb = 4;
        const int64_t terms = h.n_det;
        hipLaunchKernelGGL(k_grad_coef, dim3((unsigned)((terms + wpb - 1) / wpb)), dim3(64 * wpb), 0,
                           st, d_inst, grad_coef);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const double *Tin[2] = {T_up, T_dn};
    double *gT[2] = {grad_T_up, grad_T_dn};
    for (int s = 0; s < 2; ++s) {
        if (!gT[s]) continue;
        e = launch_grad_T(st, d_inst, h, s, Tin[s], gT[s]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// status[w] |= NONFINITE when a walker's table gradient holds a non-finite value
__global__ void k_flag_nonfinite(int W, const double *__restrict__ a, int na,
                                 const double *__restrict__ b, int nb, int32_t *__restrict__ status) {
    const int w = blockIdx.x;
    bool bad = false;
    if (a)
        for (int i = threadIdx.x; i < na; i += blockDim.x) bad |= !isfinite(a[(size_t)w * na + i]);
    if (b)
        for (int i = threadIdx.x; i < nb; i += blockDim.x) bad |= !isfinite(b[(size_t)w * nb + i]);
    if (__syncthreads_or(bad) && threadIdx.x == 0) status[w] |= 4;
}

hipError_t launch_flag_nonfinite(hipStream_t st, int W, const double *a, int na, const double *b,
                                 int nb, int32_t *status) {
    hipLaunchKernelGGL(k_flag_nonfinite, dim3(W), dim3(64), 0, st, W, a, na, b, nb, status);
    return hipGetLastError();
}

hipError_t launch_grad_T(hipStream_t st, const InstDev *d_inst, const InstDev &h, int spin,
                         const double *Tin, double *grad_T) {
    const SpinDev &S = h.s[spin];
    const size_t lds = sizeof(double) * (size_t)S.n * S.m * S.WTP;
    if (S.n * S.m > 65535 || lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_grad_T,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    // parts per tile: GT_SPLIT_ENTRIES entries per block (their lists split
    // over the block's slots) while one entry per block would stay within
    // 2^16 blocks, else enough ranges of entries to cover the chip about four
    // times over
    const int nm = S.n * S.m;
    const bool split = (size_t)S.n_tiles * nm <= 65536;
    const int parts = split ? (nm + GT_SPLIT_ENTRIES - 1) / GT_SPLIT_ENTRIES
                            : std::max(1, std::min(std::max(nm / 16, 1), (1024 + S.n_tiles - 1) / S.n_tiles));
    const int threads = GT_MAX_THREADS;
    hipLaunchKernelGGL(k_grad_T, dim3(S.n_tiles, parts), dim3(threads), lds, st, d_inst, spin, Tin,
                       grad_T, parts, split ? 1 : 0);
    return hipGetLastError();
}

}  // namespace mde
