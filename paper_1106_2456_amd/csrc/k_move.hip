// Per-walker kernels: reference LU and inverse (Sec. III: computed from
// scratch once), the table GEMM T_V = A^-1 Phi_V (Sec. III table; Algorithm 1
// step 3; Sec. V: one matrix multiplication), the single-move proposal
// (Algorithm 1 step 1 with the Sec. III Sherman-Morrison update written for a
// row change, and the Sec. IV-A derivative factors), and the commit.
#include "mde_internal.h"

namespace mde {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// LU with partial pivoting and explicit inverse, one wave per matrix
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(64)
k_lu_inverse(const InstDev *__restrict__ insts, int spin, const double *__restrict__ orb_in,
             int32_t *status) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[spin];
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    const int n = S.n, no = S.no, ld = n + 1;
    extern __shared__ double sh[];
    double *A = sh;
    double *X = sh + n * ld;
    __shared__ int pv[MAXN];
    if (orb_in) {
        for (int idx = lane; idx < n * no; idx += 64) {
            const int i = idx / no, p = idx - i * no;
            const double v = orb_in[((size_t)(w * n + i) * 5) * no + p];
            S.Phi[(size_t)w * n * no + idx] = v;
            if (I.prec >= 2 && p >= n)
                S.PhiV32[((size_t)w * n + i) * S.m + (p - n)] = (float)v;
        }
    } else if (I.prec >= 2) {
        for (int idx = lane; idx < n * S.m; idx += 64) {
            const int i = idx / S.m, p = idx - i * S.m;
            S.PhiV32[(size_t)w * n * S.m + idx] = (float)S.Phi[((size_t)w * n + i) * no + n + p];
        }
    }
    for (int idx = lane; idx < n * n; idx += 64) {
        const int i = idx / n, j = idx - i * n;
        A[i * ld + j] = orb_in ? orb_in[((size_t)(w * n + i) * 5) * no + j]
                               : S.Phi[((size_t)w * n + i) * no + j];
    }
    __syncthreads();
    double sg = 1.0, la = 0.0;
    int sing = 0;
    for (int k = 0; k < n; ++k) {
        double v = (lane >= k && lane < n) ? fabs(A[lane * ld + k]) : -1.0;
        int idx = lane;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double ov = __shfl_xor(v, off, 64);
            const int oi = __shfl_xor(idx, off, 64);
            if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
        }
        const int p = __builtin_amdgcn_readfirstlane(idx);
        if (!(v > 0.0)) { sing = 1; break; }
        if (p != k) {
            if (lane < n) {
                const double t = A[k * ld + lane];
                A[k * ld + lane] = A[p * ld + lane];
                A[p * ld + lane] = t;
            }
            sg = -sg;
        }
        if (lane == 0) pv[k] = p;
        __syncthreads();
        const double piv = A[k * ld + k];
        if (piv < 0.0) sg = -sg;
        la += log(fabs(piv));
        if (lane > k && lane < n) {
            const double f = A[lane * ld + k] / piv;
            A[lane * ld + k] = f;
            for (int j = k + 1; j < n; ++j) A[lane * ld + j] = fma(-f, A[k * ld + j], A[lane * ld + j]);
        }
        __syncthreads();
    }
    double *Bw = S.B + (size_t)w * n * n;
    if (sing) {
        for (int idx = lane; idx < n * n; idx += 64) Bw[idx] = 0.0;
        if (lane == 0) {
            S.logdet[w] = -INFINITY;
            S.sgn[w] = 0.0;
            I.st[w] |= 1;
            if (status) status[w] |= 1;
        }
        return;
    }
    if (lane < n) {
        const int c = lane;
        for (int i = 0; i < n; ++i) X[i * ld + c] = (i == c) ? 1.0 : 0.0;
        for (int k = 0; k < n; ++k) {
            const int p = pv[k];
            if (p != k) {
                const double t = X[k * ld + c];
                X[k * ld + c] = X[p * ld + c];
                X[p * ld + c] = t;
            }
        }
        for (int i = 0; i < n; ++i) {
            double s = X[i * ld + c];
            for (int kk = 0; kk < i; ++kk) s = fma(-A[i * ld + kk], X[kk * ld + c], s);
            X[i * ld + c] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = X[i * ld + c];
            for (int kk = i + 1; kk < n; ++kk) s = fma(-A[i * ld + kk], X[kk * ld + c], s);
            X[i * ld + c] = s / A[i * ld + i];
        }
    }
    __syncthreads();
    for (int idx = lane; idx < n * n; idx += 64) {
        const int i = idx / n, j = idx - i * n;
        Bw[idx] = X[i * ld + j];
    }
    if (lane == 0) {
        S.logdet[w] = la;
        S.sgn[w] = sg;
    }
}

hipError_t launch_lu_inverse(hipStream_t st, const InstDev *d_inst, const InstDev &h, int spin,
                             const double *orb_in, int32_t *status) {
    const int n = h.s[spin].n;
    const size_t lds = sizeof(double) * 2 * n * (n + 1);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_lu_inverse,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_lu_inverse, dim3(h.W), dim3(64), lds, st, d_inst, spin, orb_in, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Refresh of a spin with at most 8 electrons, eight lanes per walker: lane g
// holds row g of the walker's matrix.  LU with partial pivoting (the largest
// |A[i][k]|, the first on ties) with the pivot found and the rows swapped
// across the lane group; lane c then solves for column c of the inverse
// (forward and back substitution with the pivots' reciprocals); the columns
// are transposed through LDS and lane r writes row r of the inverse and of
// the table T_V = A^-1 Phi_V.  log|det| = log of the pivots' mantissa
// product + their exponent sum x ln 2.
// ---------------------------------------------------------------------------

template <int N>
__global__ void __launch_bounds__(64)
k_refresh_small(const InstDev *__restrict__ insts, int spin, const double *__restrict__ orb_in,
                int32_t *status) {
    constexpr int G = 8;                     // lanes per walker
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[spin];
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int w = tid / G, g = tid % G, wl = threadIdx.x / G;
    // fields read once: the stores below could alias them otherwise
    const int no = S.no, m = S.m, prec = I.prec, WT = S.WT, W = I.W;
    double *const Tg = S.T;
    float *const T32 = S.T32;
    float *const PV32 = S.PhiV32;
    __shared__ double tr[64 / G][N][N];
    const bool live = w < W;                 // uniform over a lane group
    const bool row = live && g < N;
    double *const Phw = S.Phi + (size_t)(live ? w : 0) * N * no;
    double *const Bw = S.B + (size_t)(live ? w : 0) * N * N;
    const auto orow = [&](int i) { return orb_in + ((size_t)((live ? w : 0) * N + i) * 5) * no; };
    if (row && orb_in) {
        // the kept copy of the walker's orbital rows
        for (int p0 = 0; p0 < no; p0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p0 + u < no ? orow(g)[p0 + u] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = p0 + u;
                if (p >= no) break;
                Phw[g * no + p] = v[u];
                if (prec >= 2 && p >= N) PV32[((size_t)w * N + g) * m + (p - N)] = (float)v[u];
            }
        }
    } else if (row && prec >= 2) {
        for (int p = 0; p < m; ++p) PV32[((size_t)w * N + g) * m + p] = (float)Phw[g * no + N + p];
    }
    double a[N];
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] = row ? (orb_in ? orow(g)[j] : Phw[g * no + j]) : 0.0;
    // the table's columns are read PB at a time, the next chunk issued before
    // the current one is stored (the first before the factorisation)
    constexpr int PB = 8;
    auto phi_v = [&](int i, int p) { return orb_in ? orow(i)[N + p] : Phw[i * no + N + p]; };
    double ph[PB][N];
#pragma unroll
    for (int u = 0; u < PB; ++u)
#pragma unroll
        for (int k = 0; k < N; ++k) ph[u][k] = (row && u < m) ? phi_v(k, u) : 0.0;
    double sg = 1.0, mant = 1.0, rp[N];
    int ex = 0, pv[N];
    bool sing = false;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        pv[k] = k;
        rp[k] = 0.0;
        // pivot: the largest |A[i][k]| over rows i >= k, the first on ties
        double v = (row && g >= k) ? fabs(a[k]) : -1.0;
        int idx = g;
#pragma unroll
        for (int off = G / 2; off >= 1; off >>= 1) {
            const double ov = __shfl_xor(v, off, G);
            const int oi = __shfl_xor(idx, off, G);
            if (ov > v || (ov == v && oi < idx)) {
                v = ov;
                idx = oi;
            }
        }
        if (sing) continue;
        if (!(v > 0.0)) {
            sing = true;
            continue;
        }
        const int p = idx;
        pv[k] = p;
        if (p != k) {
            const int src = g == k ? p : (g == p ? k : g);
#pragma unroll
            for (int j = 0; j < N; ++j) a[j] = __shfl(a[j], src, G);
            sg = -sg;
        }
        const double piv = __shfl(a[k], k, G);
        if (piv < 0.0) sg = -sg;
        int e;
        mant *= frexp(fabs(piv), &e);
        ex += e;
        rp[k] = 1.0 / piv;
        double rk[N];
#pragma unroll
        for (int j = k + 1; j < N; ++j) rk[j] = __shfl(a[j], k, G);
        if (row && g > k) {
            const double f = a[k] * rp[k];
            a[k] = f;
#pragma unroll
            for (int j = k + 1; j < N; ++j) a[j] = fma(-f, rk[j], a[j]);
        }
    }
    // column g of the inverse
    double x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = i == g ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int i = k + 1; i < N; ++i)
            if (pv[k] == i) {
                const double t = x[k];
                x[k] = x[i];
                x[i] = t;
            }
#pragma unroll
    for (int i = 1; i < N; ++i) {
        double s = x[i];
#pragma unroll
        for (int kk = 0; kk < i; ++kk) s = fma(-__shfl(a[kk], i, G), x[kk], s);
        x[i] = s;
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        double s = x[i];
#pragma unroll
        for (int kk = i + 1; kk < N; ++kk) s = fma(-__shfl(a[kk], i, G), x[kk], s);
        x[i] = s * rp[i];
    }
    if (row) {
#pragma unroll
        for (int i = 0; i < N; ++i) tr[wl][i][g] = sing ? 0.0 : x[i];
    }
    __syncthreads();
    if (!row) return;
    double br[N];                            // row g of the inverse
#pragma unroll
    for (int k = 0; k < N; ++k) br[k] = tr[wl][g][k];
#pragma unroll
    for (int k = 0; k < N; ++k) Bw[g * N + k] = br[k];
    if (g == 0) {
        if (sing) {
            S.logdet[w] = -INFINITY;
            S.sgn[w] = 0.0;
            I.st[w] |= 1;
            if (status) status[w] |= 1;
        } else {
            S.logdet[w] = log(mant) + ex * 0.69314718055994530942;
            S.sgn[w] = sg;
        }
    }
    // row g of T_V = A^-1 Phi_V, walker-tiled
    const size_t tb = (size_t)(w / WT) * N * m * WT + (w % WT) + (size_t)g * m * WT;
    for (int p0 = 0; p0 < m; p0 += PB) {
        double pn[PB][N];
        if (p0 + PB < m) {
#pragma unroll
            for (int u = 0; u < PB; ++u)
#pragma unroll
                for (int k = 0; k < N; ++k) pn[u][k] = p0 + PB + u < m ? phi_v(k, p0 + PB + u) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            if (p0 + u >= m) break;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) s = fma(br[k], ph[u][k], s);
            const size_t o = tb + (size_t)(p0 + u) * WT;
            if (prec == 0) Tg[o] = s;
            else T32[o] = (float)s;
        }
#pragma unroll
        for (int u = 0; u < PB; ++u)
#pragma unroll
            for (int k = 0; k < N; ++k) ph[u][k] = pn[u][k];
    }
}

hipError_t launch_refresh_small(hipStream_t st, const InstDev *d_inst, const InstDev &h, int spin,
                                const double *orb_in, int32_t *status) {
    const dim3 grid((unsigned)(((size_t)h.W * 8 + 63) / 64));
#define MDE_RS(X)                                                                          \
    case X:                                                                                \
        hipLaunchKernelGGL(k_refresh_small<X>, grid, dim3(64), 0, st, d_inst, spin, orb_in, \
                           status);                                                        \
        break;
    switch (h.s[spin].n) {
        MDE_RS(1) MDE_RS(2) MDE_RS(3) MDE_RS(4) MDE_RS(5) MDE_RS(6) MDE_RS(7) MDE_RS(8)
        default: return hipErrorInvalidValue;
    }
#undef MDE_RS
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// table GEMM in FP64 on the matrix cores: T_V[w] = A^-1[w] Phi_V[w] (Sec. III
// table; Sec. V: one matrix product instead of dot products), one block of
// four waves per walker, A^-1 staged in LDS, 16 x 16 output tiles of
// v_mfma_f64_16x16x4f64 (lanes: A[l % 16][l / 16], B[l / 16][l % 16], result
// element j at [l / 16 + 4 j][l % 16]).  In the FP32-table forms the table is
// the rounded FP64 product at a refresh.
// ---------------------------------------------------------------------------

typedef double doublex4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
k_table_gemm(const InstDev *__restrict__ insts, int spin) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[spin];
    const int w = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int n = S.n, m = S.m, no = S.no, WT = S.WT;
    extern __shared__ double sh[];
    double *Bs = sh;              // n x n
    for (int idx = tid; idx < n * n; idx += 256) Bs[idx] = S.B[(size_t)w * n * n + idx];
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    const int RT = (n + 15) >> 4, PT = (m + 15) >> 4;
    const auto Pv = MDE_G(double, S.Phi) + (size_t)w * n * no + n;     // Phi_V[k][p] at k * no + p
    const size_t tb = (size_t)(w / WT) * n * m * WT + (w % WT);
    for (int t = wave; t < RT * PT; t += 4) {
        const int rt = (t / PT) * 16, pt = (t % PT) * 16;
        const int r = rt + lr, p = pt + lr;
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < n; k0 += 4) {
            const int k = k0 + lk;
            const double a = (r < n && k < n) ? Bs[r * n + k] : 0.0;
            const double b = (k < n && p < m) ? Pv[(size_t)k * no + p] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int rr = rt + lk + 4 * j;
            if (rr >= n || p >= m) continue;
            const size_t o = tb + (size_t)(rr * m + p) * WT;
            if (I.prec == 0) S.T[o] = acc[j];
            else S.T32[o] = (float)acc[j];
        }
    }
}

hipError_t launch_table_gemm(hipStream_t st, const InstDev *d_inst, const InstDev &h, int spin) {
    const int n = h.s[spin].n;
    const size_t lds = sizeof(double) * (size_t)n * n;
    hipLaunchKernelGGL(k_table_gemm, dim3(h.W), dim3(256), lds, st, d_inst, spin);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// proposal.  Common part: c = A^-1 e_i, rho = a'.c (= det A'/det A),
// kappa^a = d^a_O . c,  q = a'^T T_V - phi'_V,  w^a = d^a_V - d^a_O^T T_V.
//
// FP64 form, in the frame of the current table T: for an excitation with
// holes h and particles p let S = T[h][p] and y = adj(S) c[h].  The updated
// table of Sec. III is T' = T - c q^T / rho; the matrix determinant lemma
// and the bordered form of the row-replaced reference (Sec. IV-A) give
//   rho R'_u   = rho det S - q[p] . y
//   rho G^a_u  = kappa^a det S + w^a[p] . y
// (R'_u = det S'_u, G^a_u = grad^a of the excited determinant over D_0(R')).
// Every quantity is a polynomial in table entries: nothing is divided by rho
// before the final per-walker quotients, so a move that lands near the
// reference determinant's node keeps full accuracy.  T' is formed only on
// acceptance.
//
// Mixed forms, in the frame of the updated table (Algorithm 1 as written):
// T'_V = T_V - c' q^T with c' = c/rho is formed in FP64 from the FP32 table
// and stored in FP32, with g^a = d^a_V - d^a_O^T T'_V = w^a + (kappa^a/rho) q;
// then R'_u = det S'_u and G^a_u = (kappa^a/rho) R'_u + g^a[p] . adj(S') c'[h].
// (With FP32 table entries the current-table frame would lose accuracy on
// moves whose ratio is much smaller than rho: rho det S and q . y then
// cancel.)
//
// One block per (walker tile, part): the tile's new orbital rows (occupied
// part and the part's slice of virtuals) are copied into LDS with coalesced
// loads; lanes are walkers.  Part 0 also writes the per-walker scalars and
// the commit's row a'^T A^-1 - e_i^T.
// ---------------------------------------------------------------------------

__host__ __device__ inline int odd_stride(int x) { return x | 1; }

template <int WT, typename TT>
__global__ void __launch_bounds__(256)
k_propose(const InstDev *__restrict__ insts, const MoveArgs *__restrict__ moves, MoveArgs m1,
          int split, int T8, int n_inst) {
    constexpr bool F64 = sizeof(TT) == 8;
    int inst, t, part;
    if (!tile_of_block(split, T8, n_inst, inst, t, part)) return;
    const InstDev &I = insts[inst];
    const MoveArgs mv = moves ? moves[inst] : m1;
    const SpinDev &S = I.s[mv.spin];
    if (t >= S.n_tiles) return;
    const int n = S.n, m = S.m, no = S.no, row = mv.row, W = I.W, nn = n * n;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int w0 = t * WT, nw = min(WT, W - w0);
    const int mc = (m + split - 1) / split, p0 = min(m, part * mc), p1 = min(m, p0 + mc);
    const int ns = n + (p1 - p0);              // staged orbitals per component
    const int ost = odd_stride(5 * ns);
    extern __shared__ double shp[];
    double *o_s = shp;                         // [WT][ost]: 5 x (occupied, slice)
    double *c_s = o_s + WT * ost;              // [n][WT]: c = A^-1 e_i
    double *r_s = c_s + n * WT;                // [5][WT]: 1/rho, kappa^a / rho (mixed)
    const auto orb = MDE_G(double, mv.new_orb) + (size_t)w0 * 5 * no;
    {
        // four loads per thread in flight before the LDS writes
        const int tot = nw * 5 * ns;
        int idx = tid;
        for (; idx < tot; idx += 4 * nthr) {
            double v[4];
            int o[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int id = min(idx + u * nthr, tot - 1);
                const int l = id / (5 * ns), r = id - l * 5 * ns, a = r / ns, j = r - a * ns;
                const int p = j < n ? j : p0 + j;  // orbital index (virtual p0.. at n + p0)
                o[u] = l * ost + r;
                v[u] = orb[(size_t)l * 5 * no + a * no + p];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (idx + u * nthr < tot) o_s[o[u]] = v[u];
        }
    }
    const auto Bg = MDE_G(double, S.B) + (size_t)w0 * nn;
    for (int idx = tid; idx < n * WT; idx += nthr) {
        const int r = idx / WT, l = idx % WT;
        c_s[idx] = (l < nw) ? Bg[(size_t)l * nn + r * n + row] : 0.0;
    }
    __syncthreads();
    if (part == 0 || !F64) {
        for (int l = tid; l < WT; l += nthr) {
            const int w = w0 + l;
            double rho = 1.0, k[4] = {0.0, 0.0, 0.0, 0.0};
            if (l < nw) {
                const double *ol = o_s + l * ost;
                rho = 0.0;
                for (int r = 0; r < n; ++r) {
                    const double c = c_s[r * WT + l];
                    rho = fma(ol[r], c, rho);
#pragma unroll
                    for (int a = 0; a < 4; ++a) k[a] = fma(ol[(1 + a) * ns + r], c, k[a]);
                }
            }
            if (!F64) {
                const double ir = 1.0 / rho;
                r_s[l] = ir;
#pragma unroll
                for (int a = 0; a < 4; ++a) r_s[(1 + a) * WT + l] = k[a] * ir;
            }
            if (part == 0 && l < nw) {
                I.rho[w] = rho;
#pragma unroll
                for (int a = 0; a < 4; ++a) I.kap[(size_t)w * 4 + a] = k[a];
                const int bits = (!isfinite(rho) || fabs(rho) < 1e-300) ? 2 : 0;
                I.st[w] = (I.st[w] & ~2) | bits;
            }
        }
    }
    if (!F64) __syncthreads();
    if (part == 0) {
        const auto cct = MDE_GW(double, I.cc) + (size_t)t * n * WT;
        const auto rrt = MDE_GW(double, I.rrow) + (size_t)t * n * WT;
        for (int idx = tid; idx < n * WT; idx += nthr) {
            const int j = idx / WT, l = idx % WT;
            double r = 0.0;
            if (l < nw) {
                const double *ol = o_s + l * ost;
#pragma unroll 4
                for (int k = 0; k < n; ++k) r = fma(ol[k], Bg[(size_t)l * nn + k * n + j], r);
                r -= (j == row) ? 1.0 : 0.0;
            }
            cct[idx] = c_s[idx];
            if (!F64) I.cc32[(size_t)t * n * WT + idx] = (float)(c_s[idx] * r_s[l]);
            rrt[idx] = r;
        }
        for (int idx = tid; idx < nw * no; idx += nthr) {
            const int l = idx / no, p = idx - l * no;
            I.newrow[(size_t)(w0 + l) * I.nomax + p] = orb[(size_t)l * 5 * no + p];
        }
    }
    // the part's slice of virtuals
    const auto Tt = MDE_G(TT, F64 ? (const void *)S.T : (const void *)S.T32) + (size_t)t * n * m * WT;
    constexpr int NE = F64 ? 5 : 4;
    const auto evt = MDE_GW(TT, F64 ? (void *)I.ev : (void *)I.ev32) + (size_t)t * NE * m * WT;
    for (int idx = p0 * WT + tid; idx < p1 * WT; idx += nthr) {
        const int p = idx / WT, l = idx % WT, jp = n + p - p0;
        double q = 0.0, wa[4] = {0.0, 0.0, 0.0, 0.0};
        if (l < nw) {
            const double *ol = o_s + l * ost;
            double v = 0.0, da[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int r = 0; r < n; ++r) {
                const double tv = (double)Tt[(size_t)(r * m + p) * WT + l];
                v = fma(ol[r], tv, v);
#pragma unroll
                for (int a = 0; a < 4; ++a) da[a] = fma(ol[(1 + a) * ns + r], tv, da[a]);
            }
            q = v - ol[jp];
#pragma unroll
            for (int a = 0; a < 4; ++a) wa[a] = ol[(1 + a) * ns + jp] - da[a];
        }
        if (F64) {
            evt[(size_t)(p * 5) * WT + l] = (TT)q;
#pragma unroll
            for (int a = 0; a < 4; ++a) evt[(size_t)(p * 5 + 1 + a) * WT + l] = (TT)wa[a];
        } else {
            const double ir = r_s[l], qi = q * ir;
#pragma unroll
            for (int a = 0; a < 4; ++a)
                evt[(size_t)(p * 4 + a) * WT + l] = (TT)fma(r_s[(1 + a) * WT + l], q, wa[a]);
            const auto Tpt = MDE_GW(float, I.Tp32) + (size_t)t * n * m * WT;
            for (int r = 0; r < n; ++r) {
                const size_t o = (size_t)(r * m + p) * WT + l;
                Tpt[o] = (float)fma(-c_s[r * WT + l], qi, (double)Tt[o]);
            }
        }
    }
}

static size_t propose_lds(int nmax, int mmax, int WT, int split) {
    const int mc = (mmax + split - 1) / split;
    return sizeof(double) * (size_t)WT * (odd_stride(5 * (nmax + mc)) + nmax + 5);
}

// proposal, MIXED_GEMM (Algorithm 1 as written: update the inverse, then
// rebuild the table with one GEMM).  FP64 part, one wave per walker:
//   c = A^-1 e_i, rho = a'.c, c' = c/rho, r = a'^T A^-1,
//   A'^-1 = A^-1 - c' (r - e_i^T)                  -> FP32 operand rows 0..n-1
//   e^a = d^a_O^T A'^-1 = d^a_O^T A^-1 - rho^a (r - e_i^T)  -> rows n..n+3
// The GEMM kernel below then forms T'_V = A'^-1 Phi'_V and g^a = d^a_V - e^a Phi'_V.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_propose_mixed(const InstDev *__restrict__ insts, const MoveArgs *__restrict__ moves, MoveArgs m1) {
    const int inst = blockIdx.y;
    const InstDev &I = insts[inst];
    const MoveArgs mv = moves ? moves[inst] : m1;
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= I.W) return;
    const SpinDev &S = I.s[mv.spin];
    const int n = S.n, no = S.no, row = mv.row, nmax = I.nmax;
    const double *__restrict__ nr = mv.new_orb + (size_t)w * 5 * no;
    const double *__restrict__ Bw = S.B + (size_t)w * n * n;
    double c = 0.0, ap = 0.0, d[4] = {0, 0, 0, 0};
    if (lane < n) {
        c = Bw[(size_t)lane * n + row];
        ap = nr[lane];
#pragma unroll
        for (int a = 0; a < 4; ++a) d[a] = nr[(1 + a) * no + lane];
    }
    const double rho = wave_sum(ap * c);
    double dc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) dc[a] = wave_sum(d[a] * c);
    const double irho = 1.0 / rho;
    double rhoA[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) rhoA[a] = dc[a] * irho;
    if (lane < n) {
        const int WT = S.WT;
        const size_t o = ((size_t)(w / WT) * n + lane) * WT + (w % WT);
        I.cc[o] = c;
        I.cc32[o] = (float)(c * irho);
    }
    if (lane == 0) {
        I.rho[w] = rho;
#pragma unroll
        for (int a = 0; a < 4; ++a) I.kap[(size_t)w * 4 + a] = dc[a];
        int bits = 0;
        if (!isfinite(rho) || fabs(rho) < 1e-300) bits |= 2;
        I.st[w] = (I.st[w] & ~2) | bits;
    }
    float *__restrict__ Ap = I.Ap32 + (size_t)w * (nmax + 4) * nmax;
    if (lane < n) {
        const int j = lane;
        double r = 0.0, f[4] = {0, 0, 0, 0};
        for (int k = 0; k < n; ++k) {
            const double b = Bw[(size_t)k * n + j];
            r = fma(nr[k], b, r);
#pragma unroll
            for (int a = 0; a < 4; ++a) f[a] = fma(nr[(1 + a) * no + k], b, f[a]);
        }
        const double rd = r - (j == row ? 1.0 : 0.0);
        I.rrow[((size_t)(w / S.WT) * n + j) * S.WT + (w % S.WT)] = rd;
        for (int rr = 0; rr < n; ++rr) {
            const double cpr = Bw[(size_t)rr * n + row] * irho;
            Ap[(size_t)rr * nmax + j] = (float)fma(-cpr, rd, Bw[(size_t)rr * n + j]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) Ap[(size_t)(n + a) * nmax + j] = (float)fma(-rhoA[a], rd, f[a]);
    }
    for (int p = lane; p < no; p += 64) I.newrow[(size_t)w * I.nomax + p] = nr[p];
}

// FP32 MFMA GEMM of the mixed proposal: one block (4 waves) per walker.
// Operand rows (n + 4) x K=n from Ap32, Phi'_V = Phi_V with row i replaced by
// the new values, both staged in LDS; v_mfma_f32_16x16x4f32 tiles (A: lane l
// holds A[l%16][l/16]; B: B[l/16][l%16]; D: lane l, element i holds
// D[4(l/16)+i][l%16]).
__global__ void __launch_bounds__(256)
k_gemm_mixed(const InstDev *__restrict__ insts, const MoveArgs *__restrict__ moves, MoveArgs m1) {
    const int inst = blockIdx.y;
    const InstDev &I = insts[inst];
    const MoveArgs mv = moves ? moves[inst] : m1;
    const int w = blockIdx.x;
    if (w >= I.W) return;
    const SpinDev &S = I.s[mv.spin];
    const int n = S.n, m = S.m, no = S.no, row = mv.row, nmax = I.nmax;
    const int rows = n + 4;
    const int rp = (rows + 15) & ~15, kp = (n + 3) & ~3, mp = (m + 15) & ~15;
    const int lda = kp + 1;
    extern __shared__ float shf[];
    float *As = shf;                 // rp x lda
    float *Bs = shf + rp * lda;      // kp x mp
    const int tid = threadIdx.x;
    const float *__restrict__ Ap = I.Ap32 + (size_t)w * (nmax + 4) * nmax;
    for (int idx = tid; idx < rp * kp; idx += 256) {
        const int r = idx / kp, k = idx - r * kp;
        As[r * lda + k] = (r < rows && k < n) ? Ap[(size_t)r * nmax + k] : 0.0f;
    }
    const double *__restrict__ nr = mv.new_orb + (size_t)w * 5 * no;
    const float *__restrict__ Pv = S.PhiV32 + (size_t)w * n * m;
    for (int idx = tid; idx < kp * mp; idx += 256) {
        const int k = idx / mp, p = idx - k * mp;
        float v = 0.0f;
        if (k < n && p < m) v = (k == row) ? (float)nr[n + p] : Pv[(size_t)k * m + p];
        Bs[idx] = v;
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int RT = rp >> 4, CT = mp >> 4;
    const int lr = lane & 15, lk = lane >> 4;
    const int WT = S.WT, tw = w / WT, lw = w % WT;
    float *__restrict__ Tp = I.Tp32 + (size_t)tw * n * m * WT + lw;
    float *__restrict__ g32 = I.ev32 + (size_t)tw * 4 * m * WT + lw;
    const bool ksum64 = I.prec == 3;
    for (int t = wave; t < RT * CT; t += 4) {
        const int rt = t / CT, ct = t - rt * CT;
        // MIXED_GEMM: one chain of MFMAs over all of K with FP32 accumulation.
        // MIXED_GEMM_KSUM64: each MFMA multiplies one K-block of 4 into a zero
        // FP32 accumulator and the K-blocks are summed in FP64.
        double acc64[4] = {0.0, 0.0, 0.0, 0.0};
        floatx4 acc32 = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int kk = 0; kk < kp; kk += 4) {
            const float a = As[(rt * 16 + lr) * lda + kk + lk];
            const float b = Bs[(kk + lk) * mp + ct * 16 + lr];
            if (ksum64) {
                const floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
                const floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, z, 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 4; ++i) acc64[i] += (double)acc[i];
            } else {
                acc32 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc32, 0, 0, 0);
            }
        }
        if (!ksum64) {
#pragma unroll
            for (int i = 0; i < 4; ++i) acc64[i] = (double)acc32[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = rt * 16 + 4 * lk + i, p = ct * 16 + lr;
            if (p >= m) continue;
            if (r < n) Tp[(size_t)(r * m + p) * WT] = (float)acc64[i];
            else if (r < rows) {
                const int a = r - n;
                g32[(size_t)(p * 4 + a) * WT] = (float)(nr[(1 + a) * no + n + p] - acc64[i]);
            }
        }
    }
}

hipError_t launch_propose(hipStream_t st, const InstDev *d_insts, int n_inst, int maxW,
                          const MoveArgs *d_moves, const MoveArgs &m1, int prec, int nmax,
                          int mmax, int WT, int max_tiles, int split) {
    if (prec >= 2) {
        dim3 grid((maxW + 3) / 4, n_inst);
        hipLaunchKernelGGL(k_propose_mixed, grid, dim3(256), 0, st, d_insts, d_moves, m1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int rp = (nmax + 4 + 15) & ~15, kp = (nmax + 3) & ~3, mp = (mmax + 15) & ~15;
        const size_t lds = sizeof(float) * ((size_t)rp * (kp + 1) + (size_t)kp * mp);
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)k_gemm_mixed,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_gemm_mixed, dim3(maxW, n_inst), dim3(256), lds, st, d_insts, d_moves,
                           m1);
        return hipGetLastError();
    }
    const size_t lds = propose_lds(nmax, mmax, WT, split);
    const int T8 = (max_tiles + NXCD - 1) / NXCD * NXCD;
    dim3 g(n_inst * T8 * split);
#define MDE_PP(X)                                                                              \
    case X:                                                                                    \
        if (prec == 0) {                                                                       \
            if (lds > 65536)                                                                   \
                (void)hipFuncSetAttribute((const void *)k_propose<X, double>,                  \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
            hipLaunchKernelGGL((k_propose<X, double>), g, dim3(256), lds, st, d_insts, d_moves, \
                               m1, split, T8, n_inst);                                         \
        } else {                                                                               \
            if (lds > 65536)                                                                   \
                (void)hipFuncSetAttribute((const void *)k_propose<X, float>,                   \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
            hipLaunchKernelGGL((k_propose<X, float>), g, dim3(256), lds, st, d_insts, d_moves, \
                               m1, split, T8, n_inst);                                         \
        }                                                                                      \
        break;
    switch (WT) {
        MDE_PP(1) MDE_PP(2) MDE_PP(4) MDE_PP(8) MDE_PP(16) MDE_PP(32) MDE_PP(64)
        default: return hipErrorInvalidValue;
    }
#undef MDE_PP
    return hipGetLastError();
}

int propose_split_limit(int nmax, int mmax, int WT, size_t lds_max) {
    // smallest split whose LDS footprint fits
    for (int s = 1; s <= mmax; ++s)
        if (propose_lds(nmax, mmax, WT, s) <= lds_max) return s;
    return 0;
}

// ---------------------------------------------------------------------------
// commit (Sec. III SM eq., row form): for accepted walkers, with c' = c/rho,
//   A^-1 <- A^-1 - c' (a'^T A^-1 - e_i^T),   Phi row i <- new,
//   T_V  <- T'_V = A'^-1 Phi'_V  (FP64: formed here as T_V - c' q^T; mixed
//                                 forms: the proposal's FP32 table),
//   log|det A| += log|rho|,  N <- N'.
// ---------------------------------------------------------------------------

template <int WT>
__global__ void __launch_bounds__(256)
k_accept(const InstDev *__restrict__ insts, const MoveArgs *__restrict__ moves, MoveArgs m1,
         int split, int T8, int n_inst) {
    int inst, t, part;
    if (!tile_of_block(split, T8, n_inst, inst, t, part)) return;
    const InstDev &I = insts[inst];
    const MoveArgs mv = moves ? moves[inst] : m1;
    const SpinDev &S = I.s[mv.spin];
    if (t >= S.n_tiles) return;
    const int n = S.n, m = S.m, no = S.no, row = mv.row, W = I.W, nm = n * m, nn = n * n;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int w0 = t * WT, nw = min(WT, W - w0);
    __shared__ int acc_s[64];
    extern __shared__ double sha[];
    double *cp_s = sha;            // [n][WT]  c' = c / rho (0 for rejected walkers)
    double *rr_s = sha + n * WT;   // [n][WT]  a'^T A^-1 - e_i^T
    const int acc_me = (tid < WT && tid < nw) ? (int)mv.accept[w0 + tid] : 0;
    if (tid < WT) acc_s[tid] = acc_me;
    // a tile none of whose walkers accepted has nothing to commit (every
    // write below is an accepted walker's); the whole block leaves together
    if (!__syncthreads_or(acc_me)) return;
    {
        const auto cc = MDE_G(double, I.cc) + (size_t)t * n * WT;
        const auto rr = MDE_G(double, I.rrow) + (size_t)t * n * WT;
        for (int idx = tid; idx < n * WT; idx += nthr) {
            const int l = idx % WT;
            const double c = cc[idx], r = rr[idx];
            const double ir = acc_s[l] ? 1.0 / I.rho[w0 + l] : 0.0;
            cp_s[idx] = c * ir;
            rr_s[idx] = r;
        }
    }
    __syncthreads();
    // A^-1 of the tile's walkers is contiguous: the part takes a slice of it
    {
        const int tot = nw * nn, ch = (tot + split - 1) / split;
        const int e0 = part * ch, e1 = min(tot, e0 + ch);
        double *Bt = S.B + (size_t)w0 * nn;
        for (int idx = e0 + tid; idx < e1; idx += nthr) {
            const int l = idx / nn, rj = idx - l * nn, r = rj / n, j = rj - r * n;
            if (!acc_s[l]) continue;
            Bt[idx] = fma(-cp_s[r * WT + l], rr_s[j * WT + l], Bt[idx]);
        }
    }
    const size_t tb = (size_t)t * nm * WT;
    const int ec = (nm * WT + split - 1) / split, e0 = part * ec, e1 = min(nm * WT, e0 + ec);
    if (I.prec == 0 && (mv.mode & MV_FUSED)) {
        // the part owns the virtual columns [p0, p1) of every row: it forms
        // q_p = a'^T T[:, p] - phi'_p from the old table, then updates them
        const int mc = (m + split - 1) / split, p0 = min(m, part * mc), p1 = min(m, p0 + mc);
        double *q_s = rr_s + n * WT;      // [mc][WT]
        for (int idx = tid; idx < (p1 - p0) * WT; idx += nthr) {
            const int pl = idx / WT, l = idx - pl * WT, p = p0 + pl;
            double q = 0.0;
            if (l < nw) {
                const auto a = MDE_G(double, I.newrow) + (size_t)(w0 + l) * I.nomax;
                for (int r = 0; r < n; ++r) q = fma(a[r], S.T[tb + (size_t)(r * m + p) * WT + l], q);
                q -= a[n + p];
            }
            q_s[idx] = q;
        }
        __syncthreads();
        for (int idx = tid; idx < n * (p1 - p0) * WT; idx += nthr) {
            const int l = idx % WT, e = idx / WT, r = e / (p1 - p0), pl = e - r * (p1 - p0);
            if (!acc_s[l]) continue;
            const size_t o = tb + (size_t)(r * m + p0 + pl) * WT + l;
            S.T[o] = fma(-cp_s[r * WT + l], q_s[pl * WT + l], S.T[o]);
        }
    } else if (I.prec == 0) {
        const auto qv = MDE_G(double, I.ev) + (size_t)t * 5 * m * WT;
        int idx = e0 + tid;
        // four entries per thread in flight
        for (; idx + 3 * nthr < e1; idx += 4 * nthr) {
            double tv[4], qp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int id = idx + u * nthr, l = id % WT, e = id / WT, r = e / m, p = e - r * m;
                tv[u] = S.T[tb + id];
                qp[u] = qv[(size_t)p * 5 * WT + l];
                (void)r;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int id = idx + u * nthr, l = id % WT, e = id / WT, r = e / m;
                if (acc_s[l]) S.T[tb + id] = fma(-cp_s[r * WT + l], qp[u], tv[u]);
            }
        }
        for (; idx < e1; idx += nthr) {
            const int l = idx % WT;
            if (!acc_s[l]) continue;
            const int e = idx / WT, r = e / m, p = e - r * m;
            S.T[tb + idx] = fma(-cp_s[r * WT + l], qv[(size_t)p * 5 * WT + l], S.T[tb + idx]);
        }
    } else {
        int idx = e0 + tid;
        for (; idx + 3 * nthr < e1; idx += 4 * nthr) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = I.Tp32[tb + idx + u * nthr];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (acc_s[(idx + u * nthr) % WT]) S.T32[tb + idx + u * nthr] = v[u];
        }
        for (; idx < e1; idx += nthr)
            if (acc_s[idx % WT]) S.T32[tb + idx] = I.Tp32[tb + idx];
    }
    // orbital row of the moved electron (walker-major, contiguous per walker)
    {
        const int tot = nw * no, ch = (tot + split - 1) / split;
        const int q0 = part * ch, q1 = min(tot, q0 + ch);
        const auto nrow = MDE_G(double, I.newrow);
        for (int idx = q0 + tid; idx < q1; idx += nthr) {
            const int l = idx / no, p = idx - l * no, w = w0 + l;
            if (!acc_s[l]) continue;
            const double v = nrow[(size_t)w * I.nomax + p];
            S.Phi[((size_t)w * n + row) * no + p] = v;
            if (I.prec >= 2 && p >= n) S.PhiV32[((size_t)w * n + row) * m + (p - n)] = (float)v;
        }
    }
    if (part == 0 && tid < nw && acc_s[tid]) {
        const int w = w0 + tid;
        const double rho = I.rho[w];
        S.logdet[w] += log(fabs(rho));
        if (rho < 0.0) S.sgn[w] = -S.sgn[w];
        I.Nold[w] = I.Nnew[w];
    }
}

// Commit of a proposal formed in the determinant kernel (FP64, 64-walker
// tiles; Sherman-Morrison row update of Sec. III with the table update
// T' = T - c' q^T, c' = c / rho): block (tile, part), part p owns the
// virtual columns p, p + P, ... of every row (it forms q from the old
// table, then updates those entries), the rows k = p, p + P, ... of each
// walker's inverse, and a share of the orbital row; every load of a thread
// is issued before its arithmetic.  Thread (g, l): walker lane l, group g.
__global__ void __launch_bounds__(256)
k_accept64f(const InstDev *__restrict__ insts, MoveArgs mv, int split, int T8) {
    constexpr int WT = 64, NMAX = 8, NG = 4;
    int inst, t, part;
    if (!tile_of_block(split, T8, 1, inst, t, part)) return;
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[mv.spin];
    if (t >= S.n_tiles) return;
    const int n = S.n, m = S.m, no = S.no, nm = n * m, nn = n * n, row = mv.row, W = I.W;
    const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int w = t * WT + l;
    if (w >= W) return;
    // the walker's inputs are loaded together with its accept flag (all
    // addresses are valid either way); a rejected walker drops them
    const bool acc = mv.accept[w] != 0;
    const double rho = I.rho[w];
    double cp[NMAX], a[NMAX];
    const auto cc = MDE_G(double, I.cc) + (size_t)t * n * WT + l;
    const auto nr = MDE_G(double, I.newrow) + (size_t)w * I.nomax;
#pragma unroll
    for (int r = 0; r < NMAX; ++r) {
        cp[r] = r < n ? cc[(size_t)r * WT] : 0.0;
        a[r] = r < n ? nr[r] : 0.0;
    }
    double *T = S.T + (size_t)t * nm * WT + l;
    const int p0 = part + split * g;
    double tv0[NMAX], q0 = 0.0;
    if (p0 < m) {
#pragma unroll
        for (int r = 0; r < NMAX; ++r) tv0[r] = r < n ? T[(size_t)(r * m + p0) * WT] : 0.0;
        q0 = -nr[n + p0];
    }
    // first row of the inverse this thread updates (k = part, j = g, g + NG)
    // and its first orbital-row entry, also ahead of the flag
    const auto rr = MDE_G(double, I.rrow) + (size_t)t * n * WT + l;
    double *B = S.B + (size_t)w * nn;
    double b0[2] = {0.0, 0.0}, r0[2] = {0.0, 0.0};
    if (part < n) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = g + h * NG;
            if (j < n) {
                b0[h] = B[part * n + j];
                r0[h] = rr[(size_t)j * WT];
            }
        }
    }
    const int pf = part * NG + g;
    const double nf = pf < no ? nr[pf] : 0.0;
    const double nnew = I.Nnew[w];
    // the remaining destinations, and the values the first thread updates,
    // also before any store (a store could alias the descriptor's fields)
    double *const Phi = S.Phi + ((size_t)w * n + row) * no;
    double *const ld_g = S.logdet;
    double *const sg_g = S.sgn;
    double *const nold_g = I.Nold;
    const bool first = part == 0 && g == 0;
    const double ld0 = first ? ld_g[w] : 0.0, sg0 = first ? sg_g[w] : 0.0;
    if (!acc) return;
    const double ir = 1.0 / rho;
#pragma unroll
    for (int r = 0; r < NMAX; ++r) cp[r] *= ir;
    // columns p = part + P * (g + NG * i): q from the old table, then update
    for (int p = p0; p < m; p += split * NG) {
        double tv[NMAX];
        double q;
        if (p == p0) {
#pragma unroll
            for (int r = 0; r < NMAX; ++r) tv[r] = tv0[r];
            q = q0;
        } else {
#pragma unroll
            for (int r = 0; r < NMAX; ++r) tv[r] = r < n ? T[(size_t)(r * m + p) * WT] : 0.0;
            q = -nr[n + p];
        }
#pragma unroll
        for (int r = 0; r < NMAX; ++r) q = fma(a[r], tv[r], q);
#pragma unroll
        for (int r = 0; r < NMAX; ++r)
            if (r < n) T[(size_t)(r * m + p) * WT] = fma(-cp[r], q, tv[r]);
    }
    // rows k = part + P * i of the inverse: B[k][j] -= c'_k r_j
    for (int k = part; k < n; k += split) {
        double ck = 0.0;
#pragma unroll
        for (int r = 0; r < NMAX; ++r)
            if (r == k) ck = cp[r];
        for (int j = g, h = 0; j < n; j += NG, ++h) {
            if (k == part && h < 2)
                B[k * n + j] = fma(-ck, r0[h], b0[h]);
            else
                B[k * n + j] = fma(-ck, rr[(size_t)j * WT], B[k * n + j]);
        }
    }
    // orbital row of the moved electron
    for (int p = pf; p < no; p += split * NG) Phi[p] = p == pf ? nf : nr[p];
    if (first) {
        ld_g[w] = ld0 + log(fabs(rho));
        if (rho < 0.0) sg_g[w] = -sg0;
        nold_g[w] = nnew;
    }
}

hipError_t launch_accept64f(hipStream_t st, const InstDev *d_inst, const MoveArgs &m1, int n_tiles,
                            int split, int n_max) {
    if (n_max > 8) return hipErrorInvalidValue;
    const int T8 = (n_tiles + NXCD - 1) / NXCD * NXCD;
    hipLaunchKernelGGL(k_accept64f, dim3(T8 * split), dim3(256), 0, st, d_inst, m1, split, T8);
    return hipGetLastError();
}

hipError_t launch_accept(hipStream_t st, const InstDev *d_insts, int n_inst, int maxW,
                         const MoveArgs *d_moves, const MoveArgs &m1, int prec, int nmax,
                         int mmax, int WT, int max_tiles, int split) {
    const int T8 = (max_tiles + NXCD - 1) / NXCD * NXCD;
    dim3 g(n_inst * T8 * split);
    const size_t lds = sizeof(double) * (2 * (size_t)nmax + (mmax + split - 1) / split) * WT;
#define MDE_AC(X)                                                                              \
    case X:                                                                                    \
        hipLaunchKernelGGL(k_accept<X>, g, dim3(256), lds, st, d_insts, d_moves, m1, split,   \
                           T8, n_inst);                                                        \
        break;
    switch (WT) {
        MDE_AC(1) MDE_AC(2) MDE_AC(4) MDE_AC(8) MDE_AC(16) MDE_AC(32) MDE_AC(64)
        default: return hipErrorInvalidValue;
    }
#undef MDE_AC
    (void)prec; (void)maxW;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------

__global__ void k_init_misc(const InstDev *__restrict__ insts) {
    const InstDev &I = insts[0];
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int s = 0; s < 2; ++s) {
        const SpinDev &S = I.s[s];
        const size_t nt = (size_t)S.n_tiles * S.WT;
        if (tid < nt) {
            const size_t t = tid / S.WT, wl = tid % S.WT;
            S.R[t * S.U * S.WT + wl] = 1.0;   // the reference: D_0 / D_0
        }
    }
    if (tid < (size_t)I.W) I.st[tid] = 0;
    if (tid < 16) I.counter[tid] = 0;
}

hipError_t launch_init_misc(hipStream_t st, const InstDev *d_inst, const InstDev &h) {
    size_t nmax = (size_t)h.W + 64;
    for (int s = 0; s < 2; ++s) {
        const size_t nt = (size_t)h.s[s].n_tiles * h.s[s].WT;
        if (nt > nmax) nmax = nt;
    }
    hipLaunchKernelGGL(k_init_misc, dim3((unsigned)((nmax + 255) / 256)), dim3(256), 0, st, d_inst);
    return hipGetLastError();
}

__global__ void k_export(const InstDev *__restrict__ insts, int what, int spin, double *dst,
                         const int32_t *__restrict__ perm_user, int n_user) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[spin];
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t W = I.W;
    if (what == 0) {
        if (tid < W * S.n * S.n) dst[tid] = S.B[tid];
    } else if (what == 1) {
        const size_t nm = (size_t)S.n * S.m;
        if (tid < W * nm) {
            const size_t w = tid / nm, e = tid % nm;
            const size_t o = ((w / S.WT) * nm + e) * S.WT + w % S.WT;
            dst[tid] = I.prec == 0 ? S.T[o] : (double)S.T32[o];
        }
    } else if (what == 2) {
        if (tid < W * (size_t)n_user) {
            const size_t w = tid / n_user, uu = tid % n_user;
            const int u = perm_user[uu];
            const size_t t = w / S.WT, wl = w % S.WT;
            dst[tid] = S.R[(t * S.U + u) * S.WT + wl];
        }
    } else if (what == 3) {
        if (tid < W) dst[tid] = S.logdet[tid];
    } else if (what == 4) {
        if (tid < W) dst[tid] = I.Nold[tid];
    }
}

hipError_t launch_export(hipStream_t st, const InstDev *d_inst, const InstDev &h, int what,
                         int spin, double *dst, const int32_t *perm_user) {
    const SpinDev &S = h.s[spin];
    size_t count = h.W;
    if (what == 0) count = (size_t)h.W * S.n * S.n;
    else if (what == 1) count = (size_t)h.W * S.n * S.m;
    else if (what == 2) count = (size_t)h.W * S.n_user;
    hipLaunchKernelGGL(k_export, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, d_inst,
                       what, spin, dst, perm_user, S.n_user);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t *p, int32_t v, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(hipStream_t st, int32_t *p, int32_t v, size_t n) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// per-instance move arguments written from kernel arguments, MOVE_BATCH at
// a time (a launch's arguments are copied by value, also into graphs)
constexpr int MOVE_BATCH = 24;
struct MoveBatch {
    MoveArgs m[MOVE_BATCH];
};
static_assert(sizeof(MoveBatch) <= 3072, "kernel argument block");

__global__ void k_set_moves(MoveArgs *__restrict__ dst, MoveBatch b, int n) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = b.m[i];
}

hipError_t launch_set_moves(hipStream_t st, MoveArgs *d_moves, const MoveArgs *h_moves, int n) {
    for (int off = 0; off < n; off += MOVE_BATCH) {
        MoveBatch b{};
        const int cnt = n - off < MOVE_BATCH ? n - off : MOVE_BATCH;
        for (int i = 0; i < cnt; ++i) b.m[i] = h_moves[off + i];
        hipLaunchKernelGGL(k_set_moves, dim3(1), dim3(64), 0, st, d_moves + off, b, cnt);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// dst[r][q] = src[r][perm[q]] over rows of no orbital values
__global__ void k_permute_orbitals(const double *__restrict__ src, double *__restrict__ dst,
                                   size_t total, int no, const int32_t *__restrict__ perm) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const size_t r = i / no;
    const int q = (int)(i - r * no);
    dst[i] = src[r * no + perm[q]];
}

hipError_t launch_permute_orbitals(hipStream_t st, const double *src, double *dst, int rows, int no,
                                   const int32_t *perm) {
    const size_t total = (size_t)rows * no;
    hipLaunchKernelGGL(k_permute_orbitals, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       src, dst, total, no, perm);
    return hipGetLastError();
}

hipError_t launch_reset_counter(hipStream_t st, int32_t *counter) {
    return launch_fill_i32(st, counter, 0, 16);
}

// ---------------------------------------------------------------------------
// synthetic orbitals: s-Gaussians chi_b = exp(-a |r - c_b|^2) with
// grad chi = -2a (r - c) chi and lap chi = (4a^2 |r - c|^2 - 6a) chi, then
// phi_p = sum_b mo[p][b] chi_b.  One block per position.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_sgauss(int nb, const double *__restrict__ centres, const double *__restrict__ expo, int n_orb,
         const double *__restrict__ mo, const double *__restrict__ pos, double *__restrict__ out) {
    extern __shared__ double chi[];   // [nb][5]
    const int q = blockIdx.x;
    const double x = pos[3 * (size_t)q], y = pos[3 * (size_t)q + 1], z = pos[3 * (size_t)q + 2];
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double dx = x - centres[3 * b], dy = y - centres[3 * b + 1], dz = z - centres[3 * b + 2];
        const double a = expo[b];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double v = exp(-a * r2);
        chi[5 * b + 0] = v;
        chi[5 * b + 1] = -2.0 * a * dx * v;
        chi[5 * b + 2] = -2.0 * a * dy * v;
        chi[5 * b + 3] = -2.0 * a * dz * v;
        chi[5 * b + 4] = (4.0 * a * a * r2 - 6.0 * a) * v;
    }
    __syncthreads();
    double *o = out + (size_t)q * 5 * n_orb;
    for (int p = threadIdx.x; p < n_orb; p += blockDim.x) {
        double acc[5] = {0, 0, 0, 0, 0};
        const double *mp = mo + (size_t)p * nb;
        for (int b = 0; b < nb; ++b) {
            const double wgt = mp[b];
#pragma unroll
            for (int c = 0; c < 5; ++c) acc[c] = fma(wgt, chi[5 * b + c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) o[(size_t)c * n_orb + p] = acc[c];
    }
}

hipError_t launch_sgauss(hipStream_t st, int nb, const double *centres, const double *expo,
                         int n_orb, const double *mo, int npos, const double *pos, double *out) {
    if (npos <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * 5 * nb;
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_sgauss,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_sgauss, dim3(npos), dim3(256), lds, st, nb, centres, expo, n_orb, mo, pos,
                       out);
    return hipGetLastError();
}

}  // namespace mde
