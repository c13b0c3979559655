// Determinant-stage kernels: the persistent gather + small-determinant + CI
// kernel (Sec. III read-off, Algorithm 1 step 4, Sec. IV-A derivative terms),
// the CI precontraction, the per-walker finish, and the N sums.
//
// Data layout on chip (LDS), walker fastest: entry e of the table for
// walker-lane wl sits at tab[e * WTP + wl].  With a walker tile of 64 the 64
// lanes of a wave are 64 walkers working on the same excitation: the
// excitation's indices are wave-uniform and every LDS gather is a
// conflict-free 512-byte row.  With small tiles (large n) the lanes of a wave
// take different excitations of the same walker(s).
#include "mde_internal.h"
#include "smalldet.h"

namespace mde {

// Excitation record: bytes 0..7 holes, bytes 8..15 local particle indices.
__device__ __forceinline__ int exc_byte(const uint4 &x, int i) {
    const uint32_t word = (i >> 2) == 0 ? x.x : (i >> 2) == 1 ? x.y : (i >> 2) == 2 ? x.z : x.w;
    return (int)((word >> ((i & 3) * 8)) & 0xffu);
}

// ---------------------------------------------------------------------------
// persistent determinant kernel
// ---------------------------------------------------------------------------
//
// Sums formed per walker over the moving spin's excitations u > 0, with
// S_u = Tab[h][p] and y = adj(S_u) c[h]:
//   acc[0]   = sum_u C_u det S_u
//   acc[1+b] = sum_u C_u sum_j e^b[p_j] y_j,   b < NE
// FP64 form (NE = 5): Tab = T, the current table, c = A^-1 e_i and
// e = (q, w^x, w^y, w^z, w^L); k_finish forms rho N' = rho N - acc[1] and
// rho sum_u C_u G^a_u = kappa^a N + acc[2+a].  Mixed forms (NE = 4): Tab = T',
// the updated table, c = c', e = g^a; k_finish forms N' = C_0 + acc[0] and
// sum_u C_u G^a_u = (kappa^a / rho) N' + acc[1+a].  (Matrix determinant
// lemma and the bordered form; the reference excitation adds C_0 to N.)
//
// LDS rows: Tab[h][p] at entry h*m + p, e^b[p] at entry NE*p + b (the
// components of one particle are consecutive rows), c[h] at entry h.

// One order-K excitation for walker-lane wl, all K x K entries gathered
// (walker tiles below 64, where the lanes of a wave hold different
// excitations).  PROPOSE accumulates into acc; VALUES returns det S.
template <int K, typename TT, int MODE>
__device__ __forceinline__ double det_one(const uint4 &ex, const TT *__restrict__ tabs,
                                          const TT *__restrict__ gs, const TT *__restrict__ cs,
                                          int m, int WTP, int wl, double Cu, double acc[NSUM]) {
    int h[K], hm[K], p[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        h[j] = exc_byte(ex, j);
        hm[j] = h[j] * m;
        p[j] = exc_byte(ex, 8 + j);
    }
    double col[K][K];
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int r = 0; r < K; ++r) col[j][r] = (double)tabs[(hm[r] + p[j]) * WTP + wl];
    double c[K], y[K];
    if (MODE == DM_VALUES) {
#pragma unroll
        for (int r = 0; r < K; ++r) c[r] = 0.0;
        return SmallDet<K, double>::run(col, c, y);
    }
#pragma unroll
    for (int r = 0; r < K; ++r) c[r] = (double)cs[h[r] * WTP + wl];
    const double dd = SmallDet<K, double>::run(col, c, y);
    acc[0] = fma(Cu, dd, acc[0]);
    constexpr int NE = sizeof(TT) == 8 ? 5 : 4;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double wy = Cu * y[j];
#pragma unroll
        for (int b = 0; b < NE; ++b)
            acc[1 + b] = fma((double)gs[(p[j] * NE + b) * WTP + wl], wy, acc[1 + b]);
    }
    return dd;
}

// With WS the e-terms go to the lane's per-particle weights Wl[p * 64]
// instead of being gathered (64-walker tiles).
template <typename TT, int MODE, bool WS = false>
__device__ double det_one_generic(int k, const uint4 &ex, const TT *__restrict__ tabs,
                                  const TT *__restrict__ gs, const TT *__restrict__ cs, int m,
                                  int WTP, int wl, double Cu, double acc[NSUM],
                                  double *Wl = nullptr) {
    int h[MAXK], p[MAXK];
    for (int j = 0; j < k; ++j) {
        h[j] = exc_byte(ex, j);
        p[j] = exc_byte(ex, 8 + j);
    }
    double col[8][8], c[8], y[8];
    for (int j = 0; j < k; ++j)
        for (int r = 0; r < k; ++r) col[j][r] = (double)tabs[(h[r] * m + p[j]) * WTP + wl];
    for (int r = 0; r < k; ++r) c[r] = (MODE == DM_VALUES) ? 0.0 : (double)cs[h[r] * WTP + wl];
    const double dd = small_det_generic<double>(k, col, c, y);
    if (MODE == DM_VALUES) return dd;
    acc[0] = fma(Cu, dd, acc[0]);
    constexpr int NE = sizeof(TT) == 8 ? 5 : 4;
    for (int j = 0; j < k; ++j) {
        const double wy = Cu * y[j];
        if (WS) {
            atomicAdd(Wl + p[j] * 64, wy);
            continue;
        }
        for (int b = 0; b < NE; ++b)
            acc[1 + b] = fma((double)gs[(p[j] * NE + b) * WTP + wl], wy, acc[1 + b]);
    }
    return dd;
}

// Loop over the item's excitations (slot-strided; records [u0, u1) read from
// global memory).  The records and CI weights of the next DP excitations of
// the lane are loaded while the current ones are evaluated (a ring of DP
// register sets, indexed statically by unrolling the loop DP-fold), so the
// lane waits on a global load once per DP excitations at most.
template <int K, typename TT, int MODE, int WT>
__device__ __forceinline__ void det_loop(const WorkItem &it, const SpinDev &S,
                                         const uint4 *__restrict__ recs, const TT *tabs,
                                         const TT *gs, const TT *cs, int wl, int slot, int nslot,
                                         double acc[NSUM]) {
    constexpr int DP = 4;
    const int len = it.u1 - it.u0;
    const size_t base = ((size_t)it.tile * S.U + it.u0) * WT;
    const auto Cb = MDE_G(double, S.C) + base;
    const auto Rb = MDE_GW(double, S.R) + base;
    const uint4 *__restrict__ rg = recs;
    const int m = S.m, WTP = S.WTP;
    uint4 exr[DP];
    double cr[DP];
#pragma unroll
    for (int i = 0; i < DP; ++i) {
        const int j = slot + i * nslot;
        exr[i] = j < len ? rg[j] : make_uint4(0, 0, 0, 0);
        cr[i] = (MODE == DM_PROPOSE && j < len) ? Cb[(size_t)j * WT + wl] : 0.0;
    }
    for (int j0 = slot; j0 < len; j0 += DP * nslot) {
#pragma unroll
        for (int i = 0; i < DP; ++i) {
            const int j = j0 + i * nslot;
            if (j >= len) break;
            const uint4 ex = exr[i];
            const double Cu = cr[i];
            const int jn = j + DP * nslot;
            if (jn < len) {
                exr[i] = rg[jn];
                if (MODE == DM_PROPOSE) cr[i] = Cb[(size_t)jn * WT + wl];
            }
            double R;
            if (K > 0)
                R = det_one<(K > 0 ? K : 1), TT, MODE>(ex, tabs, gs, cs, m, WTP, wl, Cu, acc);
            else
                R = det_one_generic<TT, MODE>(it.order, ex, tabs, gs, cs, m, WTP, wl, Cu, acc);
            if (MODE == DM_VALUES) Rb[(size_t)j * WT + wl] = R;
        }
    }
}

// ---- walker tile 64: one excitation per wave, evaluated in runs ----------
//
// The lanes of a wave are 64 walkers and every index is wave-uniform: the
// records (staged in LDS with the tables) are broadcast to the wave and all
// control flow is scalar.
// The e-terms sum_u C_u sum_j e^b[p_j] y_j are linear in e, so each lane
// collects per-particle weights W[p] += C_u y_j (one LDS add, in program
// order, into its wave's own rows: no gathers of e^b) and the block
// contracts W with e^b once per work item.
// Excitations are sorted by holes, then particles, so consecutive
// excitations of one order share their holes h_0..h_{K-1} and, often, their
// first K-1 particles (the prefix).  Within such a run only the last column
// b = T'[h][q] of S changes, and everything else is linear in b:
//   det S = u . b,                 u = cofactors of the last column
//   y_j   = v_j . b   (j < K-1),   v_j = the same with column j -> c'[h]
//   y_{K-1} = u . c'[h]            (constant over the run)
// so per excitation the wave gathers K table entries, adds C y_{K-1} to
// W[q], and the run accumulates Nrun += C det S, Yrun_j += C y_j; on
// closing the run acc[0] += Nrun and W[p_j] += Yrun_j.

__device__ __forceinline__ int byte_of(uint32_t w, int i) { return (int)((w >> (8 * i)) & 0xffu); }

// CI weights C_u are read with non-temporal loads in the proposal: a launch
// reads each weight once, and streaming them through L2 at the normal
// priority evicts the tables, inverses and partial sums that the kernels
// around the proposal hand to each other through L2.

template <int K, typename TT, int MODE>
__device__ __forceinline__ void det_runs64(const SpinDev &S, int tile, int j0, int j1,
                                           const uint32_t *exw, int u0,
                                           const TT *__restrict__ tabs, const TT *__restrict__ cs,
                                           int wl, double *Wl, double acc[NSUM]) {
    constexpr int KP = K - 1;                  // prefix length
    constexpr int KQ = KP > 0 ? KP : 1;
    constexpr uint32_t PMASK = KP == 0 ? 0u : (KP >= 4 ? 0xffffffffu : ((1u << (8 * KP)) - 1u));
    constexpr int WTP = lds_row_stride(64);
    constexpr int D = 4;                       // CI weights loaded ahead
    if (j0 >= j1) return;
    const int m = S.m;
    const size_t cb0 = (size_t)tile * S.U * 64 + wl;
    const auto Cg = MDE_G(double, S.C) + cb0;
    const auto Rg = MDE_GW(double, S.R) + cb0;
    bool open = false;
    uint32_t hx = 0, pz = 0;
    int rb[K];
    double c[K], u[K], v[KQ][K];
    double ylast = 0.0, Nrun = 0.0, Yrun[KQ];
#pragma unroll
    for (int r = 0; r < K; ++r) { rb[r] = 0; c[r] = 0.0; u[r] = 0.0; }
#pragma unroll
    for (int j = 0; j < KQ; ++j) {
        Yrun[j] = 0.0;
#pragma unroll
        for (int r = 0; r < K; ++r) v[j][r] = 0.0;
    }

    auto close_run = [&]() {
        acc[0] += Nrun;
#pragma unroll
        for (int j = 0; j < KP; ++j) atomicAdd(Wl + byte_of(pz, j) * 64, Yrun[j]);
    };

    auto step = [&](const uint32_t hw, const uint32_t pw, double Cu, int j) {
        const bool new_holes = !open || hw != hx;
        if (new_holes || ((pw ^ pz) & PMASK) != 0u) {
            if (MODE == DM_PROPOSE && open) close_run();
            if (new_holes) {
                hx = hw;
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    const int h = byte_of(hw, r);
                    rb[r] = h * m;
                    if (MODE == DM_PROPOSE) c[r] = (double)cs[h * WTP + wl];
                }
            }
            pz = pw;
            double P[KQ][K];
#pragma unroll
            for (int j = 0; j < KP; ++j) {
                const int p = byte_of(pw, j);
#pragma unroll
                for (int r = 0; r < K; ++r) P[j][r] = (double)tabs[(rb[r] + p) * WTP + wl];
            }
            if (MODE == DM_PROPOSE) {
                prefix_cofactors<K, double>(P, c, u, v, ylast);
                Nrun = 0.0;
#pragma unroll
                for (int i = 0; i < KQ; ++i) Yrun[i] = 0.0;
            }
            else
                last_cofactors<K, double>(P, u);
            open = true;
        }
        const int q = byte_of(pw, KP);
        double b[K];
#pragma unroll
        for (int r = 0; r < K; ++r) b[r] = (double)tabs[(rb[r] + q) * WTP + wl];
        double det = 0.0;
#pragma unroll
        for (int r = 0; r < K; ++r) det = fma(u[r], b[r], det);
        if (MODE == DM_VALUES) {
            Rg[(size_t)j * 64] = det;
            return;
        }
        Nrun = fma(Cu, det, Nrun);
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            double y = 0.0;
#pragma unroll
            for (int r = 0; r < K; ++r) y = fma(v[i][r], b[r], y);
            Yrun[i] = fma(Cu, y, Yrun[i]);
        }
        atomicAdd(Wl + q * 64, Cu * ylast);
    };

    // records and CI weights of the next group are loaded while the current
    // group is evaluated; indices are clamped into the range so every load
    // is unconditional (a fixed number of loads in flight).  Two register
    // sets alternate, so no copy waits for a load in flight.
    uint32_t hA[D], pA[D], hB[D], pB[D];
    double cA[D], cB[D];
    auto fetch = [&](int jb, uint32_t (&h)[D], uint32_t (&pp)[D], double (&cv)[D]) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int jj = min(jb + i, j1 - 1);
            h[i] = exw[4 * (jj - u0)];          // word x: holes 0..3
            pp[i] = exw[4 * (jj - u0) + 2];     // word z: particles 0..3
            cv[i] = MODE == DM_PROPOSE ? __builtin_nontemporal_load(&Cg[(size_t)jj * 64]) : 0.0;
        }
        // keep the compiler from moving these loads next to their use one
        // group later (an empty asm with a memory clobber emits nothing)
        __asm__ volatile("" ::: "memory");
    };
    auto run_group = [&](int jb, const uint32_t (&h)[D], const uint32_t (&pp)[D],
                         const double (&cv)[D]) {
#pragma unroll
        for (int i = 0; i < D; ++i)
            if (jb + i < j1)
                step(__builtin_amdgcn_readfirstlane(h[i]), __builtin_amdgcn_readfirstlane(pp[i]), cv[i],
                     jb + i);
    };
    fetch(j0, hA, pA, cA);
    for (int j = j0; j < j1; j += 2 * D) {
        fetch(j + D, hB, pB, cB);
        run_group(j, hA, pA, cA);
        if (j + D >= j1) break;
        fetch(j + 2 * D, hA, pA, cA);
        run_group(j + D, hB, pB, cB);
    }
    if (MODE == DM_PROPOSE && open) close_run();
}

// Orders whose prefix runs are short (triples and quadruples rarely share
// their first K-1 particles): every excitation gathers its K x K block, in
// groups of D with no branches between them but the reload of c[h] when the
// hole set changes (excitations are sorted by holes), so the LDS reads of
// one excitation overlap the arithmetic of the previous one.  Past the end
// of the range the group repeats the last excitation with weight 0 (and,
// for values, rewrites the same ratio).
template <int K, typename TT, int MODE>
__device__ __forceinline__ void det_direct64(const SpinDev &S, int tile, int j0, int j1,
                                             const uint32_t *exw, int u0,
                                             const TT *__restrict__ tabs, const TT *__restrict__ cs,
                                             int wl, double *Wl, double acc[NSUM]) {
    constexpr int WTP = lds_row_stride(64);
    constexpr int D = 4;
    if (j0 >= j1) return;
    const int m = S.m;
    const size_t cb0 = (size_t)tile * S.U * 64 + wl;
    const auto Cg = MDE_G(double, S.C) + cb0;
    const auto Rg = MDE_GW(double, S.R) + cb0;
    uint32_t hA[D], pA[D], hB[D], pB[D];
    double cA[D], cB[D];
    uint32_t hx = 0xffffffffu;      // hole set of the cached c[h]
    double c[K];
#pragma unroll
    for (int r = 0; r < K; ++r) c[r] = 0.0;
    auto fetch = [&](int jb, uint32_t (&h)[D], uint32_t (&pp)[D], double (&cv)[D]) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int jj = min(jb + i, j1 - 1);
            h[i] = exw[4 * (jj - u0)];          // word x: holes 0..3
            pp[i] = exw[4 * (jj - u0) + 2];     // word z: particles 0..3
            cv[i] = MODE == DM_PROPOSE ? __builtin_nontemporal_load(&Cg[(size_t)jj * 64]) : 0.0;
        }
        __asm__ volatile("" ::: "memory");
    };
    auto run_group = [&](int j, const uint32_t (&hc)[D], const uint32_t (&pc)[D],
                         const double (&cb)[D]) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            int hm[K], p[K];
            const uint32_t hw = __builtin_amdgcn_readfirstlane(hc[i]);
            const uint32_t pw = __builtin_amdgcn_readfirstlane(pc[i]);
#pragma unroll
            for (int r = 0; r < K; ++r) {
                hm[r] = byte_of(hw, r) * m;
                p[r] = byte_of(pw, r);
            }
            double col[K][K], y[K];
#pragma unroll
            for (int jc = 0; jc < K; ++jc)
#pragma unroll
                for (int r = 0; r < K; ++r) col[jc][r] = (double)tabs[(hm[r] + p[jc]) * WTP + wl];
            if (MODE == DM_VALUES) {
                double z[K];
#pragma unroll
                for (int r = 0; r < K; ++r) z[r] = 0.0;
                const double dd = SmallDet<K, double>::run(col, z, y);
                Rg[(size_t)min(j + i, j1 - 1) * 64] = dd;
                continue;
            }
            if (hw != hx) {
                hx = hw;
#pragma unroll
                for (int r = 0; r < K; ++r) c[r] = (double)cs[byte_of(hw, r) * WTP + wl];
            }
            const double dd = SmallDet<K, double>::run(col, c, y);
            const double Cu = (j + i < j1) ? cb[i] : 0.0;
            acc[0] = fma(Cu, dd, acc[0]);
#pragma unroll
            for (int jc = 0; jc < K; ++jc) atomicAdd(Wl + p[jc] * 64, Cu * y[jc]);
        }
    };
    fetch(j0, hA, pA, cA);
    for (int j = j0; j < j1; j += 2 * D) {
        fetch(j + D, hB, pB, cB);
        run_group(j, hA, pA, cA);
        if (j + D >= j1) break;
        fetch(j + 2 * D, hA, pA, cA);
        run_group(j + D, hB, pB, cB);
    }
}

// Orders above 4 on 64-walker tiles: one excitation at a time, elimination
// with partial pivoting (det_one_generic).
template <typename TT, int MODE>
__device__ void det_generic64(const SpinDev &S, int tile, int k, int j0, int j1,
                              const uint32_t *exw, int u0, const TT *__restrict__ tabs,
                              const TT *__restrict__ cs, int wl, double *Wl, double acc[NSUM]) {
    const size_t cb0 = (size_t)tile * S.U * 64 + wl;
    const auto Cg = MDE_G(double, S.C) + cb0;
    const auto Rg = MDE_GW(double, S.R) + cb0;
    const uint4 *exl = reinterpret_cast<const uint4 *>(exw);
    for (int j = j0; j < j1; ++j) {
        uint4 ex = exl[j - u0];
        ex.x = __builtin_amdgcn_readfirstlane(ex.x);
        ex.y = __builtin_amdgcn_readfirstlane(ex.y);
        ex.z = __builtin_amdgcn_readfirstlane(ex.z);
        ex.w = __builtin_amdgcn_readfirstlane(ex.w);
        const double Cu = MODE == DM_PROPOSE ? __builtin_nontemporal_load(&Cg[(size_t)j * 64]) : 0.0;
        const double R = det_one_generic<TT, MODE, true>(k, ex, tabs, nullptr, cs, S.m,
                                                         lds_row_stride(64), wl, Cu, acc, Wl);
        if (MODE == DM_VALUES) Rg[(size_t)j * 64] = R;
    }
}

// Copy `count` = rows x WT elements of a walker-tiled array into padded LDS
// rows (row stride WTP).  Each thread keeps eight loads in flight before it
// writes, instead of one load-wait-store round trip per element.
template <int WT, typename TT, typename ST>
__device__ __forceinline__ void stage_rows(TT *__restrict__ dst, const ST __attribute__((address_space(1))) *src,
                                           int count, int WTP, int tid, int nthr) {
    constexpr int U = 8;
    int idx = tid;
    for (; idx + (U - 1) * nthr < count; idx += U * nthr) {
        ST v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[idx + u * nthr];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = idx + u * nthr;
            dst[(e / WT) * WTP + e % WT] = (TT)v[u];
        }
    }
    for (; idx < count; idx += nthr) dst[(idx / WT) * WTP + idx % WT] = (TT)src[idx];
}

// ---------------------------------------------------------------------------
// Dense blocks of orders 1 and 2 (every excitation of the order present, in
// canonical order: hole sets ascending, particles ascending inside a hole
// set; m == M).  A hole set's table rows are held in registers and its CI
// weights are streamed in order, so no record, gather or per-excitation
// e-row is needed.  For a double with rows a = Tab[h0][.], b = Tab[h1][.],
// c0 = c[h0], c1 = c[h1] and particles p < q:
//   det S = a_p b_q - a_q b_p,   y = adj(S) (c0, c1) = (z_q, -z_p),
//   z = c0 b - c1 a,
// so with S1_p = sum_{q>p} C b_q and S2_p = sum_{q>p} C a_q (one row of
// the block):
//   sum C det S                  = sum_p (a_p S1_p - b_p S2_p)
//   sum C (e_p y_0 + e_q y_1)    = sum_p e_p (c0 S1_p - c1 S2_p)
//                                  - sum_q e_q sum_{p<q} C z_p.
// A single h -> q has det = a_q and y = c[h].  The e-terms are collected in
// registers as per-particle weights Wt[q] and added to the lane's LDS
// weights once per range.  Per excitation: one CI weight and three FMAs.
// ---------------------------------------------------------------------------

// loads of CI weights in flight: a divisor of the block length (at most
// CAP), so the ring slot of an excitation is the same in every hole set
template <int NB, int CAP>
__host__ __device__ constexpr int dense_pd() {
    int d = NB < CAP ? NB : CAP;
    while (NB % d) --d;
    return d;
}

// One unit [S0, S0 + UNIT) of the hole pair with rows a = Tab[h0][.],
// b = Tab[h1][.]; `base` is the pair's first excitation.  The ring and the
// lane's weights carry over between units.
template <int M, int S0, typename TT, int MODE>
__device__ __forceinline__ void dense2_unit(const double (&a)[M], const double (&b)[M], double c0,
                                            double c1, int base, int j1,
                                            const double __attribute__((address_space(1))) *Cg,
                                            double __attribute__((address_space(1))) *Rg,
                                            double (&cb)[Dense2Shape<M>::PD], double *Wl,
                                            double &s0) {
    constexpr int PD = Dense2Shape<M>::PD, S1E = S0 + Dense2Shape<M>::UNIT;
    int sl = 0;
#pragma unroll
    for (int p = 0; p < M - 1; ++p) {
        const int rs = sl, re = sl + (M - 1 - p);   // the row's slots
        sl = re;
        if (re <= S0 || rs >= S1E) continue;
        double S1 = 0.0, S2 = 0.0, zp = 0.0;
        if (MODE == DM_PROPOSE) zp = fma(c0, b[p], -c1 * a[p]);
#pragma unroll
        for (int q = p + 1; q < M; ++q) {
            const int x = rs + (q - p - 1);
            if (x < S0 || x >= S1E) continue;
            if (MODE == DM_VALUES) {
                Rg[(size_t)(base + x) * 64] = fma(a[p], b[q], -a[q] * b[p]);
                continue;
            }
            const double C = cb[x % PD];
            cb[x % PD] = __builtin_nontemporal_load(&Cg[(size_t)min(base + x + PD, j1 - 1) * 64]);
            __asm__ volatile("" ::: "memory");
            S1 = fma(C, b[q], S1);
            S2 = fma(C, a[q], S2);
            atomicAdd(Wl + q * 64, -C * zp);
        }
        if (MODE == DM_PROPOSE) {
            s0 = fma(a[p], S1, fma(-b[p], S2, s0));
            atomicAdd(Wl + p * 64, fma(c0, S1, -c1 * S2));
        }
    }
}

// all units of a pair in one straight-line body; units outside [g0, g1) are skipped
template <int M, int G, typename TT, int MODE>
__device__ __forceinline__ void dense2_pair(const double (&a)[M], const double (&b)[M], double c0,
                                            double c1, int base, int j1, int g0, int g1,
                                            const double __attribute__((address_space(1))) *Cg,
                                            double __attribute__((address_space(1))) *Rg,
                                            double (&cb)[Dense2Shape<M>::PD], double *Wl,
                                            double &s0) {
    if constexpr (G < Dense2Shape<M>::G) {
        if (G >= g0 && G < g1)
            dense2_unit<M, G * Dense2Shape<M>::UNIT, TT, MODE>(a, b, c0, c1, base, j1, Cg, Rg, cb,
                                                               Wl, s0);
        dense2_pair<M, G + 1, TT, MODE>(a, b, c0, c1, base, j1, g0, g1, Cg, Rg, cb, Wl, s0);
    }
}

template <int M, typename TT, int MODE>
__device__ __forceinline__ void det_dense(const SpinDev &S, int k, int tile, int j0, int j1,
                                          const TT *tabs, const TT *__restrict__ cs,
                                          int wl, double *Wl, double acc[NSUM]) {
    constexpr int WTP = lds_row_stride(64);
    if (j0 >= j1) return;
    const int n = S.n;
    const size_t cb0 = (size_t)tile * S.U * 64 + wl;
    const auto Cg = MDE_G(double, S.C) + cb0;
    const auto Rg = MDE_GW(double, S.R) + cb0;
    const int a0 = S.order_start[k];
    double Wt[M];
#pragma unroll
    for (int q = 0; q < M; ++q) Wt[q] = 0.0;
    if (k == 1) {
        constexpr int PD = dense_pd<M, 24>();
        double cb[PD];
        if (MODE == DM_PROPOSE) {
#pragma unroll
            for (int i = 0; i < PD; ++i) cb[i] = __builtin_nontemporal_load(&Cg[(size_t)min(j0 + i, j1 - 1) * 64]);
        }
        for (int base = j0; base < j1; base += M) {
            const int h = (base - a0) / M;
            double a[M];
#pragma unroll
            for (int q = 0; q < M; ++q) a[q] = (double)tabs[(h * M + q) * WTP + wl];
            if (MODE == DM_VALUES) {
#pragma unroll
                for (int q = 0; q < M; ++q) Rg[(size_t)(base + q) * 64] = a[q];
                continue;
            }
            const double ch = (double)cs[h * WTP + wl];
            double s0 = 0.0;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const double C = cb[q % PD];
                cb[q % PD] = __builtin_nontemporal_load(&Cg[(size_t)min(base + q + PD, j1 - 1) * 64]);
                __asm__ volatile("" ::: "memory");
                s0 = fma(C, a[q], s0);
                Wt[q] = fma(C, ch, Wt[q]);
            }
            acc[0] += s0;
        }
    } else {
        using SH = Dense2Shape<M>;
        constexpr int PD = SH::PD, NP = SH::NP, UNIT = SH::UNIT;
        double cb[PD];
        if (MODE == DM_PROPOSE) {
#pragma unroll
            for (int i = 0; i < PD; ++i) cb[i] = __builtin_nontemporal_load(&Cg[(size_t)min(j0 + i, j1 - 1) * 64]);
        }
        // hole pair and unit of the first excitation of the range
        int hp = (j0 - a0) / NP, h0 = 0;
        int g = (j0 - a0 - hp * NP) / UNIT;
        while (hp >= n - 1 - h0) { hp -= n - 1 - h0; ++h0; }
        int h1 = h0 + 1 + hp;
        double s0 = 0.0;
        for (int u = j0; u < j1;) {
            const int base = u - g * UNIT;
            const int g1 = min(SH::G, g + (j1 - u) / UNIT);
            double a[M], b[M];
#pragma unroll
            for (int q = 0; q < M; ++q) {
                a[q] = (double)tabs[(h0 * M + q) * WTP + wl];
                b[q] = (double)tabs[(h1 * M + q) * WTP + wl];
            }
            double c0 = 0.0, c1 = 0.0;
            if (MODE == DM_PROPOSE) {
                c0 = (double)cs[h0 * WTP + wl];
                c1 = (double)cs[h1 * WTP + wl];
            }
            dense2_pair<M, 0, TT, MODE>(a, b, c0, c1, base, j1, g, g1, Cg, Rg, cb, Wl, s0);
            u += (g1 - g) * UNIT;
            g = 0;
            if (++h1 == n) { ++h0; h1 = h0 + 1; }
        }
        acc[0] += s0;
    }
    if (MODE == DM_PROPOSE && k == 1) {
#pragma unroll
        for (int q = 0; q < M; ++q) atomicAdd(Wl + q * 64, Wt[q]);
    }
}

template <typename TT, int MODE>
__device__ __forceinline__ void det_dense_m(const SpinDev &S, int k, int tile, int j0, int j1,
                                            const TT *tabs, const TT *__restrict__ cs,
                                            int wl, double *Wl, double acc[NSUM]) {
    switch (S.m) {
        case 8: det_dense<8, TT, MODE>(S, k, tile, j0, j1, tabs, cs, wl, Wl, acc); break;
        case 12: det_dense<12, TT, MODE>(S, k, tile, j0, j1, tabs, cs, wl, Wl, acc); break;
        case 16: det_dense<16, TT, MODE>(S, k, tile, j0, j1, tabs, cs, wl, Wl, acc); break;
        case 20: det_dense<20, TT, MODE>(S, k, tile, j0, j1, tabs, cs, wl, Wl, acc); break;
        case 24: det_dense<24, TT, MODE>(S, k, tile, j0, j1, tabs, cs, wl, Wl, acc); break;
        default: break;
    }
}

// Copy of up to four segments (16-byte units) into LDS with all loads of a
// thread issued before its LDS writes: the records before and after the
// dense block, the table and c of a 64-walker tile arrive in one round trip.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
struct StageSeg {
    const u32x4_t __attribute__((address_space(1))) *src;
    u32x4_t *dst;
    int n;
};
__device__ __forceinline__ void stage_segs(const StageSeg &s0, const StageSeg &s1,
                                           const StageSeg &s2, const StageSeg &s3, int tid,
                                           int nthr) {
    constexpr int U = 16;
    const int c1 = s0.n, c2 = c1 + s1.n, c3 = c2 + s2.n, tot = c3 + s3.n;
    for (int base = tid; base < tot; base += U * nthr) {
        u32x4_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * nthr;
            if (i < tot) {
                const auto sp = i < c1 ? s0.src + i
                                       : i < c2 ? s1.src + (i - c1)
                                                : i < c3 ? s2.src + (i - c2) : s3.src + (i - c3);
                v[u] = *sp;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * nthr;
            if (i < tot) {
                u32x4_t *dp = i < c1 ? s0.dst + i
                                     : i < c2 ? s1.dst + (i - c1)
                                              : i < c3 ? s2.dst + (i - c2) : s3.dst + (i - c3);
                *dp = v[u];
            }
        }
    }
}

// End of a 64-walker item whose proposal is formed in the determinant
// kernel (FP64 current-table frame).  With W_p the per-particle weights
// summed over the waves and V_r = sum_p W_p Tab[r][p], the e-terms are
//   sum_p W_p q_p     = sum_r a'_r V_r - sum_p W_p phi'_p
//   sum_p W_p w^a_p   = sum_p W_p d^a_V[p] - sum_r d^a_O[r] V_r
// (q = a'^T T_V - phi'_V, w^a = d^a_V - d^a_O^T T_V), so only the new
// orbital values of the walker are read.  The quantities the commit needs
// (c, rho, r = a'^T A^-1 - e_i^T, q) are formed by the finishing kernel.
__device__ __forceinline__ void item64_fused_end(const WorkItem &it, const InstDev &I,
                                                 const SpinDev &S, const MoveArgs &mv,
                                                 const double *tabs, const double *cs,
                                                 double *Wall, double *Vs,
                                                 unsigned char *tab_raw, const double (&acc)[NSUM],
                                                 int tid, int nthr) {
    constexpr int WT = 64, WTP = lds_row_stride(64);
    const int n = S.n, m = S.m, no = S.no, W = I.W;
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    const int w0 = it.tile * WT;
    const auto orb = MDE_G(double, mv.new_orb);
    // with 8 waves: the first 32 entries of each of the walker's five rows
    // for the contraction below, loaded before the W and V sums
    const int l8 = wave * 8 + (lane >> 3), j8 = lane & 7, w8 = w0 + l8;
    double x0[4][5];
    if (nw == 8) {
        const auto ob = orb + (size_t)(w8 < W ? w8 : w0) * 5 * no;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = j8 + 8 * u;
#pragma unroll
            for (int bb = 0; bb < 5; ++bb) x0[u][bb] = (k < no && w8 < W) ? ob[bb * no + k] : 0.0;
        }
    }
    __syncthreads();   // all waves done: W final, Tab and c intact
    // (the sums below read all their terms before adding them, in the same
    // order as a plain loop: the reads overlap, the result is unchanged)
    constexpr int NWMAX = DET64_THREADS / 64;
    for (int idx = tid; idx < m * 64; idx += nthr) {
        const int q = idx >> 6, l = idx & 63;
        double wv[NWMAX];
#pragma unroll
        for (int v = 0; v < NWMAX; ++v) wv[v] = v < nw ? Wall[((size_t)v * m + q) * 64 + l] : 0.0;
        double w = 0.0;
#pragma unroll
        for (int v = 0; v < NWMAX; ++v)
            if (v < nw) w += wv[v];
        Wall[idx] = w;     // this thread alone reads and writes entry (q, l)
    }
    __syncthreads();
    for (int idx = tid; idx < n * 64; idx += nthr) {
        const int r = idx >> 6, l = idx & 63;
        double v = 0.0;
        int q = 0;
        for (; q + 4 <= m; q += 4) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = Wall[(q + u) * 64 + l];
                b[u] = tabs[(r * m + q + u) * WTP + l];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) v = fma(a[u], b[u], v);
        }
        for (; q < m; ++q) v = fma(Wall[q * 64 + l], tabs[(r * m + q) * WTP + l], v);
        Vs[idx] = v;
    }
    __syncthreads();
    // The contraction with the walker's new orbital values: with 8 waves,
    // wave v takes walkers 8v .. 8v + 7, eight lanes each; lane j reads
    // entries k = j, j + 8, .. of the walker's five rows (eight lanes read 64
    // contiguous bytes) and the eight partial sums are added across the lane
    // group in a fixed butterfly.  Other block sizes: thread (b, l), b = wave,
    // wave + nw, reads the walker's row b.  Component 0 carries a', the
    // others the gradient and laplacian rows, of opposite sign.
    double ctr[2] = {0.0, 0.0};
    const int w = w0 + lane;
    if (nw == 8) {
        const int j = j8;
        double pb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (w8 < W) {
            const auto ob = orb + (size_t)w8 * 5 * no;
            for (int k0 = 0; k0 < no; k0 += 32) {
                double x[4][5], gk[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = k0 + j + 8 * u;
#pragma unroll
                    for (int bb = 0; bb < 5; ++bb)
                        x[u][bb] = k0 == 0 ? x0[u][bb] : (k < no ? ob[bb * no + k] : 0.0);
                    gk[u] = k < no ? (k < n ? Vs[k * 64 + l8] : -Wall[(k - n) * 64 + l8]) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int bb = 0; bb < 5; ++bb) pb[bb] = fma(x[u][bb], gk[u], pb[bb]);
            }
        }
#pragma unroll
        for (int bb = 0; bb < 5; ++bb)
#pragma unroll
            for (int off = 4; off >= 1; off >>= 1) pb[bb] += __shfl_xor(pb[bb], off, 8);
        // lane j = b of the group keeps component b (b < 5)
#pragma unroll
        for (int bb = 0; bb < 5; ++bb)
            if (j == bb) ctr[0] = bb == 0 ? pb[bb] : -pb[bb];
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int b = wave + i * nw;
            if (b < 5 && w < W) {
                const auto ob = orb + ((size_t)w * 5 + b) * no;
                double so = 0.0, sv = 0.0;
                int k = 0;
                for (; k + 8 <= no; k += 8) {
                    double x[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) x[u] = ob[k + u];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int kk = k + u;
                        if (kk < n) so = fma(x[u], Vs[kk * 64 + lane], so);
                        else sv = fma(Wall[(kk - n) * 64 + lane], x[u], sv);
                    }
                }
                for (; k < no; ++k) {
                    const double x = ob[k];
                    if (k < n) so = fma(x, Vs[k * 64 + lane], so);
                    else sv = fma(Wall[(k - n) * 64 + lane], x, sv);
                }
                ctr[i] = b == 0 ? so - sv : sv - so;
            }
        }
    }
    __syncthreads();   // Tab, W, V read: the LDS holds the reduction now
    double *red = reinterpret_cast<double *>(tab_raw);   // [nw][NSUM][64], then [5][64]
    double *red2 = red + (size_t)nw * NSUM * 64;
#pragma unroll
    for (int q = 0; q < NSUM; ++q) red[((size_t)wave * NSUM + q) * 64 + lane] = acc[q];
    if (nw == 8) {
        const int j = lane & 7;
        if (j < 5) red2[j * 64 + wave * 8 + (lane >> 3)] = ctr[0];
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
            if (wave + i * nw < 5) red2[(wave + i * nw) * 64 + lane] = ctr[i];
    }
    __syncthreads();
    const auto pout = MDE_GW(double, S.partial);
    for (int idx = tid; idx < 64 * NSUM; idx += nthr) {
        const int l = idx / NSUM, q = idx - l * NSUM;
        double rv[NWMAX];
#pragma unroll
        for (int v = 0; v < NWMAX; ++v) rv[v] = v < nw ? red[((size_t)v * NSUM + q) * 64 + l] : 0.0;
        const double r2 = q >= 1 ? red2[(q - 1) * 64 + l] : 0.0;
        double sum = 0.0;
#pragma unroll
        for (int v = 0; v < NWMAX; ++v)
            if (v < nw) sum += rv[v];
        if (q >= 1) sum += r2;
        pout[((size_t)it.slot * 64 + l) * NSUM + q] = sum;
    }
    __syncthreads();
}

// One work item on a 64-walker tile.  LDS: [records][Tab n*m rows][c n rows]
// [W: per wave, m rows of 64 FP64 particle weights].  Each wave evaluates
// its range (dense units or a piece of the sparse range) order by order;
// the e-terms are collected in W.
// At the end the block sums W over the waves, contracts it with e^b (the
// values are loaded before the barrier) and writes the item's NSUM sums per
// walker in a fixed order.
template <typename TT, int MODE, bool GEN>
__device__ __forceinline__ void item64(const WorkItem &it, const InstDev &I, const SpinDev &S,
                                       const MoveArgs &mv, uint4 *exl, unsigned char *tab_raw,
                                       const int32_t *__restrict__ bounds, int tid, int nthr,
                                       const double *tab0, const double *tab1) {
    constexpr int WT = 64, WTP = lds_row_stride(64);
    constexpr int NE = sizeof(TT) == 8 ? 5 : 4;
    constexpr int QPT = 3;        // e-values prefetched per thread (particles wave, wave+nw, ..)
    const int n = S.n, m = S.m, W = I.W, nm = n * m;
    const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
    // FP64 proposals formed here: c from A^-1, the e-terms from the new
    // orbital values (no e^b rows), and the tile's first item writes the
    // move's quantities for the commit and the finish
    const bool fused = MODE == DM_PROPOSE && sizeof(TT) == 8 && (mv.mode & MV_FUSED);
    TT *tabs = reinterpret_cast<TT *>(tab_raw);
    TT *cs = tabs + nm * WTP;
    double *Wall = reinterpret_cast<double *>(cs + n * WTP);
    double *Wl = Wall + (size_t)wave * m * 64 + lane;
    double *Vs = Wall + (size_t)nw * m * 64;    // [n][64] (fused proposals)
    uint32_t *exw = reinterpret_cast<uint32_t *>(exl);
    // records of the item's sparse range [u0, u1) (the dense block needs
    // none): record u at exw[4 * (u - u0)]
    using G4 = const u32x4_t __attribute__((address_space(1))) *;
    const G4 exg = (G4)(S.ex);
    u32x4_t *exd = reinterpret_cast<u32x4_t *>(exl);
    StageSeg r0{exg + it.u0, exd, it.u1 - it.u0};
    StageSeg r1{exg, exd, 0};
    const int w0 = it.tile * WT;
    const size_t tn = (size_t)it.tile * nm * WT, tc = (size_t)it.tile * n * WT;
    const double *tabd = it.spin == 0 ? tab0 : tab1;
    if (fused) {
        // c = A^-1 e_i: column `row` of each walker's inverse (its rows are
        // contiguous per walker)
        const StageSeg none{exg, exd, 0};
        StageSeg st{(G4)(MDE_G(double, S.T) + tn), reinterpret_cast<u32x4_t *>(tabs),
                    nm * WT * 8 / 16};
        const int nn = n * n, row = mv.row;
        for (int idx = tid; idx < n * WT; idx += nthr) {
            const int r = idx >> 6, l = idx & 63, w = w0 + l;
            cs[idx] = (TT)(w < W ? MDE_G(double, S.B)[(size_t)w * nn + r * n + row] : 0.0);
        }
        stage_segs(r0, r1, st, none, tid, nthr);
        for (int q = 0; q < m; ++q) Wl[q * 64] = 0.0;
    } else if (MODE == DM_PROPOSE) {
        const void *tsrc = sizeof(TT) == 8 ? (const void *)S.T : (const void *)I.Tp32;
        const void *csrc = sizeof(TT) == 8 ? (const void *)I.cc : (const void *)I.cc32;
        StageSeg st{(G4)(reinterpret_cast<const TT *>(tsrc) + tn),
                    reinterpret_cast<u32x4_t *>(tabs), nm * WT * (int)sizeof(TT) / 16};
        StageSeg sc{(G4)(reinterpret_cast<const TT *>(csrc) + tc),
                    reinterpret_cast<u32x4_t *>(cs), n * WT * (int)sizeof(TT) / 16};
        stage_segs(r0, r1, st, sc, tid, nthr);
        for (int q = 0; q < m; ++q) Wl[q * 64] = 0.0;
    } else if (tabd) {
        StageSeg none{exg, exd, 0};
        stage_segs(r0, r1, none, none, tid, nthr);
        // caller's tables, per-walker layout [W][n][m]
        for (int idx = tid; idx < nm * WT; idx += nthr) {
            const int l = idx / nm, e = idx - l * nm, w = w0 + l;
            tabs[e * WTP + l] = (w < W) ? (TT)MDE_G(double, tabd)[(size_t)w * nm + e] : TT(0);
        }
    } else {
        const void *tsrc = sizeof(TT) == 8 ? (const void *)S.T : (const void *)S.T32;
        StageSeg st{(G4)(reinterpret_cast<const TT *>(tsrc) + tn),
                    reinterpret_cast<u32x4_t *>(tabs), nm * WT * (int)sizeof(TT) / 16};
        StageSeg none{exg, exd, 0};
        stage_segs(r0, r1, st, none, tid, nthr);
    }
    __syncthreads();
    double acc[NSUM] = {0, 0, 0, 0, 0, 0};
    {
        // each wave takes one cost-balanced range of the item, order by
        // order, in reverse: the ranges run from the dense block (cheapest
        // per unit of cost) to the sparse high orders, and a SIMD issues its
        // older waves first, so the last ranges go to the first waves
        const int ws = __builtin_amdgcn_readfirstlane(nw - 1 - wave);
        const int j0 = bounds[it.wb + 2 * ws], j1 = bounds[it.wb + 2 * ws + 1];
        for (int k = 1; k <= S.max_order; ++k) {
            const int a = max(j0, S.order_start[k]), b = min(j1, S.order_start[k + 1]);
            if (a >= b) continue;
            if (k <= 2 && ((S.dense_k >> (k - 1)) & 1)) {
                det_dense_m<TT, MODE>(S, k, it.tile, a, b, tabs, cs, lane, Wl, acc);
                continue;
            }
            const int rb = it.u0;
            switch (k) {
                case 1: det_runs64<1, TT, MODE>(S, it.tile, a, b, exw, rb, tabs, cs, lane, Wl, acc); break;
                case 2: det_runs64<2, TT, MODE>(S, it.tile, a, b, exw, rb, tabs, cs, lane, Wl, acc); break;
                case 3: det_direct64<3, TT, MODE>(S, it.tile, a, b, exw, rb, tabs, cs, lane, Wl, acc); break;
                case 4: det_direct64<4, TT, MODE>(S, it.tile, a, b, exw, rb, tabs, cs, lane, Wl, acc); break;
                default:
                    if constexpr (GEN)
                        det_generic64<TT, MODE>(S, it.tile, k, a, b, exw, rb, tabs, cs, lane, Wl, acc);
                    break;
            }
        }
    }
    if (MODE != DM_PROPOSE) {
        __syncthreads();   // LDS is restaged by the next item
        return;
    }
    if constexpr (sizeof(TT) == 8) {
        if (fused) {
            item64_fused_end(it, I, S, mv, tabs, cs, Wall, Vs, tab_raw, acc, tid, nthr);
            return;
        }
    }
    // e^b[q] of this thread's particles q = wave + i * nw, loaded before the
    // barrier (their latency overlaps the slowest wave)
    const auto eg = MDE_G(TT, sizeof(TT) == 8 ? (const void *)I.ev : (const void *)I.ev32) +
                    (size_t)it.tile * NE * m * WT + lane;
    double ev[QPT][NE];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const int q = min(wave + i * nw, m - 1);
#pragma unroll
        for (int b = 0; b < NE; ++b) ev[i][b] = (double)eg[(size_t)(q * NE + b) * WT];
    }
    __syncthreads();
    // W summed over the waves (wave order) and contracted with e, particle order
    double part[NE];
#pragma unroll
    for (int b = 0; b < NE; ++b) part[b] = 0.0;
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const int q = wave + i * nw;
        if (q >= m) break;
        double w = 0.0;
        for (int v = 0; v < nw; ++v) w += Wall[((size_t)v * m + q) * 64 + lane];
#pragma unroll
        for (int b = 0; b < NE; ++b) part[b] = fma(w, ev[i][b], part[b]);
    }
    for (int q = wave + QPT * nw; q < m; q += nw) {
        double w = 0.0;
        for (int v = 0; v < nw; ++v) w += Wall[((size_t)v * m + q) * 64 + lane];
#pragma unroll
        for (int b = 0; b < NE; ++b) part[b] = fma(w, (double)eg[(size_t)(q * NE + b) * WT], part[b]);
    }
    __syncthreads();   // W has been read: the LDS holds the reduction now
    double *red = reinterpret_cast<double *>(tab_raw);   // [nw][64][NSUM]
    double *red2 = red + (size_t)nw * 64 * NSUM;          // [nw][64][NE]
#pragma unroll
    for (int q = 0; q < NSUM; ++q) red[(wave * 64 + lane) * NSUM + q] = acc[q];
#pragma unroll
    for (int b = 0; b < NE; ++b) red2[(wave * 64 + lane) * NE + b] = part[b];
    __syncthreads();
    const auto pout = MDE_GW(double, S.partial);
    for (int idx = tid; idx < 64 * NSUM; idx += nthr) {
        const int l = idx / NSUM, q = idx - l * NSUM;
        double sum = 0.0;
        for (int v = 0; v < nw; ++v) sum += red[(v * 64 + l) * NSUM + q];
        if (q >= 1 && q - 1 < NE)
            for (int v = 0; v < nw; ++v) sum += red2[(v * 64 + l) * NE + (q - 1)];
        pout[((size_t)it.slot * 64 + l) * NSUM + q] = sum;
    }
    __syncthreads();
}

// GEN: the instantiation also evaluates orders 5..8 (elimination with
// pivoting, whose 8 x 8 arrays live in scratch); expansions of orders up to
// 4 run the instantiation without them.
template <typename TT, int MODE, int WT, bool GEN>
__global__ void __launch_bounds__(WT == 64 ? DET64_THREADS : 1024)
k_det(const InstDev *__restrict__ insts, const WorkItem *__restrict__ items,
      const int32_t *__restrict__ bounds, ItemQueues qs,
      int ex_cap, const MoveArgs *__restrict__ moves, MoveArgs m1, int32_t *__restrict__ counter,
      const double *tab0, const double *tab1) {
    extern __shared__ uint4 smem4[];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int wl = tid % WT;
    const int slot = tid / WT;
    const int nslot = nthr / WT;
    uint4 *exl = smem4;
    unsigned char *tab_raw = reinterpret_cast<unsigned char *>(smem4 + ex_cap);
    // Items of queue x: the first (blocks on XCD x) are taken statically, one
    // per block, without an atomic; the rest are claimed through counter[x].
    // A block whose queue is drained claims from the other queues (their
    // counters are read by eight lanes at once before any atomic is spent:
    // device-scope atomics cross the dies and cost microseconds each).
    const int home = blockIdx.x % NXCD, hb = blockIdx.x / NXCD;
    auto blocks_on = [&](int x) { return ((int)gridDim.x - x + NXCD - 1) / NXCD; };
    int stage = 0;   // 0: static item, 1: home queue, 2: other queues, 3: none left
    for (;;) {
        if (tid < 64) {
            const int lane = tid;
            int got = -1;
            if (stage == 0) {
                stage = 1;
                if (hb < qs.off[home + 1] - qs.off[home]) got = qs.off[home] + hb;
            }
            if (got < 0 && stage == 1) {
                const int nb = blocks_on(home), sz = qs.off[home + 1] - qs.off[home];
                if (nb < sz) {
                    int k = 0;
                    if (lane == 0) k = atomicAdd(&counter[home], 1);
                    k = __shfl(k, 0, 64);
                    if (nb + k < sz) got = qs.off[home] + nb + k;
                }
                if (got < 0) stage = 2;
            }
            if (got < 0 && stage == 2) {
                int avail = 0, x = 0, nb = 0, sz = 0;
                if (lane < NXCD - 1) {
                    x = (home + 1 + lane) % NXCD;
                    nb = blocks_on(x);
                    sz = qs.off[x + 1] - qs.off[x];
                    if (nb < sz)
                        avail = nb + __hip_atomic_load(&counter[x], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT) < sz;
                }
                unsigned long long mask = __ballot(avail);
                while (mask != 0ull && got < 0) {
                    const int q = __ffsll((long long)mask) - 1;
                    const int qx = __shfl(x, q, 64), qnb = __shfl(nb, q, 64), qsz = __shfl(sz, q, 64);
                    int k = 0;
                    if (lane == 0) k = atomicAdd(&counter[qx], 1);
                    k = __shfl(k, 0, 64);
                    if (qnb + k < qsz) got = qs.off[qx] + qnb + k;
                    mask &= mask - 1ull;
                }
                if (got < 0) stage = 3;
            }
            if (lane == 0) s_item = got;
        }
        __syncthreads();        const int gi = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (gi < 0) break;
        WorkItem it = items[gi];
        it.inst = __builtin_amdgcn_readfirstlane(it.inst);
        it.spin = __builtin_amdgcn_readfirstlane(it.spin);
        it.tile = __builtin_amdgcn_readfirstlane(it.tile);
        it.order = __builtin_amdgcn_readfirstlane(it.order);
        it.u0 = __builtin_amdgcn_readfirstlane(it.u0);
        it.u1 = __builtin_amdgcn_readfirstlane(it.u1);
        it.slot = __builtin_amdgcn_readfirstlane(it.slot);
        it.wb = __builtin_amdgcn_readfirstlane(it.wb);
        it.d0 = __builtin_amdgcn_readfirstlane(it.d0);
        it.d1 = __builtin_amdgcn_readfirstlane(it.d1);
        const InstDev &I = insts[it.inst];
        const SpinDev &S = I.s[it.spin];
        if (MODE == DM_PROPOSE) {
            const int mspin = moves ? moves[it.inst].spin : m1.spin;
            if (mspin != it.spin) continue;
        }
        if (WT == 64) {
            const MoveArgs mv = moves ? moves[it.inst] : m1;
            item64<TT, MODE, GEN>(it, I, S, mv, exl, tab_raw, bounds, tid, nthr, tab0, tab1);
            continue;
        }
        const int n = S.n, m = S.m, WTP = S.WTP, W = I.W;
        TT *tabs = reinterpret_cast<TT *>(tab_raw);
        constexpr int NE = sizeof(TT) == 8 ? 5 : 4;
        TT *gs = tabs + n * m * WTP;          // e^b[p] rows
        TT *cs = gs + NE * m * WTP;
        const int w0 = it.tile * WT;
        const int nm = n * m;
        // ---- stage the walker tile's tables ----
        // (the lanes read their excitation records straight from global
        // memory, where consecutive slots read consecutive records: no LDS
        // for records, so an item may span a whole order however large the
        // tables are)
        const uint4 *recs = S.ex + it.u0;
        // tables are stored walker-tiled ([tile][e][WT]): straight copies into
        // the padded LDS rows, no index division
        if (MODE == DM_PROPOSE) {
            const size_t tn = (size_t)it.tile * nm * WT, tg = (size_t)it.tile * NE * m * WT,
                         tc = (size_t)it.tile * n * WT;
            if (sizeof(TT) == 8) {
                stage_rows<WT>(tabs, MDE_G(double, S.T) + tn, nm * WT, WTP, tid, nthr);
                stage_rows<WT>(gs, MDE_G(double, I.ev) + tg, NE * m * WT, WTP, tid, nthr);
                stage_rows<WT>(cs, MDE_G(double, I.cc) + tc, n * WT, WTP, tid, nthr);
            } else {
                stage_rows<WT>(tabs, MDE_G(float, I.Tp32) + tn, nm * WT, WTP, tid, nthr);
                stage_rows<WT>(gs, MDE_G(float, I.ev32) + tg, NE * m * WT, WTP, tid, nthr);
                stage_rows<WT>(cs, MDE_G(float, I.cc32) + tc, n * WT, WTP, tid, nthr);
            }
        } else {
            const double *tabd = it.spin == 0 ? tab0 : tab1;
            if (tabd) {
                // caller's tables, per-walker layout [W][n][m]
                for (int idx = tid; idx < nm * WT; idx += nthr) {
                    const int l = idx / nm, e = idx - l * nm, w = w0 + l;
                    tabs[e * WTP + l] = (w < W) ? (TT)MDE_G(double, tabd)[(size_t)w * nm + e] : TT(0);
                }
            } else {
                const size_t tn = (size_t)it.tile * nm * WT;
                const TT *tsrc = reinterpret_cast<const TT *>(sizeof(TT) == 8 ? (const void *)S.T
                                                                               : (const void *)S.T32);
                stage_rows<WT>(tabs, MDE_G(TT, tsrc) + tn, nm * WT, WTP, tid, nthr);
            }
        }
        __syncthreads();
        double acc[NSUM] = {0, 0, 0, 0, 0, 0};
        switch (it.order) {
            case 1: det_loop<1, TT, MODE, WT>(it, S, recs, tabs, gs, cs, wl, slot, nslot, acc); break;
            case 2: det_loop<2, TT, MODE, WT>(it, S, recs, tabs, gs, cs, wl, slot, nslot, acc); break;
            case 3: det_loop<3, TT, MODE, WT>(it, S, recs, tabs, gs, cs, wl, slot, nslot, acc); break;
            case 4: det_loop<4, TT, MODE, WT>(it, S, recs, tabs, gs, cs, wl, slot, nslot, acc); break;
            default:
                if constexpr (GEN) det_loop<0, TT, MODE, WT>(it, S, recs, tabs, gs, cs, wl, slot, nslot, acc);
                break;
        }
        __syncthreads();   // tables no longer needed: reuse LDS for the reduction
        if (MODE == DM_PROPOSE) {
            // lanes with the same wl hold sums over different excitation
            // slots: fixed butterfly over the slot bits, then over waves
#pragma unroll
            for (int off = WT; off < 64; off <<= 1)
#pragma unroll
                for (int q = 0; q < NSUM; ++q) acc[q] += __shfl_xor(acc[q], off, 64);
            double *red = reinterpret_cast<double *>(tab_raw);
            const int wave = tid >> 6, lane = tid & 63;
            const int nw = nthr >> 6;
            if (lane < WT) {
#pragma unroll
                for (int q = 0; q < NSUM; ++q) red[(wave * WT + lane) * NSUM + q] = acc[q];
            }
            __syncthreads();
            const auto part = MDE_GW(double, S.partial);
            for (int idx = tid; idx < WT * NSUM; idx += nthr) {
                const int l = idx / NSUM, q = idx - l * NSUM;
                double s = 0.0;
                for (int v = 0; v < nw; ++v) s += red[(v * WT + l) * NSUM + q];
                part[((size_t)it.slot * WT + l) * NSUM + q] = s;
            }
            __syncthreads();
        }
    }
    // the last block out resets the queues for the next launch
    if (tid == 0) {
        __threadfence();
        const int done = atomicAdd(&counter[NXCD], 1);
        if (done == (int)gridDim.x - 1) {
            for (int x = 0; x <= NXCD; ++x)
                __hip_atomic_store(&counter[x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <typename TT, int MODE, bool GEN>
static hipError_t launch_det_wt(int WT, hipStream_t st, const InstDev *d_insts,
                                const WorkItem *items, const int32_t *bounds,
                                const ItemQueues &qs, int ex_cap,
                                const MoveArgs *d_moves, const MoveArgs &m1, size_t lds,
                                int threads, int grid, int32_t *counter, const double *t0,
                                const double *t1) {
#define MDE_DET_CASE(X)                                                                     \
    case X: {                                                                               \
        auto fn = k_det<TT, MODE, X, GEN>;                                                  \
        if (lds > 65536)                                                                    \
            (void)hipFuncSetAttribute((const void *)fn,                                     \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), lds, st, d_insts, items, bounds, qs, \
                           ex_cap, d_moves, m1, counter, t0, t1);                           \
        return hipGetLastError();                                                           \
    }
    switch (WT) {
        MDE_DET_CASE(1)
        MDE_DET_CASE(2)
        MDE_DET_CASE(4)
        MDE_DET_CASE(8)
        MDE_DET_CASE(16)
        MDE_DET_CASE(32)
        MDE_DET_CASE(64)
        default: return hipErrorInvalidValue;
    }
#undef MDE_DET_CASE
}

hipError_t launch_det(hipStream_t st, const InstDev *d_insts, int n_inst, const WorkItem *items,
                      const int32_t *bounds, const ItemQueues &qs, int ex_cap, const MoveArgs *d_moves, const MoveArgs &m1,
                      int mode, int prec, int WT, size_t lds, int threads, int grid,
                      int32_t *counter, const double *tab0, const double *tab1, int max_order) {
    // every instance of one launch uses the same walker tile WT
    (void)n_inst;
    if (qs.off[NXCD] <= 0) return hipSuccess;
#define MDE_DET_GEN(TT, MD, G)                                                                  \
    return launch_det_wt<TT, MD, G>(WT, st, d_insts, items, bounds, qs, ex_cap, d_moves, m1, lds, \
                                    threads, grid, counter, tab0, tab1)
    const bool gen = max_order > 4;
    if (prec == 0) {
        if (mode == DM_PROPOSE) {
            if (gen) MDE_DET_GEN(double, DM_PROPOSE, true);
            MDE_DET_GEN(double, DM_PROPOSE, false);
        }
        if (gen) MDE_DET_GEN(double, DM_VALUES, true);
        MDE_DET_GEN(double, DM_VALUES, false);
    }
    if (mode == DM_PROPOSE) {
        if (gen) MDE_DET_GEN(float, DM_PROPOSE, true);
        MDE_DET_GEN(float, DM_PROPOSE, false);
    }
    if (gen) MDE_DET_GEN(float, DM_VALUES, true);
    MDE_DET_GEN(float, DM_VALUES, false);
#undef MDE_DET_GEN
}

// ---------------------------------------------------------------------------
// CI precontraction: C_sigma[u] = sum over CI terms with this spin's
// excitation u of c_I R_other[d(I)] -- an exact regrouping of the CI sum of
// Sec. III by the moving spin's excitation (R_other does not change while
// electrons of spin sigma move).  Terms are visited in a fixed order, four
// independent loads at a time.
// ---------------------------------------------------------------------------

__global__ void k_coef_gather(const InstDev *__restrict__ insts, const double *__restrict__ coef) {
    const InstDev &I = insts[0];
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)I.n_det) return;
#pragma unroll
    for (int s = 0; s < 2; ++s)
        MDE_GW(double, I.s[s].coef_s)[k] = MDE_G(double, coef)[MDE_G(int32_t, I.s[s].ci_idx)[k]];
}

hipError_t launch_coef_gather(hipStream_t st, const InstDev *d_inst, const InstDev &h,
                              const double *coef) {
    const size_t n = (size_t)h.n_det;
    hipLaunchKernelGGL(k_coef_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d_inst,
                       coef);
    return hipGetLastError();
}

// Work units: chunks of consecutive excitations whose CI segments are short
// (chunk boundaries fall on excitation boundaries, about 64 terms each), and
// pieces of at most 64 terms of the long segments (the reference excitation
// is shared by every determinant that excites only the other spin).  A
// thread streams the terms of its unit for one walker, eight independent
// loads at a time; chunk units write C[u] directly, piece units write
// partial sums that k_pc_fix adds in piece order.
template <int WT>
__global__ void __launch_bounds__(256)
k_precontract(const InstDev *__restrict__ insts, int spin, int ublocks) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[spin];
    const SpinDev &O = I.s[1 - spin];
    constexpr int per_block = 256 / WT;
    const int wl = threadIdx.x % WT;
    // walker tile t runs on die t % 8, all unit blocks of a tile in a row:
    // the other spin's ratios of the tile stay in that die's L2 while its
    // CI terms gather them
    const int L = blockIdx.x, x = L % NXCD, li = L / NXCD;
    const int t = (li / ublocks) * NXCD + x, ub = li % ublocks;
    if (t >= S.n_tiles) return;
    int unit = ub * per_block + threadIdx.x / WT;
    if (WT == 64) unit = __builtin_amdgcn_readfirstlane(unit);
    if (unit >= S.n_chunks + S.n_pieces) return;
    const auto seg = MDE_G(int32_t, S.ci_seg);
    const auto oth = MDE_G(int32_t, S.ci_other);
    const auto cf = MDE_G(double, S.coef_s);
    const auto Ro = MDE_G(double, O.R) + (size_t)t * O.U * WT + wl;
    int u, u1, k0, k1, kend;
    double *out;
    size_t ostride;
    if (unit < S.n_chunks) {
        u = S.chunks[2 * unit];
        u1 = S.chunks[2 * unit + 1];
        k0 = seg[u];
        k1 = seg[u1];
        kend = seg[u + 1];
        out = S.C + (size_t)t * S.U * WT + wl;
        ostride = WT;
    } else {
        const int4 pc = S.pieces[unit - S.n_chunks];
        u = 0;
        u1 = 1;
        k0 = pc.y;
        k1 = pc.z;
        kend = pc.z;
        out = S.pc_part + ((size_t)(unit - S.n_chunks) * S.n_tiles + t) * WT + wl;
        ostride = 0;
    }
    const auto Cw = MDE_GW(double, out);
    double s = 0.0;
    if (WT == 64) {
        // One unit per wave, lanes = the tile's walkers.  The unit's terms
        // (other-spin excitation, coefficient, segment end) are uniform and
        // read-only: scalar loads, PC_BATCH terms at a time, with the PC_BATCH ratio
        // gathers in flight together.  A short segment's last term carries
        // its excitation, where the sum is written; excitations without
        // terms keep the zero the array was cleared to.  The weights are
        // stored non-temporally: they are read back only by later launches,
        // and the other spin's ratios the gathers reuse stay in L2.
        const int kb = __builtin_amdgcn_readfirstlane(k0);
        const int nk = __builtin_amdgcn_readfirstlane(k1) - kb;
        const auto oth_k = MDE_K(int32_t, S.ci_other) + kb;
        const auto end_k = MDE_K(int32_t, S.ci_end) + kb;
        const auto cf_k = MDE_K(double, S.coef_s) + kb;
        const bool chunk = ostride != 0;
        // past nk the loads read the next unit's terms or the padding:
        // valid indices, never used.  The next batch's gathers are issued
        // before this batch is summed.
        double r[PC_BATCH];
        {
            int oi[PC_BATCH];
#pragma unroll
            for (int i = 0; i < PC_BATCH; ++i) oi[i] = oth_k[i];
#pragma unroll
            for (int i = 0; i < PC_BATCH; ++i) r[i] = Ro[(size_t)oi[i] * WT];
        }
        for (int tb = 0; tb < nk; tb += PC_BATCH) {
            int we[PC_BATCH];
            double c[PC_BATCH], rn[PC_BATCH];
#pragma unroll
            for (int i = 0; i < PC_BATCH; ++i) {
                we[i] = end_k[tb + i];
                c[i] = cf_k[tb + i];
            }
            if (tb + PC_BATCH < nk) {
                int oi[PC_BATCH];
#pragma unroll
                for (int i = 0; i < PC_BATCH; ++i) oi[i] = oth_k[tb + PC_BATCH + i];
#pragma unroll
                for (int i = 0; i < PC_BATCH; ++i) rn[i] = Ro[(size_t)oi[i] * WT];
            }
            // keep those loads ahead of this batch's sums (an empty asm with
            // a memory clobber emits nothing)
            __asm__ volatile("" ::: "memory");
#pragma unroll
            for (int i = 0; i < PC_BATCH; ++i) {
                if (tb + i < nk) {
                    s = fma(c[i], r[i], s);
                    if (chunk && we[i] >= 0) {
                        __builtin_nontemporal_store(s, &Cw[(size_t)we[i] * WT]);
                        s = 0.0;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < PC_BATCH; ++i) r[i] = rn[i];
        }
        if (chunk) u = u1;
    } else
    for (int k = k0; k < k1; k += 8) {
        int o[8];
        double c[8], r[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool ok = k + j < k1;
            o[j] = ok ? oth[k + j] : 0;
            c[j] = ok ? cf[k + j] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) r[j] = (k + j < k1) ? Ro[(size_t)o[j] * WT] : 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (k + j < k1) {
                while (k + j >= kend) {
                    Cw[(size_t)u * ostride] = s;
                    s = 0.0;
                    ++u;
                    kend = seg[u + 1];
                }
                s = fma(c[j], r[j], s);
            }
        }
    }
    for (; u < u1; ++u) {
        Cw[(size_t)u * ostride] = s;
        s = 0.0;
    }
}

// C[u] of each long segment = sum of its pieces' partial sums, in order
__global__ void __launch_bounds__(256) k_pc_fix(const InstDev *__restrict__ insts, int spin) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[spin];
    const int WT = S.WT;
    const int idx = blockIdx.y * 256 + threadIdx.x;
    const int lg = idx / WT, wl = idx % WT, t = blockIdx.x;
    if (lg >= S.n_longs) return;
    const int4 L = S.longs[lg];
    double s = 0.0;
    const auto pp = MDE_G(double, S.pc_part) + (size_t)t * WT + wl;
    const size_t ps = (size_t)S.n_tiles * WT;
    int p = L.y;
    // eight independent loads in flight, added in piece order
    for (; p + 8 <= L.z; p += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = pp[(size_t)(p + k) * ps];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; p < L.z; ++p) s += pp[(size_t)p * ps];
    MDE_GW(double, S.C)[((size_t)t * S.U + L.x) * WT + wl] = s;
}

hipError_t launch_precontract(hipStream_t st, const InstDev *d_inst, const InstDev &h, int spin,
                              const double *coef) {
    (void)coef;
    const SpinDev &S = h.s[spin];
    const int per_block = 256 / S.WT;
    const int units = S.n_chunks + S.n_pieces;
    const int ublocks = (units + per_block - 1) / per_block;
    const int T8 = (S.n_tiles + NXCD - 1) / NXCD * NXCD;
    dim3 grid(T8 * ublocks);
#define MDE_PC(X)                                                                       \
    case X:                                                                             \
        hipLaunchKernelGGL(k_precontract<X>, grid, dim3(256), 0, st, d_inst, spin, ublocks); \
        break;
    switch (S.WT) {
        MDE_PC(1) MDE_PC(2) MDE_PC(4) MDE_PC(8) MDE_PC(16) MDE_PC(32) MDE_PC(64)
        default: return hipErrorInvalidValue;
    }
#undef MDE_PC
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || S.n_longs == 0) return e;
    dim3 g2(S.n_tiles, (S.n_longs * S.WT + 255) / 256);
    hipLaunchKernelGGL(k_pc_fix, g2, dim3(256), 0, st, d_inst, spin);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// N = sum_u C_up[u] R_up[u] per walker (thread per walker, u ascending),
// log|Psi| = log|D0up| + log|D0dn| + log|N|.
// ---------------------------------------------------------------------------

// phase 1: block (tile, part) sums u in part `part` of NSPLIT slices, fixed
// order inside (slots) and across slots; phase 2 adds the NSPLIT partials
__global__ void __launch_bounds__(256)
k_nsum_part(const InstDev *__restrict__ insts) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[0];
    const int WT = S.WT, t = blockIdx.x, part = blockIdx.y;
    const int wl = threadIdx.x % WT, slot = threadIdx.x / WT, nslot = blockDim.x / WT;
    const int uc = (S.U + NSPLIT - 1) / NSPLIT, u0 = part * uc, u1 = min(S.U, u0 + uc);
    const size_t base = (size_t)t * S.U * WT + wl;
    const auto Cb = MDE_G(double, S.C) + base;
    const auto Rb = MDE_G(double, S.R) + base;
    double s = 0.0;
    for (int u = u0 + slot; u < u1; u += nslot) s = fma(Cb[(size_t)u * WT], Rb[(size_t)u * WT], s);
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    if (slot != 0) return;
    for (int v = 1; v < nslot; ++v) s += red[v * WT + wl];
    MDE_GW(double, I.npart)[(size_t)part * S.n_tiles * WT + t * WT + wl] = s;
}

__global__ void k_nsum(const InstDev *__restrict__ insts, double *log_abs_psi, double *sign_psi,
                       int32_t *status, int with_ref) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[0];
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= I.W) return;
    double s = 0.0;
    for (int p = 0; p < NSPLIT; ++p) s += MDE_G(double, I.npart)[(size_t)p * S.n_tiles * S.WT + w];
    I.Nold[w] = s;
    int bits = I.st[w];
    if (!(s != 0.0) || !isfinite(s)) bits |= 8;
    // the reference determinant carries less than 1e-8 of Psi
    if (fabs(s) > REF_ILLCOND_N) bits |= 16;
    I.st[w] = bits;
    double la = log(fabs(s));
    double sg = (s > 0.0) ? 1.0 : (s < 0.0 ? -1.0 : 0.0);
    if (with_ref) {
        la += I.s[0].logdet[w] + I.s[1].logdet[w];
        sg *= I.s[0].sgn[w] * I.s[1].sgn[w];
    }
    if (log_abs_psi) log_abs_psi[w] = la;
    if (sign_psi) sign_psi[w] = sg;
    if (status) status[w] |= bits;
}

hipError_t launch_nsum(hipStream_t st, const InstDev *d_inst, const InstDev &h,
                       double *log_abs_psi, double *sign_psi, int32_t *status, int with_ref) {
    const SpinDev &S = h.s[0];
    hipLaunchKernelGGL(k_nsum_part, dim3(S.n_tiles, NSPLIT), dim3(256), 0, st, d_inst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nsum, dim3((h.W + 63) / 64), dim3(64), 0, st, d_inst, log_abs_psi,
                       sign_psi, status, with_ref);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// finish: per walker, sum the partials of its tile in slot order (the
// reference excitation adds C_0 to N) and form the ratio (Sec. III ratio
// eq.) and the derivatives (Sec. IV derivative eqs.).  FP64 form, with
// rho N' = rho N - Q:
//   ratio = rho N' / N,   grad^a = (kappa^a N + W^a) / (rho N'),
// Q and W^a the q- and w^a-sums.  Mixed forms, with N' the sum over the
// updated table and G^a the g^a-sums:
//   ratio = rho N' / N_old,   grad^a = ((kappa^a / rho) N' + G^a) / N'.
// ---------------------------------------------------------------------------

// the walker's results from its summed partials (C_0 included in sum[0]),
// its rho, kappa^a and status bits
__device__ __forceinline__ void finish_walker_v(const InstDev &I, const MoveArgs &mv, int w,
                                                const double (&sum)[NSUM], double rho,
                                                const double (&kap)[4], int st) {
    double ratio, rNp, d[4];
    const int prec = I.prec;
    if (prec == 0) {
        const double N = sum[0];
        rNp = fma(rho, N, -sum[1]);       // rho N'
        ratio = rNp / N;
        const double inv = 1.0 / rNp;
#pragma unroll
        for (int a = 0; a < 4; ++a) d[a] = fma(kap[a], N, sum[2 + a]) * inv;
        I.Nnew[w] = rNp / rho;
    } else {
        const double Np = sum[0], ir = 1.0 / rho;
        rNp = rho * Np;
        ratio = rNp / I.Nold[w];
        const double inv = 1.0 / Np;
#pragma unroll
        for (int a = 0; a < 4; ++a) d[a] = fma(kap[a] * ir, Np, sum[1 + a]) * inv;
        I.Nnew[w] = Np;
    }
    int bits = st & 2;
    if (!(rNp != 0.0) || !isfinite(rNp)) bits |= 8;
    if (fabs(I.Nnew[w]) > REF_ILLCOND_N) bits |= 16;
    if (!isfinite(ratio) || !isfinite(d[0]) || !isfinite(d[1]) || !isfinite(d[2]) || !isfinite(d[3]))
        bits |= 4;
    if (mv.ratio) mv.ratio[w] = ratio;
    if (mv.grad) {
        mv.grad[(size_t)w * 3 + 0] = d[0];
        mv.grad[(size_t)w * 3 + 1] = d[1];
        mv.grad[(size_t)w * 3 + 2] = d[2];
    }
    if (mv.lap) mv.lap[w] = d[3];
    if (mv.status && bits) mv.status[w] |= bits;
}

__device__ __forceinline__ void finish_walker(const InstDev &I, const MoveArgs &mv, int w,
                                              const double (&sum)[NSUM]) {
    const auto kp = MDE_G(double, I.kap) + (size_t)w * 4;
    const double kap[4] = {kp[0], kp[1], kp[2], kp[3]};
    finish_walker_v(I, mv, w, sum, I.rho[w], kap, I.st[w]);
}

__global__ void k_finish(const InstDev *__restrict__ insts, const MoveArgs *__restrict__ moves,
                         MoveArgs m1) {
    const int inst = blockIdx.y;
    const InstDev &I = insts[inst];
    const MoveArgs mv = moves ? moves[inst] : m1;
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= I.W) return;
    const SpinDev &S = I.s[mv.spin];
    const int WT = S.WT, t = w / WT, wl = w - t * WT;
    const double C0 = MDE_G(double, S.C)[(size_t)t * S.U * WT + wl];
    double sum[NSUM] = {C0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int spt = S.slots_per_tile;
    const int s0 = spt > 0 ? t * spt : MDE_G(int32_t, S.tile_slot)[t];
    const int s1 = spt > 0 ? s0 + spt : MDE_G(int32_t, S.tile_slot)[t + 1];
    const auto part = MDE_G(double, S.partial);
    // slots in order; the loads of four slots are issued before they are added
    int s = s0;
    for (; s + 4 <= s1; s += 4) {
        double v[4][NSUM];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < NSUM; ++q) v[k][q] = part[((size_t)(s + k) * WT + wl) * NSUM + q];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < NSUM; ++q) sum[q] += v[k][q];
    }
    for (; s < s1; ++s) {
#pragma unroll
        for (int q = 0; q < NSUM; ++q) sum[q] += part[((size_t)s * WT + wl) * NSUM + q];
    }
    finish_walker(I, mv, w, sum);
}

hipError_t launch_finish(hipStream_t st, const InstDev *d_insts, int n_inst, int maxW,
                         const MoveArgs *d_moves, const MoveArgs &m1, int32_t *counter) {
    (void)counter;
    const int threads = 64;
    hipLaunchKernelGGL(k_finish, dim3((maxW + threads - 1) / threads, n_inst), dim3(threads), 0, st,
                       d_insts, d_moves, m1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Finish of a proposal formed in the determinant kernel (FP64, 64-walker
// tiles), four threads per walker: c = A^-1 e_i, rho = a'.c and
// kappa^a = d^a_O.c (matrix determinant lemma, Sec. III), the results from
// the tile's partials (as k_finish), and for the commit c,
// r = a'^T A^-1 - e_i^T and the new orbital row (the commit forms
// q = a'^T T_V - phi'_V itself).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_post(const InstDev *__restrict__ insts, MoveArgs mv) {
    const InstDev &I = insts[0];
    const SpinDev &S = I.s[mv.spin];
    constexpr int WT = 64, NMAX = 8, NG = 4;
    const int t = blockIdx.x;              // block t runs on die t % 8, as the tile's items
    if (t >= S.n_tiles) return;
    const int n = S.n, no = S.no, nn = n * n, row = mv.row, W = I.W;
    // four threads per walker: thread g takes rows k = g, g + 4 of A^-1,
    // component(s) b = g (, 4) of the orbital block, a quarter of the row
    // copy, and g = 1 the partial sums
    const int l = threadIdx.x & 63, g = threadIdx.x >> 6, w = t * WT + l;
    const bool live = w < W;
    __shared__ double c_s[NMAX][WT], rr_s[NG][NMAX][WT], o_s[5][NMAX][WT], sum_s[NSUM][WT];
    const auto orb = MDE_G(double, mv.new_orb) + (size_t)(live ? w : 0) * 5 * no;
    const auto B = MDE_G(double, S.B) + (size_t)(live ? w : 0) * nn;
    double rr[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) rr[j] = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = g + h * NG;
        if (k < n && live) {
            double bk[NMAX];
#pragma unroll
            for (int j = 0; j < NMAX; ++j) bk[j] = j < n ? B[k * n + j] : 0.0;
            const double ak = orb[k];
#pragma unroll
            for (int j = 0; j < NMAX; ++j) rr[j] = fma(ak, bk[j], rr[j]);
            double ck = 0.0;
#pragma unroll
            for (int j = 0; j < NMAX; ++j)
                if (j == row) ck = bk[j];
            c_s[k][l] = ck;
        }
    }
#pragma unroll
    for (int j = 0; j < NMAX; ++j) rr_s[g][j][l] = rr[j];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int b = g + h * NG;
        if (b < 5 && live) {
            double ob[NMAX];
#pragma unroll
            for (int r = 0; r < NMAX; ++r) ob[r] = r < n ? orb[b * no + r] : 0.0;
#pragma unroll
            for (int r = 0; r < NMAX; ++r) o_s[b][r][l] = ob[r];
        }
    }
    if (g == 1 && live) {
        const double C0 = MDE_G(double, S.C)[(size_t)t * S.U * WT + l];
        double sum[NSUM] = {C0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const int spt = S.slots_per_tile;
        const int s0 = spt > 0 ? t * spt : MDE_G(int32_t, S.tile_slot)[t];
        const int s1 = spt > 0 ? s0 + spt : MDE_G(int32_t, S.tile_slot)[t + 1];
        const auto part = MDE_G(double, S.partial);
        // slots in order; the loads of four slots are issued before they are added
        int sl = s0;
        for (; sl + 4 <= s1; sl += 4) {
            double v[4][NSUM];
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int q = 0; q < NSUM; ++q) v[k][q] = part[((size_t)(sl + k) * WT + l) * NSUM + q];
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int q = 0; q < NSUM; ++q) sum[q] += v[k][q];
        }
        for (; sl < s1; ++sl) {
#pragma unroll
            for (int q = 0; q < NSUM; ++q) sum[q] += part[((size_t)sl * WT + l) * NSUM + q];
        }
#pragma unroll
        for (int q = 0; q < NSUM; ++q) sum_s[q][l] = sum[q];
    }
    // descriptor fields and the walker's status read before the first store
    // (a store through a pointer could otherwise alias them: each would be
    // read again, one round trip later)
    double *const nrow = I.newrow + (size_t)(live ? w : 0) * I.nomax;
    const auto rrow_g = MDE_GW(double, I.rrow) + (size_t)t * n * WT + l;
    const auto cc_g = MDE_GW(double, I.cc) + (size_t)t * n * WT + l;
    double *const rho_g = I.rho;
    double *const kap_g = I.kap;
    int32_t *const st_g = I.st;
    const int st_old = (g == 0 && live) ? st_g[w] : 0;
    if (live) {
        // this thread's quarter of the new orbital row, loaded, then stored
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = g + NG * i < no ? orb[g + NG * i] : 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (g + NG * i < no) nrow[g + NG * i] = v[i];
        for (int p = g + NG * 8; p < no; p += NG) nrow[p] = orb[p];
    }
    __syncthreads();
    if (!live || g > 1) return;
    if (g == 1) {
        // c and r = a'^T A^-1 - e_i^T for the commit (tiled like the tables)
        for (int j = 0; j < n; ++j) {
            double r = 0.0;
#pragma unroll
            for (int h = 0; h < NG; ++h) r += rr_s[h][j][l];
            rrow_g[(size_t)j * WT] = r - (j == row ? 1.0 : 0.0);
            cc_g[(size_t)j * WT] = c_s[j][l];
        }
        return;
    }
    // thread 0 of the walker: rho, kappa and the results
    double rk[5];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        double v = 0.0;
        for (int r = 0; r < n; ++r) v = fma(o_s[b][r][l], c_s[r][l], v);
        rk[b] = v;
    }
    rho_g[w] = rk[0];
#pragma unroll
    for (int b = 0; b < 4; ++b) kap_g[(size_t)w * 4 + b] = rk[1 + b];
    const int bits = (!isfinite(rk[0]) || fabs(rk[0]) < 1e-300) ? 2 : 0;
    const int st = (st_old & ~2) | bits;
    st_g[w] = st;
    double sum[NSUM];
#pragma unroll
    for (int q = 0; q < NSUM; ++q) sum[q] = sum_s[q][l];
    const double kap[4] = {rk[1], rk[2], rk[3], rk[4]};
    finish_walker_v(I, mv, w, sum, rk[0], kap, st);
}

hipError_t launch_post(hipStream_t st, const InstDev *d_inst, const MoveArgs &m1, int n_tiles,
                       int n_max) {
    if (n_max > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_post, dim3(n_tiles), dim3(256), 0, st, d_inst, m1);
    return hipGetLastError();
}

}  // namespace mde
