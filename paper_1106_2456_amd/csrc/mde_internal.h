// Internal device-side data structures and kernel launchers of libmde.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mde {

constexpr int MAXN = 64;     // electrons per spin
constexpr int MAXM = 256;    // virtual orbitals per spin
constexpr int MAXK = 8;      // excitation order
constexpr int NSUM = 6;      // sums over excitations: N, q-term, x, y, z, laplacian
// |Psi / (D0_up D0_dn)| above which a walker's reference determinant is
// flagged as near-singular (status bit 16: switch the reference)
constexpr double REF_ILLCOND_N = 1e8;

// One unit of determinant work: excitations [u0, u1) of spin `spin` for the
// walkers of tile `tile` of instance `inst`.  Results go to partial-sum slot
// `slot` of that instance and spin.  64-walker tiles: the range may span
// several orders and wave w of the block takes [bounds[wb + w],
// bounds[wb + w + 1]); smaller tiles: one order `order`, slot-strided.
// A work item: walker tile `tile` of instance `inst`, excitations [u0, u1)
// (records staged in LDS) and, on 64-walker tiles, also the dense-block
// excitations [d0, d1); wb indexes the per-wave (first, end) ranges.
struct WorkItem {
    int32_t inst, spin, tile, order;
    int32_t u0, u1, slot, wb;
    int32_t d0, d1;
};

// Per-spin device view of one instance.  Internal excitation order: sorted
// by order, then holes, then particles; index 0 is the reference.
struct SpinDev {
    int32_t n, m, no, U;          // electrons, virtuals, orbitals, excitations
    int32_t WT, WTP, n_tiles, n_slots;   // walker tile, LDS row stride
    int32_t order_start[MAXK + 2];       // first u of each order (k = 0..9)
    int32_t max_order;
    // Orders stored dense (bit k-1 for order k <= 2): every excitation of
    // the order is present, hole sets ascending, particles ascending within
    // a hole set, so a hole set's block is evaluated without records.
    int32_t dense_k;
    const uint4 *ex;          // [U] packed: bytes 0..7 holes, 8..15 particles - n
    const int32_t *ci_seg;    // [U+1] CI terms of this spin's excitation u
    const int32_t *ci_other;  // [n_det + PC_BATCH] other spin's excitation, per term (0 past the end)
    const int32_t *ci_end;    // [n_det + PC_BATCH] u when the term is the last of u's short CI
                              // segment, else -1
    const int32_t *ci_idx;    // [n_det] original determinant index, per term
    const int32_t *inv_off;   // [n*m+1] adjoint inverted index by entry
    const int32_t *inv_ent;   // packed (u << 6) | (j << 3) | l
    const int32_t *tile_slot; // [n_tiles+1] slots of each tile
    const WorkItem *items;    // [n_slots] work items of this spin
    double *Phi;     // [W][n][no] orbital values (current positions)
    double *B;       // [W][n][n] inverse of the reference matrix
    // Walker-tiled layout "[tile][e][WT]": element e of walker w sits at
    // ((w / WT) * E + e) * WT + w % WT, E the row length (here n*m).
    double *T;       // tiled [n*m] table, virtual block (FP64 mode)
    float *T32;      // tiled [n*m] table (mixed mode)
    float *PhiV32;   // [W][n][m] virtual orbital values in FP32 (mixed)
    double *logdet;  // [W] log|det A0|
    double *sgn;     // [W] sign det A0
    double *R;       // [n_tiles][U][WT] excited ratios at current positions
    double *C;       // [n_tiles][U][WT] CI weights: sum over terms of c_I R_other
    double *partial; // [n_slots][WT][NSUM]
    double *coef_s;  // [n_det + PC_BATCH] c_I in this spin's CI-term order
    const int32_t *chunks;   // [2*n_chunks] (first, end) excitation ranges of the precontraction
    const int4 *pieces;      // [n_pieces] (u, k0, k1, -) pieces of long CI segments
    const int4 *longs;       // [n_longs] (u, first piece, end piece, -)
    double *pc_part;         // [n_pieces][n_tiles][WT] partial sums of the pieces
    int32_t n_chunks, n_pieces, n_longs;
    int32_t n_user;          // excitations given by the caller (the dense fill follows them)
    int32_t slots_per_tile;  // k when every tile has k items (tile t's partial-sum
                             // slots are then [t k, t k + k)), else 0
};

// virtual-space sizes m for which the 64-walker kernel has a dense block
// evaluator of orders 1 and 2 (its particle loops are unrolled over m)
__host__ __device__ constexpr bool dense_m_supported(int m) {
    return m == 8 || m == 12 || m == 16 || m == 20 || m == 24;
}

// Units of a dense block handed to one wave: a single's unit is one hole
// (M excitations), a double's one hole pair (NP = M (M - 1) / 2).  The
// ring of CI weights in flight has PD entries, PD dividing NP, so an
// excitation's ring slot depends on its place in the pair only.  (The pair
// body is straight-line code: one unit per pair keeps the ring in fixed
// registers across pairs, with no wait for all loads at the loop edge.)
// All five shapes live in one kernel, whose register budget (256 per lane
// at 512 threads) is set by the deepest ring: rings of 20-38 doubles for
// every shape spilled the item loop's state to scratch on each dense entry
// (~20 MB of scratch write-back per launch); rings of 14-23 do not spill.
template <int M>
struct Dense2Shape {
    static constexpr int NP = M * (M - 1) / 2;
    static constexpr int G = 1;
    static constexpr int UNIT = NP / G;
    static constexpr int PD = M == 8 ? 14 : M == 12 ? 22 : M == 16 ? 20 : M == 20 ? 19 : 23;
    static_assert(NP % G == 0 && UNIT % PD == 0, "dense unit shape");
};

// first excitation and end of the dense block of a spin (orders 1 and 2
// when stored dense; singles are filled whenever doubles are, so the block
// is one range); da == db when there is none
__host__ __device__ inline void dense_range(const SpinDev &S, int &da, int &db) {
    const bool d1 = S.dense_k & 1, d2 = (S.dense_k >> 1) & 1;
    da = d1 ? S.order_start[1] : (d2 ? S.order_start[2] : 0);
    db = d2 ? S.order_start[3] : (d1 ? S.order_start[2] : 0);
}

struct InstDev {
    SpinDev s[2];
    int32_t W, prec, nmax, mmax, nomax, pad;
    int64_t n_det;
    const double *coef;   // [n_det] device copy
    double *Nold;    // [W] current multi-determinant sum N = Psi/(D0up D0dn)
    double *Nnew;    // [W] proposed N'
    double *rho;     // [W] det A'/det A
    // proposal of the moving spin (n, m of that spin), walker-tiled:
    double *cc;      // tiled [n]    c = A^-1 e_i
    double *kap;     // [W][4]       kappa^a = d^a_O . c
    double *ev;      // tiled [m][5] FP64 form: (q, w^x, w^y, w^z, w^L) per particle
    float *ev32;     // tiled [m][4] mixed forms: g^a of the updated table
    float *cc32;     // tiled [n]    mixed forms: c' = c / rho
    float *Tp32;     // tiled [n*m]  mixed forms: updated table T'_V
    float *Ap32;     // [W][nmax+4][nmax] MIXED_GEMM operand: rows of A'^-1, then e^a
    double *rrow;    // tiled [n]    a'^T A^-1 - e_i^T (for the commit)
    double *npart;   // [NSPLIT][n_tiles*WT] partial N sums
    double *newrow;  // [W][nomax] proposed orbital values of the moved electron
    int32_t *st;     // [W] internal status bits
    int32_t *counter;  // work-queue counter of the persistent kernel
    double *Lnew;    // [W] adjoint scratch: go / N per walker
    double *gz;      // [W][nmax * mmax] table gradient dN/dT / N of one spin (all-electron derivatives)
};

// Per-call move arguments (device array for groups, by value otherwise).
// MoveArgs.mode bit: the determinant kernel forms the proposal quantities
// itself (FP64 form on 64-walker tiles; no separate proposal launch)
constexpr int32_t MV_FUSED = 1;

struct MoveArgs {
    int32_t e, spin, row, mode;   // electron, its spin, its row in A, MV_ bits
    const double *new_orb;        // [W][5][no]
    double *ratio, *grad, *lap;
    int32_t *status;
    const uint8_t *accept;
};

enum DetMode { DM_PROPOSE = 0, DM_VALUES = 1 };

// Pointers read from descriptors are generic to the compiler; these casts
// make their loads global-memory loads (no LDS counter involvement).
#define MDE_G(T, p) ((const T __attribute__((address_space(1))) *)(p))
#define MDE_GW(T, p) ((T __attribute__((address_space(1))) *)(p))
// read-only for the whole launch (set up on the host): uniform reads become
// scalar loads
#define MDE_K(T, p) ((const T __attribute__((address_space(4))) *)(p))

// Largest excitation range of one work item (its records are staged in LDS).
constexpr int ITEM_MAX = 1024;
// threads of a 64-walker determinant block: eight waves, so each wave may
// hold a hole set's table rows in registers (up to 256 VGPRs)
constexpr int DET64_THREADS = 512;
// CI terms the 64-walker precontraction takes per step (the term arrays
// carry this many entries of padding)
constexpr int PC_BATCH = 16;
// LDS row stride of a walker tile's tables: 64-walker rows are read whole
// (one 512-byte row per wave) and need no padding; smaller tiles pad by one
// element against bank conflicts between lanes reading different rows
__host__ __device__ constexpr int lds_row_stride(int WT) {
    return WT == 64 ? 64 : (WT >= 8 ? WT + 1 : WT);
}

// The chip's workgroups are dispatched round-robin over its 8 accelerator
// dies (XCDs), each with its own L2.  Work on walker tile t is placed on XCD
// t % 8 by every per-move kernel, so a tile's tables stay in one L2.
constexpr int NXCD = 8;

// Work items grouped by XCD: queue x holds items [off[x], off[x+1]) (the
// tiles t with t % 8 == x); a block drains its own XCD's queue first, then
// helps the others.
struct ItemQueues {
    int32_t off[NXCD + 1];
};

// 1D grid of n_inst x T8 x split blocks (T8 = tiles rounded up to a multiple
// of 8): block L runs on XCD L % 8 and takes (instance, tile, part) with
// tile % 8 == L % 8.  Returns false for padding blocks.
__device__ __forceinline__ bool tile_of_block(int split, int T8, int n_inst, int &inst, int &t,
                                              int &part) {
    const int L = blockIdx.x, x = L % NXCD, li = L / NXCD;
    part = li % split;
    const int G = (li / split) * NXCD + x;
    inst = G / T8;
    t = G - inst * T8;
    return inst < n_inst;
}

// ---- launchers (stream-ordered) -------------------------------------------
// All launchers take the device array `insts` and either a single instance
// index range or work-item lists.

hipError_t launch_lu_inverse(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst,
                             int spin, const double *orb_in, int32_t *status);
// both of the above in one launch, a thread per walker (n <= 8); returns
// hipErrorInvalidValue for larger n
hipError_t launch_refresh_small(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst,
                                int spin, const double *orb_in, int32_t *status);
hipError_t launch_table_gemm(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst,
                             int spin);
hipError_t launch_propose(hipStream_t st, const InstDev *d_insts, int n_inst, int maxW,
                          const MoveArgs *d_moves, const MoveArgs &m1, int prec,
                          int nmax, int mmax, int WT, int max_tiles, int split);
hipError_t launch_det(hipStream_t st, const InstDev *d_insts, int n_inst,
                      const WorkItem *items, const int32_t *bounds, const ItemQueues &queues,
                      int ex_cap,
                      const MoveArgs *d_moves, const MoveArgs &m1, int mode, int prec,
                      int WT, size_t lds_bytes, int threads, int grid, int32_t *counter,
                      const double *tab0, const double *tab1, int max_order);
// smallest part count of the proposal whose LDS footprint fits lds_max (0: none)
int propose_split_limit(int nmax, int mmax, int WT, size_t lds_max);
hipError_t launch_post(hipStream_t st, const InstDev *d_inst, const MoveArgs &m1, int n_tiles,
                       int n_max);
hipError_t launch_finish(hipStream_t st, const InstDev *d_insts, int n_inst, int maxW,
                         const MoveArgs *d_moves, const MoveArgs &m1, int32_t *counter);
hipError_t launch_accept64f(hipStream_t st, const InstDev *d_inst, const MoveArgs &m1, int n_tiles,
                            int split, int n_max);
hipError_t launch_accept(hipStream_t st, const InstDev *d_insts, int n_inst, int maxW,
                         const MoveArgs *d_moves, const MoveArgs &m1, int prec,
                         int nmax, int mmax, int WT, int max_tiles, int split);
constexpr int NSPLIT = 16;   // parts of the excitation range in the N sum
hipError_t launch_precontract(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst,
                              int spin, const double *coef);
hipError_t launch_coef_gather(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst,
                              const double *coef);
hipError_t launch_nsum(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst,
                       double *log_abs_psi, double *sign_psi, int32_t *status, int with_ref);
hipError_t launch_init_misc(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst);
hipError_t launch_export(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst,
                         int what, int spin, double *dst, const int32_t *perm_user);
hipError_t launch_backward(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst,
                           const double *go, const double *Nw, const double *coef,
                           double *grad_coef, double *grad_T_up, double *grad_T_dn,
                           const double *T_up, const double *T_dn);
// table gradient of one spin, grad_T[w] = Lnew[w] dN/dT_V[w] ([W][n][m]);
// Tin NULL: the context's own (walker-tiled) table
hipError_t launch_grad_T(hipStream_t st, const InstDev *d_inst, const InstDev &h, int spin,
                         const double *Tin, double *grad_T);
// all-electron derivatives (k_local.hip): Lnew = 1 / N, then per spin from gz
hipError_t launch_inv_nold(hipStream_t st, const InstDev *d_inst, const InstDev &h);
// status[w] |= NONFINITE for walkers whose table gradients hold non-finite values
hipError_t launch_flag_nonfinite(hipStream_t st, int W, const double *a, int na, const double *b,
                                 int nb, int32_t *status);
size_t local_derivs_lds(int n, int m);
hipError_t launch_local_derivs(hipStream_t st, const InstDev *d_inst, const InstDev &h, int spin,
                               const double *orb, const double *Yn, double *grad, double *lap,
                               int32_t *status);
// the allocation-free variant's scratch: a device array of this many doubles
// (32 MiB), its address on the current device
constexpr size_t LOCAL_SCRATCH_DOUBLES = (size_t)4 << 20;
hipError_t local_scratch(double **out);
// Metropolis loop with drift (k_vmc.hip); phase 0 copies electron e's
// position to cur, phase 1 forms the proposal newp
hipError_t launch_vmc_drift(hipStream_t st, int W, int n_tot, int e, double tau, const double *pos,
                            const double *g0, const double *chi, double *cur, double *newp, int phase);
hipError_t launch_vmc_decide(hipStream_t st, int W, int n_tot, int e, double tau, double *pos,
                             const double *cur, const double *newp, const double *g0, const double *g1,
                             const double *ratio, const double *u, uint8_t *mask, int32_t *accepted);
hipError_t launch_eval_finish(hipStream_t st, const InstDev *d_inst, const InstDev &h_inst,
                              double *log_abs, double *sign, int32_t *status);
hipError_t launch_sgauss(hipStream_t st, int nb, const double *centres, const double *expo,
                         int n_orb, const double *mo, int npos, const double *pos,
                         double *out);
hipError_t launch_reset_counter(hipStream_t st, int32_t *counter);
// dst[r][q] = src[r][perm[q]] for rows x no values (reference switching)
hipError_t launch_permute_orbitals(hipStream_t st, const double *src, double *dst, int rows, int no,
                                   const int32_t *perm);
// copy n per-instance move arguments (host array) to d_moves, as kernel
// arguments (no host buffer is read when the copy runs)
hipError_t launch_set_moves(hipStream_t st, MoveArgs *d_moves, const MoveArgs *h_moves, int n);
hipError_t launch_fill_i32(hipStream_t st, int32_t *p, int32_t v, size_t n);

}  // namespace mde
