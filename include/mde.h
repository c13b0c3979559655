/*
 * mde.h -- C ABI of libmde.so: multi-determinant wave-function evaluation by
 * the table method on one AMD MI355X (gfx950) GPU.
 *
 * Problem statement (Sec. II): for each walker R = (r_1..r_N) and spin
 * sigma, the matrix M_sigma,k(i,j) = phi_j(r_i) (rows = electrons, columns =
 * orbitals), and
 *     Psi = sum_k alpha_k det M_up,k det M_dn,k            (Jastrow excluded)
 * where every M_sigma,k is the reference matrix (orbitals 0..n-1) with some
 * columns replaced by virtual orbitals n..n+m-1 (particle-hole excitations).
 * Per single-electron move the library returns Psi(R')/Psi(R),
 * grad_i ln Psi(R') and lap_i Psi(R')/Psi(R') (Sec. II quantities), using the
 * table T = A0^-1 Phi (Sec. III), r x r determinants of table entries
 * (Sec. III read-off, Algorithm 1 step 4), derivative tables (Sec. IV-A) and
 * the Sherman-Morrison update of A0^-1 (Sec. III, SM eq.).
 *
 * Conventions
 *  - Every function returns mde_status; MDE_OK is 0.  No exception crosses
 *    the ABI.  On failure mde_error_string(ctx) holds a message.
 *  - Arrays passed to init/propose/accept/eval/backward are DEVICE pointers
 *    owned by the caller (for example torch tensors).  Setup calls
 *    (mde_set_*) take HOST pointers and copy what they need.
 *  - All device work is ordered on the hipStream_t given to mde_create
 *    (NULL = the legacy default stream) and is asynchronous.  A context is
 *    not thread-safe; use one context per stream.
 *  - Internal state lives in a caller-allocated device workspace
 *    (mde_workspace_bytes, mde_bind_workspace): the library itself calls no
 *    device allocator after bind.
 *  - Row-major layouts, walker index slowest.  An orbital block is
 *    [5][n_orb]: component 0 = value, 1..3 = d/dx, d/dy, d/dz,
 *    4 = laplacian.  Electrons are numbered 0..n_up-1 (spin up) then
 *    n_up..n_up+n_dn-1 (spin down).  Orbitals 0..n_sigma-1 fill the reference
 *    determinant of spin sigma; orbitals n_sigma..n_orb_sigma-1 are virtual.
 *  - Excitation convention: an excitation is a list of (hole -> particle)
 *    pairs, holes ascending and particles ascending, paired in that order;
 *    the particle takes the hole's column.  Any other phase convention is
 *    folded into the CI coefficient by the caller.
 *  - Per-walker numerical problems do not fail a call: they set bits in a
 *    caller-provided int32 status[W] (MDE_ST_* below).  Bits accumulate
 *    (OR) until the caller clears the array.
 */
#ifndef MDE_H
#define MDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MDE_OK = 0,
    MDE_INVALID = 1,      /* bad argument (range, size, order of calls)      */
    MDE_NOMEM = 2,        /* workspace too small / host allocation failed    */
    MDE_DEVICE = 3,       /* a HIP runtime call failed                       */
    MDE_STATE = 4,        /* call not valid in the current state             */
    MDE_UNSUPPORTED = 5   /* size or mode outside what the library supports  */
} mde_status;

typedef enum {
    MDE_FP64 = 0,         /* every step in FP64 (the reference form)          */
    MDE_MIXED = 1,        /* tables stored in FP32 (half the LDS and memory
                             traffic of the determinant stage); the
                             Sherman-Morrison table update, the small
                             determinants, LU, denominators and CI sums are
                             computed in FP64                                 */
    MDE_MIXED_GEMM = 2,   /* as MDE_MIXED, but every proposal rebuilds the
                             table with one FP32 MFMA GEMM T' = A'^-1 Phi'_V
                             (Algorithm 1 step 3) instead of the rank-one
                             update, FP32 operands and FP32 accumulation over
                             all of K = n; its error scales with
                             |A'^-1| |Phi'_V| rather than |T'|              */
    MDE_MIXED_GEMM_KSUM64 = 3  /* as MDE_MIXED_GEMM, but each MFMA forms one
                             K-block of 4 in FP32 and the K-blocks are summed
                             in FP64 (an alternative with a smaller GEMM
                             error at the same operand precision)           */
} mde_precision;

/* per-walker status bits */
#define MDE_ST_SINGULAR_REF 1   /* zero pivot in the reference LU             */
#define MDE_ST_SMALL_RATIO  2   /* |det A'/det A| below 1e-300 or not finite  */
#define MDE_ST_NONFINITE    4   /* non-finite input or output                 */
#define MDE_ST_ZERO_PSI     8   /* multi-determinant sum exactly zero / NaN   */
#define MDE_ST_REF_ILLCOND 16   /* |Psi / (D0_up D0_dn)| > 1e8: the reference
                                   determinant is near-singular where Psi is
                                   not (Sec. V); switch the reference
                                   (mde_set_reference) for this walker       */

/* Limits of the library. */
#define MDE_MAX_ELEC  64        /* electrons per spin                         */
#define MDE_MAX_VIRT  256       /* virtual orbitals per spin                  */
#define MDE_MAX_ORDER 8         /* largest excitation order                   */

typedef struct mde_ctx mde_ctx;
typedef struct mde_group mde_group;
typedef struct mde_graph mde_graph;

typedef struct {
    int32_t n_elec[2];      /* electrons per spin, 1..MDE_MAX_ELEC            */
    int32_t n_orb[2];       /* orbitals per spin = n_elec + virtuals          */
    int32_t max_walkers;    /* upper bound on W for this context              */
    int32_t max_order;      /* largest excitation order, 1..MDE_MAX_ORDER     */
    int32_t refresh_every;  /* recompute A0^-1 and T from scratch after this
                               many accept calls (0 = never; default sweep)   */
    int32_t precision;      /* mde_precision                                  */
} mde_desc;

/* ---- lifetime ---------------------------------------------------------- */

/* Create a context for one wave function.  hip_stream: a hipStream_t (or
 * NULL).  The context keeps host metadata only until mde_bind_workspace. */
mde_status mde_create(const mde_desc *desc, void *hip_stream, mde_ctx **out);
mde_status mde_destroy(mde_ctx *ctx);
/* Last error message of ctx (static text if ctx is NULL); never NULL. */
const char *mde_error_string(const mde_ctx *ctx);
/* Library version string. */
const char *mde_version(void);

/* ---- the expansion (host pointers, copied) ----------------------------- */

/* Unique excitations of one spin in CSR form (Sec. II particle-hole
 * excitations; Sec. III table read-off).  Entry 0 must be the empty
 * excitation (the reference).  holes[offsets[u]..offsets[u+1]) are hole
 * indices in 0..n-1, ascending; particles[...] are orbital indices in
 * n..n_orb-1, ascending.  Orders above desc.max_order, repeated or
 * out-of-range indices give MDE_INVALID. */
mde_status mde_set_excitations(mde_ctx *ctx, int32_t spin, int32_t n_exc,
                               const int32_t *offsets, const int32_t *holes,
                               const int32_t *particles);

/* CI expansion (Sec. II Psi eq.): determinant I has coefficient coef[I] and
 * uses up excitation up_idx[I] and down excitation dn_idx[I].  Indices refer
 * to the lists given to mde_set_excitations (call that first). */
mde_status mde_set_ci(mde_ctx *ctx, int64_t n_det, const double *coef,
                      const int32_t *up_idx, const int32_t *dn_idx);

/* Reference switching (Sec. V: when the reference matrix is near-singular
 * while Psi is not, another determinant of the expansion serves as the
 * reference).  Makes the determinant with up excitation ref_up and down
 * excitation ref_dn (indices into the lists given to mde_set_excitations)
 * the reference of this context: its occupied orbitals become orbitals
 * 0..n-1 of the internal order, every excitation is rewritten relative to it
 * (its order can grow by the order of the new reference; MDE_UNSUPPORTED
 * above desc.max_order) and the sign of each determinant's column
 * reordering is folded into its coefficient, so Psi is unchanged.  Call
 * after mde_set_ci and before mde_bind_workspace; (0, 0) restores the
 * caller's reference.  Inputs keep the caller's orbital order (the library
 * permutes them); outputs of init/propose/grad_lap/local_derivs are the same
 * quantities; mde_export returns the rebased frame (ratios to the new
 * reference, its inverse, table and log|det|).  Contexts with a switched
 * reference cannot join a group (MDE_UNSUPPORTED). */
mde_status mde_set_reference(mde_ctx *ctx, int32_t ref_up, int32_t ref_dn);

/* ---- workspace --------------------------------------------------------- */

/* Device bytes needed for W walkers (W <= max_walkers). */
mde_status mde_workspace_bytes(const mde_ctx *ctx, int32_t W, size_t *bytes);
/* Bind caller-owned device memory (256-byte aligned, >= the size above for
 * the W passed there) and upload the expansion.  Synchronous. */
mde_status mde_bind_workspace(mde_ctx *ctx, int32_t W, void *dev, size_t bytes);

/* ---- evaluation (device pointers) -------------------------------------- */

/* From-scratch start (Sec. III: inverse and determinants computed once):
 * orb_up [W][n_up][5][n_orb_up], orb_dn [W][n_dn][5][n_orb_dn] hold every
 * electron's orbital block at its current position.  Computes A0^-1 by LU
 * with partial pivoting, T = A0^-1 Phi_V, all excited ratios and the CI sum.
 * Outputs log|Psi| and sign(Psi) per walker ([W] each, may be NULL).  W
 * must equal the walker count the workspace was bound for (MDE_INVALID). */
mde_status mde_init(mde_ctx *ctx, int32_t W, const double *orb_up, const double *orb_dn,
                    double *log_abs_psi, double *sign_psi, int32_t *status);

/* Recompute A0^-1, T and the sums from the orbital values the library keeps
 * (no inputs needed).  Same outputs as mde_init. */
mde_status mde_refresh(mde_ctx *ctx, double *log_abs_psi, double *sign_psi,
                       int32_t *status);

/* Proposal for electron e moving to r_e' (Algorithm 1; Sec. IV-A):
 * new_orb [W][5][n_orb_sigma(e)] is that electron's orbital block at r_e'.
 * Outputs ratio[W] = Psi(R')/Psi(R), grad[W][3] = grad_e ln Psi(R'),
 * lap[W] = lap_e Psi(R')/Psi(R').  The excited determinants at R' are read
 * from the current table through the matrix determinant lemma (the updated
 * table of Sec. III is formed only on acceptance), so no intermediate is
 * divided by det A'/det A; the outputs stay finite on the reference
 * determinant's node (MDE_ST_SMALL_RATIO then marks a move whose commit
 * would be singular).  State is unchanged until mde_accept. */
mde_status mde_propose(mde_ctx *ctx, int32_t e, const double *new_orb,
                       double *ratio, double *grad, double *lap, int32_t *status);

/* grad_e ln Psi(R) and lap_e Psi(R)/Psi(R) at the current position;
 * cur_orb [W][5][n_orb] is electron e's block at r_e.  Replaces any pending
 * proposal (accepting it afterwards changes nothing). */
mde_status mde_grad_lap(mde_ctx *ctx, int32_t e, const double *cur_orb,
                        double *grad, double *lap, int32_t *status);

/* grad_i ln Psi and lap_i Psi / Psi of every electron i at the current
 * positions (Sec. IV: the laplacian of all particles once per sweep, for
 * the kinetic energy).  orb_up [W][n_up][5][n_orb_up] and orb_dn hold every
 * electron's orbital block at its current position (the library keeps
 * values only).  Outputs grad [W][n_up + n_dn][3] and lap [W][n_up + n_dn]
 * (device, caller-owned); status bit MDE_ST_NONFINITE marks a walker with a
 * non-finite output.  Each excitation's derivative is the bordered
 * determinant of Sec. IV-A read at R; summed with the CI weights the
 * adjugate terms regroup by table entry into dN/dT_V (the table gradient),
 * so the call costs one cofactor gather over the excitations per spin plus
 * two n x n x m products per walker and spin.  FP64 form only
 * (MDE_UNSUPPORTED otherwise); leaves any pending proposal in place. */
mde_status mde_local_derivs(mde_ctx *ctx, const double *orb_up, const double *orb_dn,
                            double *grad, double *lap, int32_t *status);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation and outputs as mde_local_derivs, with its per-call
 * intermediate (the table gradient of one spin, W x n x m doubles) held in
 * a fixed device array of the library (32 MiB, 4 194 304 doubles, kept by
 * every GPU the library runs on until the process ends) instead of the
 * context's workspace.  The call itself allocates nothing.  MDE_UNSUPPORTED
 * when W x n x m of a spin exceeds that size.  All calls on one GPU share
 * the array: calls that overlap in time on one GPU (on different streams or
 * threads) race. */
mde_status mde_local_derivs_noalloc(mde_ctx *ctx, const double *orb_up, const double *orb_dn,
                                    double *grad, double *lap, int32_t *status);

/* Commit the pending proposal of electron e for walkers with accept[w] != 0
 * (uint8 [W]): Sherman-Morrison update of A0^-1 (Sec. III SM eq.), table,
 * reference determinant and CI sum.  Every refresh_every calls the state is
 * recomputed from scratch (mde_refresh without outputs); in the FP64
 * precision that refresh rebuilds A0^-1, T and log|det A0| only and keeps
 * the CI sum N of the moves (every FP64 proposal sums N over its own
 * determinants), and the excited ratios and CI weights are formed when the
 * next proposal or export needs them. */
mde_status mde_accept(mde_ctx *ctx, int32_t e, const uint8_t *accept);

/* Metropolis loop with drift, entirely on the device (Sec. II sampling of
 * |Psi|^2 by single-electron moves; the gradient evaluated at R for the
 * drift and at R' for the reverse move, "twice per step").  n_steps sweeps;
 * in each, electrons 0..n_up+n_dn-1 in order: g = grad_e ln Psi(R) (as
 * mde_grad_lap), r' = r_e + tau g + sqrt(tau) chi, ratio and g' at R' (as
 * mde_propose), accepted when u < |ratio|^2 G(r <- r') / G(r' <- r) with
 * G(b <- a) = exp(-|b - a - tau g(a)|^2 / (2 tau)), then committed (as
 * mde_accept).  Orbitals come from the s-Gaussian provider (set its basis
 * for both spins; MDE_STATE otherwise).  Random numbers are inputs:
 * normals [n_steps][n_up+n_dn][W][3] (chi) and uniforms
 * [n_steps][n_up+n_dn][W] (u), device.  pos [W][n_up+n_dn][3] (device,
 * in/out) holds the walkers' positions and must match the state of the last
 * mde_init; accepted [W] (int32, in/out) counts accepted moves.  No host
 * synchronisation: the loop can be captured into a graph (its host-side
 * refresh cadence is fixed at capture). */
mde_status mde_vmc(mde_ctx *ctx, int32_t n_steps, double tau, const double *normals,
                   const double *uniforms, double *pos, int32_t *accepted, int32_t *status);

/* Copy internal state for checks.  what: 0 = A0^-1 of spin s [W][n][n],
 * 1 = table T_V of spin s [W][n][m] (FP64; in MIXED mode converted from
 * FP32), 2 = excited ratios D_u/D_0 of spin s [W][n_exc] in the caller's
 * excitation order (current positions), 3 = log|det A0| of spin s [W],
 * 4 = multi-determinant sum N = Psi / (D0_up D0_dn) [W].  dst is a device
 * pointer of FP64. */
mde_status mde_export(mde_ctx *ctx, int32_t what, int32_t spin, double *dst);

/* ---- adjoint (new path; see the header of each call) ------------------- */

/* Forward from explicit tables: N = sum_I coef[I] det S_up,I det S_dn,I with
 * S[j][l] = T_sigma[h_j][p_l - n] (Sec. III r x r read-off).  T_up
 * [W][n_up][m_up], T_dn [W][n_dn][m_dn], coef [n_det] (device, FP64).
 * Outputs log|N| and sign(N) per walker.  Keeps what mde_backward needs. */
mde_status mde_eval_tables(mde_ctx *ctx, int32_t W, const double *T_up, const double *T_dn,
                           const double *coef, double *log_abs, double *sign,
                           int32_t *status);

/* Adjoint of the last mde_eval_tables: with go[W] the upstream gradient of
 * log|N_w|, grad_coef[I] = sum_w go_w dlog|N_w|/dcoef_I (deterministic order)
 * and grad_T_sigma[w] = go_w dlog|N_w|/dT_sigma[w] ([W][n][m]).  status[W]
 * (may be NULL): MDE_ST_NONFINITE for a walker whose table gradient holds a
 * non-finite value. */
mde_status mde_backward(mde_ctx *ctx, const double *go, double *grad_coef,
                        double *grad_T_up, double *grad_T_dn, int32_t *status);

/* ---- tuning -------------------------------------------------------------- */

/* Work decomposition of the determinant kernel for one spin: walker tile
 * (1..64, power of two), excitations per work item, threads per block
 * (64..1024).  0 keeps the current value.  Before mde_bind_workspace the
 * plan is kept for the bind; on a bound context it takes effect at once and
 * the walkers' state must be set again with mde_init (MDE_STATE until
 * then).  A group holding the context rebuilds its work items at its next
 * call (outside a capture). */
mde_status mde_set_plan(mde_ctx *ctx, int32_t spin, int32_t walker_tile,
                        int32_t item_exc, int32_t threads);
mde_status mde_get_plan(const mde_ctx *ctx, int32_t spin, int32_t *walker_tile,
                        int32_t *item_exc, int32_t *threads);

/* Host-only inspection of the determinant kernel's work decomposition for
 * one spin under a plan (walker tile, item size, threads) and W walkers; no
 * device call, usable before binding.  items: up to items_cap records of 10
 * int32 each (instance, spin, tile, order, u0, u1, slot, wb, d0, d1) --
 * excitations are in the library's internal order (ascending order, holes,
 * particles; 0 is the reference; orders 1 and 2 may be filled dense);
 * [u0, u1) is the item's range with staged records and [d0, d1) its share of
 * the dense block; wb indexes `ranges`.  ranges: up to ranges_cap int32, the
 * per-wave (first, end) pairs of 64-walker items (threads / 64 pairs per
 * item).  layout[0..3] = (internal excitation count, first and end of the
 * dense block, its order mask).  *n_items and *n_ranges receive the full
 * counts; MDE_NOMEM when a capacity is too small. */
mde_status mde_debug_items(const mde_ctx *ctx, int32_t spin, int32_t W, int32_t walker_tile,
                           int32_t item_exc, int32_t threads, int32_t *items, int32_t items_cap,
                           int32_t *n_items, int32_t *ranges, int32_t ranges_cap,
                           int32_t *n_ranges, int32_t *layout);

/* Time candidate plans on this context's current state (after mde_init) with
 * proposals of electron 0 and electron n_up (new_orb_up/new_orb_dn: device
 * blocks [W][5][n_orb]); keep the fastest per spin.  If cache_path is not
 * NULL the choice is read from / appended to that text file, keyed by the
 * problem shape.  Restores the state (refresh) before returning. */
mde_status mde_autotune(mde_ctx *ctx, const double *new_orb_up,
                        const double *new_orb_dn, const char *cache_path);

/* ---- profiling ---------------------------------------------------------- */

/* While enabled, every launch of the determinant kernel made by a proposal
 * (mde_propose / mde_grad_lap) is bracketed by a pair of HIP events recorded on the
 * context's stream -- inside captured graphs too, where each captured launch
 * gets its own pair.  With repeat > 1 (at most 64) the bracketed launch is
 * issued repeat times back to back between its two events, so that the
 * dispatch gap after the first event is spread over the repeats; in the
 * proposal mode the kernel writes only its partial sums (and resets its own
 * work queues), so the repeats leave the proposal's results unchanged.  At
 * most max_launches pairs are recorded; later launches are neither bracketed
 * nor repeated.  Host-side objects only; MDE_INVALID for a count out of
 * range. */
mde_status mde_profile_enable(mde_ctx *ctx, int32_t max_launches, int32_t repeat);
/* After the caller has synchronised the stream: sum of the elapsed times of
 * the recorded pairs (ms) and the number of kernel launches they hold
 * (pairs x repeat).  Pairs captured into a graph hold the times of that
 * graph's last replay. */
mde_status mde_profile_read(mde_ctx *ctx, double *total_ms, int32_t *count);
mde_status mde_profile_disable(mde_ctx *ctx);

/* ---- graphs ------------------------------------------------------------- */

/* Capture every call made on ctx's stream between begin and end into a HIP
 * graph (no host synchronisation happens in the evaluation calls).  Replays
 * repeat the captured calls with the same pointers; the caller refreshes the
 * content of its input buffers between replays.  A sequence that ends with a
 * refresh leaves the state consistent for replay. */
mde_status mde_capture_begin(mde_ctx *ctx);
mde_status mde_capture_end(mde_ctx *ctx, mde_graph **out);
mde_status mde_graph_launch(mde_graph *g, void *hip_stream);
mde_status mde_graph_destroy(mde_graph *g);

/* ---- uneven batch ------------------------------------------------------- */

/* Pack n bound contexts (same stream, same precision) so that one propose
 * runs the determinant kernel as one persistent launch per walker tile over
 * the work items of every instance of that tile (Sec. V: the tiny
 * determinants are independent): members that share a walker tile form one
 * launch; members of different tiles (each keeps the tile its tables fit,
 * chosen at bind) form one launch per tile, widest first, within the same
 * group call.  The group's work lists live in caller-owned device memory of
 * mde_group_workspace_bytes bytes.  Contexts with a switched reference are
 * refused (MDE_UNSUPPORTED). */
mde_status mde_group_workspace_bytes(mde_ctx *const *ctxs, int32_t n, size_t *bytes);
mde_status mde_group_create(mde_ctx *const *ctxs, int32_t n, void *dev, size_t bytes,
                            mde_group **out);
mde_status mde_group_destroy(mde_group *g);
/* e[n] (host): moving electron per instance; new_orb[n], ratio[n], grad[n],
 * lap[n], status[n] (host arrays of device pointers, per-instance layouts as
 * in mde_propose). */
mde_status mde_group_propose(mde_group *g, const int32_t *e,
                             const double *const *new_orb, double *const *ratio,
                             double *const *grad, double *const *lap,
                             int32_t *const *status);
/* accept[n] (host array of device uint8 [W_i] pointers). */
mde_status mde_group_accept(mde_group *g, const int32_t *e,
                            const uint8_t *const *accept);
/* Autotuner of a group: for each walker-tile class, threads per block and
 * work-item size of its members (their tiles kept) are chosen by timing
 * three group proposals of the moving electrons e[n] to new_orb[n] (as in
 * mde_group_propose) per candidate; each candidate re-evaluates the members
 * from their kept orbitals, so the state is that of the last init/refresh
 * afterwards.  Not during capture. */
mde_status mde_group_tune(mde_group *g, const int32_t *e, const double *const *new_orb);
/* Last error message of a group call. */
const char *mde_group_error_string(const mde_group *g);
/* Capture / replay work on groups exactly as on contexts. */
mde_status mde_group_capture_begin(mde_group *g);
mde_status mde_group_capture_end(mde_group *g, mde_graph **out);

/* ---- synthetic orbital provider (s-Gaussians) --------------------------- */

/* Basis of nb unnormalised s-Gaussians chi_b(r) = exp(-expo_b |r - c_b|^2)
 * and MO coefficients mo [n_orb][nb] for spin `spin` (host, copied).  Call
 * before mde_workspace_bytes: the basis lives in the workspace. */
mde_status mde_sgauss_set_basis(mde_ctx *ctx, int32_t spin, int32_t nb,
                                const double *centres, const double *expo,
                                const double *mo);
/* Orbital blocks at positions pos [npos][3] (device) -> out [npos][5][n_orb]
 * (device): value, gradient, laplacian of phi_p = sum_b mo[p][b] chi_b. */
mde_status mde_sgauss_eval(mde_ctx *ctx, int32_t spin, int32_t npos,
                           const double *pos, double *out);

#ifdef __cplusplus
}
#endif
#endif /* MDE_H */
