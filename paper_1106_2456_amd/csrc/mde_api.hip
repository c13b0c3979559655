// Host runtime and C ABI of libmde (see include/mde.h).
//
// A context owns host metadata only: the expansion in its internal order,
// work-item plans and state flags.  All device memory is the caller's
// workspace, carved here.  The evaluation calls only enqueue kernels (and,
// for groups, one small host-to-device copy of per-instance arguments), so
// they can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/mde.h"
#include "mde_internal.h"

using namespace mde;

namespace {

const char *kVersion = "mde 0.1 (gfx950)";

struct SpinHost {
    int n = 0, m = 0, no = 0, U = 0, max_order = 0;
    int n_user = 0;     // excitations given by the caller; the dense fill follows
    int dense_k = 0;    // bit k-1: order k (<= 2) stored dense
    bool have = false;
    std::vector<int> perm;       // internal -> user excitation index
    std::vector<int> iperm;      // user -> internal
    std::vector<uint4> ex;       // packed records, internal order
    std::vector<int> orders;     // order of each internal excitation
    int order_start[MAXK + 2] = {0};
    std::vector<int> ci_seg, ci_other, ci_end, ci_idx;
    std::vector<int> chunks;     // precontraction chunks (excitation boundaries)
    std::vector<int4> pieces;    // pieces of long CI segments (u, k0, k1, 0)
    std::vector<int4> longs;     // (u, first piece, end piece, 0)
    std::vector<int> inv_off, inv_ent;
    // plan
    int item_exc = 0, threads = 0;
    std::vector<double> ucost;       // cost of each excitation in the 64-walker kernel
    std::vector<WorkItem> items;     // scheduling order, grouped by XCD queue
    std::vector<int32_t> bounds;     // per item (64-walker tiles): wave range boundaries
    ItemQueues queues{};
    std::vector<int> tile_slot;
    size_t lds_prop = 0, lds_val = 0;
    int grid = 0;
    int ex_cap = 0;      // longest item (records staged in LDS)
};

struct Plan {
    int WT, item_exc[2], threads[2];
};

}  // namespace

struct mde_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct mde_ctx {
    mde_desc d{};
    hipStream_t stream = nullptr;
    std::string err;
    SpinHost sp[2];
    int WT = 64;
    std::vector<double> coef;
    std::vector<int> up_idx, dn_idx;
    int64_t n_det = 0;
    bool have_ci = false;
    int n_cu = 256;
    // s-Gaussian basis per spin (optional)
    int nb[2] = {0, 0};
    std::vector<double> centres[2], expo[2], mo[2];
    double *d_centres[2] = {nullptr, nullptr}, *d_expo[2] = {nullptr, nullptr},
           *d_mo[2] = {nullptr, nullptr};
    // device
    int W = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    InstDev h{};
    InstDev *d_inst = nullptr;
    int32_t *d_perm_user[2] = {nullptr, nullptr};
    WorkItem *d_items[2] = {nullptr, nullptr};
    int32_t *d_tile_slot[2] = {nullptr, nullptr};
    int32_t *d_bounds[2] = {nullptr, nullptr};
    size_t bounds_cap[2] = {0, 0};
    size_t items_cap[2] = {0, 0};
    size_t partial_cap[2] = {0, 0};
    size_t tileslot_cap[2] = {0, 0};
    // state
    bool initialized = false;
    bool adjoint_state = false;
    bool R_valid[2] = {false, false};
    bool coef_gathered = false;    // coef_s holds the context's own coefficients
    bool C_valid[2] = {false, false};
    int pending_e = -1;
    bool pending_fused = false;   // the pending proposal was formed in the determinant kernel
    long accept_count = 0;
    bool capturing = false;
    const double *last_T[2] = {nullptr, nullptr};   // tables of the last mde_eval_tables
    // profiling event pairs around determinant-kernel launches
    std::vector<hipEvent_t> prof_ev;
    int prof_used = 0;
    int prof_repeat = 1;
    bool prof_on = false;
    // plan fields chosen by the caller (kept when the default plan is applied)
    bool user_wt = false, user_thr[2] = {false, false}, user_item[2] = {false, false};
    // bumped whenever the work layout is re-established (apply_plan): a group
    // built over this context holds the generation it copied
    long plan_gen = 0;
    // the caller's expansion as given (kept so that the reference can be
    // switched, always relative to it)
    std::vector<int> u_off[2], u_h[2], u_p[2];
    std::vector<double> u_coef;
    std::vector<int> u_up, u_dn;
    bool in_rebase = false;
    // reference switching: internal orbital q of spin s is the caller's
    // orbital orb_perm[s][q]; empty = identity
    std::vector<int32_t> orb_perm[2];
    int32_t *d_orb_perm[2] = {nullptr, nullptr};
    double *d_vmc = nullptr;      // Metropolis loop scratch (see mde_vmc)
    uint8_t *d_vmc_mask = nullptr;
    double *d_orbx = nullptr;     // [W][5][n_orb] permuted proposal block
    double *d_orbfull = nullptr;  // [W][n][5][n_orb] up block, then the down block
    int ref_user[2] = {0, 0};
};

// default plan for W walkers, keeping the fields the caller set
static void apply_default_plan(mde_ctx *c, int W);

struct mde_group {
    std::vector<mde_ctx *> ctx;
    hipStream_t stream = nullptr;
    int prec = 0, WT = 1, threads = 256, maxW = 0, nmax = 0, mmax = 0, max_order = 0;
    size_t lds = 0;
    int grid = 0;
    int ex_cap = 16;
    InstDev *d_insts = nullptr;
    MoveArgs *d_moves = nullptr;
    WorkItem *d_items = nullptr;
    int32_t *d_bounds = nullptr;
    int n_items = 0;
    ItemQueues queues{};
    std::vector<MoveArgs> hmoves;
    std::vector<long> plan_gen;   // each member's plan generation at the last rebuild
    bool capturing = false;
    std::string err;
    // members of several walker tiles: one homogeneous group (one launch of
    // the determinant kernel) per tile, called in order of decreasing tile
    std::vector<mde_group *> subs;
    std::vector<std::vector<int>> sub_idx;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

#define MDE_FAIL(ctx, code, ...)                                    \
    do {                                                           \
        char _b[512];                                              \
        snprintf(_b, sizeof(_b), __VA_ARGS__);                     \
        if (ctx) (ctx)->err = _b;                                  \
        return code;                                               \
    } while (0)

#define MDE_HIP(ctx, call)                                                          \
    do {                                                                            \
        hipError_t _e = (call);                                                     \
        if (_e != hipSuccess)                                                       \
            MDE_FAIL(ctx, MDE_DEVICE, "%s failed: %s", #call, hipGetErrorString(_e)); \
    } while (0)

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Carver {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += sizeof(T) * std::max<size_t>(count, 1);
        return p;
    }
};

static int pow2_floor(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

// relative cost of one excitation of order k in the determinant kernel
static double order_cost(int k) {
    static const double c[9] = {0, 13, 23, 45, 95, 300, 500, 800, 1200};
    return c[std::min(std::max(k, 0), 8)];
}

// Relative cost of each excitation in the 64-walker determinant kernel (one
// wave per excitation), in units of one double excitation inside a run.
// Dense orders 1 and 2 cost per excitation of their blocks; sparse orders 1
// and 2 are evaluated in runs that share holes and leading particles (a new
// run pays for its cofactors), orders 3 and 4 one by one.  The weights are
// per-order wave times measured on MI355X with every CU busy (water-like
// system, 4 096 walkers).
static void excitation_costs(SpinHost &sp) {
    const int U = (int)sp.ex.size();
    sp.ucost.assign(U, 0.0);
    for (int u = 1; u < U; ++u) {
        const int k = sp.orders[u];
        double w;
        if (k <= 2 && ((sp.dense_k >> (k - 1)) & 1)) {
            w = k == 1 ? 0.68 : 0.44;   // dense block: per excitation
        } else if (k <= 2) {
            const uint32_t pmask = k == 1 ? 0u : 0xffu;
            const bool fresh = sp.orders[u - 1] != k || sp.ex[u].x != sp.ex[u - 1].x ||
                               ((sp.ex[u].z ^ sp.ex[u - 1].z) & pmask) != 0u;
            w = k == 1 ? 0.65 + (fresh ? 0.7 : 0.0) : 1.0 + (fresh ? 1.5 : 0.0);
        } else if (k == 3) {
            w = 2.5;
        } else if (k == 4) {
            w = 5.1;
        } else {
            w = 6.0 * k * k;
        }
        sp.ucost[u] = w;
    }
}

static int spin_of(const mde_ctx *c, int e, int *row) {
    if (e < c->d.n_elec[0]) {
        *row = e;
        return 0;
    }
    *row = e - c->d.n_elec[0];
    return 1;
}

// bytes of LDS the determinant kernel needs: staged excitation records,
// then the walker tile's tables (or the reduction scratch, whichever is larger)
static size_t det_lds(const SpinHost &s, int WT, int threads, int prec, bool propose,
                      int ex_cap = ITEM_MAX) {
    const int WTP = lds_row_stride(WT);
    const size_t esz = prec == 0 ? 8 : 4;
    const int NE = prec == 0 ? 5 : 4;
    size_t tab = (size_t)s.n * s.m * WTP * esz;
    size_t red = 0;
    if (WT == 64) {
        // c rows, then each wave's FP64 particle weights; the end-of-item
        // reduction reuses the space
        if (propose) {
            tab += (size_t)s.n * WTP * esz + (size_t)(threads / 64) * s.m * 64 * 8 + (size_t)s.n * 64 * 8;
            red = (size_t)(threads / 64) * 64 * (NSUM + NE) * 8;
        }
    } else if (propose) {
        tab += (size_t)(NE * s.m + s.n) * WTP * esz;
        red = (size_t)(threads / 64) * WT * NSUM * 8;
    }
    return (size_t)ex_cap * 16 + std::max(tab, red);
}

// work items of one spin for a plan: per tile, per order, chunks of about
// item_exc order-2-equivalent excitations (at least one per slot)
static ItemQueues queue_order(std::vector<WorkItem> &items, const std::vector<double> &cost);

// dense block [da, db) of a spin (orders 1 and 2 when stored dense)
static void dense_range(const SpinHost &s, int &da, int &db) {
    const bool d1 = s.dense_k & 1, d2 = (s.dense_k >> 1) & 1;
    da = d1 ? s.order_start[1] : (d2 ? s.order_start[2] : 0);
    db = d2 ? s.order_start[3] : (d1 ? s.order_start[2] : 0);
}

// excitations of one wave unit in the dense block of order k (0: sparse):
// a hole for singles, a fixed share of a hole pair for doubles
static int dense_unit(const SpinHost &s, int k) {
    if (k < 1 || k > 2 || !((s.dense_k >> (k - 1)) & 1)) return 0;
    if (k == 1) return s.m;
    switch (s.m) {
        case 8: return Dense2Shape<8>::UNIT;
        case 12: return Dense2Shape<12>::UNIT;
        case 16: return Dense2Shape<16>::UNIT;
        case 20: return Dense2Shape<20>::UNIT;
        case 24: return Dense2Shape<24>::UNIT;
        default: return s.m * (s.m - 1) / 2;
    }
}

// records an item stages in LDS: those of its sparse range (on 64-walker
// tiles the dense block needs none and is not part of [u0, u1))
static int item_records(const SpinHost &s, int u0, int u1, int WT) {
    (void)s;
    // only 64-walker tiles stage their records in LDS
    return WT == 64 ? u1 - u0 : 0;
}

// boundaries of nslot ranges of about equal cost over [u0, u1)
static void cost_cuts(const SpinHost &s, int u0, int u1, int nslot, std::vector<int32_t> &out) {
    double tot = 0.0;
    for (int u = u0; u < u1; ++u) tot += s.ucost[u];
    out.push_back(u0);
    double acc = 0.0;
    int u = u0;
    for (int w = 1; w < nslot; ++w) {
        const double target = tot * w / nslot;
        while (u < u1 && acc + 0.5 * s.ucost[u] < target) acc += s.ucost[u++];
        out.push_back(u);
    }
    out.push_back(u1);
}

// units of the dense block [da, db): one hole (singles) or one hole pair
static void dense_units(const SpinHost &s, int d0, int d1, std::vector<int> &starts) {
    starts.clear();
    int u = d0;
    while (u < d1) {
        starts.push_back(u);
        const int k = s.orders[u];
        u += dense_unit(s, k);
    }
    starts.push_back(d1);
}

// Per-wave ranges of a 64-walker item, 2 x nslot entries (first, end):
// some waves take whole dense units, the others equal-cost pieces of the
// sparse range, in proportion to the two costs.  Empty ranges are (0, 0).
static void item_wave_ranges(const SpinHost &s, const WorkItem &it, int nslot,
                             std::vector<int32_t> &out) {
    std::vector<int> us;
    dense_units(s, it.d0, it.d1, us);
    const int nu = (int)us.size() - 1;
    double cd = 0.0, cs = 0.0;
    for (int u = it.d0; u < it.d1; ++u) cd += s.ucost[u];
    for (int u = it.u0; u < it.u1; ++u) cs += s.ucost[u];
    int nd = 0;
    if (nu > 0) {
        nd = cs > 0.0 ? (int)std::lround(nslot * cd / (cd + cs)) : nslot;
        nd = std::max(1, std::min({nd, nu, cs > 0.0 ? nslot - 1 : nslot}));
    }
    const int ns = nslot - nd;
    // dense units over nd waves, contiguous, balanced by cost
    if (nd > 0) {
        std::vector<double> cum(nu + 1, 0.0);
        for (int i = 0; i < nu; ++i) {
            double c = 0.0;
            for (int u = us[i]; u < us[i + 1]; ++u) c += s.ucost[u];
            cum[i + 1] = cum[i] + c;
        }
        int i0 = 0;
        for (int w = 0; w < nd; ++w) {
            int i1 = i0;
            const double target = cum[nu] * (w + 1) / nd;
            while (i1 < nu && (w == nd - 1 || cum[i1 + 1] - 0.5 * (cum[i1 + 1] - cum[i1]) <= target)) ++i1;
            if (w == nd - 1) i1 = nu;
            out.push_back(us[i0]);
            out.push_back(us[i1]);
            i0 = i1;
        }
    }
    if (ns > 0) {
        std::vector<int32_t> b;
        cost_cuts(s, it.u0, it.u1, ns, b);
        for (int w = 0; w < ns; ++w) {
            out.push_back(b[w]);
            out.push_back(b[w + 1]);
        }
    }
}

static ItemQueues build_items(const SpinHost &s, int W, int WT, int item_exc, int threads,
                              std::vector<WorkItem> &items, std::vector<int> &tile_slot, int spin,
                              std::vector<int32_t> *bounds = nullptr) {
    items.clear();
    if (bounds) bounds->clear();
    const int n_tiles = (W + WT - 1) / WT;
    tile_slot.assign(n_tiles + 1, 0);
    const int nslot = threads / WT;
    std::vector<WorkItem> per;
    std::vector<double> cost;
    const int U = s.order_start[MAXK + 1];
    if (WT == 64) {
        // 64-walker tiles: each item takes a contiguous share of the dense
        // block (whole units) and a contiguous range of the sparse
        // excitations, sized so the item costs are about equal; the C stream
        // of the dense block is spread over all items of the tile
        int da, db;
        dense_range(s, da, db);
        const int sp0 = db > da ? db : 1;     // sparse excitations [sp0, U)
        std::vector<int> us;
        dense_units(s, da, db, us);
        const int nu = (int)us.size() - 1;
        std::vector<double> ucum(nu + 1, 0.0);
        for (int i = 0; i < nu; ++i) {
            double c = 0.0;
            for (int u = us[i]; u < us[i + 1]; ++u) c += s.ucost[u];
            ucum[i + 1] = ucum[i] + c;
        }
        std::vector<double> cum(U + 1, 0.0);
        for (int u = sp0; u < U; ++u) cum[u + 1] = cum[u] + s.ucost[u];
        const double total = ucum[nu] + cum[U];
        int n_it = std::max(1, (int)std::lround(total / std::max(item_exc, 1)));
        n_it = std::max(n_it, (U - sp0 + ITEM_MAX - 1) / ITEM_MAX);
        n_it = std::min(n_it, std::max(1, nu + (U - sp0)));
        // dense units: contiguous, by cost
        std::vector<int> dcut(n_it + 1, 0);
        for (int i = 1; i < n_it; ++i) {
            const double target = ucum[nu] * i / n_it;
            int j = dcut[i - 1];
            while (j < nu && ucum[j + 1] - 0.5 * (ucum[j + 1] - ucum[j]) <= target) ++j;
            dcut[i] = j;
        }
        dcut[n_it] = nu;
        // sparse cuts so that item i costs about total / n_it
        std::vector<int> cuts(n_it + 1, sp0);
        double dsum = 0.0;
        for (int i = 1; i < n_it; ++i) {
            dsum += ucum[dcut[i]] - ucum[dcut[i - 1]];
            const double target = std::max(0.0, total * i / n_it - dsum) + cum[sp0];
            int u = (int)(std::lower_bound(cum.begin() + sp0 + 1, cum.begin() + U + 1, target) - cum.begin());
            cuts[i] = std::min(std::max(u, cuts[i - 1]), U);
            cuts[i] = std::min(cuts[i], cuts[i - 1] + ITEM_MAX);
        }
        cuts[n_it] = U;
        // the last item's sparse range respects the record capacity
        while (cuts[n_it] - cuts[n_it - 1] > ITEM_MAX) {
            cuts.insert(cuts.end() - 1, cuts[n_it - 1] + ITEM_MAX);
            dcut.insert(dcut.end() - 1, nu);
            ++n_it;
        }
        for (int t = 0; t < n_tiles; ++t) {
            tile_slot[t] = (int)per.size();
            for (int i = 0; i < n_it; ++i) {
                WorkItem it{};
                it.inst = 0;
                it.spin = spin;
                it.tile = t;
                it.order = 0;
                it.u0 = cuts[i];
                it.u1 = cuts[i + 1];
                it.d0 = us[dcut[i]];
                it.d1 = us[dcut[i + 1]];
                if (it.u1 <= it.u0 && it.d1 <= it.d0) continue;
                // the tile's first item also forms the move's quantities
                // when the proposal is fused into the determinant kernel
                it.order = (int)per.size() == tile_slot[t] ? 1 : 0;
                it.slot = (int)per.size();
                it.wb = -1;
                if (bounds) {
                    it.wb = (int)bounds->size();
                    item_wave_ranges(s, it, nslot, *bounds);
                }
                per.push_back(it);
                cost.push_back(cum[it.u1] - cum[it.u0] + ucum[dcut[i + 1]] - ucum[dcut[i]]);
            }
        }
    } else {
        for (int t = 0; t < n_tiles; ++t) {
            tile_slot[t] = (int)per.size();
            for (int k = 1; k <= s.max_order; ++k) {
                const int a = s.order_start[k], b = s.order_start[k + 1];
                if (b <= a) continue;
                // (records are read from global memory: no capacity limit)
                double want = std::lround((double)item_exc * order_cost(2) / order_cost(k));
                int chunk = (int)std::min(std::max(want, (double)nslot), (double)(b - a));
                for (int u = a; u < b; u += chunk) {
                    WorkItem it{};
                    it.inst = 0;
                    it.spin = spin;
                    it.tile = t;
                    it.order = k;
                    it.u0 = u;
                    it.u1 = std::min(b, u + chunk);
                    it.slot = (int)per.size();
                    it.wb = -1;
                    per.push_back(it);
                    cost.push_back(order_cost(k) * (it.u1 - it.u0));
                }
            }
        }
    }
    tile_slot[n_tiles] = (int)per.size();
    items = per;
    return queue_order(items, cost);
}

// queue order: by XCD of the tile (t % 8), most expensive first inside a
// queue (the queue hands them out in order)
static ItemQueues queue_order(std::vector<WorkItem> &items, const std::vector<double> &cost) {
    std::vector<int> idx(items.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
        const int qx = items[x].tile % NXCD, qy = items[y].tile % NXCD;
        if (qx != qy) return qx < qy;
        return cost[x] > cost[y];
    });
    std::vector<WorkItem> out;
    out.reserve(items.size());
    ItemQueues q{};
    for (int i : idx) {
        out.push_back(items[i]);
        q.off[items[i].tile % NXCD + 1]++;
    }
    for (int x = 0; x < NXCD; ++x) q.off[x + 1] += q.off[x];
    items.swap(out);
    return q;
}

// cost of one walker tile of a spin, in the units of the item size: the
// 64-walker kernel's excitation costs, else order-2-equivalent excitations
static double tile_cost(const SpinHost &sp, int WT) {
    double t = 0.0;
    if (WT == 64) {
        for (double w : sp.ucost) t += w;
        return t;
    }
    for (int k = 1; k <= sp.max_order; ++k)
        t += order_cost(k) / order_cost(2) * (sp.order_start[k + 1] - sp.order_start[k]);
    return t;
}

// item size so that the launch has about one round of items over the CUs
// (fewer, larger items mean fewer re-stagings of the walker tile's tables
// in LDS; the 64-walker items are cost-balanced, smaller tiles' items are
// single-order and need more rounds to balance)
static int item_size_for(const mde_ctx *c, const SpinHost &sp, int W, int WT, int threads,
                         size_t lds) {
    const int n_tiles = (W + WT - 1) / WT;
    int per_cu = (int)std::min<size_t>(160 * 1024 / std::max<size_t>(lds, 1024), 2048 / threads);
    per_cu = std::max(per_cu, 1);
    const double rounds = WT == 64 ? 1.0 : 2.0;
    const double target_items = rounds * c->n_cu * per_cu;
    const double items_per_tile = std::max(1.0, target_items / n_tiles);
    const int nslot = threads / WT;
    const int sz = (int)std::ceil(tile_cost(sp, WT) / items_per_tile);
    return std::max(sz, 4 * nslot);
}

// threads of a determinant block for walker tile WT, and the most it may have
static int max_threads(int WT) { return WT == 64 ? DET64_THREADS : 1024; }
static int default_threads(int WT) { return WT == 64 ? DET64_THREADS : (WT >= 16 ? 1024 : 256); }

static Plan default_plan(const mde_ctx *c, int W) {
    Plan p{};
    const size_t esz = c->d.precision == 0 ? 8 : 4;
    // largest walker tile whose tables fit in LDS for both spins: the
    // 64-walker block (tables, c and the waves' particle weights) in the
    // 160 KB of a CU, smaller tiles in ~112 KB
    int WT = 64;
    for (int s = 0; s < 2; ++s) {
        const SpinHost &sp = c->sp[s];
        const size_t per_w = (size_t)(sp.n * sp.m + (esz == 8 ? 5 : 4) * sp.m + sp.n) * esz;
        int wt = 64;
        if (det_lds(sp, 64, DET64_THREADS, c->d.precision, true) > 160 * 1024) wt = 32;
        while (wt > 1 && wt < 64 && per_w * (wt + (wt >= 8 ? 1 : 0)) > 112 * 1024) wt /= 2;
        WT = std::min(WT, wt);
    }
    WT = std::min(WT, std::max(1, pow2_floor(std::max(W, 1))));
    p.WT = WT;
    for (int s = 0; s < 2; ++s) {
        p.threads[s] = default_threads(WT);
        const size_t lds = det_lds(c->sp[s], WT, p.threads[s], c->d.precision, true);
        p.item_exc[s] = item_size_for(c, c->sp[s], W, WT, p.threads[s], lds);
    }
    return p;
}

static void apply_default_plan(mde_ctx *c, int W) {
    const Plan p = default_plan(c, W);
    if (!c->user_wt) c->WT = p.WT;
    for (int s = 0; s < 2; ++s) {
        if (!c->user_thr[s]) c->sp[s].threads = default_threads(c->WT);
        if (!c->user_item[s]) {
            const size_t lds = det_lds(c->sp[s], c->WT, c->sp[s].threads, c->d.precision, true);
            c->sp[s].item_exc = item_size_for(c, c->sp[s], W, c->WT, c->sp[s].threads, lds);
        }
        if (c->sp[s].threads < c->WT) c->sp[s].threads = std::max(64, c->WT);
    }
}

static std::vector<Plan> candidate_plans(const mde_ctx *c, int W) {
    std::vector<Plan> out;
    Plan d = default_plan(c, W);
    out.push_back(d);
    const int wts[3] = {d.WT, std::max(1, d.WT / 2), std::max(1, d.WT / 4)};
    const int thr[3] = {256, 512, 1024};
    const double scale[3] = {0.5, 1.0, 2.0};
    for (int a = 0; a < 3; ++a) {
        if (a > 0 && wts[a] == wts[a - 1]) continue;
        for (int b = 0; b < 3; ++b) {
            if (thr[b] < wts[a] || thr[b] > max_threads(wts[a])) continue;
            for (int e = 0; e < 3; ++e) {
                Plan p{};
                p.WT = wts[a];
                for (int s = 0; s < 2; ++s) {
                    p.threads[s] = thr[b];
                    const size_t lds = det_lds(c->sp[s], p.WT, thr[b], c->d.precision, true);
                    const int base = item_size_for(c, c->sp[s], W, p.WT, thr[b], lds);
                    p.item_exc[s] = std::max((int)(base * scale[e]), 4 * (thr[b] / p.WT));
                }
                out.push_back(p);
            }
        }
    }
    return out;
}

// size the workspace for W walkers; assign pointers when base != nullptr
static size_t carve(mde_ctx *c, int W, char *base, size_t *max_items_out = nullptr) {
    Carver cv{base};
    // a sizing pass (base == nullptr) must leave the bound descriptor alone
    InstDev scratch{};
    InstDev &h = base ? c->h : scratch;
    const int prec = c->d.precision;
    const int nmax = std::max(c->sp[0].n, c->sp[1].n);
    const int mmax = std::max(c->sp[0].m, c->sp[1].m);
    const int nomax = std::max(c->sp[0].no, c->sp[1].no);
    InstDev *d_inst = cv.take<InstDev>(1);
    // plan-dependent sizes: the maximum over candidate plans
    size_t max_items[2] = {0, 0}, max_partial[2] = {0, 0}, max_tiles[2] = {0, 0};
    size_t max_bounds[2] = {0, 0};
    for (const Plan &p : candidate_plans(c, W)) {
        for (int s = 0; s < 2; ++s) {
            std::vector<WorkItem> it;
            std::vector<int> ts;
            std::vector<int32_t> bd;
            build_items(c->sp[s], W, p.WT, p.item_exc[s], p.threads[s], it, ts, s, &bd);
            max_items[s] = std::max(max_items[s], it.size());
            max_partial[s] = std::max(max_partial[s], it.size() * (size_t)p.WT * NSUM);
            max_tiles[s] = std::max(max_tiles[s], ts.size());
            max_bounds[s] = std::max(max_bounds[s], bd.size());
        }
    }
    // current plan (set by the caller) may exceed candidates
    for (int s = 0; s < 2; ++s) {
        std::vector<WorkItem> it;
        std::vector<int> ts;
        std::vector<int32_t> bd;
        build_items(c->sp[s], W, c->WT, c->sp[s].item_exc, c->sp[s].threads, it, ts, s, &bd);
        max_items[s] = std::max(max_items[s], it.size());
        max_partial[s] = std::max(max_partial[s], it.size() * (size_t)c->WT * NSUM);
        max_tiles[s] = std::max(max_tiles[s], ts.size());
        max_bounds[s] = std::max(max_bounds[s], bd.size());
    }
    const size_t Wp = (size_t)W + 64;   // room for a partial last tile of any WT (tiled buffers)
    for (int s = 0; s < 2; ++s) {
        SpinHost &sp = c->sp[s];
        SpinDev &S = h.s[s];
        S.ex = cv.take<uint4>(sp.U);
        S.ci_seg = cv.take<int32_t>(sp.U + 1);
        S.ci_other = cv.take<int32_t>(c->n_det + PC_BATCH);
        S.ci_end = cv.take<int32_t>(c->n_det + PC_BATCH);
        S.ci_idx = cv.take<int32_t>(c->n_det);
        S.inv_off = cv.take<int32_t>((size_t)sp.n * sp.m + 1);
        S.inv_ent = cv.take<int32_t>(sp.inv_ent.size());
        int32_t *ts = cv.take<int32_t>(max_tiles[s]);
        WorkItem *its = cv.take<WorkItem>(max_items[s]);
        int32_t *bds = cv.take<int32_t>(std::max<size_t>(max_bounds[s], 1));
        int32_t *pu = cv.take<int32_t>(sp.U);
        S.Phi = cv.take<double>((size_t)W * sp.n * sp.no);
        S.B = cv.take<double>((size_t)W * sp.n * sp.n);
        S.T = prec == 0 ? cv.take<double>(Wp * sp.n * sp.m) : nullptr;
        S.T32 = prec != 0 ? cv.take<float>(Wp * sp.n * sp.m) : nullptr;
        S.PhiV32 = prec >= 2 ? cv.take<float>((size_t)W * sp.n * sp.m) : nullptr;
        S.logdet = cv.take<double>(W);
        S.sgn = cv.take<double>(W);
        S.R = cv.take<double>(Wp * sp.U);
        S.C = cv.take<double>(Wp * sp.U);
        S.partial = cv.take<double>(max_partial[s]);
        S.coef_s = cv.take<double>(c->n_det + PC_BATCH);
        S.chunks = cv.take<int32_t>(sp.chunks.size());
        S.pieces = cv.take<int4>(sp.pieces.size());
        S.longs = cv.take<int4>(sp.longs.size());
        S.pc_part = cv.take<double>(sp.pieces.size() * Wp);
        if (base) {
            S.tile_slot = ts;
            S.items = its;
            c->d_tile_slot[s] = ts;
            c->d_items[s] = its;
            c->d_bounds[s] = bds;
            c->bounds_cap[s] = max_bounds[s];
            c->d_perm_user[s] = pu;
            c->items_cap[s] = max_items[s];
            c->partial_cap[s] = max_partial[s];
            c->tileslot_cap[s] = max_tiles[s];
        }
        if (c->nb[s] > 0) {
            double *cc = cv.take<double>((size_t)3 * c->nb[s]);
            double *ee = cv.take<double>(c->nb[s]);
            double *mm = cv.take<double>((size_t)sp.no * c->nb[s]);
            if (base) {
                c->d_centres[s] = cc;
                c->d_expo[s] = ee;
                c->d_mo[s] = mm;
            }
        }
    }
    h.coef = cv.take<double>(c->n_det);
    h.Nold = cv.take<double>(W);
    h.Nnew = cv.take<double>(W);
    h.rho = cv.take<double>(W);
    const size_t Wq = (size_t)W + 64;
    h.cc = cv.take<double>(Wq * nmax);
    h.kap = cv.take<double>((size_t)W * 4);
    h.rrow = cv.take<double>(Wq * nmax);
    h.npart = cv.take<double>(Wq * NSPLIT);
    h.ev = prec == 0 ? cv.take<double>(Wq * 5 * mmax) : nullptr;
    h.newrow = cv.take<double>((size_t)W * nomax);
    h.ev32 = prec != 0 ? cv.take<float>(Wq * 4 * mmax) : nullptr;
    h.cc32 = prec != 0 ? cv.take<float>(Wq * nmax) : nullptr;
    h.Tp32 = prec != 0 ? cv.take<float>(Wq * nmax * mmax) : nullptr;
    h.Ap32 = prec >= 2 ? cv.take<float>((size_t)W * (nmax + 4) * nmax) : nullptr;
    h.st = cv.take<int32_t>(W);
    h.counter = cv.take<int32_t>(64);
    h.Lnew = cv.take<double>(W);
    h.gz = prec == 0 ? cv.take<double>((size_t)W * nmax * mmax) : nullptr;
    // reference switching: orbital permutations and the permuted input blocks
    const bool rebased = !c->orb_perm[0].empty() || !c->orb_perm[1].empty();
    int32_t *op[2] = {nullptr, nullptr};
    double *ox = nullptr, *of = nullptr;
    if (rebased) {
        for (int s = 0; s < 2; ++s) op[s] = cv.take<int32_t>(c->sp[s].no);
        ox = cv.take<double>((size_t)W * 5 * nomax);
        of = cv.take<double>((size_t)W * (c->sp[0].n * c->sp[0].no + c->sp[1].n * c->sp[1].no) * 5);
    }
    // Metropolis loop: cur, new positions, g(R), g(R') [W][3] each; ratio,
    // two laplacians [W]; two orbital blocks [W][5][nomax]; the accept mask
    double *vm = cv.take<double>((size_t)W * (15 + 10 * (size_t)nomax));
    uint8_t *vmask = cv.take<uint8_t>(W);
    if (base) {
        c->d_vmc = vm;
        c->d_vmc_mask = vmask;
        for (int s = 0; s < 2; ++s) c->d_orb_perm[s] = c->orb_perm[s].empty() ? nullptr : op[s];
        c->d_orbx = ox;
        c->d_orbfull = of;
    }
    if (base) {
        c->d_inst = d_inst;
        h.W = W;
        h.prec = prec;
        h.nmax = nmax;
        h.mmax = mmax;
        h.nomax = nomax;
        h.n_det = c->n_det;
    }
    if (max_items_out) *max_items_out = max_items[0] + max_items[1];
    return cv.off;
}

// CI weights of excitations without CI terms are never written by the
// precontraction: the whole array starts at zero whenever its tile layout
// is (re)established
static mde_status zero_weights(mde_ctx *c) {
    const size_t Wp = (size_t)c->W + 64;
    for (int s = 0; s < 2; ++s)
        MDE_HIP(c, hipMemsetAsync(c->h.s[s].C, 0, sizeof(double) * Wp * c->sp[s].U, c->stream));
    return MDE_OK;
}

// apply the context's plan: items, slots, LDS sizes, grids (host + upload)
static mde_status apply_plan(mde_ctx *c) {
    for (int s = 0; s < 2; ++s) {
        SpinHost &sp = c->sp[s];
        SpinDev &S = c->h.s[s];
        std::vector<WorkItem> items;
        std::vector<int> ts;
        std::vector<int32_t> bd;
        const ItemQueues q = build_items(sp, c->W, c->WT, sp.item_exc, sp.threads, items, ts, s, &bd);
        if (items.size() > c->items_cap[s] || items.size() * (size_t)c->WT * NSUM > c->partial_cap[s] ||
            ts.size() > c->tileslot_cap[s] || bd.size() > c->bounds_cap[s])
            MDE_FAIL(c, MDE_NOMEM, "plan needs more workspace than was sized (spin %d)", s);
        sp.items = items;
        sp.bounds = bd;
        sp.queues = q;
        sp.tile_slot = ts;
        S.WT = c->WT;
        S.WTP = lds_row_stride(c->WT);
        S.n_tiles = (c->W + c->WT - 1) / c->WT;
        S.n_slots = (int)items.size();
        // slots of tile t are [ts[t], ts[t + 1]); uniform counts let the
        // finishing kernels skip that lookup
        S.slots_per_tile = 0;
        if (ts.size() >= 2) {
            const int c0 = ts[1] - ts[0];
            bool same = c0 > 0;
            for (size_t t = 0; t + 1 < ts.size() && same; ++t)
                same = ts[t + 1] - ts[t] == c0 && ts[t] == (int)t * c0;
            if (same) S.slots_per_tile = c0;
        }
        sp.ex_cap = 16;
        for (const WorkItem &it : items)
            sp.ex_cap = std::max(sp.ex_cap, item_records(sp, it.u0, it.u1, c->WT));
        sp.lds_prop = det_lds(sp, c->WT, sp.threads, c->d.precision, true, sp.ex_cap);
        sp.lds_val = det_lds(sp, c->WT, sp.threads, c->d.precision, false, sp.ex_cap);
        if (sp.lds_prop > 160 * 1024)
            MDE_FAIL(c, MDE_UNSUPPORTED, "tables of spin %d need %zu bytes of LDS", s, sp.lds_prop);
        const size_t lds = std::max<size_t>(sp.lds_prop, 1024);
        int per_cu = (int)std::min<size_t>(160 * 1024 / lds, 2048 / sp.threads);
        per_cu = std::max(per_cu, 1);
        sp.grid = (int)std::min<size_t>(items.size(), (size_t)c->n_cu * per_cu);
        sp.grid = std::max(sp.grid, 1);
        if (!items.empty()) {
            MDE_HIP(c, hipMemcpy(c->d_items[s], items.data(), sizeof(WorkItem) * items.size(),
                                 hipMemcpyHostToDevice));
        }
        MDE_HIP(c, hipMemcpy(c->d_tile_slot[s], ts.data(), sizeof(int) * ts.size(),
                             hipMemcpyHostToDevice));
        if (!bd.empty())
            MDE_HIP(c, hipMemcpy(c->d_bounds[s], bd.data(), sizeof(int32_t) * bd.size(),
                                 hipMemcpyHostToDevice));
    }
    MDE_HIP(c, hipMemcpy(c->d_inst, &c->h, sizeof(InstDev), hipMemcpyHostToDevice));
    c->R_valid[0] = c->R_valid[1] = false;
    c->C_valid[0] = c->C_valid[1] = false;
    c->plan_gen++;
    return MDE_OK;
}

// ---------------------------------------------------------------------------
// state maintenance
// ---------------------------------------------------------------------------

// parts per walker tile of the per-walker kernels: enough blocks to cover
// the CUs twice, at most `cap` (rows or columns) and 16
static int row_split(int n_cu, int blocks, int cap) {
    int s = (2 * n_cu + blocks - 1) / std::max(blocks, 1);
    s = std::min(s, std::min(std::max(cap, 1), 16));
    return std::max(s, 1);
}

// parts of the proposal grid: enough blocks to fill the chip, and enough
// parts that one part's orbital slice fits in LDS
static int prop_split(int n_cu, int blocks, int nmax, int mmax, int WT) {
    const int lim = propose_split_limit(nmax, mmax, WT, 160 * 1024);
    if (lim == 0) return 0;
    return std::max(row_split(n_cu, blocks, mmax), lim);
}

static MoveArgs no_move() {
    MoveArgs m{};
    m.spin = -1;
    return m;
}

static mde_status run_values(mde_ctx *c, int s, const double *tab0 = nullptr,
                             const double *tab1 = nullptr) {
    SpinHost &sp = c->sp[s];
    if (sp.items.empty()) {
        c->R_valid[s] = true;
        return MDE_OK;
    }
    MDE_HIP(c, launch_det(c->stream, c->d_inst, 1, c->d_items[s], c->d_bounds[s], sp.queues, sp.ex_cap,
                          nullptr, no_move(), DM_VALUES, c->d.precision, c->WT,
                          std::max<size_t>(sp.lds_val, 16), sp.threads, sp.grid, c->h.counter,
                          tab0, tab1, sp.max_order));
    c->R_valid[s] = true;
    return MDE_OK;
}

static mde_status ensure_C(mde_ctx *c, int s) {
    if (c->C_valid[s]) return MDE_OK;
    if (!c->R_valid[1 - s]) {
        mde_status st = run_values(c, 1 - s);
        if (st) return st;
    }
    MDE_HIP(c, launch_precontract(c->stream, c->d_inst, c->h, s, c->h.coef));
    c->C_valid[s] = true;
    return MDE_OK;
}

// from-scratch evaluation; orb_* NULL means "use the kept orbital values".
// Every evaluation ends in the same state -- current inverses and tables,
// the down ratios and the up CI weights marked current, the up ratios and
// the down weights marked stale -- so that a captured sequence that starts
// after one evaluation and ends with another replays consistently.  With
// need_n false (the periodic refresh inside a run of FP64 moves) N is not
// re-summed: an FP64 proposal sums N over its own determinants, and the
// up ratios, which only N would need, are formed when a down electron next
// moves (they change with every accepted up move anyway).
static mde_status full_eval(mde_ctx *c, const double *orb_up, const double *orb_dn,
                            double *log_abs, double *sign, int32_t *status, bool need_n = true) {
    const double *orb[2] = {orb_up, orb_dn};
    if (!c->coef_gathered) {
        MDE_HIP(c, launch_coef_gather(c->stream, c->d_inst, c->h, c->h.coef));
        c->coef_gathered = true;
    }
    for (int s = 0; s < 2; ++s) {
        if (c->sp[s].n <= 8) {
            MDE_HIP(c, launch_refresh_small(c->stream, c->d_inst, c->h, s, orb[s], status));
        } else {
            MDE_HIP(c, launch_lu_inverse(c->stream, c->d_inst, c->h, s, orb[s], status));
            MDE_HIP(c, launch_table_gemm(c->stream, c->d_inst, c->h, s));
        }
    }
    c->R_valid[0] = c->R_valid[1] = false;
    c->C_valid[0] = c->C_valid[1] = false;
    for (int s = need_n ? 0 : 1; s < 2; ++s) {
        mde_status st = run_values(c, s);
        if (st) return st;
    }
    mde_status st0 = ensure_C(c, 0);
    if (st0) return st0;
    // N = sum_u C_up[u] R_up[u]
    if (need_n) MDE_HIP(c, launch_nsum(c->stream, c->d_inst, c->h, log_abs, sign, status, 1));
    c->R_valid[0] = false;
    c->initialized = true;
    c->adjoint_state = false;
    c->pending_e = -1;
    return MDE_OK;
}

static void prof_free(mde_ctx *c);

// The caller's orbital blocks in the internal orbital order of a context
// whose reference was switched (rows of n_orb values, permuted in place of
// the caller's buffer into the context's scratch); unchanged otherwise.
static const double *internal_orbitals(mde_ctx *c, int s, const double *orb, int rows,
                                       double *scratch) {
    if (!orb || !c->d_orb_perm[s]) return orb;
    if (launch_permute_orbitals(c->stream, orb, scratch, rows, c->sp[s].no, c->d_orb_perm[s]) !=
        hipSuccess)
        return nullptr;
    return scratch;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *mde_version(void) { return kVersion; }

const char *mde_error_string(const mde_ctx *ctx) {
    if (!ctx) return "no context";
    return ctx->err.c_str();
}

mde_status mde_create(const mde_desc *desc, void *hip_stream, mde_ctx **out) {
    if (!desc || !out) return MDE_INVALID;
    *out = nullptr;
    for (int s = 0; s < 2; ++s) {
        if (desc->n_elec[s] < 1 || desc->n_elec[s] > MDE_MAX_ELEC) return MDE_UNSUPPORTED;
        const int m = desc->n_orb[s] - desc->n_elec[s];
        if (m < 1 || m > MDE_MAX_VIRT) return MDE_UNSUPPORTED;
    }
    if (desc->max_walkers < 1 || desc->max_order < 1 || desc->max_order > MDE_MAX_ORDER)
        return MDE_INVALID;
    if (desc->precision != MDE_FP64 && desc->precision != MDE_MIXED &&
        desc->precision != MDE_MIXED_GEMM && desc->precision != MDE_MIXED_GEMM_KSUM64)
        return MDE_INVALID;
    mde_ctx *c = new (std::nothrow) mde_ctx();
    if (!c) return MDE_NOMEM;
    c->d = *desc;
    if (c->d.refresh_every < 0) c->d.refresh_every = 0;
    c->stream = (hipStream_t)hip_stream;
    for (int s = 0; s < 2; ++s) {
        c->sp[s].n = desc->n_elec[s];
        c->sp[s].no = desc->n_orb[s];
        c->sp[s].m = desc->n_orb[s] - desc->n_elec[s];
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        c->n_cu = std::max(1, prop.multiProcessorCount);
    *out = c;
    return MDE_OK;
}

mde_status mde_destroy(mde_ctx *ctx) {
    if (ctx) prof_free(ctx);
    delete ctx;
    return MDE_OK;
}

mde_status mde_set_excitations(mde_ctx *c, int32_t spin, int32_t n_exc, const int32_t *offsets,
                               const int32_t *holes, const int32_t *particles) {
    if (!c) return MDE_INVALID;
    if (c->bound) MDE_FAIL(c, MDE_STATE, "expansion is fixed once the workspace is bound");
    if (spin < 0 || spin > 1) MDE_FAIL(c, MDE_INVALID, "spin must be 0 or 1");
    if (n_exc < 1 || !offsets) MDE_FAIL(c, MDE_INVALID, "need at least the reference excitation");
    SpinHost &sp = c->sp[spin];
    const int n = sp.n, no = sp.no;
    if (offsets[0] != 0 || offsets[1] != 0) MDE_FAIL(c, MDE_INVALID, "excitation 0 must be empty");
    struct Key {
        int k;
        std::vector<int> h, p;
        int user;
    };
    std::vector<Key> keys((size_t)n_exc);
    int max_order = 0;
    for (int u = 0; u < n_exc; ++u) {
        const int a = offsets[u], b = offsets[u + 1];
        const int k = b - a;
        if (k < 0 || k > c->d.max_order || k > n)
            MDE_FAIL(c, MDE_INVALID, "excitation %d has order %d (max_order %d)", u, k, c->d.max_order);
        if (u > 0 && k == 0) MDE_FAIL(c, MDE_INVALID, "excitation %d is empty (only 0 may be)", u);
        Key &K = keys[u];
        K.k = k;
        K.user = u;
        for (int t = a; t < b; ++t) {
            if (holes[t] < 0 || holes[t] >= n)
                MDE_FAIL(c, MDE_INVALID, "excitation %d: hole %d out of range", u, holes[t]);
            if (particles[t] < n || particles[t] >= no)
                MDE_FAIL(c, MDE_INVALID, "excitation %d: particle %d out of range", u, particles[t]);
            if (t > a && (holes[t] <= holes[t - 1] || particles[t] <= particles[t - 1]))
                MDE_FAIL(c, MDE_INVALID, "excitation %d: holes/particles must ascend", u);
            K.h.push_back(holes[t]);
            K.p.push_back(particles[t] - n);
        }
        max_order = std::max(max_order, k);
    }
    // Dense storage of orders 1 and 2: when most of the possible singles
    // (doubles) of a small virtual space are present, the missing ones are
    // appended with no determinant referring to them (their CI weight is
    // zero), so that the 64-walker kernel evaluates each hole set's block as
    // a whole, without records.
    sp.n_user = n_exc;
    sp.dense_k = 0;
    if (dense_m_supported(sp.m)) {
        const int m = sp.m;
        const int NP = m * (m - 1) / 2;
        std::vector<char> have1((size_t)n * m, 0), have2((size_t)(n * (n - 1) / 2) * NP, 0);
        auto pair_idx = [](int a, int b, int N) { return a * (2 * N - a - 1) / 2 + (b - a - 1); };
        int c1 = 0, c2 = 0;
        for (int u = 1; u < n_exc; ++u) {
            const Key &K = keys[u];
            if (K.k == 1) {
                have1[(size_t)K.h[0] * m + K.p[0]] = 1;
                ++c1;
            } else if (K.k == 2) {
                have2[(size_t)pair_idx(K.h[0], K.h[1], n) * NP + pair_idx(K.p[0], K.p[1], m)] = 1;
                ++c2;
            }
        }
        const bool d2 = c2 > 0 && n >= 2 && c2 >= 0.6 * (n * (n - 1) / 2) * NP;
        // with dense doubles the singles are filled too (at most n m of
        // them), so the sparse excitations form one range after the block
        const bool d1 = c1 > 0 && (c1 >= 0.6 * n * m || d2);
        if (d1)
            for (int h = 0; h < n; ++h)
                for (int p = 0; p < m; ++p)
                    if (!have1[(size_t)h * m + p])
                        keys.push_back(Key{1, {h}, {p}, (int)keys.size()});
        if (d2)
            for (int h0 = 0; h0 < n; ++h0)
                for (int h1 = h0 + 1; h1 < n; ++h1)
                    for (int p0 = 0; p0 < m; ++p0)
                        for (int p1 = p0 + 1; p1 < m; ++p1)
                            if (!have2[(size_t)pair_idx(h0, h1, n) * NP + pair_idx(p0, p1, m)])
                                keys.push_back(Key{2, {h0, h1}, {p0, p1}, (int)keys.size()});
        sp.dense_k = (d1 ? 1 : 0) | (d2 ? 2 : 0);
        n_exc = (int)keys.size();
    }
    std::vector<int> order((size_t)n_exc);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin() + 1, order.end(), [&](int x, int y) {
        const Key &a = keys[x], &b = keys[y];
        if (a.k != b.k) return a.k < b.k;
        if (a.h != b.h) return a.h < b.h;
        return a.p < b.p;
    });
    for (int i = 1; i < n_exc; ++i) {
        const Key &a = keys[order[i - 1]], &b = keys[order[i]];
        if (a.k == b.k && a.h == b.h && a.p == b.p)
            MDE_FAIL(c, MDE_INVALID, "excitations %d and %d are the same", a.user, b.user);
    }
    sp.U = n_exc;
    sp.max_order = max_order;
    sp.perm = order;
    sp.iperm.assign(n_exc, 0);
    for (int i = 0; i < n_exc; ++i) sp.iperm[order[i]] = i;
    sp.ex.assign(n_exc, uint4{0, 0, 0, 0});
    sp.orders.assign(n_exc, 0);
    for (int i = 0; i < n_exc; ++i) {
        const Key &K = keys[order[i]];
        uint32_t w[4] = {0, 0, 0, 0};
        for (int j = 0; j < K.k; ++j) {
            w[j >> 2] |= (uint32_t)K.h[j] << ((j & 3) * 8);
            w[2 + (j >> 2)] |= (uint32_t)K.p[j] << ((j & 3) * 8);
        }
        sp.ex[i] = uint4{w[0], w[1], w[2], w[3]};
        sp.orders[i] = K.k;
    }
    for (int k = 0; k <= MAXK + 1; ++k) sp.order_start[k] = n_exc;
    for (int i = n_exc - 1; i >= 0; --i) sp.order_start[sp.orders[i]] = i;
    for (int k = MAXK; k >= 0; --k) sp.order_start[k] = std::min(sp.order_start[k], sp.order_start[k + 1]);
    excitation_costs(sp);
    // inverted index (entry (h, p) -> (u, j, l))
    const int nm = n * sp.m;
    std::vector<int> cnt(nm + 1, 0);
    for (int i = 0; i < n_exc; ++i) {
        const Key &K = keys[order[i]];
        if (K.user >= sp.n_user) continue;   // dense fill: no determinant refers to it
        for (int j = 0; j < K.k; ++j)
            for (int l = 0; l < K.k; ++l) cnt[K.h[j] * sp.m + K.p[l] + 1]++;
    }
    for (int e = 0; e < nm; ++e) cnt[e + 1] += cnt[e];
    sp.inv_off = cnt;
    sp.inv_ent.assign(cnt[nm], 0);
    std::vector<int> pos(cnt.begin(), cnt.end() - 1);
    for (int i = 0; i < n_exc; ++i) {
        const Key &K = keys[order[i]];
        if (K.user >= sp.n_user) continue;
        for (int j = 0; j < K.k; ++j)
            for (int l = 0; l < K.k; ++l)
                sp.inv_ent[pos[K.h[j] * sp.m + K.p[l]]++] = (i << 10) | (K.k << 6) | (j << 3) | l;
    }
    if (n_exc >= (1 << 21)) MDE_FAIL(c, MDE_UNSUPPORTED, "too many excitations");
    sp.have = true;
    c->have_ci = false;
    if (!c->in_rebase) {
        c->u_off[spin].assign(offsets, offsets + sp.n_user + 1);
        c->u_h[spin].assign(holes, holes + offsets[sp.n_user]);
        c->u_p[spin].assign(particles, particles + offsets[sp.n_user]);
        c->orb_perm[spin].clear();
        c->ref_user[spin] = 0;
    }
    return MDE_OK;
}

mde_status mde_set_ci(mde_ctx *c, int64_t n_det, const double *coef, const int32_t *up_idx,
                      const int32_t *dn_idx) {
    if (!c) return MDE_INVALID;
    if (c->bound) MDE_FAIL(c, MDE_STATE, "expansion is fixed once the workspace is bound");
    if (!c->sp[0].have || !c->sp[1].have) MDE_FAIL(c, MDE_STATE, "set both excitation lists first");
    if (n_det < 1 || n_det > (int64_t)1 << 30) MDE_FAIL(c, MDE_INVALID, "bad n_det");
    const int *idx[2] = {up_idx, dn_idx};
    for (int64_t I = 0; I < n_det; ++I)
        for (int s = 0; s < 2; ++s)
            if (idx[s][I] < 0 || idx[s][I] >= c->sp[s].n_user)
                MDE_FAIL(c, MDE_INVALID, "determinant %lld: excitation index out of range", (long long)I);
    c->n_det = n_det;
    c->coef.assign(coef, coef + n_det);
    c->up_idx.assign(up_idx, up_idx + n_det);
    c->dn_idx.assign(dn_idx, dn_idx + n_det);
    for (int s = 0; s < 2; ++s) {
        SpinHost &sp = c->sp[s];
        std::vector<int> cnt(sp.U + 1, 0);
        for (int64_t I = 0; I < n_det; ++I) cnt[sp.iperm[idx[s][I]] + 1]++;
        for (int u = 0; u < sp.U; ++u) cnt[u + 1] += cnt[u];
        sp.ci_seg = cnt;
        sp.ci_other.assign(n_det, 0);
        sp.ci_idx.assign(n_det, 0);
        std::vector<int> pos(cnt.begin(), cnt.end() - 1);
        for (int64_t I = 0; I < n_det; ++I) {
            const int u = sp.iperm[idx[s][I]];
            const int k = pos[u]++;
            sp.ci_other[k] = c->sp[1 - s].iperm[idx[1 - s][I]];
            sp.ci_idx[k] = (int)I;
        }
        // precontraction work units: chunks of consecutive excitations with
        // short CI segments (about 64 terms each) and 64-term pieces of the
        // long segments
        const int PIECE = 64;
        sp.chunks.assign(1, 0);
        sp.pieces.clear();
        sp.longs.clear();
        std::vector<int> starts, ends;
        int acc = 0, cur = 0;
        for (int u = 0; u < sp.U; ++u) {
            const int len = sp.ci_seg[u + 1] - sp.ci_seg[u];
            if (len > PIECE) {
                if (u > cur) { starts.push_back(cur); ends.push_back(u); }
                const int pb = (int)sp.pieces.size();
                for (int k = sp.ci_seg[u]; k < sp.ci_seg[u + 1]; k += PIECE)
                    sp.pieces.push_back(int4{u, k, std::min(k + PIECE, sp.ci_seg[u + 1]), 0});
                sp.longs.push_back(int4{u, pb, (int)sp.pieces.size(), 0});
                cur = u + 1;
                acc = 0;
                continue;
            }
            acc += len;
            // a chunk holds at most 127 terms and 64 excitations (one wave
            // keeps them in its lanes)
            if (acc >= PIECE || u + 1 - cur >= 64) {
                starts.push_back(cur);
                ends.push_back(u + 1);
                cur = u + 1;
                acc = 0;
            }
        }
        if (cur < sp.U) { starts.push_back(cur); ends.push_back(sp.U); }
        // the last term of every short segment names its excitation; the
        // term arrays carry PC_BATCH entries of padding (read, never used)
        sp.ci_end.assign(n_det + PC_BATCH, -1);
        for (int u = 0; u < sp.U; ++u) {
            const int len = sp.ci_seg[u + 1] - sp.ci_seg[u];
            if (len > 0 && len <= PIECE) sp.ci_end[sp.ci_seg[u + 1] - 1] = u;
        }
        sp.ci_other.resize(n_det + PC_BATCH, 0);
        // chunks as (start, end) pairs flattened: chunks[2c], chunks[2c+1]
        sp.chunks.clear();
        for (size_t i = 0; i < starts.size(); ++i) {
            sp.chunks.push_back(starts[i]);
            sp.chunks.push_back(ends[i]);
        }
        if (sp.chunks.empty()) { sp.chunks.push_back(0); sp.chunks.push_back(0); }
    }
    c->have_ci = true;
    if (!c->in_rebase) {
        c->u_coef.assign(coef, coef + n_det);
        c->u_up.assign(up_idx, up_idx + n_det);
        c->u_dn.assign(dn_idx, dn_idx + n_det);
    }
    apply_default_plan(c, c->d.max_walkers);
    return MDE_OK;
}

// Reference switching (Sec. V: a near-singular reference matrix is handled by
// taking another determinant of the expansion as the reference).  The
// determinant with up excitation ref[0] and down excitation ref[1] of the
// caller's lists becomes the reference: per spin the orbitals are relabelled
// so that its columns, in their column order, are orbitals 0..n-1 and the
// others follow in ascending order; every excitation is rewritten relative
// to the new occupation (holes: new reference orbitals it lacks; particles:
// its orbitals outside the new reference; both ascending, paired in order),
// and the sign of the column permutation between the two forms of each
// determinant is folded into its CI coefficient, so Psi is unchanged.  The
// orders grow by at most the order of the new reference.
static mde_status rebase_expansion(mde_ctx *c, const int32_t ref[2]) {
    std::vector<int> offs[2], hs[2], ps[2], newidx[2];
    std::vector<double> sgn[2];
    for (int s = 0; s < 2; ++s) {
        const int n = c->sp[s].n, no = c->sp[s].no;
        const std::vector<int> &O = c->u_off[s], &H = c->u_h[s], &P = c->u_p[s];
        const int nu = (int)O.size() - 1;
        if (ref[s] < 0 || ref[s] >= nu) MDE_FAIL(c, MDE_INVALID, "reference excitation out of range");
        auto cols = [&](int u, std::vector<int> &col) {
            col.resize(n);
            for (int j = 0; j < n; ++j) col[j] = j;
            for (int t = O[u]; t < O[u + 1]; ++t) col[H[t]] = P[t];
        };
        std::vector<int> cref, perm(no), inv(no, -1);
        cols(ref[s], cref);
        std::vector<char> inref(no, 0);
        for (int j = 0; j < n; ++j) { perm[j] = cref[j]; inref[cref[j]] = 1; }
        int q = n;
        for (int o = 0; o < no; ++o)
            if (!inref[o]) perm[q++] = o;
        for (int k = 0; k < no; ++k) inv[perm[k]] = k;
        c->orb_perm[s] = std::vector<int32_t>(perm.begin(), perm.end());
        // new index: ref <-> 0 swapped, the rest unchanged
        newidx[s].resize(nu);
        for (int u = 0; u < nu; ++u) newidx[s][u] = u;
        newidx[s][ref[s]] = 0;
        newidx[s][0] = ref[s];
        std::vector<std::vector<int>> nh(nu), np_(nu);
        sgn[s].assign(nu, 1.0);
        std::vector<int> col, in_u(no);
        for (int u = 0; u < nu; ++u) {
            cols(u, col);
            std::fill(in_u.begin(), in_u.end(), 0);
            for (int j = 0; j < n; ++j) in_u[col[j]] = 1;
            std::vector<int> h2, p2;
            for (int j = 0; j < n; ++j)
                if (!in_u[perm[j]]) h2.push_back(j);
            for (int j = 0; j < n; ++j)
                if (inv[col[j]] >= n) p2.push_back(inv[col[j]]);
            std::sort(p2.begin(), p2.end());
            if ((int)h2.size() > c->d.max_order)
                MDE_FAIL(c, MDE_UNSUPPORTED, "excitation %d has order %zu relative to the new reference "
                         "(max_order %d)", u, h2.size(), c->d.max_order);
            // caller's orbitals of the new-frame column list, and the parity
            // of the permutation to the caller's column list
            std::vector<int> a(n);
            for (int j = 0; j < n; ++j) a[j] = perm[j];
            for (size_t t = 0; t < h2.size(); ++t) a[h2[t]] = perm[p2[t]];
            std::vector<int> where(no, -1), pm(n);
            for (int j = 0; j < n; ++j) where[a[j]] = j;
            for (int j = 0; j < n; ++j) pm[j] = where[col[j]];
            int inv_count = 0;
            for (int i = 0; i < n; ++i)
                for (int j = i + 1; j < n; ++j) inv_count += pm[i] > pm[j];
            sgn[s][u] = (inv_count & 1) ? -1.0 : 1.0;
            nh[newidx[s][u]] = h2;
            np_[newidx[s][u]] = p2;
        }
        offs[s].assign(1, 0);
        for (int u = 0; u < nu; ++u) {
            hs[s].insert(hs[s].end(), nh[u].begin(), nh[u].end());
            ps[s].insert(ps[s].end(), np_[u].begin(), np_[u].end());
            offs[s].push_back((int)hs[s].size());
        }
    }
    const int64_t nd = (int64_t)c->u_coef.size();
    std::vector<double> coef(nd);
    std::vector<int> up(nd), dn(nd);
    for (int64_t I = 0; I < nd; ++I) {
        coef[I] = c->u_coef[I] * sgn[0][c->u_up[I]] * sgn[1][c->u_dn[I]];
        up[I] = newidx[0][c->u_up[I]];
        dn[I] = newidx[1][c->u_dn[I]];
    }
    c->in_rebase = true;
    mde_status st = MDE_OK;
    for (int s = 0; s < 2 && st == MDE_OK; ++s)
        st = mde_set_excitations(c, s, (int)offs[s].size() - 1, offs[s].data(), hs[s].data(),
                                 ps[s].data());
    if (st == MDE_OK) st = mde_set_ci(c, nd, coef.data(), up.data(), dn.data());
    c->in_rebase = false;
    if (st == MDE_OK) {
        c->ref_user[0] = ref[0];
        c->ref_user[1] = ref[1];
        if (ref[0] == 0) c->orb_perm[0].clear();
        if (ref[1] == 0) c->orb_perm[1].clear();
    }
    return st;
}

mde_status mde_sgauss_set_basis(mde_ctx *c, int32_t spin, int32_t nb, const double *centres,
                                const double *expo, const double *mo) {
    if (!c) return MDE_INVALID;
    if (c->bound) MDE_FAIL(c, MDE_STATE, "set the basis before binding the workspace");
    if (spin < 0 || spin > 1 || nb < 1 || nb > 3072) MDE_FAIL(c, MDE_INVALID, "bad basis (1..3072 functions)");
    c->nb[spin] = nb;
    c->centres[spin].assign(centres, centres + 3 * (size_t)nb);
    c->expo[spin].assign(expo, expo + nb);
    c->mo[spin].assign(mo, mo + (size_t)c->sp[spin].no * nb);
    return MDE_OK;
}

mde_status mde_workspace_bytes(const mde_ctx *cc, int32_t W, size_t *bytes) {
    mde_ctx *c = const_cast<mde_ctx *>(cc);
    if (!c || !bytes) return MDE_INVALID;
    if (!c->have_ci) MDE_FAIL(c, MDE_STATE, "set excitations and CI first");
    if (W < 1 || W > c->d.max_walkers) MDE_FAIL(c, MDE_INVALID, "W out of range");
    if (!c->bound) apply_default_plan(c, W);
    *bytes = carve(c, W, nullptr) + 256;
    return MDE_OK;
}

mde_status mde_bind_workspace(mde_ctx *c, int32_t W, void *dev, size_t bytes) {
    if (!c || !dev) return MDE_INVALID;
    if (c->bound) MDE_FAIL(c, MDE_STATE, "workspace already bound");
    if (!c->have_ci) MDE_FAIL(c, MDE_STATE, "set excitations and CI first");
    if (W < 1 || W > c->d.max_walkers) MDE_FAIL(c, MDE_INVALID, "W out of range");
    if (((uintptr_t)dev) % 256) MDE_FAIL(c, MDE_INVALID, "workspace must be 256-byte aligned");
    size_t need = 0;
    apply_default_plan(c, W);
    need = carve(c, W, nullptr);
    if (bytes < need) MDE_FAIL(c, MDE_NOMEM, "workspace has %zu bytes, needs %zu", bytes, need);
    c->W = W;
    c->ws = (char *)dev;
    c->ws_bytes = bytes;
    carve(c, W, c->ws);
    // upload the expansion
    for (int s = 0; s < 2; ++s) {
        SpinHost &sp = c->sp[s];
        SpinDev &S = c->h.s[s];
        S.n = sp.n;
        S.m = sp.m;
        S.no = sp.no;
        S.U = sp.U;
        S.max_order = sp.max_order;
        S.dense_k = sp.dense_k;
        S.n_user = sp.n_user;
        for (int k = 0; k < MAXK + 2; ++k) S.order_start[k] = sp.order_start[k];
        MDE_HIP(c, hipMemcpy((void *)S.ex, sp.ex.data(), sizeof(uint4) * sp.U, hipMemcpyHostToDevice));
        MDE_HIP(c, hipMemcpy((void *)S.ci_seg, sp.ci_seg.data(), sizeof(int) * (sp.U + 1),
                             hipMemcpyHostToDevice));
        MDE_HIP(c, hipMemcpy((void *)S.ci_other, sp.ci_other.data(), sizeof(int) * (c->n_det + PC_BATCH),
                             hipMemcpyHostToDevice));
        MDE_HIP(c, hipMemcpy((void *)S.ci_end, sp.ci_end.data(), sizeof(int) * (c->n_det + PC_BATCH),
                             hipMemcpyHostToDevice));
        MDE_HIP(c, hipMemset(S.coef_s + c->n_det, 0, sizeof(double) * PC_BATCH));
        MDE_HIP(c, hipMemcpy((void *)S.ci_idx, sp.ci_idx.data(), sizeof(int) * c->n_det,
                             hipMemcpyHostToDevice));
        MDE_HIP(c, hipMemcpy((void *)S.chunks, sp.chunks.data(), sizeof(int) * sp.chunks.size(),
                             hipMemcpyHostToDevice));
        if (!sp.pieces.empty()) {
            MDE_HIP(c, hipMemcpy((void *)S.pieces, sp.pieces.data(), sizeof(int4) * sp.pieces.size(),
                                 hipMemcpyHostToDevice));
            MDE_HIP(c, hipMemcpy((void *)S.longs, sp.longs.data(), sizeof(int4) * sp.longs.size(),
                                 hipMemcpyHostToDevice));
        }
        S.n_chunks = (int)sp.chunks.size() / 2;
        S.n_pieces = (int)sp.pieces.size();
        S.n_longs = (int)sp.longs.size();
        MDE_HIP(c, hipMemcpy((void *)S.inv_off, sp.inv_off.data(), sizeof(int) * sp.inv_off.size(),
                             hipMemcpyHostToDevice));
        if (!sp.inv_ent.empty())
            MDE_HIP(c, hipMemcpy((void *)S.inv_ent, sp.inv_ent.data(),
                                 sizeof(int) * sp.inv_ent.size(), hipMemcpyHostToDevice));
        MDE_HIP(c, hipMemcpy(c->d_perm_user[s], sp.iperm.data(), sizeof(int) * sp.U,
                             hipMemcpyHostToDevice));
        if (c->d_orb_perm[s])
            MDE_HIP(c, hipMemcpy(c->d_orb_perm[s], c->orb_perm[s].data(), sizeof(int32_t) * sp.no,
                                 hipMemcpyHostToDevice));
        if (c->nb[s] > 0) {
            MDE_HIP(c, hipMemcpy(c->d_centres[s], c->centres[s].data(),
                                 sizeof(double) * c->centres[s].size(), hipMemcpyHostToDevice));
            MDE_HIP(c, hipMemcpy(c->d_expo[s], c->expo[s].data(), sizeof(double) * c->expo[s].size(),
                                 hipMemcpyHostToDevice));
            MDE_HIP(c, hipMemcpy(c->d_mo[s], c->mo[s].data(), sizeof(double) * c->mo[s].size(),
                                 hipMemcpyHostToDevice));
        }
    }
    c->coef_gathered = false;
    MDE_HIP(c, hipMemcpy((void *)c->h.coef, c->coef.data(), sizeof(double) * c->n_det,
                         hipMemcpyHostToDevice));
    c->bound = true;
    mde_status st = apply_plan(c);
    if (st) return st;
    MDE_HIP(c, launch_init_misc(c->stream, c->d_inst, c->h));
    if (mde_status zs = zero_weights(c)) return zs;
    MDE_HIP(c, hipStreamSynchronize(c->stream));
    return MDE_OK;
}

mde_status mde_init(mde_ctx *c, int32_t W, const double *orb_up, const double *orb_dn,
                    double *log_abs_psi, double *sign_psi, int32_t *status) {
    if (!c) return MDE_INVALID;
    if (!c->bound) MDE_FAIL(c, MDE_STATE, "bind a workspace first");
    if (W != c->W) MDE_FAIL(c, MDE_INVALID, "W = %d, but the workspace is bound for %d walkers", W, c->W);
    if (!orb_up || !orb_dn) MDE_FAIL(c, MDE_INVALID, "orbital blocks required");
    MDE_HIP(c, launch_fill_i32(c->stream, c->h.st, 0, c->W));
    c->accept_count = 0;
    const double *ou = internal_orbitals(c, 0, orb_up, c->W * c->sp[0].n * 5, c->d_orbfull);
    const double *od = internal_orbitals(
        c, 1, orb_dn, c->W * c->sp[1].n * 5,
        c->d_orbfull ? c->d_orbfull + (size_t)c->W * c->sp[0].n * 5 * c->sp[0].no : nullptr);
    if (!ou || !od) MDE_FAIL(c, MDE_DEVICE, "orbital permutation launch failed");
    return full_eval(c, ou, od, log_abs_psi, sign_psi, status);
}

mde_status mde_set_reference(mde_ctx *c, int32_t ref_up, int32_t ref_dn) {
    if (!c) return MDE_INVALID;
    if (c->bound) MDE_FAIL(c, MDE_STATE, "the reference is fixed once the workspace is bound");
    if (!c->have_ci || c->u_coef.empty()) MDE_FAIL(c, MDE_STATE, "set excitations and CI first");
    const int32_t ref[2] = {ref_up, ref_dn};
    return rebase_expansion(c, ref);
}

mde_status mde_refresh(mde_ctx *c, double *log_abs_psi, double *sign_psi, int32_t *status) {
    if (!c) return MDE_INVALID;
    if (!c->initialized) MDE_FAIL(c, MDE_STATE, "call mde_init first");
    return full_eval(c, nullptr, nullptr, log_abs_psi, sign_psi, status);
}

static mde_status do_propose(mde_ctx *c, int32_t e, const double *orb, double *ratio, double *grad,
                             double *lap, int32_t *status) {
    if (!c) return MDE_INVALID;
    if (!c->initialized || c->adjoint_state) MDE_FAIL(c, MDE_STATE, "call mde_init/mde_refresh first");
    if (e < 0 || e >= c->d.n_elec[0] + c->d.n_elec[1]) MDE_FAIL(c, MDE_INVALID, "electron out of range");
    if (!orb) MDE_FAIL(c, MDE_INVALID, "orbital block required");
    int row;
    const int s = spin_of(c, e, &row);
    mde_status st = ensure_C(c, s);
    if (st) return st;
    orb = internal_orbitals(c, s, orb, c->W * 5, c->d_orbx);
    if (!orb) MDE_FAIL(c, MDE_DEVICE, "orbital permutation launch failed");
    MoveArgs m{};
    m.e = e;
    m.spin = s;
    m.row = row;
    m.new_orb = orb;
    m.ratio = ratio;
    m.grad = grad;
    m.lap = lap;
    m.status = status;
    const int nmax = c->h.nmax, mmax = c->h.mmax;
    SpinHost &sp = c->sp[s];
    // FP64 on 64-walker tiles (at most 8 electrons per spin): the
    // determinant kernel forms the proposal, k_post the commit's quantities
    const bool fused = c->d.precision == 0 && c->WT == 64 && !sp.items.empty() && sp.n <= 8;
    if (fused) {
        m.mode |= MV_FUSED;
    } else {
        const int split = prop_split(c->n_cu, c->h.s[s].n_tiles, nmax, mmax, c->WT);
        if (split == 0) MDE_FAIL(c, MDE_UNSUPPORTED, "proposal does not fit in LDS");
        MDE_HIP(c, launch_propose(c->stream, c->d_inst, 1, c->W, nullptr, m, c->d.precision, nmax,
                                  mmax, c->WT, c->h.s[s].n_tiles, split));
    }
    const bool prof = c->prof_on && 2 * (c->prof_used + 1) <= (int)c->prof_ev.size();
    if (prof) MDE_HIP(c, hipEventRecord(c->prof_ev[2 * c->prof_used], c->stream));
    // a profiled launch is issued prof_repeat times back to back: in this mode
    // the kernel writes only its partial sums and resets its own queues, so
    // every repeat leaves the same result
    const int reps = prof ? c->prof_repeat : 1;
    for (int r = 0; r < reps && !sp.items.empty(); ++r)
        MDE_HIP(c, launch_det(c->stream, c->d_inst, 1, c->d_items[s], c->d_bounds[s], sp.queues, sp.ex_cap,
                              nullptr, m, DM_PROPOSE, c->d.precision, c->WT, sp.lds_prop, sp.threads,
                              sp.grid, c->h.counter, nullptr, nullptr, sp.max_order));
    if (prof) {
        MDE_HIP(c, hipEventRecord(c->prof_ev[2 * c->prof_used + 1], c->stream));
        c->prof_used++;
    }
    if (fused)
        MDE_HIP(c, launch_post(c->stream, c->d_inst, m, c->h.s[s].n_tiles, sp.n));
    else
        MDE_HIP(c, launch_finish(c->stream, c->d_inst, 1, c->W, nullptr, m, c->h.counter));
    c->pending_e = e;
    c->pending_fused = fused;
    return MDE_OK;
}

mde_status mde_propose(mde_ctx *c, int32_t e, const double *new_orb, double *ratio, double *grad,
                       double *lap, int32_t *status) {
    return do_propose(c, e, new_orb, ratio, grad, lap, status);
}

mde_status mde_grad_lap(mde_ctx *c, int32_t e, const double *cur_orb, double *grad, double *lap,
                        int32_t *status) {
    return do_propose(c, e, cur_orb, nullptr, grad, lap, status);
}

mde_status mde_accept(mde_ctx *c, int32_t e, const uint8_t *accept) {
    if (!c) return MDE_INVALID;
    if (!c->initialized || c->adjoint_state) MDE_FAIL(c, MDE_STATE, "call mde_init first");
    if (c->pending_e != e) MDE_FAIL(c, MDE_STATE, "no pending proposal for electron %d", e);
    if (!accept) MDE_FAIL(c, MDE_INVALID, "accept mask required");
    int row;
    const int s = spin_of(c, e, &row);
    MoveArgs m{};
    m.e = e;
    m.spin = s;
    m.row = row;
    m.accept = accept;
    if (c->pending_fused) {
        m.mode |= MV_FUSED;
        MDE_HIP(c, launch_accept64f(c->stream, c->d_inst, m, c->h.s[s].n_tiles,
                                    row_split(c->n_cu, c->h.s[s].n_tiles, c->sp[s].n), c->sp[s].n));
    } else {
        MDE_HIP(c, launch_accept(c->stream, c->d_inst, 1, c->W, nullptr, m, c->d.precision, c->h.nmax,
                                 c->h.mmax, c->WT, c->h.s[s].n_tiles,
                                 row_split(c->n_cu, c->h.s[s].n_tiles, c->sp[s].n)));
    }
    c->R_valid[s] = false;
    c->C_valid[1 - s] = false;
    c->pending_e = -1;
    c->accept_count++;
    if (c->d.refresh_every > 0 && c->accept_count % c->d.refresh_every == 0)
        return full_eval(c, nullptr, nullptr, nullptr, nullptr, nullptr, c->d.precision != 0);
    return MDE_OK;
}

static mde_status local_derivs(mde_ctx *c, const double *orb_up, const double *orb_dn,
                               double *grad, double *lap, int32_t *status, bool no_alloc) {
    if (!c) return MDE_INVALID;
    if (!c->initialized || c->adjoint_state) MDE_FAIL(c, MDE_STATE, "call mde_init first");
    if (c->d.precision != MDE_FP64)
        MDE_FAIL(c, MDE_UNSUPPORTED, "all-electron derivatives are computed in the FP64 form");
    if (!orb_up || !orb_dn || !grad || !lap) MDE_FAIL(c, MDE_INVALID, "orbital blocks and outputs required");
    for (int s = 0; s < 2; ++s) {
        if (local_derivs_lds(c->sp[s].n, c->sp[s].m) > 160 * 1024 ||
            sizeof(double) * (size_t)c->sp[s].n * c->sp[s].m * lds_row_stride(c->WT) > 160 * 1024)
            MDE_FAIL(c, MDE_UNSUPPORTED, "spin %d: tables too large for the derivative kernels", s);
    }
    // ratios of both spins and the CI weights of both spins at the current positions
    for (int s = 0; s < 2; ++s)
        if (!c->R_valid[s]) {
            mde_status st = run_values(c, s);
            if (st) return st;
        }
    for (int s = 0; s < 2; ++s) {
        mde_status st = ensure_C(c, s);
        if (st) return st;
    }
    double *yz = c->h.gz;
    if (no_alloc) {
        for (int s = 0; s < 2; ++s)
            if ((size_t)c->W * c->sp[s].n * c->sp[s].m > LOCAL_SCRATCH_DOUBLES)
                MDE_FAIL(c, MDE_UNSUPPORTED,
                         "W x n x m = %zu exceeds the %zu doubles of the allocation-free scratch",
                         (size_t)c->W * c->sp[s].n * c->sp[s].m, LOCAL_SCRATCH_DOUBLES);
        MDE_HIP(c, local_scratch(&yz));
    }
    MDE_HIP(c, launch_inv_nold(c->stream, c->d_inst, c->h));
    const double *orb[2] = {orb_up, orb_dn};
    for (int s = 0; s < 2; ++s) {
        const double *o = internal_orbitals(c, s, orb[s], c->W * c->sp[s].n * 5, c->d_orbfull);
        if (!o) MDE_FAIL(c, MDE_DEVICE, "orbital permutation launch failed");
        MDE_HIP(c, launch_grad_T(c->stream, c->d_inst, c->h, s, nullptr, yz));
        MDE_HIP(c, launch_local_derivs(c->stream, c->d_inst, c->h, s, o, yz, grad, lap, status));
    }
    return MDE_OK;
}

mde_status mde_local_derivs(mde_ctx *c, const double *orb_up, const double *orb_dn, double *grad,
                            double *lap, int32_t *status) {
    return local_derivs(c, orb_up, orb_dn, grad, lap, status, false);
}

mde_status mde_local_derivs_noalloc(mde_ctx *c, const double *orb_up, const double *orb_dn,
                                    double *grad, double *lap, int32_t *status) {
    return local_derivs(c, orb_up, orb_dn, grad, lap, status, true);
}

mde_status mde_vmc(mde_ctx *c, int32_t n_steps, double tau, const double *normals,
                   const double *uniforms, double *pos, int32_t *accepted, int32_t *status) {
    if (!c) return MDE_INVALID;
    if (!c->initialized || c->adjoint_state) MDE_FAIL(c, MDE_STATE, "call mde_init first");
    if (c->nb[0] <= 0 || c->nb[1] <= 0)
        MDE_FAIL(c, MDE_STATE, "the loop evaluates orbitals with the s-Gaussian provider: set its basis");
    if (n_steps < 0 || !(tau > 0.0)) MDE_FAIL(c, MDE_INVALID, "need n_steps >= 0 and tau > 0");
    if (n_steps > 0 && (!normals || !uniforms || !pos || !accepted))
        MDE_FAIL(c, MDE_INVALID, "random inputs, positions and the acceptance counts are required");
    const int W = c->W, n_tot = c->d.n_elec[0] + c->d.n_elec[1];
    const int nomax = c->h.nomax;
    double *cur = c->d_vmc, *newp = cur + (size_t)W * 3, *g0 = newp + (size_t)W * 3;
    double *g1 = g0 + (size_t)W * 3, *ratio = g1 + (size_t)W * 3, *lap0 = ratio + W;
    double *lap1 = lap0 + W, *blk0 = lap1 + W, *blk1 = blk0 + (size_t)W * 5 * nomax;
    for (int step = 0; step < n_steps; ++step)
        for (int e = 0; e < n_tot; ++e) {
            int row;
            const int s = spin_of(c, e, &row);
            const size_t mv = (size_t)step * n_tot + e;
            // grad_e ln Psi at the current position (the drift)
            MDE_HIP(c, launch_vmc_drift(c->stream, W, n_tot, e, tau, pos, g0, nullptr, cur, newp, 0));
            MDE_HIP(c, launch_sgauss(c->stream, c->nb[s], c->d_centres[s], c->d_expo[s], c->sp[s].no,
                                     c->d_mo[s], W, cur, blk0));
            mde_status st = do_propose(c, e, blk0, nullptr, g0, lap0, status);
            if (st) return st;
            // the proposal and its ratio and gradient at R'
            MDE_HIP(c, launch_vmc_drift(c->stream, W, n_tot, e, tau, pos, g0, normals + mv * W * 3,
                                        cur, newp, 1));
            MDE_HIP(c, launch_sgauss(c->stream, c->nb[s], c->d_centres[s], c->d_expo[s], c->sp[s].no,
                                     c->d_mo[s], W, newp, blk1));
            st = do_propose(c, e, blk1, ratio, g1, lap1, status);
            if (st) return st;
            MDE_HIP(c, launch_vmc_decide(c->stream, W, n_tot, e, tau, pos, cur, newp, g0, g1, ratio,
                                         uniforms + mv * W, c->d_vmc_mask, accepted));
            st = mde_accept(c, e, c->d_vmc_mask);
            if (st) return st;
        }
    return MDE_OK;
}

mde_status mde_export(mde_ctx *c, int32_t what, int32_t spin, double *dst) {
    if (!c || !dst) return MDE_INVALID;
    if (!c->initialized) MDE_FAIL(c, MDE_STATE, "nothing to export yet");
    if (spin < 0 || spin > 1 || what < 0 || what > 4) MDE_FAIL(c, MDE_INVALID, "bad export request");
    if (what == 2 && !c->R_valid[spin]) {
        mde_status st = run_values(c, spin);
        if (st) return st;
    }
    MDE_HIP(c, launch_export(c->stream, c->d_inst, c->h, what, spin, dst, c->d_perm_user[spin]));
    return MDE_OK;
}

mde_status mde_eval_tables(mde_ctx *c, int32_t W, const double *T_up, const double *T_dn,
                           const double *coef, double *log_abs, double *sign, int32_t *status) {
    if (!c) return MDE_INVALID;
    if (!c->bound) MDE_FAIL(c, MDE_STATE, "bind a workspace first");
    if (W != c->W) MDE_FAIL(c, MDE_INVALID, "W = %d, but the workspace is bound for %d walkers", W, c->W);
    if (c->d.precision != MDE_FP64) MDE_FAIL(c, MDE_UNSUPPORTED, "the adjoint path is FP64");
    if (!T_up || !T_dn || !coef) MDE_FAIL(c, MDE_INVALID, "tables and coefficients required");
    MDE_HIP(c, launch_fill_i32(c->stream, c->h.st, 0, c->W));
    MDE_HIP(c, launch_coef_gather(c->stream, c->d_inst, c->h, coef));
    c->coef_gathered = false;
    mde_status st = run_values(c, 0, T_up, T_dn);
    if (st) return st;
    st = run_values(c, 1, T_up, T_dn);
    if (st) return st;
    for (int s = 0; s < 2; ++s)
        MDE_HIP(c, launch_precontract(c->stream, c->d_inst, c->h, s, coef));
    MDE_HIP(c, launch_nsum(c->stream, c->d_inst, c->h, log_abs, sign, status, 0));
    // the context's move state is now that of the explicit tables
    c->last_T[0] = T_up;
    c->last_T[1] = T_dn;
    c->adjoint_state = true;
    c->R_valid[0] = c->R_valid[1] = true;
    c->C_valid[0] = c->C_valid[1] = true;
    c->pending_e = -1;
    return MDE_OK;
}

mde_status mde_backward(mde_ctx *c, const double *go, double *grad_coef, double *grad_T_up,
                        double *grad_T_dn, int32_t *status) {
    if (!c) return MDE_INVALID;
    if (!c->adjoint_state) MDE_FAIL(c, MDE_STATE, "call mde_eval_tables first");
    if (!go) MDE_FAIL(c, MDE_INVALID, "upstream gradient required");
    // the cofactors are taken from the tables given to mde_eval_tables; the
    // caller keeps those buffers unchanged until this call
    MDE_HIP(c, launch_backward(c->stream, c->d_inst, c->h, go, nullptr, nullptr, grad_coef,
                               grad_T_up, grad_T_dn, c->last_T[0], c->last_T[1]));
    if (status && (grad_T_up || grad_T_dn))
        MDE_HIP(c, launch_flag_nonfinite(c->stream, c->W, grad_T_up, c->sp[0].n * c->sp[0].m,
                                         grad_T_dn, c->sp[1].n * c->sp[1].m, status));
    return MDE_OK;
}


mde_status mde_set_plan(mde_ctx *c, int32_t spin, int32_t walker_tile, int32_t item_exc,
                        int32_t threads) {
    if (!c) return MDE_INVALID;
    if (spin < 0 || spin > 1) MDE_FAIL(c, MDE_INVALID, "spin must be 0 or 1");
    if (c->capturing) MDE_FAIL(c, MDE_STATE, "cannot re-plan during capture");
    if (walker_tile) {
        if (walker_tile < 1 || walker_tile > 64 || (walker_tile & (walker_tile - 1)))
            MDE_FAIL(c, MDE_INVALID, "walker tile must be a power of two in 1..64");
    }
    const int wt_new = walker_tile ? walker_tile : c->WT;
    if (threads) {
        if (threads < 64 || threads > max_threads(wt_new) || threads % 64)
            MDE_FAIL(c, MDE_INVALID, "bad thread count (64..%d, a multiple of 64, for walker tile %d)",
                     max_threads(wt_new), wt_new);
    }
    if (c->user_thr[1 - spin] && c->sp[1 - spin].threads > max_threads(wt_new))
        MDE_FAIL(c, MDE_INVALID, "the other spin's thread count exceeds %d for walker tile %d",
                 max_threads(wt_new), wt_new);
    if (walker_tile) {
        c->WT = walker_tile;
        c->user_wt = true;
    }
    if (threads) {
        c->sp[spin].threads = threads;
        c->user_thr[spin] = true;
    }
    for (int s = 0; s < 2; ++s)
        if (c->sp[s].threads > max_threads(c->WT)) c->sp[s].threads = default_threads(c->WT);
    if (item_exc) {
        if (item_exc < 1) MDE_FAIL(c, MDE_INVALID, "bad item size");
        c->sp[spin].item_exc = item_exc;
        c->user_item[spin] = true;
    }
    for (int s = 0; s < 2; ++s)
        if (c->sp[s].threads < c->WT) c->sp[s].threads = std::max(64, c->WT);
    if (!c->bound) return MDE_OK;
    mde_status st = apply_plan(c);
    if (st) return st;
    c->initialized = false;   // R and C layouts depend on the tile: re-init needed
    MDE_HIP(c, launch_init_misc(c->stream, c->d_inst, c->h));
    if (mde_status zs = zero_weights(c)) return zs;
    return MDE_OK;
}

mde_status mde_debug_items(const mde_ctx *c, int32_t spin, int32_t W, int32_t walker_tile,
                           int32_t item_exc, int32_t threads, int32_t *items, int32_t items_cap,
                           int32_t *n_items, int32_t *ranges, int32_t ranges_cap,
                           int32_t *n_ranges, int32_t *layout) {
    if (!c || spin < 0 || spin > 1 || W < 1 || item_exc < 1 || !n_items || !n_ranges)
        return MDE_INVALID;
    if (walker_tile < 1 || walker_tile > 64 || (walker_tile & (walker_tile - 1))) return MDE_INVALID;
    if (threads < walker_tile || threads > max_threads(walker_tile) || threads % 64) return MDE_INVALID;
    const SpinHost &sp = c->sp[spin];
    if (!sp.have || sp.ucost.empty()) return MDE_STATE;
    std::vector<WorkItem> it;
    std::vector<int> ts;
    std::vector<int32_t> bd;
    build_items(sp, W, walker_tile, item_exc, threads, it, ts, spin, &bd);
    *n_items = (int32_t)it.size();
    *n_ranges = (int32_t)bd.size();
    if (layout) {
        int da, db;
        dense_range(sp, da, db);
        layout[0] = sp.U;
        layout[1] = da;
        layout[2] = db;
        layout[3] = sp.dense_k;
    }
    if ((int)it.size() > items_cap || (int)bd.size() > ranges_cap) return MDE_NOMEM;
    for (size_t i = 0; i < it.size(); ++i) {
        const WorkItem &w = it[i];
        const int32_t v[10] = {w.inst, w.spin, w.tile, w.order, w.u0, w.u1, w.slot, w.wb, w.d0, w.d1};
        if (items) std::copy(v, v + 10, items + 10 * i);
    }
    if (ranges) std::copy(bd.begin(), bd.end(), ranges);
    return MDE_OK;
}

mde_status mde_get_plan(const mde_ctx *c, int32_t spin, int32_t *walker_tile, int32_t *item_exc,
                        int32_t *threads) {
    if (!c || spin < 0 || spin > 1) return MDE_INVALID;
    if (walker_tile) *walker_tile = c->WT;
    if (item_exc) *item_exc = c->sp[spin].item_exc;
    if (threads) *threads = c->sp[spin].threads;
    return MDE_OK;
}

// internal re-plan that keeps the state valid (values + C + N recomputed
// from the kept orbitals)
static mde_status replan_keep_state(mde_ctx *c, const Plan &p) {
    c->WT = p.WT;
    for (int s = 0; s < 2; ++s) {
        c->sp[s].threads = std::max(p.threads[s], std::max(64, p.WT));
        c->sp[s].item_exc = p.item_exc[s];
    }
    mde_status st = apply_plan(c);
    if (st) return st;
    MDE_HIP(c, launch_init_misc(c->stream, c->d_inst, c->h));
    if (mde_status zs = zero_weights(c)) return zs;
    return full_eval(c, nullptr, nullptr, nullptr, nullptr, nullptr);
}

static std::string shape_key(const mde_ctx *c) {
    std::ostringstream o;
    o << "v1 prec=" << c->d.precision << " W=" << c->W;
    for (int s = 0; s < 2; ++s) {
        const SpinHost &sp = c->sp[s];
        o << " s" << s << ":n=" << sp.n << ",m=" << sp.m << ",U=" << sp.U << ",k=";
        for (int k = 1; k <= sp.max_order; ++k)
            o << (sp.order_start[k + 1] - sp.order_start[k]) << (k < sp.max_order ? "/" : "");
    }
    o << " ndet=" << c->n_det;
    return o.str();
}

mde_status mde_autotune(mde_ctx *c, const double *new_orb_up, const double *new_orb_dn,
                        const char *cache_path) {
    if (!c) return MDE_INVALID;
    if (!c->initialized || c->adjoint_state) MDE_FAIL(c, MDE_STATE, "call mde_init first");
    if (c->capturing) MDE_FAIL(c, MDE_STATE, "cannot tune during capture");
    const std::string key = shape_key(c);
    if (cache_path) {
        std::ifstream f(cache_path);
        std::string line;
        while (std::getline(f, line)) {
            const size_t bar = line.find(" | ");
            if (bar == std::string::npos || line.substr(0, bar) != key) continue;
            Plan p{};
            if (sscanf(line.c_str() + bar + 3, "%d %d %d %d %d", &p.WT, &p.item_exc[0], &p.threads[0],
                       &p.item_exc[1], &p.threads[1]) == 5)
                return replan_keep_state(c, p);
        }
    }
    const double *orb[2] = {new_orb_up, new_orb_dn};
    const int e_of[2] = {0, c->d.n_elec[0]};
    hipEvent_t e0, e1;
    MDE_HIP(c, hipEventCreate(&e0));
    MDE_HIP(c, hipEventCreate(&e1));
    double best_t = 1e30;
    Plan best = default_plan(c, c->W);
    best.WT = c->WT;
    for (int s = 0; s < 2; ++s) {
        best.item_exc[s] = c->sp[s].item_exc;
        best.threads[s] = c->sp[s].threads;
    }
    std::vector<Plan> cands = candidate_plans(c, c->W);
    cands.insert(cands.begin(), best);
    for (const Plan &p : cands) {
        mde_status st = replan_keep_state(c, p);
        if (st) {
            c->err.clear();
            continue;
        }
        // one warm proposal per spin, then timed: 3 proposals per spin
        double total = 0.0;
        bool ok = true;
        for (int s = 0; s < 2 && ok; ++s) {
            if (!orb[s]) continue;
            if (do_propose(c, e_of[s], orb[s], nullptr, nullptr, nullptr, nullptr)) { ok = false; break; }
            MDE_HIP(c, hipEventRecord(e0, c->stream));
            for (int r = 0; r < 3; ++r)
                if (do_propose(c, e_of[s], orb[s], nullptr, nullptr, nullptr, nullptr)) ok = false;
            MDE_HIP(c, hipEventRecord(e1, c->stream));
            MDE_HIP(c, hipEventSynchronize(e1));
            float ms = 0.f;
            MDE_HIP(c, hipEventElapsedTime(&ms, e0, e1));
            total += ms;
        }
        if (ok && total < best_t) {
            best_t = total;
            best = p;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    mde_status st = replan_keep_state(c, best);
    if (st) return st;
    c->pending_e = -1;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        f << key << " | " << best.WT << " " << best.item_exc[0] << " " << best.threads[0] << " "
          << best.item_exc[1] << " " << best.threads[1] << "\n";
    }
    return MDE_OK;
}

// ---- profiling ----------------------------------------------------------------

static void prof_free(mde_ctx *c) {
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    c->prof_ev.clear();
    c->prof_used = 0;
    c->prof_on = false;
}

mde_status mde_profile_enable(mde_ctx *c, int32_t max_launches, int32_t repeat) {
    if (!c) return MDE_INVALID;
    if (max_launches < 1 || max_launches > 1 << 16) MDE_FAIL(c, MDE_INVALID, "bad launch count");
    if (repeat < 1 || repeat > 64) MDE_FAIL(c, MDE_INVALID, "bad repeat count");
    if (c->capturing) MDE_FAIL(c, MDE_STATE, "enable profiling before capture");
    prof_free(c);
    c->prof_ev.resize(2 * (size_t)max_launches);
    for (auto &e : c->prof_ev)
        MDE_HIP(c, hipEventCreate(&e));
    c->prof_repeat = repeat;
    c->prof_on = true;
    return MDE_OK;
}

mde_status mde_profile_read(mde_ctx *c, double *total_ms, int32_t *count) {
    if (!c || !total_ms || !count) return MDE_INVALID;
    double t = 0.0;
    for (int i = 0; i < c->prof_used; ++i) {
        float ms = 0.f;
        MDE_HIP(c, hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]));
        t += ms;
    }
    *total_ms = t;
    *count = c->prof_used * c->prof_repeat;
    return MDE_OK;
}

mde_status mde_profile_disable(mde_ctx *c) {
    if (!c) return MDE_INVALID;
    prof_free(c);
    return MDE_OK;
}

// ---- graphs -----------------------------------------------------------------

mde_status mde_capture_begin(mde_ctx *c) {
    if (!c) return MDE_INVALID;
    if (c->capturing) MDE_FAIL(c, MDE_STATE, "already capturing");
    MDE_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    return MDE_OK;
}

mde_status mde_capture_end(mde_ctx *c, mde_graph **out) {
    if (!c || !out) return MDE_INVALID;
    if (!c->capturing) MDE_FAIL(c, MDE_STATE, "not capturing");
    c->capturing = false;
    mde_graph *g = new (std::nothrow) mde_graph();
    if (!g) return MDE_NOMEM;
    hipError_t e = hipStreamEndCapture(c->stream, &g->graph);
    if (e != hipSuccess) {
        delete g;
        MDE_FAIL(c, MDE_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        delete g;
        MDE_FAIL(c, MDE_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    *out = g;
    return MDE_OK;
}

mde_status mde_graph_launch(mde_graph *g, void *hip_stream) {
    if (!g) return MDE_INVALID;
    return hipGraphLaunch(g->exec, (hipStream_t)hip_stream) == hipSuccess ? MDE_OK : MDE_DEVICE;
}

mde_status mde_graph_destroy(mde_graph *g) {
    if (!g) return MDE_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return MDE_OK;
}

// ---- s-Gaussian provider ------------------------------------------------------

mde_status mde_sgauss_eval(mde_ctx *c, int32_t spin, int32_t npos, const double *pos, double *out) {
    if (!c) return MDE_INVALID;
    if (!c->bound) MDE_FAIL(c, MDE_STATE, "bind a workspace first");
    if (spin < 0 || spin > 1 || c->nb[spin] == 0) MDE_FAIL(c, MDE_STATE, "no basis for this spin");
    if (npos < 0 || (npos > 0 && (!pos || !out))) MDE_FAIL(c, MDE_INVALID, "bad positions");
    MDE_HIP(c, launch_sgauss(c->stream, c->nb[spin], c->d_centres[spin], c->d_expo[spin],
                             c->sp[spin].no, c->d_mo[spin], npos, pos, out));
    return MDE_OK;
}

// ---- uneven batch --------------------------------------------------------------

#define MDE_GFAIL(g, code, ...)                                  \
    do {                                                         \
        char _b[512];                                            \
        snprintf(_b, sizeof(_b), __VA_ARGS__);                   \
        if (g) (g)->err = _b;                                    \
        return code;                                             \
    } while (0)

static size_t group_items(mde_ctx *const *ctxs, int n) {
    size_t t = 0;
    for (int i = 0; i < n; ++i) t += ctxs[i]->sp[0].items.size() + ctxs[i]->sp[1].items.size();
    return t;
}

static mde_status hgroup_workspace_bytes(mde_ctx *const *ctxs, int32_t n, size_t *bytes) {
    if (!ctxs || n < 1 || !bytes) return MDE_INVALID;
    size_t max_items = 0;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i] || !ctxs[i]->bound) return MDE_STATE;
        size_t mi = 0;
        carve(ctxs[i], ctxs[i]->W, nullptr, &mi);
        max_items += mi;
    }
    Carver cv{nullptr};
    cv.take<InstDev>(n);
    cv.take<MoveArgs>(n);
    cv.take<WorkItem>(max_items);
    cv.take<int32_t>(max_items * 2 * (1024 / 64));
    *bytes = cv.off + 256;
    return MDE_OK;
}

static mde_status group_rebuild(mde_group *g) {
    const int n = (int)g->ctx.size();
    std::vector<WorkItem> all;
    std::vector<double> cost;
    std::vector<int32_t> bounds;
    g->lds = 0;
    g->maxW = 0;
    g->nmax = 0;
    g->mmax = 0;
    {
        int thr = 64;
        for (int i = 0; i < n; ++i)
            for (int s = 0; s < 2; ++s) thr = std::max(thr, g->ctx[i]->sp[s].threads);
        g->threads = std::min(std::max(thr, g->WT), max_threads(g->WT));
    }
    for (int i = 0; i < n; ++i) {
        mde_ctx *c = g->ctx[i];
        g->maxW = std::max(g->maxW, c->W);
        g->max_order = std::max(g->max_order, std::max(c->sp[0].max_order, c->sp[1].max_order));
        g->nmax = std::max(g->nmax, c->h.nmax);
        g->mmax = std::max(g->mmax, c->h.mmax);
        for (int s = 0; s < 2; ++s) {
            g->ex_cap = std::max(g->ex_cap, c->sp[s].ex_cap);
            for (WorkItem it : c->sp[s].items) {
                it.inst = i;
                if (g->WT == 64) {
                    double cst = 0.0;
                    for (int u = it.u0; u < it.u1; ++u) cst += c->sp[s].ucost[u];
                    for (int u = it.d0; u < it.d1; ++u) cst += c->sp[s].ucost[u];
                    cost.push_back(cst);
                    it.wb = (int)bounds.size();
                    item_wave_ranges(c->sp[s], it, g->threads / 64, bounds);
                } else {
                    cost.push_back(order_cost(it.order) * (it.u1 - it.u0) * c->WT);
                }
                all.push_back(it);
            }
        }
    }
    for (int i = 0; i < n; ++i)
        for (int s = 0; s < 2; ++s) {
            mde_ctx *c = g->ctx[i];
            g->lds = std::max(g->lds, det_lds(c->sp[s], c->WT, g->threads, c->d.precision, true,
                                              g->ex_cap));
        }
    std::vector<WorkItem> sorted = all;
    g->queues = queue_order(sorted, cost);
    g->n_items = (int)sorted.size();
    if (!sorted.empty())
        if (hipMemcpy(g->d_items, sorted.data(), sizeof(WorkItem) * sorted.size(),
                      hipMemcpyHostToDevice) != hipSuccess)
            MDE_GFAIL(g, MDE_DEVICE, "upload of group items failed");
    if (!bounds.empty())
        if (hipMemcpy(g->d_bounds, bounds.data(), sizeof(int32_t) * bounds.size(),
                      hipMemcpyHostToDevice) != hipSuccess)
            MDE_GFAIL(g, MDE_DEVICE, "upload of group wave ranges failed");
    std::vector<InstDev> insts(n);
    for (int i = 0; i < n; ++i) insts[i] = g->ctx[i]->h;
    if (hipMemcpy(g->d_insts, insts.data(), sizeof(InstDev) * n, hipMemcpyHostToDevice) != hipSuccess)
        MDE_GFAIL(g, MDE_DEVICE, "upload of group descriptors failed");
    const size_t lds = std::max<size_t>(g->lds, 1024);
    int per_cu = (int)std::min<size_t>(160 * 1024 / lds, 2048 / g->threads);
    per_cu = std::max(per_cu, 1);
    g->grid = std::max(1, (int)std::min<size_t>(sorted.size(), (size_t)g->ctx[0]->n_cu * per_cu));
    g->plan_gen.resize(n);
    for (int i = 0; i < n; ++i) g->plan_gen[i] = g->ctx[i]->plan_gen;
    return MDE_OK;
}

static mde_status hgroup_create(mde_ctx *const *ctxs, int32_t n, void *dev, size_t bytes,
                               mde_group **out) {
    if (!ctxs || n < 1 || !out || !dev) return MDE_INVALID;
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i] || !ctxs[i]->bound) return MDE_STATE;
        if (ctxs[i]->stream != ctxs[0]->stream || ctxs[i]->d.precision != ctxs[0]->d.precision)
            return MDE_INVALID;
        if (ctxs[i]->d_orb_perm[0] || ctxs[i]->d_orb_perm[1]) return MDE_UNSUPPORTED;
    }
    size_t need = 0;
    if (hgroup_workspace_bytes(ctxs, n, &need) != MDE_OK || bytes < need) return MDE_NOMEM;
    mde_group *g = new (std::nothrow) mde_group();
    if (!g) return MDE_NOMEM;
    g->ctx.assign(ctxs, ctxs + n);
    g->stream = ctxs[0]->stream;
    g->prec = ctxs[0]->d.precision;
    // every instance of the launch must share one walker tile (set it with
    // mde_set_plan before binding); blocks use the largest thread count
    int thr = 64;
    for (int i = 0; i < n; ++i) {
        if (ctxs[i]->WT != ctxs[0]->WT) {
            delete g;
            return MDE_INVALID;
        }
        for (int s = 0; s < 2; ++s) thr = std::max(thr, ctxs[i]->sp[s].threads);
    }
    g->WT = ctxs[0]->WT;
    g->threads = std::min(std::max(thr, g->WT), max_threads(g->WT));
    Carver cv{(char *)dev};
    g->d_insts = cv.take<InstDev>(n);
    g->d_moves = cv.take<MoveArgs>(n);
    size_t max_items = 0;
    for (int i = 0; i < n; ++i) {
        size_t mi = 0;
        carve(ctxs[i], ctxs[i]->W, nullptr, &mi);
        max_items += mi;
    }
    g->d_items = cv.take<WorkItem>(max_items);
    g->d_bounds = cv.take<int32_t>(max_items * 2 * (1024 / 64));
    g->hmoves.assign(n, MoveArgs{});
    mde_status st = group_rebuild(g);
    if (st) {
        delete g;
        return st;
    }
    *out = g;
    return MDE_OK;
}

static void hgroup_destroy(mde_group *g) { delete g; }

// Write the per-instance move arguments to the device array the kernels
// read, stream-ordered, as arguments of small copy kernels: nothing is read
// from host memory when the copy runs, so a captured graph carries the
// arguments of the captured call by value and the call allocates nothing.
static mde_status group_upload(mde_group *g) {
    const int n = (int)g->ctx.size();
    if (launch_set_moves(g->stream, g->d_moves, g->hmoves.data(), n) != hipSuccess)
        MDE_GFAIL(g, MDE_DEVICE, "argument upload");
    return MDE_OK;
}

// A member whose plan changed since the group copied its work items (a
// mde_set_plan + refresh or mde_autotune) has a new table layout: rebuild
// the group's items from it, outside a capture; members must still share
// one walker tile.
static mde_status group_check_plans(mde_group *g) {
    bool stale = false;
    for (size_t i = 0; i < g->ctx.size(); ++i) stale |= g->ctx[i]->plan_gen != g->plan_gen[i];
    if (!stale) return MDE_OK;
    if (g->capturing)
        MDE_GFAIL(g, MDE_STATE, "a member's plan changed since the group was built; "
                                "call the group outside a capture first");
    for (size_t i = 0; i < g->ctx.size(); ++i)
        if (g->ctx[i]->WT != g->WT)
            MDE_GFAIL(g, MDE_STATE, "instance %zu changed its walker tile (%d, group %d)", i,
                      g->ctx[i]->WT, g->WT);
    return group_rebuild(g);
}

static mde_status hgroup_propose(mde_group *g, const int32_t *e, const double *const *new_orb,
                                 double *const *ratio, double *const *grad, double *const *lap,
                                 int32_t *const *status) {
    if (!g || !e || !new_orb) return MDE_INVALID;
    const int n = (int)g->ctx.size();
    {
        mde_status pst = group_check_plans(g);
        if (pst) return pst;
    }
    for (int i = 0; i < n; ++i) {
        mde_ctx *c = g->ctx[i];
        if (!c->initialized || c->adjoint_state) MDE_GFAIL(g, MDE_STATE, "instance %d not initialised", i);
        if (e[i] < 0 || e[i] >= c->d.n_elec[0] + c->d.n_elec[1])
            MDE_GFAIL(g, MDE_INVALID, "instance %d: electron out of range", i);
        int row;
        const int s = spin_of(c, e[i], &row);
        mde_status st = ensure_C(c, s);
        if (st) MDE_GFAIL(g, st, "instance %d: %s", i, c->err.c_str());
        MoveArgs &m = g->hmoves[i];
        m = MoveArgs{};
        m.e = e[i];
        m.spin = s;
        m.row = row;
        m.new_orb = new_orb[i];
        m.ratio = ratio ? ratio[i] : nullptr;
        m.grad = grad ? grad[i] : nullptr;
        m.lap = lap ? lap[i] : nullptr;
        m.status = status ? status[i] : nullptr;
    }
    mde_status st = group_upload(g);
    if (st) return st;
    const MoveArgs none = no_move();
    const int gt = (g->maxW + g->WT - 1) / g->WT;
    const int split = prop_split(g->ctx[0]->n_cu, gt * n, g->nmax, g->mmax, g->WT);
    if (split == 0) MDE_GFAIL(g, MDE_UNSUPPORTED, "proposal does not fit in LDS");
    if (launch_propose(g->stream, g->d_insts, n, g->maxW, g->d_moves, none, g->prec, g->nmax,
                       g->mmax, g->WT, gt, split) != hipSuccess)
        MDE_GFAIL(g, MDE_DEVICE, "propose launch");
    if (launch_det(g->stream, g->d_insts, n, g->d_items, g->d_bounds, g->queues, g->ex_cap, g->d_moves, none,
                   DM_PROPOSE, g->prec, g->WT, g->lds, g->threads, g->grid, g->ctx[0]->h.counter,
                   nullptr, nullptr, g->max_order) != hipSuccess)
        MDE_GFAIL(g, MDE_DEVICE, "determinant launch");
    if (launch_finish(g->stream, g->d_insts, n, g->maxW, g->d_moves, none, nullptr) != hipSuccess)
        MDE_GFAIL(g, MDE_DEVICE, "finish launch");
    for (int i = 0; i < n; ++i) {
        g->ctx[i]->pending_e = e[i];
        g->ctx[i]->pending_fused = false;
    }
    return MDE_OK;
}

static mde_status hgroup_accept(mde_group *g, const int32_t *e, const uint8_t *const *accept) {
    if (!g || !e || !accept) return MDE_INVALID;
    const int n = (int)g->ctx.size();
    {
        mde_status pst = group_check_plans(g);
        if (pst) return pst;
    }
    for (int i = 0; i < n; ++i) {
        mde_ctx *c = g->ctx[i];
        if (c->pending_e != e[i]) MDE_GFAIL(g, MDE_STATE, "instance %d: no pending proposal", i);
        int row;
        const int s = spin_of(c, e[i], &row);
        MoveArgs &m = g->hmoves[i];
        m = MoveArgs{};
        m.e = e[i];
        m.spin = s;
        m.row = row;
        m.accept = accept[i];
    }
    mde_status st = group_upload(g);
    if (st) return st;
    const MoveArgs none = no_move();
    const int gt = (g->maxW + g->WT - 1) / g->WT;
    if (launch_accept(g->stream, g->d_insts, n, g->maxW, g->d_moves, none, g->prec, g->nmax,
                      g->mmax, g->WT, gt, row_split(g->ctx[0]->n_cu, gt * n, g->nmax)) != hipSuccess)
        MDE_GFAIL(g, MDE_DEVICE, "accept launch");
    for (int i = 0; i < n; ++i) {
        mde_ctx *c = g->ctx[i];
        int row;
        const int s = spin_of(c, e[i], &row);
        c->R_valid[s] = false;
        c->C_valid[1 - s] = false;
        c->pending_e = -1;
        c->accept_count++;
        if (c->d.refresh_every > 0 && c->accept_count % c->d.refresh_every == 0) {
            mde_status r = full_eval(c, nullptr, nullptr, nullptr, nullptr, nullptr,
                                     c->d.precision != 0);
            if (r) MDE_GFAIL(g, r, "instance %d refresh: %s", i, c->err.c_str());
        }
    }
    return MDE_OK;
}

mde_status mde_group_capture_begin(mde_group *g) {
    if (!g) return MDE_INVALID;
    if (g->capturing) MDE_GFAIL(g, MDE_STATE, "already capturing");
    if (hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        MDE_GFAIL(g, MDE_DEVICE, "begin capture");
    g->capturing = true;
    for (mde_group *q : g->subs) q->capturing = true;
    for (mde_ctx *c : g->ctx) c->capturing = true;
    return MDE_OK;
}

mde_status mde_group_capture_end(mde_group *g, mde_graph **out) {
    if (!g || !out) return MDE_INVALID;
    if (!g->capturing) MDE_GFAIL(g, MDE_STATE, "not capturing");
    g->capturing = false;
    for (mde_group *q : g->subs) q->capturing = false;
    for (mde_ctx *c : g->ctx) c->capturing = false;
    mde_graph *gr = new (std::nothrow) mde_graph();
    if (!gr) return MDE_NOMEM;
    if (hipStreamEndCapture(g->stream, &gr->graph) != hipSuccess) {
        delete gr;
        MDE_GFAIL(g, MDE_DEVICE, "end capture");
    }
    if (hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(gr->graph);
        delete gr;
        MDE_GFAIL(g, MDE_DEVICE, "instantiate");
    }
    *out = gr;
    return MDE_OK;
}

// members grouped by walker tile, widest first
static std::vector<std::vector<int>> tile_classes(mde_ctx *const *ctxs, int n) {
    std::map<int, std::vector<int>, std::greater<int>> m;
    for (int i = 0; i < n; ++i) m[ctxs[i]->WT].push_back(i);
    std::vector<std::vector<int>> out;
    for (auto &kv : m) out.push_back(kv.second);
    return out;
}

mde_status mde_group_workspace_bytes(mde_ctx *const *ctxs, int32_t n, size_t *bytes) {
    if (!ctxs || n < 1 || !bytes) return MDE_INVALID;
    for (int i = 0; i < n; ++i)
        if (!ctxs[i] || !ctxs[i]->bound) return MDE_STATE;
    const auto cls = tile_classes(ctxs, n);
    if (cls.size() == 1) return hgroup_workspace_bytes(ctxs, n, bytes);
    size_t tot = 0;
    for (const auto &idx : cls) {
        std::vector<mde_ctx *> cs;
        for (int i : idx) cs.push_back(ctxs[i]);
        size_t b = 0;
        mde_status st = hgroup_workspace_bytes(cs.data(), (int)cs.size(), &b);
        if (st) return st;
        tot += align_up(b, 256);
    }
    *bytes = tot;
    return MDE_OK;
}

mde_status mde_group_create(mde_ctx *const *ctxs, int32_t n, void *dev, size_t bytes,
                            mde_group **out) {
    if (!ctxs || n < 1 || !out || !dev) return MDE_INVALID;
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i] || !ctxs[i]->bound) return MDE_STATE;
        if (ctxs[i]->stream != ctxs[0]->stream || ctxs[i]->d.precision != ctxs[0]->d.precision)
            return MDE_INVALID;
    }
    const auto cls = tile_classes(ctxs, n);
    if (cls.size() == 1) return hgroup_create(ctxs, n, dev, bytes, out);
    size_t need = 0;
    if (mde_group_workspace_bytes(ctxs, n, &need) != MDE_OK || bytes < need) return MDE_NOMEM;
    mde_group *g = new (std::nothrow) mde_group();
    if (!g) return MDE_NOMEM;
    g->ctx.assign(ctxs, ctxs + n);
    g->stream = ctxs[0]->stream;
    g->prec = ctxs[0]->d.precision;
    size_t off = 0;
    for (const auto &idx : cls) {
        std::vector<mde_ctx *> cs;
        for (int i : idx) cs.push_back(ctxs[i]);
        size_t b = 0;
        mde_group *sub = nullptr;
        mde_status st = hgroup_workspace_bytes(cs.data(), (int)cs.size(), &b);
        if (st == MDE_OK) st = hgroup_create(cs.data(), (int)cs.size(), (char *)dev + off, b, &sub);
        if (st) {
            for (mde_group *q : g->subs) hgroup_destroy(q);
            delete g;
            return st;
        }
        g->subs.push_back(sub);
        g->sub_idx.push_back(idx);
        off += align_up(b, 256);
    }
    *out = g;
    return MDE_OK;
}

mde_status mde_group_destroy(mde_group *g) {
    if (!g) return MDE_OK;
    for (mde_group *q : g->subs) hgroup_destroy(q);
    hgroup_destroy(g);
    return MDE_OK;
}

}  // extern "C"

template <typename T>
static std::vector<T> gather_args(const T *a, const std::vector<int> &idx) {
    std::vector<T> out;
    if (!a) return out;
    for (int i : idx) out.push_back(a[i]);
    return out;
}

template <typename T>
static const T *ptr_or_null(const std::vector<T> &v) {
    return v.empty() ? nullptr : v.data();
}

extern "C" {

mde_status mde_group_propose(mde_group *g, const int32_t *e, const double *const *new_orb,
                             double *const *ratio, double *const *grad, double *const *lap,
                             int32_t *const *status) {
    if (!g || !e || !new_orb) return MDE_INVALID;
    if (g->subs.empty()) return hgroup_propose(g, e, new_orb, ratio, grad, lap, status);
    for (size_t k = 0; k < g->subs.size(); ++k) {
        const auto &idx = g->sub_idx[k];
        const auto ee = gather_args(e, idx);
        const auto no = gather_args(new_orb, idx);
        const auto ra = gather_args(ratio, idx);
        const auto gr = gather_args(grad, idx);
        const auto la = gather_args(lap, idx);
        const auto stt = gather_args(status, idx);
        mde_status st = hgroup_propose(g->subs[k], ee.data(), no.data(), ptr_or_null(ra), ptr_or_null(gr),
                                       ptr_or_null(la), ptr_or_null(stt));
        if (st) MDE_GFAIL(g, st, "walker-tile class %zu: %s", k, g->subs[k]->err.c_str());
    }
    return MDE_OK;
}

mde_status mde_group_accept(mde_group *g, const int32_t *e, const uint8_t *const *accept) {
    if (!g || !e || !accept) return MDE_INVALID;
    if (g->subs.empty()) return hgroup_accept(g, e, accept);
    for (size_t k = 0; k < g->subs.size(); ++k) {
        const auto &idx = g->sub_idx[k];
        const auto ee = gather_args(e, idx);
        const auto ac = gather_args(accept, idx);
        mde_status st = hgroup_accept(g->subs[k], ee.data(), ac.data());
        if (st) MDE_GFAIL(g, st, "walker-tile class %zu: %s", k, g->subs[k]->err.c_str());
    }
    return MDE_OK;
}

// Autotuner of a homogeneous group: threads per block and item size of its
// members (their walker tile kept), each candidate applied to every member
// (state kept: re-evaluated from the kept orbitals) and timed over three
// group proposals after a warm one; the fastest stays.
static mde_status hgroup_tune(mde_group *g, const int32_t *e, const double *const *new_orb) {
    const int n = (int)g->ctx.size();
    const int WT = g->WT;
    struct Cand {
        int thr;
        double scale;
    };
    std::vector<Cand> cands;
    for (int thr : {256, 512, 1024})
        if (thr >= WT && thr <= max_threads(WT))
            for (double sc : {0.5, 1.0, 2.0}) cands.push_back({thr, sc});
    auto apply = [&](const Cand &cd) -> mde_status {
        for (int i = 0; i < n; ++i) {
            mde_ctx *c = g->ctx[i];
            Plan p{};
            p.WT = c->WT;
            for (int s = 0; s < 2; ++s) {
                p.threads[s] = cd.thr;
                const size_t lds = det_lds(c->sp[s], c->WT, cd.thr, c->d.precision, true);
                const int base = item_size_for(c, c->sp[s], c->W, c->WT, cd.thr, lds);
                p.item_exc[s] = std::max((int)(base * cd.scale), 4 * (cd.thr / c->WT));
            }
            mde_status st = replan_keep_state(c, p);
            if (st) return st;
        }
        return group_rebuild(g);
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        MDE_GFAIL(g, MDE_DEVICE, "event creation");
    double best_t = 1e30;
    int best = -1;
    for (size_t k = 0; k < cands.size(); ++k) {
        if (apply(cands[k]) != MDE_OK) continue;
        if (hgroup_propose(g, e, new_orb, nullptr, nullptr, nullptr, nullptr) != MDE_OK) continue;
        (void)hipEventRecord(e0, g->stream);
        bool ok = true;
        for (int r = 0; r < 3; ++r)
            ok &= hgroup_propose(g, e, new_orb, nullptr, nullptr, nullptr, nullptr) == MDE_OK;
        (void)hipEventRecord(e1, g->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ok && ms < best_t) {
            best_t = ms;
            best = (int)k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best < 0) MDE_GFAIL(g, MDE_DEVICE, "no candidate plan ran");
    mde_status st = apply(cands[best]);
    if (st) MDE_GFAIL(g, st, "applying the chosen plan");
    for (mde_ctx *c : g->ctx) c->pending_e = -1;
    return MDE_OK;
}

mde_status mde_group_tune(mde_group *g, const int32_t *e, const double *const *new_orb) {
    if (!g || !e || !new_orb) return MDE_INVALID;
    if (g->capturing) MDE_GFAIL(g, MDE_STATE, "cannot tune during capture");
    for (mde_ctx *c : g->ctx)
        if (!c->initialized || c->adjoint_state) MDE_GFAIL(g, MDE_STATE, "initialise every member first");
    if (g->subs.empty()) return hgroup_tune(g, e, new_orb);
    for (size_t k = 0; k < g->subs.size(); ++k) {
        const auto ee = gather_args(e, g->sub_idx[k]);
        const auto no = gather_args(new_orb, g->sub_idx[k]);
        mde_status st = hgroup_tune(g->subs[k], ee.data(), no.data());
        if (st) MDE_GFAIL(g, st, "walker-tile class %zu: %s", k, g->subs[k]->err.c_str());
    }
    return MDE_OK;
}

const char *mde_group_error_string(const mde_group *g) { return g ? g->err.c_str() : "no group"; }

}  // extern "C"
