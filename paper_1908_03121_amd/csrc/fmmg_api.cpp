// fmmg_api.cpp -- the C-ABI declared in include/fmmg.h: plan creation (host
// planning, device tables and workspaces), the solve's launch sequence in its
// two shapes (one launch per class, or one persistent launch over all work
// items), hipGraph capture/replay, the launch-shape tuner, statistics and
// error reporting.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/fmmg.h"
#include "fmmg_internal.h"
#include "launch.h"
#include "planner.hpp"

using namespace fmmg;

namespace {

thread_local std::string g_err;

fmmg_status fail(fmmg_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

fmmg_status hip_fail(hipError_t e, const char* what) {
    return fail(FMMG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, what)                                  \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, what);     \
    } while (0)

std::mutex g_tab_mutex;
bool g_tab_uploaded[64] = {false};

template <typename T>
fmmg_status dev_upload(T** dst, const std::vector<T>& src, size_t capacity, hipStream_t st,
                       const char* what) {
    *dst = nullptr;
    size_t n = capacity > src.size() ? capacity : src.size();
    if (n == 0) return FMMG_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), n * sizeof(T));
    if (e != hipSuccess) return fail(FMMG_ENOMEM, std::string("hipMalloc ") + what + ": " + hipGetErrorString(e));
    if (!src.empty()) {
        e = hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    return FMMG_OK;
}

fmmg_status dev_alloc(double** dst, size_t n, const char* what) {
    *dst = nullptr;
    if (n == 0) return FMMG_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), n * sizeof(double));
    if (e != hipSuccess) return fail(FMMG_ENOMEM, std::string("hipMalloc ") + what + ": " + hipGetErrorString(e));
    return FMMG_OK;
}

std::vector<TreeIn> to_trees(const fmmg_tree_desc* trees, int32_t n_trees) {
    std::vector<TreeIn> v(size_t(n_trees > 0 ? n_trees : 0));
    for (int t = 0; t < n_trees; ++t) {
        v[size_t(t)].n = trees[t].n_subgrids;
        v[size_t(t)].level = trees[t].level;
        v[size_t(t)].coord = trees[t].coord;
        for (int a = 0; a < 3; ++a) v[size_t(t)].origin[a] = trees[t].origin[a];
        v[size_t(t)].L0 = trees[t].L0;
    }
    return v;
}

constexpr int TOP_CHUNKS = MAX_TOP_PARTS;

int prec_form(fmmg_precision pr) {
    return pr == FMMG_MIXED ? PR_MIX : pr == FMMG_MIXED_F32 ? PR_F32 : PR_F64;
}
constexpr int MAX_LAUNCH_STREAMS = 128;  // stream pool of the per-sub-grid launch model
constexpr int COUNTER_STRIDE = 16;  // ints per branch of the persistent-launch counters (>= NQUEUE + 1)
static_assert(COUNTER_STRIDE >= NQUEUE + 1, "persistent-launch counters");

}  // namespace

// Per-solve device workspaces of a plan.
struct fmmg_ws {
    double* mass = nullptr;   // [n_leaf][512]
    double* rec = nullptr;    // [n_ref][512][16]
    double* com = nullptr;    // [n_ref][3][512]
    double* Lp = nullptr;     // [groups][n_ref][19][512]
    double* Lr = nullptr;     // [n_ref][19][512]
    double* Lf = nullptr;     // [n_leaf][4][512]
    double* Lf3 = nullptr;    // [n_slot3][4][512]
    double* part = nullptr;   // [top partial slots][19][512]
    int* counter = nullptr;   // persistent-launch counters: NQUEUE + 1 per branch, COUNTER_STRIDE apart
};

struct fmmg_plan {
    int device = -1;
    int n_cu = 0;
    int max_bpc = 0;
    int max_groups = MAX_GROUPS;   // plane groups the partial buffers are sized for
    fmmg_options opt;
    HostPlan hp;
    hipStream_t capture_stream = nullptr;
    hipStream_t side_stream = nullptr;     // coarse branch of an overlapped solve
    hipStream_t mono_stream = nullptr;     // fine monopole class (overlap 2)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join_mono = nullptr;
    SubDev* d_subs = nullptr;
    int32_t* d_leaf_sub = nullptr;
    M2MTask* d_m2m_tasks = nullptr;
    int32_t* d_top_leaf = nullptr;
    L2LTask* d_l2l_tasks = nullptr;
    int32_t* d_top_src = nullptr;
    TopItem* d_top_items = nullptr;
    TopReduce* d_top_reduce = nullptr;
    Item* d_items_class = nullptr;
    Item* d_items_lpt = nullptr;
    Item* d_items_xcd = nullptr;
    size_t items_capacity = 0;
    fmmg_ws ws;                            // plan-owned workspaces
    unsigned long long* d_bad = nullptr;   // fmmg_check_density's result
    unsigned long long* h_bad = nullptr;
    unsigned long long* d_rho_bad = nullptr;      // the solves' density flag (see check_rho)
    unsigned long long* h_rho_bad = nullptr;      // pinned host word it is handed to
    unsigned long long* h_rho_bad_dev = nullptr;  // the host word's device address
    // launch shape
    fmmg_launch_shape shape;
    bool tuned = false;
    // graph cache
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const double* g_rho = nullptr;
    double* g_phi = nullptr;
    double* g_g = nullptr;
    int64_t launches = 0;
    int64_t solves = 0;
    // stage timing (eager solves with options.timing)
    std::vector<std::array<hipEvent_t, FMMG_N_STAGES + 1>> events;
    size_t n_timed = 0;
    int64_t stage_launches[FMMG_N_STAGES] = {0, 0, 0, 0, 0, 0, 0, 0};
    // per-sub-grid launch model (options.launch_streams > 0): the work items of
    // one target sub-grid and class form a run, launched on its own
    struct Run {
        int32_t kind, begin, n;
    };
    std::vector<Run> runs;                 // coarse level first, then sub-grid, then class
    std::vector<hipStream_t> pool;
    std::vector<hipEvent_t> pool_join;
};

namespace {

void drop_graph(fmmg_plan* p) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
}

void release(fmmg_plan* p) {
    if (!p) return;
    drop_graph(p);
    void* bufs[] = {p->d_subs, p->d_leaf_sub, p->d_m2m_tasks, p->d_top_leaf, p->d_l2l_tasks,
                    p->d_top_src, p->d_top_items, p->d_top_reduce, p->d_items_class, p->d_items_lpt, p->d_items_xcd,
                    p->ws.counter, p->ws.mass, p->ws.rec, p->ws.com, p->ws.Lp, p->ws.Lr, p->ws.Lf, p->ws.Lf3,
                    p->ws.part, p->d_bad, p->d_rho_bad};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (p->h_bad) (void)hipHostFree(p->h_bad);
    if (p->h_rho_bad) (void)hipHostFree(p->h_rho_bad);
    for (auto& set : p->events)
        for (hipEvent_t ev : set)
            if (ev) (void)hipEventDestroy(ev);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->mono_stream) (void)hipStreamDestroy(p->mono_stream);
    if (p->ev_join_mono) (void)hipEventDestroy(p->ev_join_mono);
    for (hipStream_t q : p->pool)
        if (q) (void)hipStreamDestroy(q);
    for (hipEvent_t ev : p->pool_join)
        if (ev) (void)hipEventDestroy(ev);
    delete p;
}

Ctx make_ctx(const fmmg_plan* p, const fmmg_ws& w, hipStream_t st) {
    Ctx a;
    a.subs = p->d_subs;
    a.leaf_sub = p->d_leaf_sub;
    a.mass = w.mass;
    a.rec = w.rec;
    a.com = w.com;
    a.rec_zero = int64_t(p->hp.ref_sub.size()) * NCELL;
    a.Lp = w.Lp;
    a.Lr = w.Lr;
    a.Lf = w.Lf;
    a.Lf3 = w.Lf3;
    a.part = w.part;
    a.rho_bad = p->d_rho_bad;
    a.rho_bad_host = p->h_rho_bad_dev;
    a.flag_out = 0;
    a.top_items = p->d_top_items;
    a.top_src = p->d_top_src;
    a.top_reds = p->d_top_reduce;
    a.rho = nullptr;
    a.part_stride = int64_t(p->hp.ref_sub.size()) * NLOC * NCELL;
    a.G = p->opt.G;
    a.corr = p->opt.angular_correction ? 1 : 0;
    a.prec = prec_form(p->opt.precision);
    a.ngroups = p->hp.ngroups;
    a.st = st;
    return a;
}

// Rebuilds and uploads the work items for a launch shape.
// Runs of the per-sub-grid launch model: the class list split at every change
// of (class, target sub-grid), ordered like a top-down walk of the trees
// (coarse level first), then by sub-grid and class.
void build_runs(fmmg_plan* p) {
    const HostPlan& hp = p->hp;
    struct Keyed {
        int32_t level, target, kind;
        fmmg_plan::Run r;
    };
    std::vector<Keyed> v;
    const int32_t n = int32_t(hp.items_class.size());
    for (int32_t i = 0; i < n;) {
        const Item& it = hp.items_class[size_t(i)];
        auto target = [&](const Item& x) {
            return x.kind == IT_TOP ? hp.top_items[size_t(x.sub)].target : x.sub;
        };
        const int32_t t = target(it);
        int32_t j = i + 1;
        while (j < n && hp.items_class[size_t(j)].kind == it.kind && target(hp.items_class[size_t(j)]) == t) ++j;
        v.push_back({hp.subs[size_t(t)].level, t, it.kind, {it.kind, i, j - i}});
        i = j;
    }
    std::stable_sort(v.begin(), v.end(), [](const Keyed& a, const Keyed& b) {
        if (a.level != b.level) return a.level < b.level;
        if (a.target != b.target) return a.target < b.target;
        return a.kind < b.kind;
    });
    p->runs.clear();
    for (const Keyed& k : v) p->runs.push_back(k.r);
}

// plane_pairs -1 (automatic): paired refined-target items when they number
// at least 8 per compute unit
int resolve_pairs(const fmmg_plan* p, int pairs, int groups) {
    if (pairs >= 0) return pairs;
    return int64_t(p->hp.mp_ref.size()) * (NS / 2) * groups >= 8 * int64_t(p->n_cu) ? 1 : 0;
}

fmmg_status apply_shape(fmmg_plan* p, int persistent, int groups, int bpc, int overlap, int queues, int pairs,
                        hipStream_t st) {
    if (queues != 0 && queues != 1) return fail(FMMG_EINVAL, "xcd_queues must be 0 or 1");
    if (pairs != 0 && pairs != 1) return fail(FMMG_EINVAL, "plane_pairs must be -1, 0 or 1");
    if (groups < 1 || groups > p->max_groups)
        return fail(FMMG_EINVAL, "plane_groups must be 1.." + std::to_string(p->max_groups) + " for this plan");
    if (bpc < 0) return fail(FMMG_EINVAL, "blocks_per_cu must be >= 0");
    if (bpc == 0 || bpc > p->max_bpc) bpc = p->max_bpc;
    if (overlap < 0 || overlap > 2) return fail(FMMG_EINVAL, "overlap must be 0, 1 or 2");
    // without overlap every class is one launch (no coarse branch)
    const bool split = overlap > 0 && p->hp.split_natural > 0;
    if (groups != p->hp.ngroups || split != (p->hp.split > 0) || pairs != p->hp.pairs) {
        build_items(&p->hp, groups, split, pairs);
        if (p->hp.items_class.size() > p->items_capacity) return fail(FMMG_EINVAL, "work-item capacity exceeded");
        if (!p->hp.items_class.empty()) {
            HIP_TRY(hipMemcpyAsync(p->d_items_class, p->hp.items_class.data(),
                                   p->hp.items_class.size() * sizeof(Item), hipMemcpyHostToDevice, st), "item upload");
            HIP_TRY(hipMemcpyAsync(p->d_items_lpt, p->hp.items_lpt.data(),
                                   p->hp.items_lpt.size() * sizeof(Item), hipMemcpyHostToDevice, st), "item upload");
            HIP_TRY(hipMemcpyAsync(p->d_items_xcd, p->hp.items_xcd.data(),
                                   p->hp.items_xcd.size() * sizeof(Item), hipMemcpyHostToDevice, st), "item upload");
        }
        HIP_TRY(hipStreamSynchronize(st), "item upload");
        build_runs(p);
    }
    if (p->hp.split == 0) overlap = 0;
    if (p->shape.persistent != persistent || p->shape.plane_groups != groups || p->shape.blocks_per_cu != bpc ||
        p->shape.overlap != overlap || p->shape.xcd_queues != queues || p->shape.plane_pairs != pairs)
        drop_graph(p);
    p->shape.persistent = persistent;
    p->shape.plane_groups = groups;
    p->shape.blocks_per_cu = bpc;
    p->shape.overlap = overlap;
    p->shape.split_level = p->hp.split;
    p->shape.launch_streams = int32_t(p->pool.size());
    p->shape.use_graph = p->opt.use_graph ? 1 : 0;
    p->shape.xcd_queues = queues;
    p->shape.plane_pairs = pairs;
    return FMMG_OK;
}

// The solve's launch sequence; returns the number of launches.  ev (may be
// null) receives an event at every stage boundary; it forces one stream.
//
// Levels below the split level s form the coarse branch.  Dependencies: the
// same-level items of level l need the upward pass down to level l - 1 (the
// masses of level-l leaves); the downward task of a level-l parent needs its
// own items (level l), its inherited part (the level l - 1 task) and, for
// leaf children, their own items (level l + 1).  Overlapped order:
//   caller's stream: upward levels max-1 .. s-1 (.. s when level s has no
//                    leaves) | fork | fine items | join |
//                    leaf children of level s-1, downward levels s .. max-1
//   side stream:     (after fork) the remaining upward levels, parentless-leaf
//                    masses, coarse items, parentless-leaf output, refined
//                    children of levels 0 .. s-1, leaf children of levels
//                    0 .. s-2 | join
int64_t enqueue_solve(fmmg_plan* p, const fmmg_ws& w, const double* rho, double* phi, double* g,
                      hipStream_t st, const hipEvent_t* ev) {
    const HostPlan& hp = p->hp;
    const int s = hp.split;
    const bool fork = !ev && p->shape.overlap && s > 0;
    hipStream_t side = fork ? p->side_stream : st;
    Ctx a = make_ctx(p, w, st);
    a.rho = rho;
    Ctx c = a;
    c.st = side;
    int64_t per[FMMG_N_STAGES] = {0, 0, 0, 0, 0, 0, 0, 0};
    int stage = 0;
    auto mark = [&](int sg) {
        stage = sg;
        if (ev) (void)hipEventRecord(ev[sg], st);
    };
    auto cnt = [&](int n) { if (n > 0) per[stage] += 1; };
    auto m2m = [&](const Ctx& x, int l) {
        const int b = hp.level_ref_begin[size_t(l)], m = hp.level_leafpar_end[size_t(l)],
                  e = hp.level_ref_begin[size_t(l) + 1];
        launch_m2m_leafpar(x, p->d_m2m_tasks + b, m - b);
        cnt(m - b);
        launch_m2m(x, p->d_m2m_tasks + m, e - m);
        cnt(e - m);
    };
    const int kinds[IT_KINDS] = {IT_TOP, IT_MONO, IT_MP_REF, IT_MP_LEAF};
    auto one_class = [&](const Ctx& x, int br, int k) {
        const int n = hp.class_begin[br][k + 1] - hp.class_begin[br][k];
        launch_class(x, k, p->d_items_class + hp.class_begin[br][k], n);
        cnt(n);
    };
    auto fused = [&](const Ctx& x, int br) {
        const int n = hp.lpt_begin[br + 1] - hp.lpt_begin[br];
        const int grid = br == 0 ? p->shape.blocks_per_cu * p->n_cu : p->n_cu;
        // one queue per XCD, or the largest-first list as queue 0 (blocks
        // whose own queue is empty move on to it)
        Queues qs;
        const bool xq = p->shape.xcd_queues != 0;
        for (int q = 0; q <= NQUEUE; ++q) qs.begin[q] = xq ? hp.queue_begin[br][q] - hp.lpt_begin[br] : (q ? n : 0);
        launch_persist(x, (xq ? p->d_items_xcd : p->d_items_lpt) + hp.lpt_begin[br], qs, grid,
                       w.counter + COUNTER_STRIDE * br);
        cnt(n);
    };
    auto items = [&](const Ctx& x, int br) {
        if (p->shape.persistent) fused(x, br);
        else
            for (int k : kinds) one_class(x, br, k);
    };
    // The solve's last launch (the leaf children of the deepest parents, or
    // the output of a forest of parentless leaves) also hands the density
    // flag to the host; every path below ends with it on the caller's stream.
    auto last = [&](const Ctx& x) {
        Ctx y = x;
        y.flag_out = 1;
        return y;
    };
    auto l2l = [&](const Ctx& x, int l, int kind) {  // kind 1: refined children, 0: leaf children
        const int b = hp.l2l_begin[size_t(2 * l + (1 - kind))], e = hp.l2l_begin[size_t(2 * l + (2 - kind))];
        const int mode = l > 0 ? PARENT_TOTAL : (hp.top_full ? PARENT_TOP_PARTS : PARENT_OWN_PARTS);
        const bool final_launch = kind == 0 && l == hp.max_level - 1;
        launch_l2l(final_launch ? last(x) : x, p->d_l2l_tasks + b, e - b, mode, phi, g);
        cnt(e - b);
    };
    const int n_tl = int(hp.top_leaf.size());
    // parentless leaves' output: the last launch when there is no level 1
    auto leaf_out = [&](const Ctx& x) {
        launch_leaf_out(hp.max_level == 0 ? last(x) : x, p->d_top_leaf, n_tl, phi, g);
        cnt(n_tl);
    };
    if (!p->pool.empty()) {
        // the execution model of Sec. 5.1: many small launches, one per target
        // sub-grid and class, spread over a pool of streams; the passes stay
        // on the solve's stream
        launch_p2m_top(a, p->d_top_leaf, n_tl);
        cnt(n_tl);
        for (int l = hp.max_level - 1; l >= 0; --l) m2m(a, l);
        const size_t used = std::min(p->pool.size(), p->runs.size());
        (void)hipEventRecord(p->ev_fork, st);
        for (size_t k = 0; k < used; ++k) (void)hipStreamWaitEvent(p->pool[k], p->ev_fork, 0);
        size_t k = 0;
        for (const fmmg_plan::Run& r : p->runs) {
            Ctx x = a;
            x.st = p->pool[k];
            launch_class(x, r.kind, p->d_items_class + r.begin, r.n);
            cnt(r.n);
            k = k + 1 == used ? 0 : k + 1;
        }
        for (size_t q = 0; q < used; ++q) {
            (void)hipEventRecord(p->pool_join[q], p->pool[q]);
            (void)hipStreamWaitEvent(st, p->pool_join[q], 0);
        }
        leaf_out(a);
        for (int l = 0; l < hp.max_level; ++l) {
            l2l(a, l, 1);
            l2l(a, l, 0);
        }
    } else if (!fork) {
        // one stream, stage by stage
        mark(FMMG_STAGE_P2M);
        launch_p2m_top(a, p->d_top_leaf, n_tl);
        cnt(n_tl);
        mark(FMMG_STAGE_M2M);
        for (int l = hp.max_level - 1; l >= 0; --l) m2m(a, l);
        const int stage_of[IT_KINDS] = {FMMG_STAGE_MP_REFINED, FMMG_STAGE_MP_LEAF, FMMG_STAGE_MONO, FMMG_STAGE_TOP};
        for (int k : kinds) {
            mark(stage_of[k]);
            if (!p->shape.persistent) {
                one_class(a, 0, k);
                one_class(a, 1, k);
            }
        }
        mark(FMMG_STAGE_FUSED);
        if (p->shape.persistent) {
            fused(a, 0);
            fused(a, 1);
        }
        mark(FMMG_STAGE_DOWN);
        leaf_out(a);
        for (int l = 0; l < hp.max_level; ++l) {
            l2l(a, l, 1);
            l2l(a, l, 0);
        }
    } else {
        // the fine items need the records of levels >= s and the masses of
        // leaves at levels >= s (level s's come from the level s-1 step)
        const int lo = hp.level_leaves[size_t(s)] > 0 ? s - 1 : s;
        for (int l = hp.max_level - 1; l >= lo; --l) m2m(a, l);
        (void)hipEventRecord(p->ev_fork, st);
        (void)hipStreamWaitEvent(side, p->ev_fork, 0);
        const bool mono_apart = p->shape.overlap == 2 && !p->shape.persistent;
        if (mono_apart) {
            // the fine monopole class on a third stream, beside the fine
            // multipole classes (their blocks fill each other's idle slots)
            Ctx m = a;
            m.st = p->mono_stream;
            (void)hipStreamWaitEvent(p->mono_stream, p->ev_fork, 0);
            one_class(m, 0, IT_MONO);
            (void)hipEventRecord(p->ev_join_mono, p->mono_stream);
            for (int k : kinds)
                if (k != IT_MONO) one_class(a, 0, k);
        } else {
            items(a, 0);
        }
        for (int l = lo - 1; l >= 0; --l) m2m(c, l);
        launch_p2m_top(c, p->d_top_leaf, n_tl);
        cnt(n_tl);
        items(c, 1);
        leaf_out(c);  // (max_level >= 1 here: the split level is > 0)
        for (int l = 0; l < s; ++l) l2l(c, l, 1);
        for (int l = 0; l < s - 1; ++l) l2l(c, l, 0);
        (void)hipEventRecord(p->ev_join, side);
        (void)hipStreamWaitEvent(st, p->ev_join, 0);
        if (mono_apart) (void)hipStreamWaitEvent(st, p->ev_join_mono, 0);
        l2l(a, s - 1, 0);
        for (int l = s; l < hp.max_level; ++l) {
            l2l(a, l, 1);
            l2l(a, l, 0);
        }
    }
    if (ev) (void)hipEventRecord(ev[FMMG_N_STAGES], st);
    int64_t n = 0;
    for (int k = 0; k < FMMG_N_STAGES; ++k) {
        p->stage_launches[k] = per[k];
        n += per[k];
    }
    return n;
}

// ---------------------------------------------------------------------------
// launch-shape tuner
// ---------------------------------------------------------------------------
std::string signature(const fmmg_plan* p) {
    std::ostringstream o;
    const HostPlan& hp = p->hp;
    o << "fmmg2 trees=" << hp.n_trees << " sub=" << hp.subs.size() << " ref=" << hp.ref_sub.size()
      << " leaf=" << hp.leaf_sub.size() << " lev=" << hp.max_level << " k3=" << hp.n_slot3
      << " top=" << (p->opt.top_mode == FMMG_TOP_FULL ? "full" : "stencil")
      << " prec=" << (p->opt.precision == FMMG_MIXED ? "mixed" : p->opt.precision == FMMG_MIXED_F32 ? "mixed_f32" : "fp64")
      << " cu=" << p->n_cu
      << " split=" << hp.split_natural << " ovl=" << p->opt.overlap
      << " graph=" << (p->opt.use_graph ? 1 : 0);
    return o.str();
}

// Cache file: a JSON object, one entry per line:
//   "signature": {"persistent": P, "plane_groups": G, "blocks_per_cu": B, "overlap": O,
//                 "xcd_queues": Q, "plane_pairs": R, "ms": T},
bool cache_lookup(const char* path, const std::string& sig, int* pers, int* groups, int* bpc, int* ovl,
                  int* queues, int* pairs) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line, key = "\"" + sig + "\":";
    while (std::getline(f, line)) {
        size_t at = line.find(key);
        if (at == std::string::npos) continue;
        int a = -1, b = -1, c = -1, d = -1, q = -1, r = -1;
        const char* s = line.c_str() + at + key.size();
        if (std::sscanf(s,
                        " {\"persistent\": %d, \"plane_groups\": %d, \"blocks_per_cu\": %d, \"overlap\": %d, "
                        "\"xcd_queues\": %d, \"plane_pairs\": %d",
                        &a, &b, &c, &d, &q, &r) == 6 &&
            (a == 0 || a == 1) && b >= 1 && b <= MAX_GROUPS && c >= 0 && d >= 0 && d <= 2 && (q == 0 || q == 1) &&
            (r == 0 || r == 1)) {
            // (a group count above the plan's buffers is rejected by apply_shape)
            *pers = a;
            *groups = b;
            *bpc = c;
            *ovl = d;
            *queues = q;
            *pairs = r;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& sig, int pers, int groups, int bpc, int ovl, int queues,
                 int pairs, double ms) {
    if (!path) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line)) {
            if (line.find("\": {\"persistent\"") == std::string::npos) continue;
            if (line.find("\"" + sig + "\":") != std::string::npos) continue;
            while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
            keep.push_back(line);
        }
    }
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "  \"%s\": {\"persistent\": %d, \"plane_groups\": %d, \"blocks_per_cu\": %d, \"overlap\": %d, "
                  "\"xcd_queues\": %d, \"plane_pairs\": %d, \"ms\": %.6f}",
                  sig.c_str(), pers, groups, bpc, ovl, queues, pairs, ms);
    keep.push_back(buf);
    std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp);
        if (!o) return;
        o << "{\n";
        for (size_t i = 0; i < keep.size(); ++i) o << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
        o << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

fmmg_status tune(fmmg_plan* p, const double* rho, double* phi, double* g, hipStream_t st) {
    int pers = 0, groups = 0, bpc = 0, ovl = 0, queues = 1, pairs = 0;
    const std::string sig = signature(p);
    if (cache_lookup(p->opt.tuning_cache, sig, &pers, &groups, &bpc, &ovl, &queues, &pairs)) {
        fmmg_status s = apply_shape(p, pers, groups, bpc, ovl, queues, pairs, st);
        if (s != FMMG_OK) return s;
        p->shape.from_cache = 1;
        p->tuned = true;
        return FMMG_OK;
    }
    struct Cand { int pers, groups, bpc, ovl, queues, pairs; };
    std::vector<Cand> cands;
    const int max_ov = p->hp.split_natural > 0 ? p->opt.overlap : 0;
    for (int ov = 0; ov <= max_ov; ++ov)
        for (int gr : {1, 2, 3, 5}) {
            if (gr > p->max_groups) continue;
            const int pr = resolve_pairs(p, p->opt.plane_pairs, gr);
            cands.push_back({0, gr, 0, ov, p->opt.xcd_queues, pr});
            if (ov == 2) continue;  // the third stream applies to per-class launches only
            for (int b = 1; b <= p->max_bpc; ++b)
                for (int q : {1, 0}) cands.push_back({1, gr, b, ov, q, pr});
        }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(FMMG_EHIP, "hipEventCreate"); }
    if (p->opt.use_graph && !p->capture_stream &&
        hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(FMMG_EHIP, "hipStreamCreate");
    }
    double best = 1e300;
    Cand bc = cands[0];
    fmmg_status status = FMMG_OK;
    // the winner's captured graph becomes the plan's graph (it was captured
    // for these buffers), so the solves replay the very instance that was
    // timed
    hipGraph_t best_cg = nullptr;
    hipGraphExec_t best_ce = nullptr;
    int64_t best_launches = 0;
    // each candidate runs the way the plan will: graph replays when the plan
    // uses graphs, else eager launches; it is timed as the best of 3 runs of
    // enough solves to last about 1 ms
    // after the candidates above, the fastest is tried once more with the
    // other item form when the plan leaves it to the tuner
    const size_t n_first = cands.size();
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        const Cand c = cands[ci];
        status = apply_shape(p, c.pers, c.groups, c.bpc, c.ovl, c.queues, c.pairs, st);
        if (status != FMMG_OK) break;
        hipGraph_t cg = nullptr;
        hipGraphExec_t ce = nullptr;
        int64_t launches = 0;
        if (p->opt.use_graph) {
            hipError_t e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                launches = enqueue_solve(p, p->ws, rho, phi, g, p->capture_stream, nullptr);
                hipError_t le = hipGetLastError();
                e = hipStreamEndCapture(p->capture_stream, &cg);
                if (e == hipSuccess) e = le;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&ce, cg, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                if (cg) (void)hipGraphDestroy(cg);
                status = hip_fail(e, "tuning capture");
                break;
            }
        }
        auto run = [&]() {
            if (ce) (void)hipGraphLaunch(ce, st);
            else enqueue_solve(p, p->ws, rho, phi, g, st, nullptr);
        };
        auto timed = [&](int n, double* ms_out) {
            (void)hipEventRecord(e0, st);
            for (int i = 0; i < n; ++i) run();
            (void)hipEventRecord(e1, st);
            hipError_t e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            *ms_out = double(ms) / n;
            return e;
        };
        double t = 1e300, one = 0;
        run();  // warm
        hipError_t e = timed(1, &one);
        const int reps = one > 0 ? std::max(1, std::min(8, int(1.0 / one))) : 8;
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {
            double ms = 0;
            e = timed(reps, &ms);
            t = std::min(t, ms);
        }
        const bool better = e == hipSuccess && t < best;
        if (better) {
            if (best_ce) (void)hipGraphExecDestroy(best_ce);
            if (best_cg) (void)hipGraphDestroy(best_cg);
            best_ce = ce;
            best_cg = cg;
            best_launches = launches;
        } else {
            if (ce) (void)hipGraphExecDestroy(ce);
            if (cg) (void)hipGraphDestroy(cg);
        }
        if (e != hipSuccess) { status = hip_fail(e, "tuning run"); break; }
        if (better) { best = t; bc = c; }
        if (ci + 1 == n_first && p->opt.plane_pairs < 0) {
            Cand f = bc;
            f.pairs = 1 - bc.pairs;
            cands.push_back(f);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    auto drop_best = [&]() {
        if (best_ce) (void)hipGraphExecDestroy(best_ce);
        if (best_cg) (void)hipGraphDestroy(best_cg);
    };
    if (status != FMMG_OK) { drop_best(); return status; }
    status = apply_shape(p, bc.pers, bc.groups, bc.bpc, bc.ovl, bc.queues, bc.pairs, st);
    if (status != FMMG_OK) { drop_best(); return status; }
    if (best_ce) {
        drop_graph(p);
        p->graph = best_cg;
        p->graph_exec = best_ce;
        p->g_rho = rho;
        p->g_phi = phi;
        p->g_g = g;
        p->launches = best_launches;
    }
    p->shape.from_cache = 0;
    p->shape.tuned_ms = best;
    p->tuned = true;
    cache_store(p->opt.tuning_cache, sig, bc.pers, bc.groups, p->shape.blocks_per_cu, p->shape.overlap, bc.queues,
                bc.pairs, best);
    return FMMG_OK;
}

}  // namespace

extern "C" {

int32_t fmmg_version(void) { return FMMG_VERSION; }

const char* fmmg_last_error(void) { return g_err.c_str(); }

void fmmg_default_options(fmmg_options* opt) {
    if (!opt) return;
    memset(opt, 0, sizeof(*opt));
    opt->precision = FMMG_FP64;
    opt->top_mode = FMMG_TOP_FULL;
    opt->G = 1.0;
    opt->angular_correction = 1;
    opt->use_graph = -1;
    opt->persistent = 0;
    opt->timing = 0;
    opt->plane_groups = 0;
    opt->blocks_per_cu = 0;
    opt->autotune = 0;
    opt->tuning_cache = nullptr;
    opt->overlap = 1;
    opt->xcd_queues = 1;
    opt->plane_pairs = -1;
}

fmmg_status fmmg_count_pairs(const fmmg_tree_desc* trees, int32_t n_trees, fmmg_top_mode top_mode,
                             fmmg_stats* stats) {
    try {
        if (!trees || !stats || n_trees < 1) return fail(FMMG_EINVAL, "fmmg_count_pairs: null argument or n_trees < 1");
        if (top_mode != FMMG_TOP_FULL && top_mode != FMMG_TOP_STENCIL_ONLY)
            return fail(FMMG_EINVAL, "fmmg_count_pairs: bad top_mode");
        std::vector<TreeIn> tv = to_trees(trees, n_trees);
        HostPlan hp;
        std::string err;
        int rc = build_host_plan(tv.data(), n_trees, top_mode == FMMG_TOP_FULL, TOP_CHUNKS, &hp, &err);
        if (rc) return fail(rc == -2 ? FMMG_ETREE : FMMG_EINVAL, err);
        memset(stats, 0, sizeof(*stats));
        for (int c = 0; c < 4; ++c) stats->pairs[c] = hp.counts.cls[c];
        stats->pairs_top = hp.counts.top;
        stats->paper_flops = hp.counts.paper_flops();
        stats->n_leaves = int64_t(hp.leaf_sub.size());
        stats->n_refined = int64_t(hp.ref_sub.size());
        stats->max_level = hp.max_level;
        stats->n_trees = n_trees;
        stats->sweep_y_targets = hp.sweep_y_targets;
        stats->sweep_x_targets = hp.sweep_x_targets;
        return FMMG_OK;
    } catch (const std::bad_alloc&) {
        return fail(FMMG_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(FMMG_EINVAL, "unexpected host error");
    }
}

fmmg_status fmmg_plan_create(fmmg_plan** out, const fmmg_tree_desc* trees, int32_t n_trees,
                             const fmmg_options* opt, void* hip_stream) {
    if (!out) return fail(FMMG_EINVAL, "fmmg_plan_create: out is NULL");
    *out = nullptr;
    if (!trees || n_trees < 1) return fail(FMMG_EINVAL, "fmmg_plan_create: need n_trees >= 1 trees");
    fmmg_plan* p = nullptr;
    try {
        p = new fmmg_plan();
        if (opt) p->opt = *opt;
        else fmmg_default_options(&p->opt);
        // use_graph < 0: capture batched plans, unless their stages are timed
        if (p->opt.use_graph < 0) p->opt.use_graph = (n_trees > 1 && !p->opt.timing) ? 1 : 0;
        const fmmg_options& o = p->opt;
        std::string bad;
        if (o.precision != FMMG_FP64 && o.precision != FMMG_MIXED && o.precision != FMMG_MIXED_F32)
            bad = "bad precision";
        else if (o.top_mode != FMMG_TOP_FULL && o.top_mode != FMMG_TOP_STENCIL_ONLY) bad = "bad top_mode";
        else if (o.timing && o.use_graph) bad = "timing needs eager launches (use_graph = 0)";
        else if (o.timing && o.autotune) bad = "timing and autotune cannot be combined";
        else if (o.plane_groups < 0 || o.plane_groups > MAX_GROUPS) bad = "plane_groups must be 0..5";
        else if (o.blocks_per_cu < 0) bad = "blocks_per_cu must be >= 0";
        else if (o.overlap < 0 || o.overlap > 2) bad = "overlap must be 0, 1 or 2";
        else if (o.launch_streams < 0 || o.launch_streams > MAX_LAUNCH_STREAMS) bad = "launch_streams must be 0..128";
        else if (o.launch_streams && o.timing) bad = "timing needs launch_streams = 0";
        else if (o.launch_streams && o.autotune) bad = "autotune needs launch_streams = 0";
        else if (o.xcd_queues != 0 && o.xcd_queues != 1) bad = "xcd_queues must be 0 or 1";
        else if (o.plane_pairs < -1 || o.plane_pairs > 1) bad = "plane_pairs must be -1, 0 or 1";
        if (!bad.empty()) { release(p); return fail(FMMG_EINVAL, bad); }
        hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
        hipError_t e = hipGetDevice(&p->device);
        if (e != hipSuccess) { release(p); return fail(FMMG_EUNSUPPORTED, std::string("no HIP device: ") + hipGetErrorString(e)); }
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, p->device);
        if (e != hipSuccess) { release(p); return hip_fail(e, "hipGetDeviceProperties"); }
        if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            release(p);
            return fail(FMMG_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
        }
        p->n_cu = prop.multiProcessorCount;
        p->max_bpc = persist_blocks_per_cu(prec_form(o.precision));
        if (p->max_bpc < 1) p->max_bpc = 1;
        std::vector<TreeIn> tv = to_trees(trees, n_trees);
        std::string err;
        int rc = build_host_plan(tv.data(), n_trees, o.top_mode == FMMG_TOP_FULL, TOP_CHUNKS, &p->hp, &err);
        if (rc) { release(p); return fail(rc == -2 ? FMMG_ETREE : FMMG_EINVAL, err); }
        HostPlan& hp = p->hp;
        // partial buffers and item capacity for the plane-group counts this plan may use
        p->max_groups = (o.plane_groups > 0 && !o.autotune) ? o.plane_groups : MAX_GROUPS;
        if (!o.autotune && o.plane_groups == 0) p->max_groups = 2;
        build_items(&hp, p->max_groups, true, 0);  // the larger item form
        p->items_capacity = hp.items_class.size();
        fmmg_status s;
#define UP(dst, src, cap, what) if ((s = dev_upload(&(dst), (src), (cap), st, what)) != FMMG_OK) { release(p); return s; }
        UP(p->d_subs, hp.subs, 0, "sub-grid table");
        UP(p->d_leaf_sub, hp.leaf_sub, 0, "leaf list");
        UP(p->d_m2m_tasks, hp.m2m_tasks, 0, "upward tasks");
        UP(p->d_top_leaf, hp.top_leaf, 0, "top leaf list");
        UP(p->d_l2l_tasks, hp.l2l_tasks, 0, "downward tasks");
        UP(p->d_top_src, hp.top_src, 0, "top source list");
        UP(p->d_top_items, hp.top_items, 0, "top items");
        UP(p->d_top_reduce, hp.top_reduce, 0, "top reductions");
        UP(p->d_items_class, std::vector<Item>(), p->items_capacity, "work items");
        UP(p->d_items_lpt, std::vector<Item>(), p->items_capacity, "work items");
        UP(p->d_items_xcd, std::vector<Item>(), p->items_capacity, "work items");
#undef UP
        size_t nl = hp.leaf_sub.size(), nr = hp.ref_sub.size();
#define AL(dst, n, what) if ((s = dev_alloc(&(dst), (n), what)) != FMMG_OK) { release(p); return s; }
        AL(p->ws.mass, nl * NCELL, "leaf masses");
        AL(p->ws.rec, (nr * NCELL + 1) * NREC, "multipole records");  // + one zero record
        AL(p->ws.com, nr * 3 * NCELL, "centre-of-mass offsets");
        AL(p->ws.Lp, size_t(p->max_groups) * nr * NLOC * NCELL, "refined own terms");
        AL(p->ws.Lr, nr * NLOC * NCELL, "refined expansions");
        AL(p->ws.Lf, nl * NLEAF * NCELL, "leaf terms");
        AL(p->ws.Lf3, size_t(hp.n_slot3) * NLEAF * NCELL, "leaf terms from refined sources");
        AL(p->ws.part, size_t(hp.n_top_parts) * NLOC * NCELL, "top partial sums");
#undef AL
        e = hipMalloc(reinterpret_cast<void**>(&p->ws.counter), 2 * COUNTER_STRIDE * sizeof(int));
        if (e != hipSuccess) { release(p); return fail(FMMG_ENOMEM, "hipMalloc counter"); }
        e = hipMemsetAsync(p->ws.counter, 0, 2 * COUNTER_STRIDE * sizeof(int), st);
        if (e != hipSuccess) { release(p); return hip_fail(e, "counter clear"); }
        // the zero record after the last refined cell (read for leaf and
        // absent source cells when a plane window is staged)
        e = hipMemsetAsync(p->ws.rec + nr * NCELL * NREC, 0, NREC * sizeof(double), st);
        if (e != hipSuccess) { release(p); return hip_fail(e, "zero record clear"); }
        // the solves' density flag and the pinned host word it is handed to
        e = hipMalloc(reinterpret_cast<void**>(&p->d_rho_bad), sizeof(unsigned long long));
        if (e != hipSuccess) { release(p); return fail(FMMG_ENOMEM, "hipMalloc density flag"); }
        launch_fill_u64(p->d_rho_bad, 1, ~0ull, st);
        e = hipGetLastError();
        if (e != hipSuccess) { release(p); return hip_fail(e, "density flag clear"); }
        e = hipHostMalloc(reinterpret_cast<void**>(&p->h_rho_bad), sizeof(unsigned long long),
                          hipHostMallocMapped);
        if (e != hipSuccess) { release(p); return fail(FMMG_ENOMEM, "hipHostMalloc density flag"); }
        __atomic_store_n(p->h_rho_bad, ~0ull, __ATOMIC_RELEASE);
        e = hipHostGetDevicePointer(reinterpret_cast<void**>(&p->h_rho_bad_dev), p->h_rho_bad, 0);
        if (e != hipSuccess) { release(p); return hip_fail(e, "density flag host mapping"); }
        e = hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->mono_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join_mono, hipEventDisableTiming);
        if (e != hipSuccess) { release(p); return hip_fail(e, "second stream"); }
        for (int k = 0; k < o.launch_streams && e == hipSuccess; ++k) {
            hipStream_t q = nullptr;
            hipEvent_t ev = nullptr;
            e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
            if (e == hipSuccess) p->pool.push_back(q);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) p->pool_join.push_back(ev);
        }
        if (e != hipSuccess) { release(p); return hip_fail(e, "launch stream pool"); }
        e = hipMalloc(reinterpret_cast<void**>(&p->d_bad), sizeof(unsigned long long));
        if (e != hipSuccess) { release(p); return fail(FMMG_ENOMEM, "hipMalloc flag"); }
        e = hipHostMalloc(reinterpret_cast<void**>(&p->h_bad), sizeof(unsigned long long), hipHostMallocDefault);
        if (e != hipSuccess) { release(p); return fail(FMMG_ENOMEM, "hipHostMalloc flag"); }
        {
            std::lock_guard<std::mutex> lk(g_tab_mutex);
            if (p->device < 0 || p->device >= 64) { release(p); return fail(FMMG_EUNSUPPORTED, "device index >= 64"); }
            if (!g_tab_uploaded[p->device]) {
                StencilTables tab;
                build_stencil_tables(&tab);
                e = upload_tables(&tab, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) { release(p); return hip_fail(e, "stencil table upload"); }
                g_tab_uploaded[p->device] = true;
            }
        }
        p->hp.ngroups = 0;  // force the first item upload
        memset(&p->shape, 0, sizeof(p->shape));
        {
            const int gr = o.plane_groups ? o.plane_groups : 2;
            s = apply_shape(p, o.persistent ? 1 : 0, gr, o.blocks_per_cu, o.overlap, o.xcd_queues,
                            resolve_pairs(p, o.plane_pairs, gr), st);
        }
        if (s != FMMG_OK) { release(p); return s; }
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) { release(p); return hip_fail(e, "plan upload"); }
        *out = p;
        return FMMG_OK;
    } catch (const std::bad_alloc&) {
        release(p);
        return fail(FMMG_ENOMEM, "host allocation failed");
    } catch (...) {
        release(p);
        return fail(FMMG_EINVAL, "unexpected host error");
    }
}

fmmg_status fmmg_plan_n_leaves(const fmmg_plan* p, int64_t* n) {
    if (!p || !n) return fail(FMMG_EINVAL, "null argument");
    *n = int64_t(p->hp.leaf_sub.size());
    return FMMG_OK;
}

fmmg_status fmmg_leaf_order(const fmmg_plan* p, int32_t* idx) {
    if (!p || !idx) return fail(FMMG_EINVAL, "null argument");
    memcpy(idx, p->hp.leaf_desc.data(), p->hp.leaf_desc.size() * sizeof(int32_t));
    return FMMG_OK;
}

fmmg_status fmmg_get_launch_shape(const fmmg_plan* p, fmmg_launch_shape* out) {
    if (!p || !out) return fail(FMMG_EINVAL, "null argument");
    *out = p->shape;
    return FMMG_OK;
}

namespace {

// Checks shared by the solve entry points: buffers, device, and a bad
// density that a completed solve on this plan has reported (taken, so that
// it is reported once).
fmmg_status solve_checks(fmmg_plan* p, const double* rho, double* phi, double* g, const char* who) {
    if (!p) return fail(FMMG_EINVAL, std::string(who) + ": plan is NULL");
    if (!p->hp.leaf_sub.empty() && (!rho || !phi || !g)) return fail(FMMG_EINVAL, std::string(who) + ": null buffer");
    {
        // the kernels read rho while writing phi and g: no two may share memory
        const uintptr_t n = uintptr_t(p->hp.leaf_sub.size()) * NCELL * sizeof(double);
        const uintptr_t r0 = reinterpret_cast<uintptr_t>(rho), p0 = reinterpret_cast<uintptr_t>(phi),
                        g0 = reinterpret_cast<uintptr_t>(g);
        auto overlap = [](uintptr_t a, uintptr_t na, uintptr_t b, uintptr_t nb) { return a < b + nb && b < a + na; };
        if (n > 0 && (overlap(r0, n, p0, n) || overlap(r0, n, g0, 3 * n) || overlap(p0, n, g0, 3 * n)))
            return fail(FMMG_EINVAL, std::string(who) + ": rho, phi and g overlap");
    }
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p->device) return fail(FMMG_EINVAL, std::string(who) + ": plan belongs to another device");
    const unsigned long long bad = __atomic_exchange_n(p->h_rho_bad, ~0ull, __ATOMIC_ACQ_REL);
    if (bad != ~0ull)
        return fail(FMMG_EINVAL, std::string(who) + ": a completed solve on this plan read a negative or non-finite "
                                 "density at flat index " + std::to_string(bad) + "; nothing was enqueued");
    return FMMG_OK;
}

}  // namespace

fmmg_status fmmg_solve(fmmg_plan* p, const double* rho, double* phi, double* g, void* hip_stream) {
    fmmg_status cs = solve_checks(p, rho, phi, g, "fmmg_solve");
    if (cs != FMMG_OK) return cs;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    try {
        if (p->opt.autotune && !p->tuned) {
            fmmg_status s = tune(p, rho, phi, g, st);
            if (s != FMMG_OK) return s;
        }
        if (!p->opt.use_graph) {
            const hipEvent_t* ev = nullptr;
            if (p->opt.timing) {
                if (p->n_timed == p->events.size()) {
                    if (p->events.size() >= 100000)
                        return fail(FMMG_EINVAL, "fmmg_solve: call fmmg_get_timings at least every 100000 solves");
                    std::array<hipEvent_t, FMMG_N_STAGES + 1> set;
                    set.fill(nullptr);
                    for (auto& e : set) {
                        hipError_t ee = hipEventCreate(&e);
                        if (ee != hipSuccess) {
                            for (auto& d : set)
                                if (d) (void)hipEventDestroy(d);
                            return hip_fail(ee, "hipEventCreate");
                        }
                    }
                    p->events.push_back(set);
                }
                ev = p->events[p->n_timed++].data();
            }
            p->launches = enqueue_solve(p, p->ws, rho, phi, g, st, ev);
            HIP_TRY(hipGetLastError(), "kernel launch");
        } else {
            if (!p->graph_exec || p->g_rho != rho || p->g_phi != phi || p->g_g != g) {
                drop_graph(p);
                if (!p->capture_stream)
                    HIP_TRY(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
                HIP_TRY(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
                p->launches = enqueue_solve(p, p->ws, rho, phi, g, p->capture_stream, nullptr);
                hipError_t le = hipGetLastError();
                hipError_t ce = hipStreamEndCapture(p->capture_stream, &p->graph);
                if (le != hipSuccess) return hip_fail(le, "kernel launch during capture");
                if (ce != hipSuccess) return hip_fail(ce, "end capture");
                HIP_TRY(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0), "graph instantiate");
                p->g_rho = rho;
                p->g_phi = phi;
                p->g_g = g;
            }
            HIP_TRY(hipGraphLaunch(p->graph_exec, st), "graph launch");
        }
        p->solves++;
        return FMMG_OK;
    } catch (...) {
        return fail(FMMG_EINVAL, "unexpected host error in fmmg_solve");
    }
}

fmmg_status fmmg_density_status(fmmg_plan* p, int64_t* bad_index) {
    if (!p || !bad_index) return fail(FMMG_EINVAL, "fmmg_density_status: null argument");
    const unsigned long long bad = __atomic_exchange_n(p->h_rho_bad, ~0ull, __ATOMIC_ACQ_REL);
    *bad_index = bad == ~0ull ? -1 : int64_t(bad);
    if (bad != ~0ull)
        return fail(FMMG_EINVAL, "a completed solve read a negative or non-finite density at flat index " +
                                     std::to_string(bad));
    return FMMG_OK;
}

fmmg_status fmmg_check_density(fmmg_plan* p, const double* rho, void* hip_stream) {
    if (!p || (!rho && !p->hp.leaf_sub.empty())) return fail(FMMG_EINVAL, "fmmg_check_density: null argument");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    int64_t n = int64_t(p->hp.leaf_sub.size()) * NCELL;
    launch_check_density(rho, n, p->d_bad, st);
    HIP_TRY(hipGetLastError(), "density check launch");
    HIP_TRY(hipMemcpyAsync(p->h_bad, p->d_bad, sizeof(unsigned long long), hipMemcpyDeviceToHost, st), "copy flag");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    if (*p->h_bad != ~0ull)
        return fail(FMMG_EINVAL, "density at flat index " + std::to_string(*p->h_bad) + " is negative or not finite");
    return FMMG_OK;
}

fmmg_status fmmg_check_density_noalloc(const double* rho, int64_t n, int64_t* bad_index, void* hip_stream) {
    if (n < 0) return fail(FMMG_EINVAL, "fmmg_check_density_noalloc: negative size");
    if (n > FMMG_NOALLOC_MAX_DENSITIES)
        return fail(FMMG_EINVAL, "fmmg_check_density_noalloc: " + std::to_string(n) +
                                     " densities exceed the maximum of " + std::to_string(FMMG_NOALLOC_MAX_DENSITIES) +
                                     " that its static array covers");
    if (!bad_index || (!rho && n > 0)) return fail(FMMG_EINVAL, "fmmg_check_density_noalloc: null argument");
    static_assert(FMMG_NOALLOC_MAX_DENSITIES == int64_t(NOALLOC_SLOTS) * NOALLOC_CHUNK, "static array size");
    std::string what;
    const hipError_t e = noalloc_check_density(rho, n, bad_index, reinterpret_cast<hipStream_t>(hip_stream), &what);
    if (e != hipSuccess) return hip_fail(e, what.c_str());
    return FMMG_OK;
}

fmmg_status fmmg_get_timings(fmmg_plan* p, fmmg_timings* out) {
    if (!p || !out) return fail(FMMG_EINVAL, "null argument");
    if (!p->opt.timing) return fail(FMMG_EINVAL, "plan was created without timing");
    memset(out, 0, sizeof(*out));
    for (size_t i = 0; i < p->n_timed; ++i) {
        const auto& ev = p->events[i];
        for (int s = 0; s < FMMG_N_STAGES; ++s) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[size_t(s)], ev[size_t(s) + 1]), "hipEventElapsedTime");
            out->ms[s] += double(ms);
        }
    }
    for (int s = 0; s < FMMG_N_STAGES; ++s) out->launches[s] = p->stage_launches[s];
    out->solves = int64_t(p->n_timed);
    p->n_timed = 0;
    return FMMG_OK;
}

fmmg_status fmmg_get_stats(const fmmg_plan* p, fmmg_stats* s) {
    if (!p || !s) return fail(FMMG_EINVAL, "null argument");
    memset(s, 0, sizeof(*s));
    for (int c = 0; c < 4; ++c) s->pairs[c] = p->hp.counts.cls[c];
    s->pairs_top = p->hp.counts.top;
    s->launches = p->launches;
    s->solves = p->solves;
    s->paper_flops = p->hp.counts.paper_flops();
    s->n_leaves = int64_t(p->hp.leaf_sub.size());
    s->n_refined = int64_t(p->hp.ref_sub.size());
    s->max_level = p->hp.max_level;
    s->n_trees = p->hp.n_trees;
    s->sweep_y_targets = p->hp.sweep_y_targets;
    s->sweep_x_targets = p->hp.sweep_x_targets;
    return FMMG_OK;
}

void fmmg_plan_destroy(fmmg_plan* p) { release(p); }

}  // extern "C"
