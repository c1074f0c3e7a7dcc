// fmmg_api.cpp -- the C-ABI declared in include/fmmg.h: plan creation (host
// planning, device tables and workspaces), the solve's launch sequence, hipGraph
// capture/replay, statistics and error reporting.
#include <hip/hip_runtime.h>
#include <string.h>

#include <array>
#include <mutex>
#include <new>
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

#define HIP_TRY(call, what)                       \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

std::mutex g_tab_mutex;
bool g_tab_uploaded[64] = {false};

template <typename T>
fmmg_status dev_upload(T** dst, const std::vector<T>& src, hipStream_t st, const char* what) {
    *dst = nullptr;
    if (src.empty()) return FMMG_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T));
    if (e != hipSuccess) return fail(FMMG_ENOMEM, std::string("hipMalloc ") + what + ": " + hipGetErrorString(e));
    e = hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, what);
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

constexpr int TOP_CHUNKS = 32;

}  // namespace

struct fmmg_plan {
    int device = -1;
    fmmg_options opt;
    HostPlan hp;
    hipStream_t capture_stream = nullptr;
    SubDev* d_subs = nullptr;
    int32_t* d_leaf_sub = nullptr;
    int32_t* d_mp_ref = nullptr;
    int32_t* d_mono_leaf = nullptr;
    int32_t* d_mp_leaf = nullptr;
    int32_t* d_ref_by_level = nullptr;
    int32_t* d_top_leaf = nullptr;
    int32_t* d_top_src = nullptr;
    TopItem* d_top_items = nullptr;
    TopReduce* d_top_reduce = nullptr;
    double* d_mass = nullptr;
    double* d_rec = nullptr;
    double* d_Lr = nullptr;
    double* d_Lf = nullptr;
    double* d_part = nullptr;
    unsigned long long* d_bad = nullptr;
    unsigned long long* h_bad = nullptr;
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
    int64_t stage_launches[FMMG_N_STAGES] = {0, 0, 0, 0, 0, 0, 0};
};

namespace {

void release(fmmg_plan* p) {
    if (!p) return;
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    void* bufs[] = {p->d_subs, p->d_leaf_sub, p->d_mp_ref, p->d_mono_leaf, p->d_mp_leaf,
                    p->d_ref_by_level, p->d_top_leaf, p->d_top_src, p->d_top_items, p->d_top_reduce,
                    p->d_mass, p->d_rec, p->d_Lr, p->d_Lf, p->d_part, p->d_bad};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (p->h_bad) (void)hipHostFree(p->h_bad);
    for (auto& set : p->events)
        for (hipEvent_t ev : set)
            if (ev) (void)hipEventDestroy(ev);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    delete p;
}

Launch make_launch(const fmmg_plan* p, hipStream_t st) {
    Launch a;
    a.subs = p->d_subs;
    a.leaf_sub = p->d_leaf_sub;
    a.mass = p->d_mass;
    a.rec = p->d_rec;
    a.Lr = p->d_Lr;
    a.Lf = p->d_Lf;
    a.part = p->d_part;
    a.G = p->opt.G;
    a.corr = p->opt.angular_correction ? 1 : 0;
    a.mixed = p->opt.precision == FMMG_MIXED ? 1 : 0;
    a.st = st;
    return a;
}

// The solve's launch sequence; returns the number of launches.  ev (may be
// null) receives an event at every stage boundary.
int64_t enqueue_solve(fmmg_plan* p, const double* rho, double* phi, double* g, hipStream_t st,
                      const hipEvent_t* ev) {
    const HostPlan& hp = p->hp;
    Launch a = make_launch(p, st);
    int64_t n = 0;
    int64_t per[FMMG_N_STAGES] = {0, 0, 0, 0, 0, 0, 0};
    auto mark = [&](int stage) { if (ev) (void)hipEventRecord(ev[stage], st); };
    auto cnt = [&](int stage, int items) { if (items > 0) { ++n; ++per[stage]; } };
    // step 1: leaf masses, then moments bottom-up
    mark(FMMG_STAGE_P2M);
    launch_p2m(a, rho, int(hp.leaf_sub.size()));
    cnt(FMMG_STAGE_P2M, int(hp.leaf_sub.size()));
    mark(FMMG_STAGE_M2M);
    for (int l = hp.max_level - 1; l >= 0; --l) {
        int b = hp.level_ref_begin[size_t(l)], e = hp.level_ref_begin[size_t(l) + 1];
        launch_m2m(a, p->d_ref_by_level + b, e - b);
        cnt(FMMG_STAGE_M2M, e - b);
    }
    // step 2: same-level interactions
    mark(FMMG_STAGE_TOP);
    if (!hp.top_items.empty()) {
        launch_top(a, p->d_top_items, int(hp.top_items.size()), p->d_top_src, p->d_top_reduce,
                   int(hp.top_reduce.size()));
        n += 2;
        per[FMMG_STAGE_TOP] += 2;
    }
    mark(FMMG_STAGE_MONO);
    launch_mono(a, p->d_mono_leaf, int(hp.mono_leaf.size()));
    cnt(FMMG_STAGE_MONO, int(hp.mono_leaf.size()));
    mark(FMMG_STAGE_MP_REFINED);
    launch_mp(a, p->d_mp_ref, int(hp.mp_ref.size()), false);
    cnt(FMMG_STAGE_MP_REFINED, int(hp.mp_ref.size()));
    mark(FMMG_STAGE_MP_LEAF);
    launch_mp(a, p->d_mp_leaf, int(hp.mp_leaf.size()), true);
    cnt(FMMG_STAGE_MP_LEAF, int(hp.mp_leaf.size()));
    // step 3: leaves without parents, then top-down re-expansion
    mark(FMMG_STAGE_DOWN);
    launch_leaf_out(a, p->d_top_leaf, int(hp.top_leaf.size()), phi, g);
    cnt(FMMG_STAGE_DOWN, int(hp.top_leaf.size()));
    for (int l = 0; l < hp.max_level; ++l) {
        int b = hp.level_ref_begin[size_t(l)], e = hp.level_ref_begin[size_t(l) + 1];
        launch_l2l(a, p->d_ref_by_level + b, e - b, phi, g);
        cnt(FMMG_STAGE_DOWN, e - b);
    }
    mark(FMMG_N_STAGES);
    for (int s = 0; s < FMMG_N_STAGES; ++s) p->stage_launches[s] = per[s];
    return n;
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
    opt->use_graph = 0;
    opt->persistent = 0;
    opt->timing = 0;
    opt->tuning_cache = nullptr;
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
        if (p->opt.precision != FMMG_FP64 && p->opt.precision != FMMG_MIXED) {
            release(p);
            return fail(FMMG_EINVAL, "bad precision");
        }
        if (p->opt.top_mode != FMMG_TOP_FULL && p->opt.top_mode != FMMG_TOP_STENCIL_ONLY) {
            release(p);
            return fail(FMMG_EINVAL, "bad top_mode");
        }
        if (p->opt.timing && p->opt.use_graph) {
            release(p);
            return fail(FMMG_EINVAL, "timing needs eager launches (use_graph = 0)");
        }
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
        std::vector<TreeIn> tv = to_trees(trees, n_trees);
        std::string err;
        int rc = build_host_plan(tv.data(), n_trees, p->opt.top_mode == FMMG_TOP_FULL, TOP_CHUNKS, &p->hp, &err);
        if (rc) { release(p); return fail(rc == -2 ? FMMG_ETREE : FMMG_EINVAL, err); }
        const HostPlan& hp = p->hp;
        fmmg_status s;
#define UP(dst, src, what) if ((s = dev_upload(&(dst), (src), st, what)) != FMMG_OK) { release(p); return s; }
        UP(p->d_subs, hp.subs, "sub-grid table");
        UP(p->d_leaf_sub, hp.leaf_sub, "leaf list");
        UP(p->d_mp_ref, hp.mp_ref, "refined target list");
        UP(p->d_mono_leaf, hp.mono_leaf, "leaf target list");
        UP(p->d_mp_leaf, hp.mp_leaf, "leaf multipole target list");
        UP(p->d_ref_by_level, hp.ref_by_level, "level lists");
        UP(p->d_top_leaf, hp.top_leaf, "top leaf list");
        UP(p->d_top_src, hp.top_src, "top source list");
        UP(p->d_top_items, hp.top_items, "top items");
        UP(p->d_top_reduce, hp.top_reduce, "top reductions");
#undef UP
        size_t nl = hp.leaf_sub.size(), nr = hp.ref_sub.size();
#define AL(dst, n, what) if ((s = dev_alloc(&(dst), (n), what)) != FMMG_OK) { release(p); return s; }
        AL(p->d_mass, nl * NCELL, "leaf masses");
        AL(p->d_rec, nr * NREC * NCELL, "multipole records");
        AL(p->d_Lr, nr * NLOC * NCELL, "refined expansions");
        AL(p->d_Lf, nl * NLEAF * NCELL, "leaf terms");
        AL(p->d_part, size_t(hp.n_top_parts) * NLOC * NCELL, "top partial sums");
#undef AL
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

fmmg_status fmmg_solve(fmmg_plan* p, const double* rho, double* phi, double* g, void* hip_stream) {
    if (!p) return fail(FMMG_EINVAL, "fmmg_solve: plan is NULL");
    if (!p->hp.leaf_sub.empty() && (!rho || !phi || !g)) return fail(FMMG_EINVAL, "fmmg_solve: null buffer");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p->device) return fail(FMMG_EINVAL, "fmmg_solve: plan belongs to another device");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    try {
        if (!p->opt.use_graph) {
            const hipEvent_t* ev = nullptr;
            if (p->opt.timing) {
                if (p->n_timed == p->events.size()) {
                    if (p->events.size() >= 100000) return fail(FMMG_EINVAL, "fmmg_solve: call fmmg_get_timings at least every 100000 solves");
                    std::array<hipEvent_t, FMMG_N_STAGES + 1> set;
                    set.fill(nullptr);
                    for (auto& e : set) {
                        hipError_t ee = hipEventCreate(&e);
                        if (ee != hipSuccess) {
                            for (auto& d : set) if (d) (void)hipEventDestroy(d);
                            return hip_fail(ee, "hipEventCreate");
                        }
                    }
                    p->events.push_back(set);
                }
                ev = p->events[p->n_timed++].data();
            }
            p->launches = enqueue_solve(p, rho, phi, g, st, ev);
            HIP_TRY(hipGetLastError(), "kernel launch");
        } else {
            if (!p->graph_exec || p->g_rho != rho || p->g_phi != phi || p->g_g != g) {
                if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
                if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
                if (!p->capture_stream)
                    HIP_TRY(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
                HIP_TRY(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
                p->launches = enqueue_solve(p, rho, phi, g, p->capture_stream, nullptr);
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
    return FMMG_OK;
}

void fmmg_plan_destroy(fmmg_plan* p) { release(p); }

}  // extern "C"
