// Host driver for the sanitizer test of the planner: reads a dump of octree
// descriptors (written by tests/test_planner_sanitized.py), builds the host
// plan for both top-level modes and the work-item lists for every plane-group
// count with and without the coarse-level split, and prints the pair counts.
// Built with g++ and AddressSanitizer / UndefinedBehaviorSanitizer; no GPU.
#include "planner.hpp"

#include <cstdio>
#include <string>
#include <vector>

using namespace fmmg;

static bool rd(FILE* f, void* p, size_t sz, size_t n) { return fread(p, sz, n, f) == n; }

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int nsets = 0;
    if (!rd(f, &nsets, 4, 1)) return 2;
    for (int si = 0; si < nsets; ++si) {
        char name[17] = {0};
        int nt = 0;
        if (!rd(f, name, 16, 1) || !rd(f, &nt, 4, 1)) return 2;
        std::vector<std::vector<int32_t>> lv(static_cast<size_t>(nt)), co(static_cast<size_t>(nt));
        std::vector<TreeIn> tv(static_cast<size_t>(nt));
        for (int t = 0; t < nt; ++t) {
            int n = 0;
            double o[3], L0;
            if (!rd(f, &n, 4, 1) || !rd(f, o, 8, 3) || !rd(f, &L0, 8, 1)) return 2;
            lv[size_t(t)].resize(size_t(n));
            co[size_t(t)].resize(size_t(n) * 3);
            if (!rd(f, lv[size_t(t)].data(), 4, size_t(n)) || !rd(f, co[size_t(t)].data(), 4, size_t(n) * 3)) return 2;
            tv[size_t(t)] = TreeIn{n, lv[size_t(t)].data(), co[size_t(t)].data(), {o[0], o[1], o[2]}, L0};
        }
        for (int top_full = 0; top_full < 2; ++top_full) {
            HostPlan hp;
            std::string err;
            const int rc = build_host_plan(tv.data(), nt, top_full, 8, &hp, &err);
            if (rc) {
                printf("%s top_full=%d error %d %s\n", name, top_full, rc, err.c_str());
                return 1;
            }
            for (int g = 1; g <= MAX_GROUPS; ++g)
                for (int split = 0; split < 2; ++split) build_items(&hp, g, split != 0);
            printf("%s %d %zu %zu %lld %lld %lld %lld %lld\n", name, top_full, hp.leaf_sub.size(),
                   hp.ref_sub.size(), (long long)hp.counts.cls[0], (long long)hp.counts.cls[1],
                   (long long)hp.counts.cls[2], (long long)hp.counts.cls[3], (long long)hp.counts.top);
        }
    }
    fclose(f);
    StencilTables st;
    build_stencil_tables(&st);
    printf("done\n");
    return 0;
}
