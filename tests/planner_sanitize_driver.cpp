// Host driver for the sanitizer test of the planner: reads a dump of octree
// descriptors (written by tests/test_planner_sanitized.py), builds the host
// plan for both top-level modes and the work-item lists for every plane-group
// count with and without the coarse-level split, and prints the pair counts.
// Built with g++ and AddressSanitizer / UndefinedBehaviorSanitizer; no GPU.
#include "planner.hpp"

#include <algorithm>
#include <array>
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
            // the upward and downward passes' task records agree with the
            // sub-grid table they summarise
            {
                size_t n_ref = 0;
                for (const SubDev& S : hp.subs) n_ref += S.kind == 1;
                // every refined sub-grid is a parent once upward and 8 times downward
                bool ok = hp.m2m_tasks.size() == hp.ref_by_level.size() && hp.ref_by_level.size() == n_ref &&
                          hp.l2l_tasks.size() == 8 * n_ref;
                for (size_t i = 0; ok && i < hp.m2m_tasks.size(); ++i) {
                    const M2MTask& tk = hp.m2m_tasks[i];
                    const SubDev& Ps = hp.subs[size_t(hp.ref_by_level[i])];
                    ok = tk.pidx == Ps.idx && tk.ph == Ps.h;
                    for (int e = 0; ok && e < 8; ++e) {
                        const SubDev& Cs = hp.subs[size_t(Ps.child[e])];
                        ok = tk.cidx[e] == Cs.idx && ((tk.ckinds >> e) & 1) == Cs.kind && Cs.h == 0.5 * Ps.h;
                    }
                }
                for (size_t i = 0; ok && i < hp.l2l_tasks.size(); ++i) {
                    const L2LTask& tk = hp.l2l_tasks[i];
                    const SubDev& Ps = hp.subs[size_t(tk.psub)];
                    const int e = (tk.flags >> 1) & 7;
                    const SubDev& Cs = hp.subs[size_t(Ps.child[e])];
                    ok = Ps.kind == 1 && tk.pidx == Ps.idx && tk.pred == Ps.red && tk.cidx == Cs.idx &&
                         (tk.flags & 1) == Cs.kind && (tk.flags >> 4) == Cs.n3 && tk.slot3 == Cs.slot3 &&
                         tk.ch == Cs.h;
                }
                if (!ok) {
                    printf("%s top_full=%d pass task records wrong\n", name, top_full);
                    return 1;
                }
            }
            for (int g = 1; g <= MAX_GROUPS; ++g)
                for (int split = 0; split < 2; ++split)
                for (int pairs = 0; pairs < 2; ++pairs) {
                    build_items(&hp, g, split != 0, pairs);
                    // the refined-target items cover every (target, plane,
                    // group) once, each with both planes of its parent plane
                    // when paired and one plane otherwise
                    {
                        std::vector<int> cover(hp.subs.size() * NS * size_t(g), 0);
                        bool ok = true;
                        size_t n_ref_items = 0;
                        for (const Item& it : hp.items_class) {
                            if (it.kind != IT_MP_REF) continue;
                            ++n_ref_items;
                            const int zt0 = it.a & 15, m = it.a >> 4, grp = it.b & 7;
                            ok = ok && zt0 % 2 == 0 && zt0 < NS && grp < g && (pairs ? m == 3 : (m == 1 || m == 2));
                            for (int pl = 0; pl < 2 && ok; ++pl)
                                if (m >> pl & 1) ++cover[(size_t(it.sub) * NS + size_t(zt0 + pl)) * size_t(g) + size_t(grp)];
                        }
                        for (int32_t sref : hp.mp_ref)
                            for (int z = 0; z < NS; ++z)
                                for (int gg = 0; gg < g; ++gg)
                                    ok = ok && cover[(size_t(sref) * NS + size_t(z)) * size_t(g) + size_t(gg)] == 1;
                        ok = ok && n_ref_items == hp.mp_ref.size() * size_t(NS / (pairs ? 2 : 1) * g);
                        if (!ok) {
                            printf("%s refined-target items wrong (groups %d split %d pairs %d)\n", name, g, split, pairs);
                            return 1;
                        }
                    }
                    // the persistent queues of each branch partition it, and
                    // hold the same items as the per-class lists
                    for (int b = 0; b < 2; ++b) {
                        bool ok = hp.queue_begin[b][0] == hp.lpt_begin[b] &&
                                  hp.queue_begin[b][NQUEUE] == hp.lpt_begin[b + 1];
                        for (int q = 0; q < NQUEUE; ++q) ok = ok && hp.queue_begin[b][q] <= hp.queue_begin[b][q + 1];
                        std::vector<std::array<int32_t, 4>> a, x, c;
                        for (int32_t i = hp.lpt_begin[b]; i < hp.lpt_begin[b + 1]; ++i) {
                            const Item& it = hp.items_lpt[size_t(i)];
                            a.push_back({it.kind, it.sub, it.a, it.b});
                            const Item& jt = hp.items_xcd[size_t(i)];
                            x.push_back({jt.kind, jt.sub, jt.a, jt.b});
                        }
                        for (int32_t i = hp.class_begin[b][0]; i < hp.class_begin[b][IT_KINDS]; ++i) {
                            const Item& it = hp.items_class[size_t(i)];
                            c.push_back({it.kind, it.sub, it.a, it.b});
                        }
                        std::sort(a.begin(), a.end());
                        std::sort(x.begin(), x.end());
                        std::sort(c.begin(), c.end());
                        if (!ok || a != c || x != c) {
                            printf("%s persistent queues wrong (groups %d split %d pairs %d branch %d)\n", name, g, split,
                                   pairs, b);
                            return 1;
                        }
                    }
                }
            // class-4 items: each leaf's refined neighbours covered exactly
            // once, in slot order, by its own consecutive Lf3 slots
            std::vector<int> covered(hp.subs.size() * 27, 0);
            int32_t next_slot = 0;
            for (const HostPlan::C4Chunk& c : hp.c4_chunks) {
                const SubDev& S = hp.subs[size_t(c.sub)];
                if (c.slot != next_slot++ || c.slot < S.slot3 || c.slot >= S.slot3 + S.n3 || c.o_begin < 0 ||
                    c.o_end > 27 || c.o_begin >= c.o_end) {
                    printf("%s class-4 chunk slots wrong\n", name);
                    return 1;
                }
                for (int o = c.o_begin; o < c.o_end; ++o)  // the item visits only refined neighbours
                    if (o != 13 && S.nbr[o] >= 0 && (S.nbr[o] & 1)) covered[size_t(c.sub) * 27 + size_t(o)]++;
            }
            if (next_slot != hp.n_slot3) { printf("%s class-4 slot count wrong\n", name); return 1; }
            for (size_t s = 0; s < hp.subs.size(); ++s)
                for (int o = 0; o < 27; ++o) {
                    const SubDev& S = hp.subs[s];
                    const bool want = S.kind == 0 && S.n3 > 0 && o != 13 && S.nbr[o] >= 0 && (S.nbr[o] & 1);
                    if (covered[s * 27 + size_t(o)] != (want ? 1 : 0)) {
                        printf("%s class-4 neighbour coverage wrong\n", name);
                        return 1;
                    }
                }
            printf("%s %d %zu %zu %lld %lld %lld %lld %lld\n", name, top_full, hp.leaf_sub.size(),
                   hp.ref_sub.size(), (long long)hp.counts.cls[0], (long long)hp.counts.cls[1],
                   (long long)hp.counts.cls[2], (long long)hp.counts.cls[3], (long long)hp.counts.top);
        }
    }
    fclose(f);
    StencilTables st;
    build_stencil_tables(&st);
    // class-4 tables against a brute-force count: for every neighbour slot,
    // the (target parent, source parent) steps must cover each leaf-target /
    // source cell pair of the rule (parents within |D|^2 <= 8) exactly once
    bool ok = st.c4_grp_begin[0] == 0 && st.c4_grp_begin[27] <= C4_MAX_GROUPS;
    for (int o = 0; o < 27 && ok; ++o) {
        const int off[3] = {o / 9 - 1, (o / 3) % 3 - 1, o % 3 - 1};
        std::vector<int> seen(size_t(NCELL) * NCELL, 0);
        if (o == 13) {
            ok = st.c4_grp_begin[14] == st.c4_grp_begin[13];
            continue;
        }
        const int sl = st.c4_slab[o];
        const int n[3] = {sl & 15, (sl >> 4) & 15, (sl >> 8) & 15};
        const int p0[3] = {(sl >> 12) & 3, (sl >> 14) & 3, (sl >> 16) & 3};
        if (n[0] * n[1] * n[2] > C4_SLAB) ok = false;
        for (int g = st.c4_grp_begin[o]; g < st.c4_grp_begin[o + 1] && ok; ++g) {
            const int pt = st.c4_grp[g] & 63, first = (st.c4_grp[g] >> 6) & 4095, cnt = st.c4_grp[g] >> 18;
            if (first + cnt > C4_MAX_TASKS) { ok = false; break; }
            for (int k = first; k < first + cnt; ++k) {
                const int sp = st.c4_task[k];
                const int ip[3] = {sp / (n[1] * n[2]), (sp / n[2]) % n[1], sp % n[2]};
                for (int tc = 0; tc < 8; ++tc)
                    for (int sc = 0; sc < 8; ++sc) {
                        const int tq = ((2 * (pt & 3) + (tc & 1)) * 8 + 2 * ((pt >> 2) & 3) + ((tc >> 1) & 1)) * 8 +
                                       2 * (pt >> 4) + (tc >> 2);
                        const int scl[3] = {sc >> 2, (sc >> 1) & 1, sc & 1};
                        int cs[3];
                        for (int a = 0; a < 3; ++a) cs[a] = 2 * (p0[a] + ip[a]) + scl[a];
                        const int sq = (cs[2] * 8 + cs[1]) * 8 + cs[0];
                        seen[size_t(tq) * NCELL + size_t(sq)]++;
                    }
            }
        }
        for (int tq = 0; tq < NCELL && ok; ++tq)
            for (int sq = 0; sq < NCELL; ++sq) {
                const int t[3] = {tq & 7, (tq >> 3) & 7, tq >> 6}, s[3] = {sq & 7, (sq >> 3) & 7, sq >> 6};
                int d2 = 0;
                for (int a = 0; a < 3; ++a) {
                    const int D = 4 * off[a] + (s[a] >> 1) - (t[a] >> 1);  // parent offset
                    d2 += D * D;
                }
                if (seen[size_t(tq) * NCELL + size_t(sq)] != (d2 <= 8 ? 1 : 0)) { ok = false; break; }
            }
    }
    printf("%s\n", ok ? "c4 tables ok" : "c4 tables WRONG");
    printf("done\n");
    return 0;
}
