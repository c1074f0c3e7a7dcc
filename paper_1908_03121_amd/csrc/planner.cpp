// planner.cpp -- host-side planning of the octree FMM solve: tree validation,
// neighbour/child tables, the canonical stencil, work lists and pair counts.
//
// The interaction rule (opening criterion, arXiv:1908.03121 Sec. 4.3) for
// same-level cells cA, cB with d = cB - cA and D = floor(cB/2) - floor(cA/2):
// evaluated iff (all-pairs top level or |D|^2 <= 8) and (|d|^2 >= 9 or one
// side is a leaf).  Per parity of cA the parent-near set has 743 offsets
// (651 far, 92 near); the 8 parity sets are mirror images of one another,
// so one canonical table (parity 0,0,0) serves every cell.
#include "planner.hpp"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <unordered_map>

namespace fmmg {

namespace {

int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

uint64_t key_of(int l, int x, int y, int z) {
    return (uint64_t(l) << 57) | (uint64_t(x) << 38) | (uint64_t(y) << 19) | uint64_t(z);
}

// canonical (parity 0,0,0) parent-near offsets
struct Canon {
    std::vector<int> dx, dy, dz;
    std::vector<int> far;
};

const Canon& canon() {
    static Canon c = [] {
        Canon k;
        for (int dz = -REACH; dz <= REACH; ++dz)
            for (int dx = -REACH; dx <= REACH; ++dx)
                for (int dy = -REACH; dy <= REACH; ++dy) {
                    if (!dx && !dy && !dz) continue;
                    int Dx = floordiv(dx, 2), Dy = floordiv(dy, 2), Dz = floordiv(dz, 2);
                    if (Dx * Dx + Dy * Dy + Dz * Dz > 8) continue;
                    k.dx.push_back(dx);
                    k.dy.push_back(dy);
                    k.dz.push_back(dz);
                    k.far.push_back(dx * dx + dy * dy + dz * dz >= 9);
                }
        return k;
    }();
    return c;
}

// Per neighbour slot, the number of (target cell, stencil offset) pairs whose
// source falls into that slot, far and near separately.
struct SlotCounts {
    int64_t far[27], nearc[27];
};

const SlotCounts& slot_counts() {
    static SlotCounts s = [] {
        SlotCounts k;
        memset(&k, 0, sizeof(k));
        const Canon& c = canon();
        for (int q = 0; q < NCELL; ++q) {
            int x = q & 7, y = (q >> 3) & 7, z = q >> 6;
            int sx = 1 - 2 * (x & 1), sy = 1 - 2 * (y & 1), sz = 1 - 2 * (z & 1);
            for (size_t e = 0; e < c.dx.size(); ++e) {
                int bx = x + sx * c.dx[e], by = y + sy * c.dy[e], bz = z + sz * c.dz[e];
                int slot = (floordiv(bx, 8) + 1) * 9 + (floordiv(by, 8) + 1) * 3 + (floordiv(bz, 8) + 1);
                if (c.far[e]) k.far[slot]++;
                else k.nearc[slot]++;
            }
        }
        return k;
    }();
    return s;
}

// far pairs between two refined top-level sub-grids at offset o (|o_i| <= 1)
int64_t top_far_pairs(int ox, int oy, int oz) {
    static int64_t tab[27];
    static bool init = false;
    if (!init) {
        for (int t = 0; t < 27; ++t) {
            int px = t / 9 - 1, py = (t / 3) % 3 - 1, pz = t % 3 - 1;
            int64_t n = 0;
            for (int a = 0; a < NCELL; ++a)
                for (int b = 0; b < NCELL; ++b) {
                    int dx = 8 * px + (b >> 6) - (a >> 6);
                    int dy = 8 * py + ((b >> 3) & 7) - ((a >> 3) & 7);
                    int dz = 8 * pz + (b & 7) - (a & 7);
                    if (dx * dx + dy * dy + dz * dz >= 9) ++n;
                }
            tab[t] = n;
        }
        init = true;
    }
    if (ox < -1 || ox > 1 || oy < -1 || oy > 1 || oz < -1 || oz > 1) return int64_t(NCELL) * NCELL;
    return tab[(ox + 1) * 9 + (oy + 1) * 3 + (oz + 1)];
}

}  // namespace

// Class-4 tables: for every neighbour slot o, the slab of source parents
// within reach and, per target parent of the leaf, its partner parents in the
// slab (|D|^2 <= 8 for the parent offset D; every such pair of parents gives
// the 64 cell pairs of their children, none of them the self pair).
static void build_c4_tables(StencilTables* t) {
    int ng = 0, nt = 0;
    for (int o = 0; o < 27; ++o) {
        t->c4_grp_begin[o] = ng;
        t->c4_slab[o] = 0;
        if (o == 13) continue;
        const int off[3] = {o / 9 - 1, (o / 3) % 3 - 1, o % 3 - 1};
        int n[3], p0[3];
        for (int a = 0; a < 3; ++a) {
            n[a] = off[a] ? 2 : 4;
            p0[a] = off[a] < 0 ? 2 : 0;
        }
        t->c4_slab[o] = n[0] | (n[1] << 4) | (n[2] << 8) | (p0[0] << 12) | (p0[1] << 14) | (p0[2] << 16);
        struct Grp { int pt; std::vector<int> src; };
        std::vector<Grp> grp;
        for (int pt = 0; pt < 64; ++pt) {
            const int tp[3] = {pt >> 4, (pt >> 2) & 3, pt & 3};
            Grp g{pt, {}};
            for (int sp = 0; sp < n[0] * n[1] * n[2]; ++sp) {
                const int ip[3] = {sp / (n[1] * n[2]), (sp / n[2]) % n[1], sp % n[2]};
                int d2 = 0;
                for (int a = 0; a < 3; ++a) {
                    const int D = 4 * off[a] + p0[a] + ip[a] - tp[a];
                    d2 += D * D;
                }
                if (d2 <= 8) g.src.push_back(sp);
            }
            if (!g.src.empty()) grp.push_back(std::move(g));
        }
        std::stable_sort(grp.begin(), grp.end(), [](const Grp& a, const Grp& b) { return a.src.size() > b.src.size(); });
        for (const Grp& g : grp) {
            t->c4_grp[ng++] = g.pt | (nt << 6) | (int(g.src.size()) << 18);
            for (int sp : g.src) t->c4_task[nt++] = sp;
        }
    }
    t->c4_grp_begin[27] = ng;
}

void build_stencil_tables(StencilTables* t) {
    memset(t, 0, sizeof(*t));
    const Canon& c = canon();
    int pos = 0;
    for (int g = 0; g < NDZ; ++g) {
        int dz = DZ0 + g;
        for (int pass = 0; pass < 2; ++pass) {
            int begin = pos;
            for (size_t e = 0; e < c.dx.size(); ++e) {
                if (c.dz[e] != dz || c.far[e] != (pass == 0)) continue;
                // byte offsets of the source cell in a component group of
                // the plane window (16 bytes per cell, MP_PRS cells per row)
                const uint32_t ox = uint16_t(int16_t(16 * c.dx[e]));
                const uint32_t oy = uint16_t(int16_t(16 * MP_PRS * c.dy[e]));
                t->mp_entry[pos++] = int32_t(ox | (oy << 16));
            }
            if (pass == 0) { t->mp_far_begin[g] = begin; t->mp_far_count[g] = pos - begin; }
            else { t->mp_near_begin[g] = begin; t->mp_near_count[g] = pos - begin; }
        }
    }
    // monopole columns by dz-range class: [-4,5], [-2,3], [0,1]
    const int lo_of[3] = {-4, -2, 0}, n_of[3] = {10, 6, 2};
    int nc = 0;
    for (int cls = 0; cls < 3; ++cls) {
        t->mono_class_begin[cls] = nc;
        for (int dx = -REACH; dx <= REACH; ++dx)
            for (int dy = -REACH; dy <= REACH; ++dy) {
                int lo = 100, hi = -100;
                for (size_t e = 0; e < c.dx.size(); ++e)
                    if (c.dx[e] == dx && c.dy[e] == dy) { lo = std::min(lo, c.dz[e]); hi = std::max(hi, c.dz[e]); }
                if (dx == 0 && dy == 0) { lo = -4; hi = 5; }  // the self offset sits inside this column
                if (lo > hi || lo != lo_of[cls] || hi != lo_of[cls] + n_of[cls] - 1) continue;
                t->mono_col[nc++] = (dx + 8) | ((dy + 8) << 8);
            }
    }
    t->mono_class_begin[3] = nc;
    build_c4_tables(t);
    for (int n2 = 1; n2 < MONO_R2; ++n2) {
        const double a = 1.0 / sqrt(double(n2)), b = 1.0 / (double(n2) * sqrt(double(n2)));
        t->mono_r[n2][0] = a;
        t->mono_r[n2][1] = b;
        t->mono_rf[n2][0] = float(a);
        t->mono_rf[n2][1] = float(b);
    }
}

int build_host_plan(const TreeIn* trees, int n_trees, int top_full, int top_chunks,
                    HostPlan* out, std::string* err) {
    HostPlan& P = *out;
    P = HostPlan();
    if (!trees || n_trees < 1) { *err = "need at least one tree"; return -1; }
    if (top_chunks < 1) top_chunks = 1;
    P.n_trees = n_trees;
    P.top_full = top_full;
    int64_t total = 0;
    for (int t = 0; t < n_trees; ++t) {
        const TreeIn& T = trees[t];
        if (T.n < 1 || !T.level || !T.coord) { *err = "tree " + std::to_string(t) + ": empty or null arrays"; return -1; }
        if (!(T.L0 > 0.0) || !isfinite(T.L0)) { *err = "tree " + std::to_string(t) + ": L0 must be finite and > 0"; return -1; }
        total += T.n;
    }
    if (total > (int64_t(1) << 30)) { *err = "too many sub-grids"; return -1; }
    P.subs.resize(size_t(total));
    P.nbr_sub.assign(size_t(total) * 27, -1);
    std::vector<int> refined(size_t(total), 0);
    std::vector<std::unordered_map<uint64_t, int32_t>> maps(n_trees);
    int64_t base = 0;
    for (int t = 0; t < n_trees; ++t) {
        const TreeIn& T = trees[t];
        P.sub_tree_base.push_back(int32_t(base));
        auto& M = maps[t];
        M.reserve(size_t(T.n) * 2);
        for (int i = 0; i < T.n; ++i) {
            int l = T.level[i], x = T.coord[3 * i], y = T.coord[3 * i + 1], z = T.coord[3 * i + 2];
            if (l < 0 || l > 19 || x < 0 || y < 0 || z < 0 || x >= (1 << 19) || y >= (1 << 19) || z >= (1 << 19)) {
                *err = "tree " + std::to_string(t) + ", sub-grid " + std::to_string(i) + ": level/coordinate out of range";
                return -2;
            }
            if (!M.emplace(key_of(l, x, y, z), int32_t(base + i)).second) {
                *err = "tree " + std::to_string(t) + ", sub-grid " + std::to_string(i) + ": duplicate";
                return -2;
            }
        }
        for (int i = 0; i < T.n; ++i) {
            int l = T.level[i], x = T.coord[3 * i], y = T.coord[3 * i + 1], z = T.coord[3 * i + 2];
            SubDev& S = P.subs[size_t(base + i)];
            memset(&S, 0, sizeof(S));
            S.slot3 = -1;
            S.red = -1;
            S.level = l;
            S.tree = t;
            S.coord[0] = x; S.coord[1] = y; S.coord[2] = z;
            S.h = T.L0 / (8.0 * ldexp(1.0, l));
            if (l > 0 && !M.count(key_of(l - 1, x >> 1, y >> 1, z >> 1))) {
                *err = "tree " + std::to_string(t) + ", sub-grid " + std::to_string(i) + ": parent missing";
                return -2;
            }
            int nchild = 0;
            for (int e = 0; e < 8; ++e) {
                auto it = M.find(key_of(l + 1, 2 * x + (e >> 2), 2 * y + ((e >> 1) & 1), 2 * z + (e & 1)));
                S.child[e] = it == M.end() ? -1 : it->second;
                nchild += it != M.end();
            }
            if (nchild != 0 && nchild != 8) {
                *err = "tree " + std::to_string(t) + ", sub-grid " + std::to_string(i) + ": has " +
                       std::to_string(nchild) + " of 8 children";
                return -2;
            }
            refined[size_t(base + i)] = nchild == 8;
            if (l > P.max_level) P.max_level = l;
            for (int o = 0; o < 27; ++o) {
                int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
                int nx = x + ox, ny = y + oy, nz = z + oz;
                int32_t id = -1;
                if (nx >= 0 && ny >= 0 && nz >= 0) {
                    auto it = M.find(key_of(l, nx, ny, nz));
                    if (it != M.end()) id = it->second;
                }
                P.nbr_sub[size_t(base + i) * 27 + size_t(o)] = id;
            }
        }
        base += T.n;
    }
    // leaf / refined numbering in descriptor order, trees concatenated
    for (int t = 0; t < n_trees; ++t) {
        for (int i = 0; i < trees[t].n; ++i) {
            int32_t s = P.sub_tree_base[t] + i;
            SubDev& S = P.subs[size_t(s)];
            if (refined[size_t(s)]) {
                S.kind = 1;
                S.idx = int32_t(P.ref_sub.size());
                P.ref_sub.push_back(s);
            } else {
                S.kind = 0;
                S.idx = int32_t(P.leaf_sub.size());
                P.leaf_sub.push_back(s);
                P.leaf_desc.push_back(i);
            }
        }
    }
    for (size_t s = 0; s < P.subs.size(); ++s) {
        SubDev& S = P.subs[s];
        for (int o = 0; o < 27; ++o) {
            int32_t id = P.nbr_sub[s * 27 + size_t(o)];
            if (id < 0) { S.nbr[o] = -1; continue; }
            const SubDev& N = P.subs[size_t(id)];
            S.nbr[o] = (N.idx << 1) | N.kind;
            if (o != 13) S.flags |= N.kind ? 2 : 1;
        }
    }
    // work lists and pair counts of the stencil step
    const SlotCounts& sc = slot_counts();
    for (int32_t s = 0; s < int32_t(P.subs.size()); ++s) {
        const SubDev& S = P.subs[size_t(s)];
        bool top = S.level == 0 && top_full;
        if (S.level == 0 && S.kind == 0) P.top_leaf.push_back(s);
        if (top) continue;
        if (S.kind) P.mp_ref.push_back(s);
        else {
            P.mono_leaf.push_back(s);
            if (S.flags & 2) P.mp_leaf.push_back(s);
        }
        for (int o = 0; o < 27; ++o) {
            int32_t id = P.nbr_sub[size_t(s) * 27 + size_t(o)];
            if (id < 0) continue;
            int nk = P.subs[size_t(id)].kind;
            if (S.kind) {
                if (nk) P.counts.cls[1] += sc.far[o];
                else P.counts.cls[0] += sc.far[o] + sc.nearc[o];
            } else {
                if (nk) P.counts.cls[3] += sc.far[o] + sc.nearc[o];
                else P.counts.cls[2] += sc.far[o] + sc.nearc[o];
            }
        }
    }
    // class-4 items: each leaf's refined neighbours in slot order, cut after
    // C4_ITEM_STEPS steps; one Lf3 slot per item, a leaf's slots consecutive
    {
        static const std::array<int, 27> steps = [] {
            std::array<int, 27> k{};
            StencilTables t;
            build_stencil_tables(&t);
            for (int o = 0; o < 27; ++o)
                for (int g = t.c4_grp_begin[o]; g < t.c4_grp_begin[o + 1]; ++g) k[size_t(o)] += t.c4_grp[g] >> 18;
            return k;
        }();
        P.c4_chunks.clear();
        int32_t slot = 0;
        for (int32_t s : P.mp_leaf) {
            SubDev& S = P.subs[size_t(s)];
            S.slot3 = slot;
            int o0 = -1, acc = 0;
            for (int o = 0; o < 27; ++o) {
                if (o == 13 || S.nbr[o] < 0 || !(S.nbr[o] & 1)) continue;
                if (o0 < 0) o0 = o;
                acc += steps[size_t(o)];
                if (acc >= C4_ITEM_STEPS) {
                    P.c4_chunks.push_back({s, o0, o + 1, slot++, acc});
                    o0 = -1;
                    acc = 0;
                }
            }
            if (o0 >= 0) P.c4_chunks.push_back({s, o0, 27, slot++, acc});
            S.n3 = slot - S.slot3;
        }
        P.n_slot3 = slot;
    }
    // refined sub-grids level by level; within a level, those whose 8
    // children are all leaves first (their upward step has its own kernel)
    P.level_ref_begin.assign(size_t(P.max_level) + 2, 0);
    P.level_leafpar_end.assign(size_t(P.max_level) + 1, 0);
    for (int l = 0; l <= P.max_level; ++l) {
        P.level_ref_begin[size_t(l)] = int32_t(P.ref_by_level.size());
        for (int pass = 0; pass < 2; ++pass) {
            for (int32_t s : P.ref_sub) {
                const SubDev& S = P.subs[size_t(s)];
                if (S.level != l) continue;
                bool leaves = true;
                for (int e = 0; e < 8; ++e) leaves &= P.subs[size_t(S.child[e])].kind == 0;
                if (leaves == (pass == 0)) P.ref_by_level.push_back(s);
            }
            if (pass == 0) P.level_leafpar_end[size_t(l)] = int32_t(P.ref_by_level.size());
        }
    }
    P.level_ref_begin[size_t(P.max_level) + 1] = int32_t(P.ref_by_level.size());
    P.m2m_tasks.clear();
    for (int32_t s : P.ref_by_level) {
        const SubDev& Ps = P.subs[size_t(s)];
        M2MTask tk;
        tk.pidx = Ps.idx;
        tk.ckinds = 0;
        for (int e = 0; e < 8; ++e) {
            const SubDev& Cs = P.subs[size_t(Ps.child[e])];
            tk.cidx[e] = Cs.idx;
            tk.ckinds |= Cs.kind << e;
        }
        tk.ph = Ps.h;
        P.m2m_tasks.push_back(tk);
    }
    P.level_leaves.assign(size_t(P.max_level) + 1, 0);
    for (const SubDev& S : P.subs)
        if (S.kind == 0) P.level_leaves[size_t(S.level)]++;
    // downward tasks, one launch per (level, child kind).  Sibling children
    // read halves of the same lines of their parent's coefficients, and
    // work-groups go to the 8 XCDs (each with its own L2) in turn by block
    // index: each parent's children are therefore placed on one lane
    // (position mod 8), parents spread over the lanes by load
    P.l2l_begin.assign(size_t(2 * P.max_level) + 1, 0);
    for (int l = 0; l < P.max_level; ++l) {
        for (int kind = 1; kind >= 0; --kind) {
            P.l2l_begin[size_t(2 * l + (1 - kind))] = int32_t(P.l2l_tasks.size());
            std::vector<int32_t> lane[8];
            for (int i = P.level_ref_begin[size_t(l)]; i < P.level_ref_begin[size_t(l) + 1]; ++i) {
                const int32_t ps = P.ref_by_level[size_t(i)];
                int j = 0;
                for (int k = 1; k < 8; ++k)
                    if (lane[k].size() < lane[j].size()) j = k;
                for (int e = 0; e < 8; ++e)
                    if (P.subs[size_t(P.subs[size_t(ps)].child[e])].kind == kind) lane[j].push_back(ps * 8 + e);
            }
            size_t longest = 0;
            for (const auto& v : lane) longest = std::max(longest, v.size());
            for (size_t r = 0; r < longest; ++r)
                for (const auto& v : lane)
                    if (r < v.size()) {
                        const SubDev& Ps = P.subs[size_t(v[r] >> 3)];
                        const int e = v[r] & 7;
                        const SubDev& Cs = P.subs[size_t(Ps.child[e])];
                        L2LTask tk;
                        tk.pidx = Ps.idx;
                        tk.pred = -1;  // set below, with the top level's reductions
                        tk.cidx = Cs.idx;
                        tk.flags = Cs.kind | (e << 1) | (Cs.n3 << 4);
                        tk.slot3 = Cs.slot3;
                        tk.psub = v[r] >> 3;
                        tk.ch = Cs.h;
                        P.l2l_tasks.push_back(tk);
                    }
        }
    }
    P.l2l_begin[size_t(2 * P.max_level)] = int32_t(P.l2l_tasks.size());
    // top level under the all-pairs rule
    if (top_full) {
        for (int t = 0; t < n_trees; ++t) {
            int32_t list_off = int32_t(P.top_src.size());
            std::vector<int32_t> tops;
            for (int i = 0; i < trees[t].n; ++i)
                if (trees[t].level[i] == 0) tops.push_back(P.sub_tree_base[t] + i);
            P.top_src.insert(P.top_src.end(), tops.begin(), tops.end());
            int64_t ncells = int64_t(tops.size()) * NCELL;
            int nchunk = int(std::min<int64_t>(top_chunks, ncells));
            int64_t chunk = (ncells + nchunk - 1) / nchunk;
            nchunk = int((ncells + chunk - 1) / chunk);
            for (int32_t T : tops) {
                TopReduce R;
                memset(&R, 0, sizeof(R));
                R.target = T;
                R.part_begin = P.n_top_parts;
                R.n_part = nchunk;
                for (int k = 0; k < nchunk; ++k) {
                    for (int zt = 0; zt < NS; ++zt) {
                        TopItem it;
                        memset(&it, 0, sizeof(it));
                        it.target = T;
                        it.zt = zt;
                        it.src_begin = int32_t(k * chunk);
                        it.src_end = int32_t(std::min<int64_t>(ncells, (k + 1) * chunk));
                        it.part = P.n_top_parts + k;
                        it.src_list = list_off;
                        P.top_items.push_back(it);
                    }
                }
                P.n_top_parts += nchunk;
                P.subs[size_t(T)].red = int32_t(P.top_reduce.size());
                P.top_reduce.push_back(R);
                const SubDev& ST = P.subs[size_t(T)];
                for (int32_t Sb : tops) {
                    const SubDev& SS = P.subs[size_t(Sb)];
                    int64_t n;
                    if (!ST.kind || !SS.kind) n = int64_t(NCELL) * NCELL - (Sb == T ? NCELL : 0);
                    else n = top_far_pairs(SS.coord[0] - ST.coord[0], SS.coord[1] - ST.coord[1],
                                           SS.coord[2] - ST.coord[2]);
                    P.counts.top += n;
                }
            }
        }
    }
    for (L2LTask& tk : P.l2l_tasks) tk.pred = P.subs[size_t(tk.psub)].red;
    build_items(&P, 1, true, 0);
    return 0;
}

void build_items(HostPlan* Pp, int ngroups, bool split, int pairs) {
    HostPlan& P = *Pp;
    if (ngroups < 1) ngroups = 1;
    if (ngroups > MAX_GROUPS) ngroups = MAX_GROUPS;
    P.ngroups = ngroups;
    P.pairs = pairs ? 1 : 0;
    StencilTables tab;
    build_stencil_tables(&tab);
    // estimated cost of an item, in refined-pair units, and its level
    struct Costed { Item it; double cost; int level; };
    std::vector<Costed> all;
    // a source plane with no usable neighbour among the 9 at its offset along
    // the sweep axis (z for sweep 0, y for sweep 1, x for sweep 2) is skipped
    // by the kernels; the estimates count the planes they visit.  Neighbour-
    // code strides of the frame axes (u, v, w): (x, y, z), (x, z, y), (z, y, x)
    auto plane_used = [&](const SubDev& S, int sweep, int ws) {
        const int ow = ws < 0 ? -1 : (ws >= NS ? 1 : 0);
        const int UN = sweep == 2 ? 1 : 9, VN = sweep == 1 ? 1 : 3;
        const int WN = sweep == 0 ? 1 : (sweep == 1 ? 3 : 9);
        for (int o = 0; o < 9; ++o)
            if (S.nbr[(o / 3) * UN + (o % 3) * VN + (ow + 1) * WN] >= 0) return true;
        return false;
    };
    // stencil entries that target plane zt visits over the canonical plane
    // offsets [i0, i1)
    auto visited = [&](const SubDev& S, int sweep, int zt, int i0, int i1, bool nearc) {
        double n = 0;
        for (int i = i0; i < i1; ++i)
            if (plane_used(S, sweep, zt + (1 - 2 * (zt & 1)) * (DZ0 + i)))
                n += tab.mp_far_count[i] + (nearc ? tab.mp_near_count[i] : 0);
        return n;
    };
    // the sweep of a target: the frame that visits the fewest entries (on a
    // tie the first of z, y, x)
    auto best_sweep = [&](const SubDev& S, bool nearc) {
        double n[3] = {0, 0, 0};
        for (int sw = 0; sw < 3; ++sw)
            for (int zt = 0; zt < NS; ++zt) n[sw] += visited(S, sw, zt, 0, NDZ, nearc);
        int best = 0;
        for (int sw = 1; sw < 3; ++sw)
            if (n[sw] < n[best]) best = sw;
        return best;
    };
    P.sweep_y_targets = 0;
    P.sweep_x_targets = 0;
    for (int32_t s : P.mp_ref) {
        const SubDev& S = P.subs[size_t(s)];
        const bool nearc = (S.flags & 1) != 0;
        const int sw = best_sweep(S, nearc);
        P.sweep_y_targets += sw == 1;
        P.sweep_x_targets += sw == 2;
        // per plane of parent cells (target planes 2 pz, 2 pz + 1) and group
        // of staged source planes j (canonical offsets j of the even plane and
        // NDZ - 1 - j of the odd one): one item of both planes, or one per plane
        for (int pz = 0; pz < NS / 2; ++pz)
            for (int g = 0; g < ngroups; ++g) {
                const int j0 = g * NDZ / ngroups, j1 = (g + 1) * NDZ / ngroups;
                const double ne = visited(S, sw, 2 * pz, j0, j1, nearc);
                const double no = visited(S, sw, 2 * pz + 1, NDZ - j1, NDZ - j0, nearc);
                const int b = g | (sw << 3);
                if (P.pairs) {
                    all.push_back({Item{IT_MP_REF, s, 2 * pz | 3 << 4, b}, 64.0 * (ne + no) + 3000.0, S.level});
                } else {
                    all.push_back({Item{IT_MP_REF, s, 2 * pz | 1 << 4, b}, 64.0 * ne + 2000.0, S.level});
                    all.push_back({Item{IT_MP_REF, s, 2 * pz | 2 << 4, b}, 64.0 * no + 2000.0, S.level});
                }
            }
    }
    // class-4 items: cost of their (target parent, source parent) steps of
    // 64 pairs each, plus the staging of every refined neighbour's slab
    for (const HostPlan::C4Chunk& c : P.c4_chunks) {
        int nn = 0;
        for (int o = c.o_begin; o < c.o_end; ++o) nn += o != 13 && P.subs[size_t(c.sub)].nbr[o] >= 0 && (P.subs[size_t(c.sub)].nbr[o] & 1);
        all.push_back({Item{IT_MP_LEAF, c.sub, c.o_begin | (c.o_end << 8), c.slot},
                       64.0 * 0.65 * c.steps + 1500.0 * nn + 2000.0, P.subs[size_t(c.sub)].level});
    }
    for (int32_t s : P.mono_leaf)
        all.push_back({Item{IT_MONO, s, 0, 0}, 512.0 * 743.0 * 0.025 + 4000.0, P.subs[size_t(s)].level});
    for (size_t k = 0; k < P.top_items.size(); ++k) {
        const TopItem& ti = P.top_items[k];
        all.push_back({Item{IT_TOP, int32_t(k), 0, 0}, 64.0 * double(ti.src_end - ti.src_begin) + 1000.0, 0});
    }
    // split level: the coarse levels below it carry at most a fifth of the work
    std::vector<double> lc(size_t(P.max_level) + 1, 0.0);
    double total = 0;
    for (const Costed& c : all) {
        lc[size_t(c.level)] += c.cost;
        total += c.cost;
    }
    P.split_natural = 0;
    double below = 0;
    for (int s = 1; s <= P.max_level; ++s) {
        below += lc[size_t(s) - 1];
        if (below <= 0.2 * total) P.split_natural = s;
    }
    P.split = split ? P.split_natural : 0;
    auto branch = [&](const Costed& c) { return c.level < P.split ? 1 : 0; };
    // class lists in sub-grid order (measured no slower than largest first,
    // since neighbouring items share sources in the caches); the persistent
    // list largest estimated cost first
    P.items_class.clear();
    for (int b = 0; b < 2; ++b) {
        const int order[IT_KINDS] = {IT_MP_REF, IT_MP_LEAF, IT_MONO, IT_TOP};
        for (int k : order) {
            P.class_begin[b][k] = int32_t(P.items_class.size());
            for (const Costed& c : all)
                if (c.it.kind == k && branch(c) == b) P.items_class.push_back(c.it);
        }
        P.class_begin[b][IT_KINDS] = int32_t(P.items_class.size());
    }
    // persistent lists: per branch, NQUEUE queues, one per XCD (the blocks of
    // a persistent launch are dealt to the XCDs in turn, and each XCD has its
    // own L2).  Items in the order of their target sub-grid along a Z-order
    // curve (tree by tree, positions scaled to the finest level), so that a
    // queue holds a compact region whose source records stay in its XCD's
    // L2, cut into NQUEUE runs of equal estimated cost; top-level items lead
    // their run, the small monopole items trail it (a short tail).
    // (19 bits per axis below the tree index: the coarsest bits are kept for
    // deep trees; the key orders only, so a lost bit costs locality, not
    // correctness)
    int lmax = 0, c0max = 1;
    for (const SubDev& S : P.subs) {
        lmax = std::max(lmax, int(S.level));
        if (S.level == 0)
            for (int a = 0; a < 3; ++a) c0max = std::max(c0max, int(S.coord[a]) + 1);
    }
    int top_bits = 0;  // bits of a level-0 coordinate
    while ((1 << top_bits) < c0max) ++top_bits;
    const int nbits = lmax + top_bits, drop = nbits > 19 ? nbits - 19 : 0;
    auto zkey = [&](const Costed& c) -> uint64_t {
        if (c.it.kind == IT_TOP) return 0;
        const SubDev& S = P.subs[size_t(c.it.sub)];
        uint64_t x[3];
        for (int a = 0; a < 3; ++a) x[a] = (uint64_t(uint32_t(S.coord[a])) << (lmax - S.level)) >> drop;
        uint64_t k = 0;
        for (int bit = nbits - drop - 1; bit >= 0; --bit)
            for (int a = 0; a < 3; ++a) k = (k << 1) | ((x[a] >> bit) & 1);
        return (uint64_t(uint32_t(S.tree) & 63) << 57) | k;
    };
    std::vector<std::pair<uint64_t, size_t>> order;
    order.reserve(all.size());
    for (size_t i = 0; i < all.size(); ++i) order.push_back({zkey(all[i]), i});
    std::stable_sort(order.begin(), order.end());
    P.items_xcd.clear();
    for (int b = 0; b < 2; ++b) {
        double total = 0;
        for (const auto& o : order)
            if (branch(all[o.second]) == b) total += all[o.second].cost;
        std::vector<size_t> run[NQUEUE];
        double acc = 0;
        for (const auto& o : order) {
            const Costed& c = all[o.second];
            if (branch(c) != b) continue;
            int q = total > 0 ? int(acc / total * NQUEUE) : 0;
            if (q >= NQUEUE) q = NQUEUE - 1;
            run[q].push_back(o.second);
            acc += c.cost;
        }
        for (int q = 0; q < NQUEUE; ++q) {
            P.queue_begin[b][q] = int32_t(P.items_xcd.size());
            for (int pass = 0; pass < 3; ++pass)
                for (size_t i : run[q]) {
                    const int k = all[i].it.kind;
                    if ((pass == 0) == (k == IT_TOP) && (pass == 2) == (k == IT_MONO)) P.items_xcd.push_back(all[i].it);
                }
        }
        P.queue_begin[b][NQUEUE] = int32_t(P.items_xcd.size());
    }
    // the single list: largest estimated cost first
    std::vector<Costed> lpt = all;
    std::stable_sort(lpt.begin(), lpt.end(), [](const Costed& a, const Costed& b) { return a.cost > b.cost; });
    P.items_lpt.clear();
    for (int b = 0; b < 2; ++b) {
        P.lpt_begin[b] = int32_t(P.items_lpt.size());
        for (const Costed& c : lpt)
            if (branch(c) == b) P.items_lpt.push_back(c.it);
    }
    P.lpt_begin[2] = int32_t(P.items_lpt.size());
}

}  // namespace fmmg
