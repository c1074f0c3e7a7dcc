// planner.hpp -- host-side planning of the octree FMM solve (no device code).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "fmmg_internal.h"

namespace fmmg {

struct TreeIn {
    int32_t n;
    const int32_t* level;
    const int32_t* coord;
    double origin[3];
    double L0;
};

struct PairCounts {
    int64_t cls[4] = {0, 0, 0, 0};  // refined<-leaf, refined<-refined, leaf<-leaf, leaf<-refined
    int64_t top = 0;
    double paper_flops() const {
        return 12.0 * double(cls[2]) + 455.0 * double(cls[0] + cls[1] + cls[3] + top);
    }
};

struct HostPlan {
    int n_trees = 0;
    int top_full = 1;
    int max_level = 0;
    std::vector<SubDev> subs;          // all sub-grids, trees concatenated
    std::vector<int32_t> sub_tree_base;  // first global sub id of each tree
    std::vector<int32_t> leaf_sub;     // global leaf order -> sub id
    std::vector<int32_t> leaf_desc;    // global leaf order -> descriptor index in its tree
    std::vector<int32_t> ref_sub;      // refined index -> sub id
    std::vector<int32_t> nbr_sub;      // [n_sub][27] neighbour sub ids (-1 absent)

    // work lists (global sub ids)
    std::vector<int32_t> mp_ref;       // refined targets of the stencil step
    std::vector<int32_t> mono_leaf;    // leaf targets of the stencil step
    std::vector<int32_t> mp_leaf;      // leaf targets with a refined neighbour
    std::vector<int32_t> level_ref_begin;  // refined sub ids sorted by level: [l, l+1)
    std::vector<int32_t> ref_by_level;
    std::vector<M2MTask> m2m_tasks;          // the upward pass's record of each, same order
    std::vector<int32_t> level_leafpar_end;  // level l's parents with 8 leaf children:
                                             // [level_ref_begin[l], level_leafpar_end[l])
    std::vector<int32_t> top_leaf;     // top-level leaves (output straight from own terms)
    std::vector<int32_t> level_leaves; // number of leaf sub-grids per level
    // downward tasks, parent sub id * 8 + child slot, grouped by parent level
    // and child kind: level l's refined children are [l2l_begin[2l],
    // l2l_begin[2l+1]), its leaf children [l2l_begin[2l+1], l2l_begin[2l+2])
    std::vector<L2LTask> l2l_tasks;
    std::vector<int32_t> l2l_begin;
    int32_t n_slot3 = 0;               // Lf3 slots: one per class-4 item
    struct C4Chunk { int32_t sub, o_begin, o_end, slot, steps; };
    std::vector<C4Chunk> c4_chunks;    // class-4 items: a leaf's neighbour slots [o_begin, o_end)

    // same-level work items for a given number of plane groups, in two
    // branches: 0 = levels >= split (fine), 1 = levels < split (coarse)
    int ngroups = 1;
    int pairs = 0;                     // 1: a refined-target item takes both planes of a parent plane
    int split = 0;                     // split level of the current lists (0: one branch)
    int split_natural = 0;             // split level the estimates give
    int32_t sweep_y_targets = 0;       // refined targets whose plane items run along y
    int32_t sweep_x_targets = 0;       // refined targets whose plane items run along x
    std::vector<Item> items_class;     // grouped by branch, then kind, in list order
    int32_t class_begin[2][IT_KINDS + 1] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
    // persistent lists, branch 0 then branch 1 (the same items per branch in
    // both): items_lpt largest estimated cost first; items_xcd cut into
    // NQUEUE queues, one per XCD, of about equal estimated cost
    std::vector<Item> items_lpt;
    std::vector<Item> items_xcd;
    int32_t lpt_begin[3] = {0, 0, 0};  // branch b: [lpt_begin[b], lpt_begin[b + 1]) in both lists
    int32_t queue_begin[2][NQUEUE + 1] = {};  // queue q of branch b: [queue_begin[b][q], [q + 1]) in items_xcd

    // top level under the all-pairs rule
    std::vector<int32_t> top_src;      // per tree, its level-0 sub ids (concatenated)
    std::vector<TopItem> top_items;
    std::vector<TopReduce> top_reduce;
    int32_t n_top_parts = 0;

    PairCounts counts;
};

// Validates trees and builds every host table.  Returns 0, or -1 (argument)
// / -2 (malformed tree) with a message in *err.
int build_host_plan(const TreeIn* trees, int n_trees, int top_full, int top_chunks,
                    HostPlan* out, std::string* err);

// (Re)builds the work-item lists with ngroups (1..MAX_GROUPS) plane groups
// per refined-target plane item, an item taking both target planes of a
// parent plane (pairs = 1) or one (pairs = 0).  The natural split level is
// the largest s <= max_level whose levels below s carry at most a fifth of
// the estimated same-level work (0: none); the lists use it when split is
// true (a coarse branch for the overlapped solve), else split = 0 (every
// class one list).
void build_items(HostPlan* P, int ngroups, bool split, int pairs);

// Fills the canonical stencil tables.
void build_stencil_tables(StencilTables* t);

}  // namespace fmmg
