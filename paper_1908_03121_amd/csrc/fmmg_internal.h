// fmmg_internal.h -- data layouts shared by the host planner, the API layer
// and the gfx950 kernels of the octree FMM gravity solve.
//
// Device layouts (all float64 unless noted; "q" is the internal cell index
// q = (z*8 + y)*8 + x inside a sub-grid, x fastest, so that a z-plane of a
// sub-grid is 64 contiguous values):
//   mass [n_leaf][512]            leaf cell masses m = rho h^3
//   rec  [n_ref][512][16]         refined cells, 16 contiguous values per
//                                 cell (read and written as 8 16-byte
//                                 groups): m, COM offset from the cell
//                                 centre (3), trace-free quadrupole (5:
//                                 xx yy xy xz yz), trace-free octupole
//                                 (7: xxx xxy xxz xyy xyz yyy yyz)
//                                 followed by one all-zero record
//   com  [n_ref][3][512]          the COM offsets again, component-major,
//                                 for the downward pass
//   Lp   [groups][n_ref][19][512] refined cells' own (same-level) Taylor
//                                 coefficients, one partial per group of
//                                 source planes: L0, L1 (3), trace-free L2 (5),
//                                 trace-free L3 (7), correction dg (3)
//   Lr   [n_ref][19][512]         refined cells' total coefficients (step 3)
//   Lf   [n_leaf][4][512]         leaf cells' own potential and acceleration
//                                 from leaf sources (or the top level)
//   Lf3  [n_slot3][4][512]        the same from refined sources, for leaves
//                                 that have refined neighbours: one slot per
//                                 class-4 item, a leaf's slots consecutive
// Trace-free storage is exact here: every contraction of the method is with a
// derivative tensor of 1/r, which is harmonic (trace-free), and trace parts
// of children's moments contribute only trace parts to the parent's.
#pragma once

#include <stdint.h>

namespace fmmg {

constexpr int NS = 8;          // cells per sub-grid edge
constexpr int NCELL = 512;     // cells per sub-grid
constexpr int REACH = 5;       // max |d_i| of the stencil
constexpr int PW = NS + 2 * REACH;  // 18: edge of the source window around a sub-grid
constexpr int PCELLS = PW * PW;     // 324 cells in one source plane window
constexpr int PRS = 20;             // LDS row stride (cells) of the monopole mass box: with
                                    // lanes y-fastest (lane = x*8 + y), each pass of 32
                                    // lanes reading 8-byte words over 64 banks hits
                                    // distinct banks for every mirrored stencil offset
constexpr int PSLOTS = PW * PRS;    // 360 LDS cells per box plane
constexpr int MP_PRS = PW;          // 18: row stride of the multipole plane window, whose
                                    // records sit in 16-byte groups of components: each
                                    // pass of 16 lanes reading 16-byte groups then hits
                                    // distinct bank groups (rows of both lane parities
                                    // differ mod 8, and 2 * 18 = 2 mod 16 spreads them)
constexpr int MP_SLOTS = PW * MP_PRS;  // 324
constexpr int NREC = 16;       // record components of a refined cell
constexpr int NLOC = 19;       // Taylor components of a refined cell
constexpr int NLEAF = 4;       // phi, gx, gy, gz of a leaf cell
constexpr int NDZ = 10;        // canonical dz range [-4, 5] of the parity-000 stencil
constexpr int DZ0 = -4;
constexpr int MONO_COLS = 100; // canonical (dx, dy) columns
constexpr int MONO_R2 = 76;     // squared canonical offsets |d|^2 of the monopole columns: 0..75

// record component indices
enum { R_M = 0, R_DX = 1, R_DY = 2, R_DZ = 3, R_Q = 4, R_O = 9 };
// Taylor component indices
enum { T_L0 = 0, T_L1 = 1, T_L2 = 4, T_L3 = 9, T_S = 16 };
// Arithmetic of the same-level pair terms.  PR_F64: FP64 throughout.
// PR_MIX: sources staged in FP64; the Taylor coefficients' pair terms in FP32
// with FP32 partial sums per source plane, flushed into FP64 sums; the
// angular-momentum correction's pair terms evaluated and summed in FP64.
// PR_F32: sources staged in FP32 and every pair term, the correction's
// included, in FP32 with FP32 partial sums per source plane.
enum { PR_F64 = 0, PR_MIX = 1, PR_F32 = 2 };

struct SubDev {
    double h;          // cell edge
    int32_t kind;      // 0 leaf, 1 refined
    int32_t idx;       // index into the leaf or the refined arrays
    int32_t level;
    int32_t tree;
    int32_t nbr[27];   // same-level neighbours: -1 absent, else (idx << 1) | kind
                       // (idx into the leaf or refined arrays); slot
                       // (ox+1)*9 + (oy+1)*3 + (oz+1) for offset (ox,oy,oz)
    int32_t child[8];  // refined: child sub-grid ids, slot ex*4 + ey*2 + ez
    int32_t coord[3];
    int32_t flags;     // bit0: has a leaf neighbour; bit1: has a refined neighbour
    int32_t slot3;     // leaf with refined neighbours: its first Lf3 slot, else -1
    int32_t red;       // top level under the all-pairs rule: its TopReduce index, else -1
    int32_t n3;        // leaf with refined neighbours: its number of Lf3 slots (one per
                       // class-4 item), else 0
};

// Same-level work items.  A block of 256 threads (4 waves) runs one item.
enum { IT_MP_REF = 0, IT_MP_LEAF = 1, IT_MONO = 2, IT_TOP = 3, IT_KINDS = 4 };
constexpr int MAX_GROUPS = 5;   // source-plane groups of a refined-target item (of the 10 canonical dz)
constexpr int NQUEUE = 8;       // persistent-launch queues: one per XCD of the MI355X
struct Item {
    int32_t kind;
    int32_t sub;   // target sub-grid (IT_TOP: index into the top items)
    int32_t a;     // IT_MP_REF: 2 pz in bits 0..3 for the parent plane pz along
                   // the sweep axis, bit 4: target plane 2 pz, bit 5: 2 pz + 1;
                   // IT_MP_LEAF: neighbour slots [a & 255, a >> 8)
    int32_t b;     // IT_MP_REF: plane group in bits 0..2, sweep in bits 3..4
                   // (0: planes along z, lanes on (x, y); 1: along y, lanes on
                   // (x, z); 2: along x, lanes on (z, y));
                   // IT_MP_LEAF: its Lf3 slot
};

// Upward-pass task: a refined parent sub-grid with what the kernels need of
// it and its 8 children, read as one record per block.
struct M2MTask {
    int32_t pidx;     // parent: index into the refined arrays
    int32_t ckinds;   // bit e: child e is refined
    int32_t cidx[8];  // child e: index into the leaf or the refined arrays
    double ph;        // parent cell edge
};

// Downward-pass task: child slot e of a refined parent sub-grid, with what
// the kernel needs of both, so that a block reads one record instead of the
// task, then the parent's and then the child's sub-grid entries in turn.
struct L2LTask {
    int32_t pidx;   // parent: index into the refined arrays
    int32_t pred;   // parent: its TopReduce index (top level under the all-pairs rule), else -1
    int32_t cidx;   // child: index into the leaf or the refined arrays
    int32_t flags;  // child kind in bit 0 (1 refined), child slot e = ex*4 + ey*2 + ez in
                    // bits 1..3, the child's number of Lf3 slots from bit 4
    int32_t slot3;  // leaf child: its first Lf3 slot
    int32_t psub;   // parent sub-grid id
    double ch;      // child cell edge
};

// Leaf targets with refined sources (class 4) are grouped by target parent
// cell: the rule selects a leaf target's partners by the offset D of the two
// parent cells alone (|D|^2 <= 8), so the 8 children of one parent cell share
// one partner set, the 8 children of each partner parent.  Per neighbour
// slot, the source parents within reach form a slab of 2 or 4 parent cells
// per axis (2 on the side facing the target, 4 along a shared face), at most
// C4_SLAB of them.
constexpr int C4_SLAB = 32;        // source parents of a face neighbour's slab (2 x 4 x 4)
constexpr int C4_MAX_TASKS = 3584; // (target parent, source parent) pairs over the 26 slots: 3560
constexpr int C4_MAX_GROUPS = 448; // (slot, target parent) groups: 6 x 32 + 12 x 16 + 8 x 4
// A leaf's refined neighbours are taken in slot order and cut into items of
// at least this many (target parent, source parent) steps (a face neighbour
// has 444, an edge 70, a corner 7), each with its own Lf3 slot.
constexpr int C4_ITEM_STEPS = 400;

// Canonical stencil tables (parity (0,0,0); other parities are mirror images:
// a cell of parity p uses offset (sx*dx, sy*dy, sz*dz) with s = 1 - 2p).
struct StencilTables {
    // refined-target multipole kernel: entries 16 dx (low signed 16 bits)
    // and 16 MP_PRS dy (high signed 16 bits), the byte offsets of the source
    // cell in the plane window, grouped by canonical dz (DZ0..DZ0+NDZ-1), far
    // entries first, then near ones
    int32_t mp_entry[743];
    int32_t mp_far_begin[NDZ], mp_far_count[NDZ];
    int32_t mp_near_begin[NDZ], mp_near_count[NDZ];
    // monopole kernel: the 100 columns (dx, dy) of the canonical stencil fall
    // into three classes by their dz range: [-4,5] (52 columns), [-2,3] (32),
    // [0,1] (16).  Columns are sorted by class; entry = (dx+8) | (dy+8) << 8.
    // The kernel values depend on |d|^2 only: mono_r[n] = {n^-1/2, n^-3/2}
    // (zero for n = 0, the self term), 1.2 KB, so they stay in the scalar
    // cache; dz |d|^-3 is formed in the kernel.
    int32_t mono_col[MONO_COLS];
    int32_t mono_class_begin[4];
    double mono_r[MONO_R2][2];
    float mono_rf[MONO_R2][2];
    // class 4 by target parent cell.  Neighbour slot o = (ox+1)*9 + (oy+1)*3 +
    // (oz+1): c4_slab[o] = nx | ny << 4 | nz << 8 | x0 << 12 | y0 << 14 |
    // z0 << 16, the slab's extent (2 or 4) and first parent coordinate (0 or
    // 2) per axis in the neighbour's 4^3 parent cells, slab parent index
    // (ix * ny + iy) * nz + iz.  Groups [c4_grp_begin[o], c4_grp_begin[o+1])
    // (largest first): c4_grp[g] = pt | first << 6 | count << 18, the target
    // parent pt = (px * 4 + py) * 4 + pz of the leaf and its partner parents
    // c4_task[first .. first + count) as slab parent indices.
    int32_t c4_slab[27];
    int32_t c4_grp_begin[28];
    int32_t c4_grp[C4_MAX_GROUPS];
    int32_t c4_task[C4_MAX_TASKS];  // 32-bit: the wave-uniform index is a scalar load
};

// Top-level (all pairs) tile: 64 target cells (plane zt of sub-grid target)
// against the source cells [src_begin, src_end) of the tree's top-level
// source list; partial sums go to slot part.
struct TopItem {
    int32_t target;
    int32_t zt;
    int32_t src_begin;
    int32_t src_end;
    int32_t part;      // partial slot
    int32_t src_list;  // offset of the tree's top-level source list
    int32_t pad0, pad1;
};

// Reduction of the partial slots (at most MAX_TOP_PARTS) of one top-level
// target sub-grid.
constexpr int MAX_TOP_PARTS = 8;
struct TopReduce {
    int32_t target;
    int32_t part_begin;
    int32_t n_part;
    int32_t pad;
};

}  // namespace fmmg
