// launch.h -- host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <string>

#include "fmmg_internal.h"

namespace fmmg {

// Device buffers and scalars of one solve, passed by value to the kernels.
struct Ctx {
    const SubDev* subs;
    const int32_t* leaf_sub;
    double* mass;
    double* rec;            // [n_ref][512][16] records, cell-major
    double* com;            // [n_ref][3][512] their centre-of-mass offsets (downward pass)
    int64_t rec_zero;       // cell index of the all-zero record after the last refined cell
    double* Lp;             // [MAX_GROUPS][n_ref][19][512] own terms per plane group
    double* Lr;             // [n_ref][19][512] totals
    double* Lf;             // [n_leaf][4][512]
    double* Lf3;            // [n_slot3][4][512]
    double* part;           // top-level partial sums
    const TopItem* top_items;
    const int32_t* top_src;
    const TopReduce* top_reds;  // partial slots of each top-level target
    const double* rho;          // caller's densities (I/O cell order)
    unsigned long long* rho_bad;       // smallest flat index of a negative or non-finite
                                       // density read by the upward pass, ~0 if none
    unsigned long long* rho_bad_host;  // device address of the host word it is copied to
    int flag_out;                      // 1 in the solve's last launch: block 0 copies a
                                       // set rho_bad to the host word and clears it
    int64_t part_stride;    // elements between plane groups of Lp
    double G;
    int corr;
    int prec;               // PR_F64, PR_MIX or PR_F32
    int ngroups;
    hipStream_t st;
};

// parent expansions of one downward level: inherited part + own plane-group
// sums; top-level partial slots; own plane-group sums only
enum { PARENT_TOTAL = 0, PARENT_TOP_PARTS = 1, PARENT_OWN_PARTS = 2 };

hipError_t upload_tables(const StencilTables* t, hipStream_t st);
void launch_p2m_top(const Ctx& a, const int32_t* list, int n);
void launch_m2m(const Ctx& a, const M2MTask* list, int n);
// parents whose 8 children are all leaves: one block per parent
void launch_m2m_leafpar(const Ctx& a, const M2MTask* list, int n);
void launch_class(const Ctx& a, int kind, const Item* items, int n);
// The item queues of a persistent launch: queue q is items [begin[q],
// begin[q + 1]) (offsets into the launch's list; begin[0] = 0).
struct Queues {
    int32_t begin[NQUEUE + 1];
};
// ctr: NQUEUE + 1 ints, zero before the first launch and re-armed by each launch
void launch_persist(const Ctx& a, const Item* items, const Queues& qs, int grid, int* ctr);
int persist_blocks_per_cu(int prec);
void launch_l2l(const Ctx& a, const L2LTask* tasks, int n, int parent_mode, double* phi, double* g);
void launch_leaf_out(const Ctx& a, const int32_t* list, int n, double* phi, double* g);
void launch_check_density(const double* rho, int64_t n, unsigned long long* bad, hipStream_t st);
void launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st);

// Density check without allocation (noalloc.hip): partial results in a
// static device array of NOALLOC_SLOTS words, one per chunk of NOALLOC_CHUNK
// densities, so n <= NOALLOC_SLOTS * NOALLOC_CHUNK.  On failure *err names
// the failing step.
constexpr int NOALLOC_SLOTS = 65536;
constexpr int NOALLOC_CHUNK = 4096;
hipError_t noalloc_check_density(const double* rho, int64_t n, int64_t* out, hipStream_t st,
                                 std::string* err);

}  // namespace fmmg
