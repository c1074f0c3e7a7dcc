// launch.h -- host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "fmmg_internal.h"

namespace fmmg {

// Device buffers and scalars shared by every launch of one solve.
struct Launch {
    const SubDev* subs;
    const int32_t* leaf_sub;
    double* mass;
    double* rec;
    double* Lr;
    double* Lf;
    double* part;
    double G;
    int corr;
    int mixed;
    hipStream_t st;
};

hipError_t upload_tables(const StencilTables* t, hipStream_t st);
void launch_p2m(const Launch& a, const double* rho, int n_leaf);
void launch_m2m(const Launch& a, const int32_t* list, int n);
void launch_mp(const Launch& a, const int32_t* list, int n, bool leaf_targets);
void launch_mono(const Launch& a, const int32_t* list, int n);
void launch_top(const Launch& a, const TopItem* items, int n_items, const int32_t* top_src,
                const TopReduce* reds, int n_red);
void launch_l2l(const Launch& a, const int32_t* list, int n, double* phi, double* g);
void launch_leaf_out(const Launch& a, const int32_t* list, int n, double* phi, double* g);
void launch_check_density(const double* rho, int64_t n, unsigned long long* bad, hipStream_t st);

}  // namespace fmmg
