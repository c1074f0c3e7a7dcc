/*
 * oracle.h -- plain, slow, FP64 CPU reference for the octree fast-multipole
 * gravity solve over 8x8x8 sub-grids (Octo-Tiger's FMM, arXiv:1908.03121,
 * Sec. 4.3 "The FMM hotspot").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no source with the GPU path.
 *
 * Tree convention (same logical input as the C-ABI): n sub-grids, each with a
 * level l >= 0 and non-negative integer coordinates s.  A sub-grid covers
 * origin + L0 * 2^-l * [s, s+1) and holds 8^3 cells of size h = L0/(8*2^l).
 * A sub-grid is refined iff its 8 children are listed.  Sub-grids without a
 * parent must be at level 0.  Leaf order = order of leaves in the descriptor.
 * Densities are [leaf][i][j][k] with k (z) fastest.
 *
 * Return codes: 0 ok, -1 bad argument, -2 malformed tree, -3 out of memory.
 */
#ifndef FMM_ORACLE_H
#define FMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* statistics: ordered pair counts */
typedef struct {
    int64_t cls[4];        /* 1: refined<-leaf, 2: refined<-refined, 3: leaf<-leaf, 4: leaf<-refined */
    int64_t top;           /* pairs evaluated at the top level under the all-pairs rule  */
    int64_t per_level[16]; /* all evaluated pairs, by level                              */
} oracle_stats;

/* --- building blocks (exposed so that tests can pin them) -------------- */

/* Derivatives of 1/|R|: D0, D1[3], D2[3][3], D3[3][3][3], D4[3][3][3][3]. */
void oracle_dtensors(const double R[3], double* D0, double* D1, double* D2,
                     double* D3, double* D4);

/* Interaction rule: returns 1 iff the ordered pair of same-level cells with
 * integer coordinates ca, cb is evaluated at that level.  all_pairs = 1 at a
 * top level under the all-pairs rule. */
int oracle_pair_rule(int all_pairs, const int ca[3], const int cb[3], int a_leaf, int b_leaf);

/* Contribution of source B (mass mb, COM xb, raw moments M2b[9], M3b[27]) to
 * the expansion of target A (mass ma, COM xa, raw octupole M3a[27]).
 * Adds into L0[1], L1[3], L2[9], L3[27], dg[3]. */
void oracle_m2l_pair(double G, int correction,
                     double ma, const double xa[3], const double* M3a,
                     double mb, const double xb[3], const double* M2b, const double* M3b,
                     double* L0, double* L1, double* L2, double* L3, double* dg);

/* Re-expansion of a cubic Taylor polynomial L (L0, L1[3], L2[9], L3[27])
 * about a point displaced by r; writes the shifted coefficients. */
void oracle_l2l(const double* L0, const double* L1, const double* L2, const double* L3,
                const double r[3], double* o0, double* o1, double* o2, double* o3);

/* Upward pass: per cell of every sub-grid (descriptor order, 512 cells in
 * [i][j][k] order) the mass, centre of mass X[3], raw quadrupole M2[9] and
 * raw octupole M3[27] about X.  Any output pointer may be NULL. */
int oracle_upward(int n, const int32_t* level, const int32_t* coord, const double origin[3],
                  double L0, const double* rho, double* m, double* X, double* M2, double* M3);

/* --- full solves --------------------------------------------------------- */

/* FMM solve: phi[leaf][512], g[leaf][3][512] (cell order [i][j][k]).
 * top_all_pairs: 1 = the top level evaluates all its pairs (complete solve);
 *                0 = the top level uses the same parent-near stencil as the
 *                    others (kernel test of a single sub-grid neighbourhood).
 * stats may be NULL. */
int oracle_solve(int n, const int32_t* level, const int32_t* coord, const double origin[3],
                 double L0, const double* rho, double G, int top_all_pairs, int correction,
                 double* phi, double* g, oracle_stats* stats);

/* Same as oracle_solve, but only for the n_sample listed leaf cells
 * (leaf index, cell index 0..511); phi[n_sample], g[n_sample][3]. */
int oracle_solve_sampled(int n, const int32_t* level, const int32_t* coord,
                         const double origin[3], double L0, const double* rho, double G,
                         int top_all_pairs, int correction, int n_sample,
                         const int32_t* sample_leaf, const int32_t* sample_cell,
                         double* phi, double* g);

/* OpenMP threads of the solve loops: oracle_set_threads(n) sets the team
 * size (n < 1: the runtime default) and returns it; oracle_max_threads()
 * returns the current one. */
int oracle_set_threads(int n);
int oracle_max_threads(void);

/* O(N^2) direct sum over leaf cells as point masses (self excluded). */
int oracle_direct_sum(int n, const int32_t* level, const int32_t* coord, const double origin[3],
                      double L0, const double* rho, double G, double* phi, double* g);

/* The same plain sum at sampled leaf cells only: phi[i], g[3 i .. 3 i + 2] for
 * leaf sample_leaf[i] (leaf order), cell sample_cell[i] (caller's cell order). */
int oracle_direct_sum_sampled(int n, const int32_t* level, const int32_t* coord,
                              const double origin[3], double L0, const double* rho, double G,
                              int n_sample, const int32_t* sample_leaf,
                              const int32_t* sample_cell, double* phi, double* g);

/* Exact-once check: cover[a * nleafcells + b] counts how many evaluated pairs
 * (A, B) have leaf cell a below (or equal to) A and b below (or equal to) B.
 * nleafcells = 512 * number of leaves.  uint8 saturates at 255. */
int oracle_pair_coverage(int n, const int32_t* level, const int32_t* coord, int top_all_pairs,
                         uint8_t* cover);

#ifdef __cplusplus
}
#endif
#endif
