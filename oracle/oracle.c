/*
 * oracle.c -- plain FP64 CPU reference for the octree FMM gravity solve.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Parity unpinned parts are listed
 * in the header comment of each function below; everything else is pinned by
 * the tests in tests/test_oracle_*.py.
 *
 * What the method computes (arXiv:1908.03121, Sec. 4.3):
 *   step 1 (upward):  leaf cells are point masses m = rho h^3 at their centres
 *                     (every cell's density determines its mass); refined
 *                     cells get mass, centre of mass and multipole moments
 *                     from their 8 children, bottom-up.
 *   step 2 (same level): each cell interacts with the same-level cells that
 *                     the opening criterion selects (1074-element stencil),
 *                     giving Taylor coefficients of the potential.  Four
 *                     interaction classes arise from AMR (refined/leaf target
 *                     x refined/leaf source).
 *   step 3 (downward): the parent's Taylor expansion is passed to its
 *                     children and accumulated, top-down.
 * plus the angular-momentum-conserving correction of the same-level step
 * (Sec. 4.2, Sec. 4.3: linear and angular momentum conserved to machine
 * precision).
 *
 * The expansions are the textbook Cartesian Taylor series of 1/r, written with
 * full index loops (3^k components for rank k), raw (not trace-free) moments
 * about the centre of mass, multipoles and Taylor coefficients of orders 0..3,
 * and the truncation n + m <= 3 (source order n, target order m).
 */
#include "oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define NS 8
#define NCELL 512
#define REACH 5

/* ------------------------------------------------------------------------ */
/* tree                                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    const int32_t* level;
    const int32_t* coord;
    double origin[3];
    double L0;
    int maxlev;
    int* refined;   /* [n] */
    int* leaf_of;   /* [n] leaf index or -1 */
    int* leaves;    /* [nleaf] descriptor index of each leaf */
    int nleaf;
    int64_t* hkey;
    int* hval;
    int hcap;
} tree_t;

static int64_t pack_key(int l, int x, int y, int z) {
    return ((int64_t)l << 57) | ((int64_t)x << 38) | ((int64_t)y << 19) | (int64_t)z;
}

static uint64_t mix(uint64_t k) {
    k ^= k >> 33; k *= 0xff51afd7ed558ccdULL; k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL; k ^= k >> 33;
    return k;
}

static int tree_find(const tree_t* t, int l, int x, int y, int z) {
    if (l < 0 || x < 0 || y < 0 || z < 0) return -1;
    if (x >= (1 << 19) || y >= (1 << 19) || z >= (1 << 19)) return -1;
    int64_t key = pack_key(l, x, y, z);
    uint64_t h = mix((uint64_t)key) & (uint64_t)(t->hcap - 1);
    for (;;) {
        if (t->hval[h] < 0) return -1;
        if (t->hkey[h] == key) return t->hval[h];
        h = (h + 1) & (uint64_t)(t->hcap - 1);
    }
}

static void tree_free(tree_t* t) {
    free(t->refined); free(t->leaf_of); free(t->leaves); free(t->hkey); free(t->hval);
    memset(t, 0, sizeof(*t));
}

/* returns 0, -1 (argument) or -2 (malformed tree) */
static int tree_build(tree_t* t, int n, const int32_t* level, const int32_t* coord,
                      const double* origin, double L0) {
    memset(t, 0, sizeof(*t));
    if (n <= 0 || !level || !coord) return -1;
    t->n = n; t->level = level; t->coord = coord;
    t->origin[0] = origin ? origin[0] : 0.0;
    t->origin[1] = origin ? origin[1] : 0.0;
    t->origin[2] = origin ? origin[2] : 0.0;
    t->L0 = L0;
    if (!(L0 > 0.0)) return -1;
    t->hcap = 1;
    while (t->hcap < 2 * n + 16) t->hcap <<= 1;
    t->hkey = (int64_t*)malloc(sizeof(int64_t) * t->hcap);
    t->hval = (int*)malloc(sizeof(int) * t->hcap);
    t->refined = (int*)calloc(n, sizeof(int));
    t->leaf_of = (int*)malloc(sizeof(int) * n);
    t->leaves = (int*)malloc(sizeof(int) * n);
    if (!t->hkey || !t->hval || !t->refined || !t->leaf_of || !t->leaves) { tree_free(t); return -3; }
    for (int i = 0; i < t->hcap; ++i) t->hval[i] = -1;
    t->maxlev = 0;
    for (int i = 0; i < n; ++i) {
        int l = level[i], x = coord[3 * i], y = coord[3 * i + 1], z = coord[3 * i + 2];
        if (l < 0 || l > 30 || x < 0 || y < 0 || z < 0 ||
            x >= (1 << 19) || y >= (1 << 19) || z >= (1 << 19)) { tree_free(t); return -2; }
        if (l > t->maxlev) t->maxlev = l;
        int64_t key = pack_key(l, x, y, z);
        uint64_t h = mix((uint64_t)key) & (uint64_t)(t->hcap - 1);
        while (t->hval[h] >= 0) {
            if (t->hkey[h] == key) { tree_free(t); return -2; } /* duplicate */
            h = (h + 1) & (uint64_t)(t->hcap - 1);
        }
        t->hkey[h] = key; t->hval[h] = i;
    }
    for (int i = 0; i < n; ++i) {
        int l = level[i], x = coord[3 * i], y = coord[3 * i + 1], z = coord[3 * i + 2];
        if (l > 0 && tree_find(t, l - 1, x / 2, y / 2, z / 2) < 0) { tree_free(t); return -2; }
        int nchild = 0;
        for (int e = 0; e < 8; ++e)
            if (tree_find(t, l + 1, 2 * x + (e >> 2), 2 * y + ((e >> 1) & 1), 2 * z + (e & 1)) >= 0) ++nchild;
        if (nchild != 0 && nchild != 8) { tree_free(t); return -2; }
        t->refined[i] = (nchild == 8);
    }
    t->nleaf = 0;
    for (int i = 0; i < n; ++i) {
        if (t->refined[i]) t->leaf_of[i] = -1;
        else { t->leaf_of[i] = t->nleaf; t->leaves[t->nleaf++] = i; }
    }
    return 0;
}

static double cell_size(const tree_t* t, int l) { return t->L0 / (NS * ldexp(1.0, l)); }

/* global integer cell coordinates of local cell q = (i*8+j)*8+k of sub-grid s */
static void cell_coords(const tree_t* t, int s, int q, int c[3]) {
    c[0] = NS * t->coord[3 * s] + (q >> 6);
    c[1] = NS * t->coord[3 * s + 1] + ((q >> 3) & 7);
    c[2] = NS * t->coord[3 * s + 2] + (q & 7);
}

static void cell_centre(const tree_t* t, int l, const int c[3], double X[3]) {
    double h = cell_size(t, l);
    for (int a = 0; a < 3; ++a) X[a] = t->origin[a] + (c[a] + 0.5) * h;
}

/* cell (level l, global coords c) -> sub-grid index and local cell index */
static int find_cell(const tree_t* t, int l, const int c[3], int* q) {
    if (c[0] < 0 || c[1] < 0 || c[2] < 0) return -1;
    int s = tree_find(t, l, c[0] / NS, c[1] / NS, c[2] / NS);
    if (s >= 0) *q = ((c[0] % NS) * NS + (c[1] % NS)) * NS + (c[2] % NS);
    return s;
}

static int check_rho(const tree_t* t, const double* rho) {
    if (!rho) return -1;
    long long nv = (long long)t->nleaf * NCELL;
    for (long long i = 0; i < nv; ++i)
        if (!(rho[i] >= 0.0) || !isfinite(rho[i])) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* expansions                                                                */
/* ------------------------------------------------------------------------ */
static double kd(int i, int j) { return i == j ? 1.0 : 0.0; }

/* D^(k) = k-th derivative tensor of 1/|R| (textbook):
 *   D0 = 1/r,  D1_i = -R_i/r^3,  D2_ij = 3 R_i R_j/r^5 - d_ij/r^3,
 *   D3_ijk = -15 R_i R_j R_k/r^7 + 3 (R_i d_jk + R_j d_ik + R_k d_ij)/r^5,
 *   D4_ijkl = 105 R_i R_j R_k R_l/r^9
 *             - 15 (R_i R_j d_kl + R_i R_k d_jl + R_i R_l d_jk
 *                   + R_j R_k d_il + R_j R_l d_ik + R_k R_l d_ij)/r^7
 *             + 3 (d_ij d_kl + d_ik d_jl + d_il d_jk)/r^5.
 * order selects how many are filled (1..4); unused pointers may be NULL. */
static void dtensors_order(const double R[3], int order, double* D0, double* D1, double* D2,
                           double* D3, double* D4) {
    double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    double r = sqrt(r2);
    double i1 = 1.0 / r, i2 = i1 * i1;
    double i3 = i1 * i2, i5 = i3 * i2, i7 = i5 * i2, i9 = i7 * i2;
    if (D0) *D0 = i1;
    if (D1) for (int i = 0; i < 3; ++i) D1[i] = -R[i] * i3;
    if (order >= 2 && D2)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                D2[3 * i + j] = 3.0 * R[i] * R[j] * i5 - kd(i, j) * i3;
    if (order >= 3 && D3)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k)
                    D3[9 * i + 3 * j + k] = -15.0 * R[i] * R[j] * R[k] * i7
                        + 3.0 * (R[i] * kd(j, k) + R[j] * kd(i, k) + R[k] * kd(i, j)) * i5;
    if (order >= 4 && D4)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l)
                        D4[27 * i + 9 * j + 3 * k + l] =
                            105.0 * R[i] * R[j] * R[k] * R[l] * i9
                            - 15.0 * (R[i] * R[j] * kd(k, l) + R[i] * R[k] * kd(j, l)
                                      + R[i] * R[l] * kd(j, k) + R[j] * R[k] * kd(i, l)
                                      + R[j] * R[l] * kd(i, k) + R[k] * R[l] * kd(i, j)) * i7
                            + 3.0 * (kd(i, j) * kd(k, l) + kd(i, k) * kd(j, l)
                                     + kd(i, l) * kd(j, k)) * i5;
}

void oracle_dtensors(const double R[3], double* D0, double* D1, double* D2, double* D3, double* D4) {
    dtensors_order(R, 4, D0, D1, D2, D3, D4);
}

static int floordiv2(int a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

/* Interaction rule (opening criterion, Sec. 4.3).  For an ordered pair of
 * distinct same-level cells with offset d = cb - ca and parent offset
 * D = floor(cb/2) - floor(ca/2):
 *   parents-near  <=>  |D|^2 <= 8,     far  <=>  |d|^2 >= 9,
 *   evaluated at this level  <=>  (all_pairs or parents-near)
 *                                 and (far or A is a leaf or B is a leaf).
 * Refined-refined near pairs are deferred to the children.  Per parent parity
 * this selects 743 partners (651 of them far); the union over the 8 parities
 * is the 1074-element stencil of Sec. 4.3 (1074 x 512 = 549,888 interactions
 * per sub-grid). */
int oracle_pair_rule(int all_pairs, const int ca[3], const int cb[3], int a_leaf, int b_leaf) {
    int d2 = 0, D2 = 0;
    for (int a = 0; a < 3; ++a) {
        int d = cb[a] - ca[a];
        int D = floordiv2(cb[a]) - floordiv2(ca[a]);
        d2 += d * d;
        D2 += D * D;
    }
    if (d2 == 0) return 0;
    if (!all_pairs && D2 > 8) return 0;
    return (d2 >= 9) || a_leaf || b_leaf;
}

/* Source B (moments about its COM xb) seen from target A (COM xa), R = xa - xb.
 * The potential of B near xa, Taylor-expanded about xa:
 *   L^(m) = -G sum_n (-1)^n/n! M_B^(n) . D^(n+m)(R),  truncated at n + m <= 3,
 * with M^(1) = 0 about the COM:
 *   L0   = -G [ mb D0 + 1/2 M2b:D2 - 1/6 M3b:D3 ]
 *   L1_i = -G [ mb D1_i + 1/2 M2b_jk D3_ijk ]
 *   L2   = -G mb D2,      L3 = -G mb D3.
 * Angular-momentum correction (Sec. 4.2): the order-4 forces that the
 * truncation drops from the octupole-monopole energy terms, applied as a
 * uniform acceleration of A,
 *   dg_i = -(G/6) D4_ijkl ( M3b_jkl - (mb/ma) M3a_jkl ),
 * so that the pair forces are equal and opposite and their torques cancel.
 * M2b/M3b NULL means a point mass; M3a NULL means the target is a point mass.
 * full_target = 0 skips L2/L3 (a leaf target's expansion is only evaluated at
 * its own centre). */
static void m2l_pair(double G, int correction, int full_target,
                     double ma, const double xa[3], const double* M3a,
                     double mb, const double xb[3], const double* M2b, const double* M3b,
                     double* L0, double* L1, double* L2, double* L3, double* dg) {
    double R[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
    int need_d4 = correction && (M3a || M3b) && ma > 0.0;
    int need_d3 = full_target || M2b || M3b;
    int order = need_d4 ? 4 : (need_d3 ? 3 : 1);
    double D0, D1[3], D2[9], D3[27], D4[81];
    dtensors_order(R, order, &D0, D1, D2, D3, D4);

    double s0 = mb * D0;
    if (M2b) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) s0 += 0.5 * M2b[3 * i + j] * D2[3 * i + j];
    }
    if (M3b) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k)
                    s0 -= (1.0 / 6.0) * M3b[9 * i + 3 * j + k] * D3[9 * i + 3 * j + k];
    }
    *L0 += -G * s0;
    for (int i = 0; i < 3; ++i) {
        double s1 = mb * D1[i];
        if (M2b)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) s1 += 0.5 * M2b[3 * j + k] * D3[9 * i + 3 * j + k];
        L1[i] += -G * s1;
    }
    if (full_target) {
        for (int a = 0; a < 9; ++a) L2[a] += -G * mb * D2[a];
        for (int a = 0; a < 27; ++a) L3[a] += -G * mb * D3[a];
    }
    if (need_d4) {
        double ratio = mb / ma;
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) {
                        double q = (M3b ? M3b[9 * j + 3 * k + l] : 0.0)
                                 - ratio * (M3a ? M3a[9 * j + 3 * k + l] : 0.0);
                        s += D4[27 * i + 9 * j + 3 * k + l] * q;
                    }
            dg[i] += -(G / 6.0) * s;
        }
    }
}

void oracle_m2l_pair(double G, int correction, double ma, const double xa[3], const double* M3a,
                     double mb, const double xb[3], const double* M2b, const double* M3b,
                     double* L0, double* L1, double* L2, double* L3, double* dg) {
    m2l_pair(G, correction, 1, ma, xa, M3a, mb, xb, M2b, M3b, L0, L1, L2, L3, dg);
}

/* Step 3: the parent's cubic Taylor polynomial re-expanded about a point
 * displaced by r (exact for a cubic):
 *   o0   = L0 + L1_i r_i + 1/2 L2_ij r_i r_j + 1/6 L3_ijk r_i r_j r_k
 *   o1_i = L1_i + L2_ij r_j + 1/2 L3_ijk r_j r_k
 *   o2_ij = L2_ij + L3_ijk r_k,      o3 = L3. */
void oracle_l2l(const double* L0, const double* L1, const double* L2, const double* L3,
                const double r[3], double* o0, double* o1, double* o2, double* o3) {
    double s = *L0;
    for (int i = 0; i < 3; ++i) s += L1[i] * r[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s += 0.5 * L2[3 * i + j] * r[i] * r[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) s += (1.0 / 6.0) * L3[9 * i + 3 * j + k] * r[i] * r[j] * r[k];
    double t1[3], t2[9], t3[27];
    for (int i = 0; i < 3; ++i) {
        double v = L1[i];
        for (int j = 0; j < 3; ++j) v += L2[3 * i + j] * r[j];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) v += 0.5 * L3[9 * i + 3 * j + k] * r[j] * r[k];
        t1[i] = v;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double v = L2[3 * i + j];
            for (int k = 0; k < 3; ++k) v += L3[9 * i + 3 * j + k] * r[k];
            t2[3 * i + j] = v;
        }
    for (int a = 0; a < 27; ++a) t3[a] = L3[a];
    *o0 = s;
    memcpy(o1, t1, sizeof(t1));
    memcpy(o2, t2, sizeof(t2));
    memcpy(o3, t3, sizeof(t3));
}

/* ------------------------------------------------------------------------ */
/* step 1: upward pass                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    double* m;   /* [n*512]     */
    double* X;   /* [n*512*3]   */
    double* M2;  /* [n*512*9]   */
    double* M3;  /* [n*512*27]  */
} moments_t;

static void moments_free(moments_t* mo) { free(mo->m); free(mo->X); free(mo->M2); free(mo->M3); }

static int moments_alloc(moments_t* mo, int n) {
    size_t nc = (size_t)n * NCELL;
    mo->m = (double*)calloc(nc, sizeof(double));
    mo->X = (double*)calloc(nc * 3, sizeof(double));
    mo->M2 = (double*)calloc(nc * 9, sizeof(double));
    mo->M3 = (double*)calloc(nc * 27, sizeof(double));
    if (!mo->m || !mo->X || !mo->M2 || !mo->M3) { moments_free(mo); return -3; }
    return 0;
}

/* Leaf cell: point mass m = rho h^3 at the cell centre (M2 = M3 = 0).
 * Refined cell with children c (r_c = X_c - X):
 *   m = sum m_c,   X = sum m_c X_c / m   (geometric centre if m = 0),
 *   M2_ij  = sum ( M2c_ij + m_c r_i r_j ),
 *   M3_ijk = sum ( M3c_ijk + M2c_ij r_k + M2c_ik r_j + M2c_jk r_i + m_c r_i r_j r_k ). */
static void upward(const tree_t* t, const double* rho, moments_t* mo) {
    for (int li = 0; li < t->nleaf; ++li) {
        int s = t->leaves[li];
        int l = t->level[s];
        double h = cell_size(t, l), vol = h * h * h;
        for (int q = 0; q < NCELL; ++q) {
            size_t cq = (size_t)s * NCELL + q;
            int c[3];
            cell_coords(t, s, q, c);
            mo->m[cq] = rho[(size_t)li * NCELL + q] * vol;
            cell_centre(t, l, c, &mo->X[3 * cq]);
        }
    }
    for (int l = t->maxlev - 1; l >= 0; --l) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int s = 0; s < t->n; ++s) {
            if (t->level[s] != l || !t->refined[s]) continue;
            for (int q = 0; q < NCELL; ++q) {
                size_t cq = (size_t)s * NCELL + q;
                int c[3];
                cell_coords(t, s, q, c);
                size_t kids[8];
                double m = 0.0, X[3] = {0, 0, 0};
                for (int e = 0; e < 8; ++e) {
                    int cc[3] = {2 * c[0] + (e >> 2), 2 * c[1] + ((e >> 1) & 1), 2 * c[2] + (e & 1)};
                    int qc = 0;
                    int sc = find_cell(t, l + 1, cc, &qc);
                    kids[e] = (size_t)sc * NCELL + qc;
                    m += mo->m[kids[e]];
                }
                if (m > 0.0) {
                    for (int e = 0; e < 8; ++e)
                        for (int a = 0; a < 3; ++a) X[a] += mo->m[kids[e]] * mo->X[3 * kids[e] + a];
                    for (int a = 0; a < 3; ++a) X[a] /= m;
                } else {
                    cell_centre(t, l, c, X);
                }
                double M2[9] = {0}, M3[27] = {0};
                for (int e = 0; e < 8; ++e) {
                    size_t k = kids[e];
                    double mc = mo->m[k];
                    const double* M2c = &mo->M2[9 * k];
                    const double* M3c = &mo->M3[27 * k];
                    double r[3];
                    for (int a = 0; a < 3; ++a) r[a] = mo->X[3 * k + a] - X[a];
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) M2[3 * i + j] += M2c[3 * i + j] + mc * r[i] * r[j];
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j)
                            for (int kk = 0; kk < 3; ++kk)
                                M3[9 * i + 3 * j + kk] += M3c[9 * i + 3 * j + kk]
                                    + M2c[3 * i + j] * r[kk] + M2c[3 * i + kk] * r[j]
                                    + M2c[3 * j + kk] * r[i] + mc * r[i] * r[j] * r[kk];
                }
                mo->m[cq] = m;
                memcpy(&mo->X[3 * cq], X, sizeof(X));
                memcpy(&mo->M2[9 * cq], M2, sizeof(M2));
                memcpy(&mo->M3[27 * cq], M3, sizeof(M3));
            }
        }
    }
}

int oracle_upward(int n, const int32_t* level, const int32_t* coord, const double origin[3],
                  double L0, const double* rho, double* m, double* X, double* M2, double* M3) {
    tree_t t;
    int rc = tree_build(&t, n, level, coord, origin, L0);
    if (rc) return rc;
    if (check_rho(&t, rho)) { tree_free(&t); return -1; }
    moments_t mo;
    if (moments_alloc(&mo, n)) { tree_free(&t); return -3; }
    upward(&t, rho, &mo);
    size_t nc = (size_t)n * NCELL;
    if (m) memcpy(m, mo.m, nc * sizeof(double));
    if (X) memcpy(X, mo.X, nc * 3 * sizeof(double));
    if (M2) memcpy(M2, mo.M2, nc * 9 * sizeof(double));
    if (M3) memcpy(M3, mo.M3, nc * 27 * sizeof(double));
    moments_free(&mo);
    tree_free(&t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* step 2: same-level interactions of one target cell                        */
/* ------------------------------------------------------------------------ */
typedef struct { double L0, L1[3], L2[9], L3[27], dg[3]; } local_t;

typedef struct { int64_t cls[4], top, lev; } cnt_t;

static void pair_into(const tree_t* t, const moments_t* mo, double G, int corr,
                      int sa, size_t ca_idx, int sb, size_t cb_idx, local_t* L) {
    int a_leaf = !t->refined[sa], b_leaf = !t->refined[sb];
    m2l_pair(G, corr, !a_leaf,
             mo->m[ca_idx], &mo->X[3 * ca_idx], a_leaf ? NULL : &mo->M3[27 * ca_idx],
             mo->m[cb_idx], &mo->X[3 * cb_idx],
             b_leaf ? NULL : &mo->M2[9 * cb_idx], b_leaf ? NULL : &mo->M3[27 * cb_idx],
             &L->L0, L->L1, L->L2, L->L3, L->dg);
}

static void count_pair(cnt_t* k, int all_pairs_here, int a_leaf, int b_leaf) {
    k->lev++;
    if (all_pairs_here) { k->top++; return; }
    int cls = a_leaf ? (b_leaf ? 3 : 4) : (b_leaf ? 1 : 2);
    k->cls[cls - 1]++;
}

/* Own (same-level) expansion of cell q of sub-grid sa. */
static void cell_own(const tree_t* t, const moments_t* mo, double G, int top_all, int corr,
                     int sa, int q, local_t* L, cnt_t* k) {
    memset(L, 0, sizeof(*L));
    int l = t->level[sa];
    int ca[3];
    cell_coords(t, sa, q, ca);
    size_t ia = (size_t)sa * NCELL + q;
    int a_leaf = !t->refined[sa];
    if (top_all && l == 0) {
        /* top level: every pair of the level is a candidate */
        for (int sb = 0; sb < t->n; ++sb) {
            if (t->level[sb] != 0) continue;
            int b_leaf = !t->refined[sb];
            for (int qb = 0; qb < NCELL; ++qb) {
                int cb[3];
                cell_coords(t, sb, qb, cb);
                if (!oracle_pair_rule(1, ca, cb, a_leaf, b_leaf)) continue;
                pair_into(t, mo, G, corr, sa, ia, sb, (size_t)sb * NCELL + qb, L);
                if (k) count_pair(k, 1, a_leaf, b_leaf);
            }
        }
        return;
    }
    for (int dx = -REACH; dx <= REACH; ++dx)
        for (int dy = -REACH; dy <= REACH; ++dy)
            for (int dz = -REACH; dz <= REACH; ++dz) {
                int cb[3] = {ca[0] + dx, ca[1] + dy, ca[2] + dz};
                int qb = 0;
                int sb = find_cell(t, l, cb, &qb);
                if (sb < 0) continue;
                int b_leaf = !t->refined[sb];
                if (!oracle_pair_rule(0, ca, cb, a_leaf, b_leaf)) continue;
                pair_into(t, mo, G, corr, sa, ia, sb, (size_t)sb * NCELL + qb, L);
                if (k) count_pair(k, 0, a_leaf, b_leaf);
            }
}

/* ------------------------------------------------------------------------ */
/* full solve                                                                */
/* ------------------------------------------------------------------------ */
static void add_stats(oracle_stats* st, const cnt_t* k, int l) {
    for (int c = 0; c < 4; ++c) st->cls[c] += k->cls[c];
    st->top += k->top;
    if (l < 16) st->per_level[l] += k->lev;
}

int oracle_solve(int n, const int32_t* level, const int32_t* coord, const double origin[3],
                 double L0, const double* rho, double G, int top_all_pairs, int correction,
                 double* phi, double* g, oracle_stats* stats) {
    tree_t t;
    int rc = tree_build(&t, n, level, coord, origin, L0);
    if (rc) return rc;
    if (check_rho(&t, rho) || !phi || !g) { tree_free(&t); return -1; }
    moments_t mo;
    if (moments_alloc(&mo, n)) { tree_free(&t); return -3; }
    upward(&t, rho, &mo);

    size_t nc = (size_t)n * NCELL;
    local_t* L = (local_t*)calloc(nc, sizeof(local_t));
    if (!L) { moments_free(&mo); tree_free(&t); return -3; }
    if (stats) memset(stats, 0, sizeof(*stats));

    /* step 2: every cell of every sub-grid, own interactions only */
    #pragma omp parallel
    {
        oracle_stats loc;
        memset(&loc, 0, sizeof(loc));
        #pragma omp for schedule(dynamic, 64)
        for (long long idx = 0; idx < (long long)nc; ++idx) {
            int s = (int)(idx / NCELL), q = (int)(idx % NCELL);
            cnt_t k;
            memset(&k, 0, sizeof(k));
            cell_own(&t, &mo, G, top_all_pairs, correction, s, q, &L[idx], &k);
            add_stats(&loc, &k, t.level[s]);
        }
        if (stats) {
            #pragma omp critical
            {
                for (int c = 0; c < 4; ++c) stats->cls[c] += loc.cls[c];
                stats->top += loc.top;
                for (int l = 0; l < 16; ++l) stats->per_level[l] += loc.per_level[l];
            }
        }
    }

    /* step 3: top-down, child += parent's expansion re-expanded at the child COM */
    for (int l = 1; l <= t.maxlev; ++l) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int s = 0; s < n; ++s) {
            if (t.level[s] != l) continue;
            for (int q = 0; q < NCELL; ++q) {
                int c[3], cp[3] = {0, 0, 0}, qp = 0;
                cell_coords(&t, s, q, c);
                for (int a = 0; a < 3; ++a) cp[a] = c[a] / 2;
                int sp = find_cell(&t, l - 1, cp, &qp);
                size_t ic = (size_t)s * NCELL + q, ip = (size_t)sp * NCELL + qp;
                double r[3];
                for (int a = 0; a < 3; ++a) r[a] = mo.X[3 * ic + a] - mo.X[3 * ip + a];
                local_t sh;
                oracle_l2l(&L[ip].L0, L[ip].L1, L[ip].L2, L[ip].L3, r, &sh.L0, sh.L1, sh.L2, sh.L3);
                L[ic].L0 += sh.L0;
                for (int a = 0; a < 3; ++a) L[ic].L1[a] += sh.L1[a];
                for (int a = 0; a < 9; ++a) L[ic].L2[a] += sh.L2[a];
                for (int a = 0; a < 27; ++a) L[ic].L3[a] += sh.L3[a];
                for (int a = 0; a < 3; ++a) L[ic].dg[a] += L[ip].dg[a];
            }
        }
    }

    /* leaf output: phi = L0, g = -L1 + dg at the cell centre */
    for (int li = 0; li < t.nleaf; ++li) {
        int s = t.leaves[li];
        for (int q = 0; q < NCELL; ++q) {
            size_t ic = (size_t)s * NCELL + q;
            phi[(size_t)li * NCELL + q] = L[ic].L0;
            for (int a = 0; a < 3; ++a)
                g[((size_t)li * 3 + a) * NCELL + q] = -L[ic].L1[a] + L[ic].dg[a];
        }
    }
    free(L);
    moments_free(&mo);
    tree_free(&t);
    return 0;
}

int oracle_solve_sampled(int n, const int32_t* level, const int32_t* coord,
                         const double origin[3], double L0, const double* rho, double G,
                         int top_all_pairs, int correction, int n_sample,
                         const int32_t* sample_leaf, const int32_t* sample_cell,
                         double* phi, double* g) {
    tree_t t;
    int rc = tree_build(&t, n, level, coord, origin, L0);
    if (rc) return rc;
    if (check_rho(&t, rho) || n_sample < 0 || (n_sample > 0 && (!sample_leaf || !sample_cell || !phi || !g))) {
        tree_free(&t);
        return -1;
    }
    for (int i = 0; i < n_sample; ++i)
        if (sample_leaf[i] < 0 || sample_leaf[i] >= t.nleaf || sample_cell[i] < 0 || sample_cell[i] >= NCELL) {
            tree_free(&t);
            return -1;
        }
    moments_t mo;
    if (moments_alloc(&mo, n)) { tree_free(&t); return -3; }
    upward(&t, rho, &mo);

    #pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_sample; ++i) {
        int s = t.leaves[sample_leaf[i]];
        int lk = t.level[s];
        int c[3];
        cell_coords(&t, s, sample_cell[i], c);
        local_t acc;
        memset(&acc, 0, sizeof(acc));
        size_t iprev = 0;
        for (int l = 0; l <= lk; ++l) {
            int ca[3] = {c[0] >> (lk - l), c[1] >> (lk - l), c[2] >> (lk - l)};
            int qa = 0;
            int sa = find_cell(&t, l, ca, &qa);
            size_t ia = (size_t)sa * NCELL + qa;
            local_t own;
            cell_own(&t, &mo, G, top_all_pairs, correction, sa, qa, &own, NULL);
            if (l > 0) {
                double r[3];
                for (int a = 0; a < 3; ++a) r[a] = mo.X[3 * ia + a] - mo.X[3 * iprev + a];
                local_t sh;
                oracle_l2l(&acc.L0, acc.L1, acc.L2, acc.L3, r, &sh.L0, sh.L1, sh.L2, sh.L3);
                acc.L0 = sh.L0;
                memcpy(acc.L1, sh.L1, sizeof(sh.L1));
                memcpy(acc.L2, sh.L2, sizeof(sh.L2));
                memcpy(acc.L3, sh.L3, sizeof(sh.L3));
            }
            acc.L0 += own.L0;
            for (int a = 0; a < 3; ++a) acc.L1[a] += own.L1[a];
            for (int a = 0; a < 9; ++a) acc.L2[a] += own.L2[a];
            for (int a = 0; a < 27; ++a) acc.L3[a] += own.L3[a];
            for (int a = 0; a < 3; ++a) acc.dg[a] += own.dg[a];
            iprev = ia;
        }
        phi[i] = acc.L0;
        for (int a = 0; a < 3; ++a) g[3 * i + a] = -acc.L1[a] + acc.dg[a];
    }
    moments_free(&mo);
    tree_free(&t);
    return 0;
}

/* OpenMP team size of the parallel loops (the solve loops over target
 * cells); n < 1 restores the runtime default.  Used to report the thread
 * count a timing ran with and to time the oracle on one core. */
int oracle_set_threads(int n) {
#ifdef _OPENMP
    static int dflt = 0;
    if (!dflt) dflt = omp_get_max_threads();
    omp_set_num_threads(n >= 1 ? n : dflt);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* plain definitions                                                         */
/* ------------------------------------------------------------------------ */
/* phi_a = -G sum_{b != a} m_b / |x_a - x_b|,
 * g_a   = -G sum_{b != a} m_b (x_a - x_b) / |x_a - x_b|^3,  leaf cells as point masses. */

/* leaf cells as point masses: centres x[3N] and masses m[N], N = 512 * leaves,
 * in leaf order and the caller's cell order */
static int point_masses(const tree_t* t, const double* rho, double** xo, double** mo) {
    size_t N = (size_t)t->nleaf * NCELL;
    double* x = (double*)malloc(sizeof(double) * 3 * N);
    double* m = (double*)malloc(sizeof(double) * N);
    if (!x || !m) { free(x); free(m); return -3; }
    for (int li = 0; li < t->nleaf; ++li) {
        int s = t->leaves[li];
        int l = t->level[s];
        double h = cell_size(t, l);
        for (int q = 0; q < NCELL; ++q) {
            int c[3];
            cell_coords(t, s, q, c);
            size_t i = (size_t)li * NCELL + q;
            cell_centre(t, l, c, &x[3 * i]);
            m[i] = rho[i] * h * h * h;
        }
    }
    *xo = x;
    *mo = m;
    return 0;
}

/* Newton's sum at point a over every other point */
static void newton_at(size_t N, const double* x, const double* m, size_t a, double G,
                      double* phi, double g[3]) {
    double p = 0.0, ga[3] = {0, 0, 0};
    for (size_t b = 0; b < N; ++b) {
        if (b == a) continue;
        double R[3] = {x[3 * a] - x[3 * b], x[3 * a + 1] - x[3 * b + 1], x[3 * a + 2] - x[3 * b + 2]};
        double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
        double r = sqrt(r2);
        p += m[b] / r;
        double w = m[b] / (r2 * r);
        for (int k = 0; k < 3; ++k) ga[k] += w * R[k];
    }
    *phi = -G * p;
    for (int k = 0; k < 3; ++k) g[k] = -G * ga[k];
}

int oracle_direct_sum(int n, const int32_t* level, const int32_t* coord, const double origin[3],
                      double L0, const double* rho, double G, double* phi, double* g) {
    tree_t t;
    int rc = tree_build(&t, n, level, coord, origin, L0);
    if (rc) return rc;
    if (check_rho(&t, rho) || !phi || !g) { tree_free(&t); return -1; }
    size_t N = (size_t)t.nleaf * NCELL;
    double *x, *m;
    if (point_masses(&t, rho, &x, &m)) { tree_free(&t); return -3; }
    #pragma omp parallel for schedule(dynamic, 64)
    for (long long a = 0; a < (long long)N; ++a) {
        double ga[3];
        size_t li = (size_t)a / NCELL, q = (size_t)a % NCELL;
        newton_at(N, x, m, (size_t)a, G, &phi[a], ga);
        for (int k = 0; k < 3; ++k) g[(li * 3 + k) * NCELL + q] = ga[k];
    }
    free(x);
    free(m);
    tree_free(&t);
    return 0;
}

int oracle_direct_sum_sampled(int n, const int32_t* level, const int32_t* coord,
                              const double origin[3], double L0, const double* rho, double G,
                              int n_sample, const int32_t* sample_leaf,
                              const int32_t* sample_cell, double* phi, double* g) {
    tree_t t;
    int rc = tree_build(&t, n, level, coord, origin, L0);
    if (rc) return rc;
    if (check_rho(&t, rho) || n_sample < 0 || (n_sample > 0 && (!sample_leaf || !sample_cell || !phi || !g))) {
        tree_free(&t);
        return -1;
    }
    for (int i = 0; i < n_sample; ++i) {
        if (sample_leaf[i] < 0 || sample_leaf[i] >= t.nleaf || sample_cell[i] < 0 || sample_cell[i] >= NCELL) {
            tree_free(&t);
            return -1;
        }
    }
    size_t N = (size_t)t.nleaf * NCELL;
    double *x, *m;
    if (point_masses(&t, rho, &x, &m)) { tree_free(&t); return -3; }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_sample; ++i) {
        size_t a = (size_t)sample_leaf[i] * NCELL + (size_t)sample_cell[i];
        newton_at(N, x, m, a, G, &phi[i], &g[3 * (size_t)i]);
    }
    free(x);
    free(m);
    tree_free(&t);
    return 0;
}

/* collect leaf-cell ids below (or equal to) cell c of level l */
static int leaf_cells_below(const tree_t* t, int l, const int c[3], int32_t* out, int cap) {
    int q = 0;
    int s = find_cell(t, l, c, &q);
    if (s < 0) return 0;
    if (!t->refined[s]) {
        if (cap < 1) return 0;
        out[0] = t->leaf_of[s] * NCELL + q;
        return 1;
    }
    int k = 0;
    for (int e = 0; e < 8; ++e) {
        int cc[3] = {2 * c[0] + (e >> 2), 2 * c[1] + ((e >> 1) & 1), 2 * c[2] + (e & 1)};
        k += leaf_cells_below(t, l + 1, cc, out + k, cap - k);
    }
    return k;
}

int oracle_pair_coverage(int n, const int32_t* level, const int32_t* coord, int top_all_pairs,
                         uint8_t* cover) {
    tree_t t;
    double origin[3] = {0, 0, 0};
    int rc = tree_build(&t, n, level, coord, origin, 1.0);
    if (rc) return rc;
    if (!cover) { tree_free(&t); return -1; }
    size_t N = (size_t)t.nleaf * NCELL;
    memset(cover, 0, N * N);
    int cap = (int)N;
    int32_t* la = (int32_t*)malloc(sizeof(int32_t) * cap);
    int32_t* lb = (int32_t*)malloc(sizeof(int32_t) * cap);
    if (!la || !lb) { free(la); free(lb); tree_free(&t); return -3; }
    for (int sa = 0; sa < n; ++sa) {
        int l = t.level[sa];
        int a_leaf = !t.refined[sa];
        for (int q = 0; q < NCELL; ++q) {
            int ca[3];
            cell_coords(&t, sa, q, ca);
            int na = leaf_cells_below(&t, l, ca, la, cap);
            if (top_all_pairs && l == 0) {
                for (int sb = 0; sb < n; ++sb) {
                    if (t.level[sb] != 0) continue;
                    for (int qb = 0; qb < NCELL; ++qb) {
                        int cb[3];
                        cell_coords(&t, sb, qb, cb);
                        if (!oracle_pair_rule(1, ca, cb, a_leaf, !t.refined[sb])) continue;
                        int nb = leaf_cells_below(&t, l, cb, lb, cap);
                        for (int i = 0; i < na; ++i)
                            for (int j = 0; j < nb; ++j) {
                                uint8_t* p = &cover[(size_t)la[i] * N + lb[j]];
                                if (*p < 255) ++*p;
                            }
                    }
                }
                continue;
            }
            for (int dx = -REACH; dx <= REACH; ++dx)
                for (int dy = -REACH; dy <= REACH; ++dy)
                    for (int dz = -REACH; dz <= REACH; ++dz) {
                        int cb[3] = {ca[0] + dx, ca[1] + dy, ca[2] + dz};
                        int qb = 0;
                        int sb = find_cell(&t, l, cb, &qb);
                        if (sb < 0) continue;
                        if (!oracle_pair_rule(0, ca, cb, a_leaf, !t.refined[sb])) continue;
                        int nb = leaf_cells_below(&t, l, cb, lb, cap);
                        for (int i = 0; i < na; ++i)
                            for (int j = 0; j < nb; ++j) {
                                uint8_t* p = &cover[(size_t)la[i] * N + lb[j]];
                                if (*p < 255) ++*p;
                            }
                    }
        }
    }
    free(la);
    free(lb);
    tree_free(&t);
    return 0;
}
