// kernels.hip -- gfx950 kernels of the octree FMM gravity solve
// (arXiv:1908.03121, Sec. 4.3: upward pass, same-level stencil interactions
// with order-3 multipoles and the angular-momentum correction, downward pass).
//
// Thread mapping of the same-level kernels: a wavefront holds one plane of
// 8x8 target cells (multipole items: a z- or y-plane, lane = u*8 + v in the
// plane's frame; monopole items: a lane owns a z-column of 8 targets; top
// level: z-plane, lane = y*8 + x).  Cells of different parity use mirror
// images of one canonical stencil, so every lane of a wave walks the same
// entry list (uniform control flow, scalar table loads) with its own signs.
// Sources are staged in LDS one 18 x 18 plane window (multipole items) or
// the 18^3 box (monopole items) at a time.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fmmg_internal.h"
#include "launch.h"
#include <type_traits>

namespace fmmg {

// two signed 16-bit lanes of a 32-bit register (packed dot products)
typedef short short2_t __attribute__((ext_vector_type(2)));

__constant__ StencilTables c_tab;

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_full(double x) {
    // hardware estimate (~2^-23 relative) refined by one third-order
    // Newton-Householder step: y (1 + e/2 + 3e^2/8), e = 1 - x y^2
    double y = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-x * y, y, 1.0);
    double t = __builtin_fma(0.375, e, 0.5);
    return __builtin_fma(y * e, t, y);
}
__device__ __forceinline__ float rsqrt_full(float x) { return __builtin_amdgcn_rsqf(x); }

// threadIdx.x made opaque to the optimiser: index arithmetic derived from it
// then stays inside the work item instead of being hoisted out of the
// persistent loop, where it would stay live across every item
__device__ __forceinline__ int item_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Density check of the upward pass: a negative or non-finite density sets
// cx.rho_bad to the smallest such flat index (rho[flat]); lanes_contiguous:
// the wave's lanes read consecutive flat indices, so its lowest bad lane holds
// its smallest one and a single atomic suffices.
__device__ __forceinline__ void check_rho(const Ctx& cx, double v, unsigned long long flat,
                                          bool lanes_contiguous) {
    const bool bad = !(v >= 0.0) || !(v < __builtin_inf());
    const unsigned long long mask = __ballot(bad);
    if (!mask) return;
    if (lanes_contiguous ? int(__lane_id()) == __ffsll((long long)mask) - 1 : bad)
        atomicMin(cx.rho_bad, flat);
}

// The solve's last launch: block 0 hands a recorded bad density to the host
// word (system scope) and re-arms the device flag for the next solve.
__device__ __forceinline__ void rho_flag_out(const Ctx& cx) {
    if (!cx.flag_out || blockIdx.x != 0 || threadIdx.x != 0) return;
    const unsigned long long v = __hip_atomic_load(cx.rho_bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v != ~0ull) {
        __hip_atomic_store(cx.rho_bad_host, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(cx.rho_bad, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// internal cell index (x fastest) -> I/O index (z fastest)
__device__ __forceinline__ int io_index(int q) {
    int x = q & 7, y = (q >> 3) & 7, z = q >> 6;
    return (x * 8 + y) * 8 + z;
}

// The 16 record values of refined cell `cell` (refined index * 512 + cell
// index): 8 16-byte loads from one address.
__device__ __forceinline__ void load_rec(const double* __restrict__ rec, size_t cell, double (&v)[NREC]) {
    const double2* p = reinterpret_cast<const double2*>(rec + cell * NREC);
#pragma unroll
    for (int j = 0; j < NREC / 2; ++j) {
        const double2 t = p[j];
        v[2 * j] = t.x;
        v[2 * j + 1] = t.y;
    }
}

// Scale of record component k as the pair terms take a staged source:
// quadrupole times -3, octupole divided by 2, mass and position unchanged.
__device__ __forceinline__ constexpr double stage_scale(int k) {
    return k >= R_O ? 0.5 : (k >= R_Q ? -3.0 : 1.0);
}

// A double moved across lanes by a DPP control (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(b)), CTRL, 0xF, 0xF, false));
    const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), CTRL, 0xF, 0xF, false));
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

// Sum over the 8 lanes 8k .. 8k + 7 of a full wave, in every one of them:
// lane ^ 1 and lane ^ 2 within a quad (quad_perm), then the lane mirrored
// within the 8 (row_half_mirror), which lies in the other quad.  DPP moves,
// no LDS; a fixed order, so the result is reproducible.
__device__ __forceinline__ double sum8_lanes(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    return v;
}

// Index into a launch's list for this block: the blocks of a launch are dealt
// to the NQUEUE XCDs in turn, so XCD x (blocks b with b % NQUEUE = x) gets a
// contiguous run of the list (neighbouring sub-grids: shared data in its L2).
__device__ __forceinline__ int xcd_run_index() {
    const int nb = int(gridDim.x), b = int(blockIdx.x);
    const int per = nb / NQUEUE, rem = nb % NQUEUE, x = b % NQUEUE;
    return x * per + (x < rem ? x : rem) + b / NQUEUE;
}

// Accumulators of one target cell.  Refined targets carry all 19 components,
// leaf targets only L0, L1 and the correction sum S.  L2 and L3 are summed
// in the forms the pair terms produce most cheaply (see pair_terms): l2 sums
// mb e2 times (XX - ZZ, YY - ZZ, 2XY, 2XZ, 2YZ), l3 the components xzz,
// xxy, xxz, xyy, 2xyz, yzz, yyz of mb D3 divided by -3.  Since D2 and D3
// are trace-free, out() recovers L2 xx, yy and L3 xxx, yyy from them.
template <typename P>
struct Acc {
    P l0, l1[3], l2[5], l3[7], s[3];
    __device__ __forceinline__ void zero() {
        l0 = 0;
        for (int i = 0; i < 3; ++i) l1[i] = 0, s[i] = 0;
        for (int i = 0; i < 5; ++i) l2[i] = 0;
        for (int i = 0; i < 7; ++i) l3[i] = 0;
    }
    template <typename Q>
    __device__ __forceinline__ void add(const Acc<Q>& o, bool full, bool with_s = true) {
        l0 += P(o.l0);
        for (int i = 0; i < 3; ++i) l1[i] += P(o.l1[i]);
        if (with_s)
            for (int i = 0; i < 3; ++i) s[i] += P(o.s[i]);
        if (full) {
            for (int i = 0; i < 5; ++i) l2[i] += P(o.l2[i]);
            for (int i = 0; i < 7; ++i) l3[i] += P(o.l3[i]);
        }
    }
    // the 19 output components: with P = l2[0], Q = l2[1] (mb e2 summed
    // over XX - ZZ and YY - ZZ) and mb d1 = mb e2 r^2, L2 xx = mb e2 (r^2 -
    // 3 XX) = Q - 2P and L2 yy = P - 2Q; L3 xxx = -(xyy + xzz) and
    // yyy = -(xxy + yzz); the rest undo the factors -1/3 and 2
    __device__ __forceinline__ void out(double v[NLOC]) const {
        v[T_L0] = double(l0);
        for (int i = 0; i < 3; ++i) v[T_L1 + i] = double(l1[i]);
        const double P2 = double(l2[0]), Q2 = double(l2[1]);
        v[T_L2 + 0] = fma(-2.0, P2, Q2);
        v[T_L2 + 1] = fma(-2.0, Q2, P2);
        for (int i = 2; i < 5; ++i) v[T_L2 + i] = -1.5 * double(l2[i]);
        v[T_L3 + 0] = 3.0 * (double(l3[3]) + double(l3[0]));
        v[T_L3 + 5] = 3.0 * (double(l3[1]) + double(l3[5]));
        for (int i : {1, 2, 3, 6}) v[T_L3 + i] = -3.0 * double(l3[i]);
        v[T_L3 + 4] = -1.5 * double(l3[4]);
        for (int i = 0; i < 3; ++i) v[T_S + i] = double(s[i]);
    }
};

__device__ __forceinline__ double fmaP(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaP(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// o:RR for a trace-free rank-3 tensor o (xxx xxy xxz xyy xyz yyy yyz, with
// o_xzz = -o_xxx - o_xyy and o_yzz = -o_xxy - o_yyy passed in oxzz, oyzz),
// written with XmZ = XX - ZZ, YmZ = YY - ZZ and the doubled mixed products.
template <typename P>
__device__ __forceinline__ void oct_rr(const P o[7], P oxzz, P oyzz, P XmZ, P YmZ, P XY2, P XZ2,
                                       P YZ2, P w[3]) {
    w[0] = fmaP(o[0], XmZ, fmaP(o[3], YmZ, fmaP(o[1], XY2, fmaP(o[2], XZ2, o[4] * YZ2))));
    w[1] = fmaP(o[1], XmZ, fmaP(o[5], YmZ, fmaP(o[3], XY2, fmaP(o[4], XZ2, o[6] * YZ2))));
    w[2] = fmaP(o[2], XmZ, fmaP(o[6], YmZ, fmaP(o[4], XY2, fmaP(oxzz, XZ2, oyzz * YZ2))));
}

// One ordered pair: source B (mass mb, trace-free quadrupole q, octupole o)
// seen from target A at separation R = X_A - X_B.  Taylor coefficients of the
// potential truncated at (source order + target order) <= 3, without the
// factor -G (applied once per target):
//   L0 += mb D0 + 1/2 q:D2 - 1/6 o:D3,  L1 += mb D1 + 1/2 q:D3,
//   L2 += mb D2,  L3 += mb D3,
//   dg += -G/6 D4:(o_B - (mb/mA) o_A)   (angular-momentum correction)
// With trace-free tensors and D^(n) = sum of R^k delta^j terms these reduce to
//   q:D2 = d2 RqR,  (q:D3)_i = d3 R_i RqR + 2 d2 (qR)_i,  o:D3 = d3 o:RRR,
//   (D4:Q)_i = d4 R_i Q:RRR + 3 d3 (Q:RR)_i,
// where d0 = 1/r, d1 = -1/r^3, d2 = 3/r^5, d3 = -15/r^7, d4 = 105/r^9.
// The constants are folded into the staged data and the output scales: the
// kernel forms e2 = d2/-3 = -1/r^5, e3 = d3/-3 and g4 = -7/3 e3/r^2 = -d4/9,
// the source quadrupole arrives times -3 (q holds -3 q_B) and its octupole
// divided by 2 (o holds o_B/2), the target's octupole divided by 2 mA (oa
// holds o_A/(2 mA), zero for mA = 0, so that its weight in the correction is
// -mb).  Then the L0, L1 sums are the plain ones, the L2 (without its trace
// term mb d1) and L3 sums carry the factor -1/3, the mixed ones (L2 xy xz
// yz, L3 xyz, formed from the doubled products) -2/3 (Acc::out), and S sums
//   e3 (Q:RR)_i + g4 R_i Q:RRR = -(D4:Q)_i / 18,  Q = o_B/2 - mb o_A/(2 mA),
// so that dg = 3G S.
// FULL: refined target (L2, L3 and its own octupole oa enter; oa[7], oa[8]
// hold its dependent components xzz, yzz).
template <bool FULL, typename P>
__device__ __forceinline__ void pair_terms(P X, P Y, P Z, P mb, const P q[5], const P o[7],
                                           const P oa[9], bool corr, Acc<P>& a) {
    const P XX = X * X, YY = Y * Y, ZZ = Z * Z;
    const P r2 = XX + YY + ZZ;
    const P d0 = rsqrt_full(r2);
    const P ir2 = d0 * d0;
    const P d1 = -d0 * ir2;
    const P e2 = ir2 * d1;            // d2 / -3
    const P e3 = P(-5) * ir2 * e2;    // d3 / -3
    const P X2 = X + X, Y2 = Y + Y;
    const P XY2 = X2 * Y, XZ2 = X2 * Z, YZ2 = Y2 * Z;  // doubled mixed products
    const P XmZ = XX - ZZ, YmZ = YY - ZZ;
    const P qzz = -q[0] - q[1];
    const P ux = fmaP(q[0], X, fmaP(q[2], Y, q[3] * Z));
    const P uy = fmaP(q[2], X, fmaP(q[1], Y, q[4] * Z));
    const P uz = fmaP(q[3], X, fmaP(q[4], Y, qzz * Z));
    const P hRqR = P(0.5) * fmaP(X, ux, fmaP(Y, uy, Z * uz));
    P wb[3];
    oct_rr(o, -o[0] - o[3], -o[1] - o[5], XmZ, YmZ, XY2, XZ2, YZ2, wb);
    const P BRRR = fmaP(X, wb[0], fmaP(Y, wb[1], Z * wb[2]));  // o_B:RRR / 2
    a.l0 = fmaP(mb, d0, fmaP(e2, hRqR, fmaP(e3, BRRR, a.l0)));
    const P c1 = fmaP(mb, d1, e3 * hRqR);
    a.l1[0] = fmaP(c1, X, fmaP(e2, ux, a.l1[0]));
    a.l1[1] = fmaP(c1, Y, fmaP(e2, uy, a.l1[1]));
    a.l1[2] = fmaP(c1, Z, fmaP(e2, uz, a.l1[2]));
    if (FULL) {
        // -1/3 of mb D2 and mb D3 in the forms of Acc
        const P md2 = mb * e2, md3 = mb * e3;
        a.l2[0] = fmaP(md2, XmZ, a.l2[0]);
        a.l2[1] = fmaP(md2, YmZ, a.l2[1]);
        a.l2[2] = fmaP(md2, XY2, a.l2[2]);
        a.l2[3] = fmaP(md2, XZ2, a.l2[3]);
        a.l2[4] = fmaP(md2, YZ2, a.l2[4]);
        const P bx = fmaP(md3, XX, md2), cy = fmaP(md3, YY, md2), cz = fmaP(md3, ZZ, md2);
        a.l3[0] = fmaP(X, cz, a.l3[0]);
        a.l3[1] = fmaP(Y, bx, a.l3[1]);
        a.l3[2] = fmaP(Z, bx, a.l3[2]);
        a.l3[3] = fmaP(X, cy, a.l3[3]);
        a.l3[4] = fmaP(md3 * XY2, Z, a.l3[4]);
        a.l3[5] = fmaP(Y, cz, a.l3[5]);
        a.l3[6] = fmaP(Z, cy, a.l3[6]);
    }
    // correction terms: always accumulated (no branch in the pair body); the
    // output scale of S is zero when the correction is off
    {
        const P g4 = P(-7.0 / 3.0) * ir2 * e3;  // -d4 / 9
        P Qx = wb[0], Qy = wb[1], Qz = wb[2];
        if (FULL) {
            P wa[3];
            oct_rr(oa, oa[7], oa[8], XmZ, YmZ, XY2, XZ2, YZ2, wa);
            Qx = fmaP(-mb, wa[0], Qx);
            Qy = fmaP(-mb, wa[1], Qy);
            Qz = fmaP(-mb, wa[2], Qz);
        }
        const P QRRR = fmaP(X, Qx, fmaP(Y, Qy, Z * Qz));
        const P t4 = g4 * QRRR;
        a.s[0] = fmaP(t4, X, fmaP(e3, Qx, a.s[0]));
        a.s[1] = fmaP(t4, Y, fmaP(e3, Qy, a.s[1]));
        a.s[2] = fmaP(t4, Z, fmaP(e3, Qz, a.s[2]));
    }
}

// The same pair in the mixed form: the separation, the derivative scalars
// and the correction term S (with the source and target octupoles) in FP64,
// S added straight into the FP64 sums s; the Taylor coefficients L0..L3 in
// FP32 from the rounded separation, scalars and moments, into the FP32
// partial sums a.
template <bool FULL>
__device__ __forceinline__ void pair_terms_mix(double X, double Y, double Z, double mb, const double q[5],
                                               const double o[7], const double oa[9], Acc<float>& a,
                                               double (&s)[3]) {
    const double XX = X * X, YY = Y * Y, ZZ = Z * Z;
    const double r2 = XX + YY + ZZ;
    const double d0 = rsqrt_full(r2);
    const double ir2 = d0 * d0;
    const double d1 = -d0 * ir2;
    const double e2 = ir2 * d1;                  // as in pair_terms
    const double e3 = -5.0 * ir2 * e2;
    const double g4 = (-7.0 / 3.0) * ir2 * e3;
    const double X2 = X + X, Y2 = Y + Y;
    const double XY2 = X2 * Y, XZ2 = X2 * Z, YZ2 = Y2 * Z;
    const double XmZ = XX - ZZ, YmZ = YY - ZZ;
    double wb[3];
    oct_rr(o, -o[0] - o[3], -o[1] - o[5], XmZ, YmZ, XY2, XZ2, YZ2, wb);
    const double BRRR = fmaP(X, wb[0], fmaP(Y, wb[1], Z * wb[2]));  // o_B:RRR / 2
    {
        double Qx = wb[0], Qy = wb[1], Qz = wb[2];
        if (FULL) {
            double wa[3];
            oct_rr(oa, oa[7], oa[8], XmZ, YmZ, XY2, XZ2, YZ2, wa);
            Qx = fmaP(-mb, wa[0], Qx);
            Qy = fmaP(-mb, wa[1], Qy);
            Qz = fmaP(-mb, wa[2], Qz);
        }
        const double QRRR = fmaP(X, Qx, fmaP(Y, Qy, Z * Qz));
        const double t4 = g4 * QRRR;
        s[0] = fmaP(t4, X, fmaP(e3, Qx, s[0]));
        s[1] = fmaP(t4, Y, fmaP(e3, Qy, s[1]));
        s[2] = fmaP(t4, Z, fmaP(e3, Qz, s[2]));
    }
    const float x = float(X), y = float(Y), z = float(Z), m = float(mb);
    const float f0 = float(d0), f1 = float(d1), f2 = float(e2), f3 = float(e3);
    const float q0 = float(q[0]), q1 = float(q[1]), q2 = float(q[2]), q3 = float(q[3]), q4 = float(q[4]);
    const float qzz = -q0 - q1;
    const float ux = fmaP(q0, x, fmaP(q2, y, q3 * z));
    const float uy = fmaP(q2, x, fmaP(q1, y, q4 * z));
    const float uz = fmaP(q3, x, fmaP(q4, y, qzz * z));
    const float hRqR = 0.5f * fmaP(x, ux, fmaP(y, uy, z * uz));
    a.l0 = fmaP(m, f0, fmaP(f2, hRqR, fmaP(f3, float(BRRR), a.l0)));
    const float c1 = fmaP(m, f1, f3 * hRqR);
    a.l1[0] = fmaP(c1, x, fmaP(f2, ux, a.l1[0]));
    a.l1[1] = fmaP(c1, y, fmaP(f2, uy, a.l1[1]));
    a.l1[2] = fmaP(c1, z, fmaP(f2, uz, a.l1[2]));
    if (FULL) {
        const float md2 = m * f2, md3 = m * f3;
        const float xx = x * x, yy = y * y, zz = z * z;
        a.l2[0] = fmaP(md2, xx - zz, a.l2[0]);
        a.l2[1] = fmaP(md2, yy - zz, a.l2[1]);
        const float x2 = x + x;
        a.l2[2] = fmaP(md2, x2 * y, a.l2[2]);
        a.l2[3] = fmaP(md2, x2 * z, a.l2[3]);
        a.l2[4] = fmaP(md2, (y + y) * z, a.l2[4]);
        const float bx = fmaP(md3, xx, md2), cy = fmaP(md3, yy, md2), cz = fmaP(md3, zz, md2);
        a.l3[0] = fmaP(x, cz, a.l3[0]);
        a.l3[1] = fmaP(y, bx, a.l3[1]);
        a.l3[2] = fmaP(z, bx, a.l3[2]);
        a.l3[3] = fmaP(x, cy, a.l3[3]);
        a.l3[4] = fmaP(md3 * x2 * y, z, a.l3[4]);
        a.l3[5] = fmaP(y, cz, a.l3[5]);
        a.l3[6] = fmaP(z, cy, a.l3[6]);
    }
}

// One pair in the arithmetic of precision form PR (sources staged as P =
// double for PR_F64 and PR_MIX, float for PR_F32): FP64 terms go to acc, the
// FP32 forms' Taylor terms to the partial sums part (PR_F64: part is acc).
template <bool FULL, int PR, typename P, typename PA>
__device__ __forceinline__ void pair_any(P X, P Y, P Z, const P* src, const P oa[9], Acc<double>& acc,
                                         Acc<PA>& part) {
    if constexpr (PR == PR_MIX)
        pair_terms_mix<FULL>(X, Y, Z, src[R_M], &src[R_Q], &src[R_O], oa, part, acc.s);
    else
        pair_terms<FULL, P>(X, Y, Z, src[R_M], &src[R_Q], &src[R_O], oa, true, part);
}

// ---------------------------------------------------------------------------
// step 1: leaf masses and the upward pass
// ---------------------------------------------------------------------------
// Leaves without a parent: m = rho h^3 in the internal cell order.
// grid: one block of 512 per listed leaf.
__global__ __launch_bounds__(512) void k_p2m_top(Ctx cx, const int32_t* __restrict__ list) {
    const SubDev& S = cx.subs[list[blockIdx.x]];
    const int q = threadIdx.x;
    const double h = S.h;
    const size_t io = size_t(S.idx) * NCELL + io_index(q);
    const double v = cx.rho[io];
    check_rho(cx, v, io, false);
    cx.mass[size_t(S.idx) * NCELL + q] = v * (h * h * h);
}

// The summed contributions v (m, S1, S2 in xx yy zz xy xz yz, S3 in xxx xxy
// xxz xyy xyz xzz yyy yyz yzz zzz, all about the parent cell centre) moved to
// the COM offset d = S1/m and stored trace-free as the record at out (16
// contiguous values), the COM offset also at com (stride NCELL per axis).
__device__ __forceinline__ void m2m_store(double (&v)[20], double* out, double* com) {
    const double m = v[0];
    double ox = 0, oy = 0, oz = 0;
    if (m > 0) {
        const double im = 1.0 / m;
        ox = v[1] * im;
        oy = v[2] * im;
        oz = v[3] * im;
    }
    double* p2 = v + 4;    // xx yy zz xy xz yz
    double* p3 = v + 10;   // xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
    // shift to the COM: M3 = S3 - sym(S2 d) + 2 m d d d (S2 before its shift)
    const double m2 = 2 * m;
    p3[0] += -3 * p2[0] * ox + m2 * ox * ox * ox;
    p3[1] += -(p2[0] * oy + 2 * p2[3] * ox) + m2 * ox * ox * oy;
    p3[2] += -(p2[0] * oz + 2 * p2[4] * ox) + m2 * ox * ox * oz;
    p3[3] += -(2 * p2[3] * oy + p2[1] * ox) + m2 * ox * oy * oy;
    p3[4] += -(p2[3] * oz + p2[4] * oy + p2[5] * ox) + m2 * ox * oy * oz;
    p3[5] += -(2 * p2[4] * oz + p2[2] * ox) + m2 * ox * oz * oz;
    p3[6] += -3 * p2[1] * oy + m2 * oy * oy * oy;
    p3[7] += -(p2[1] * oz + 2 * p2[5] * oy) + m2 * oy * oy * oz;
    p3[8] += -(2 * p2[5] * oz + p2[2] * oy) + m2 * oy * oz * oz;
    p3[9] += -3 * p2[2] * oz + m2 * oz * oz * oz;
    p2[0] -= m * ox * ox;
    p2[1] -= m * oy * oy;
    p2[2] -= m * oz * oz;
    p2[3] -= m * ox * oy;
    p2[4] -= m * ox * oz;
    p2[5] -= m * oy * oz;
    const double tr = (p2[0] + p2[1] + p2[2]) * (1.0 / 3.0);
    const double tx = p3[0] + p3[3] + p3[5];
    const double ty = p3[1] + p3[6] + p3[8];
    const double tz = p3[2] + p3[7] + p3[9];
    double w[NREC];
    w[R_M] = m;
    w[R_DX] = ox;
    w[R_DY] = oy;
    w[R_DZ] = oz;
    w[R_Q + 0] = p2[0] - tr;
    w[R_Q + 1] = p2[1] - tr;
    w[R_Q + 2] = p2[3];
    w[R_Q + 3] = p2[4];
    w[R_Q + 4] = p2[5];
    w[R_O + 0] = p3[0] - 0.6 * tx;
    w[R_O + 1] = p3[1] - 0.2 * ty;
    w[R_O + 2] = p3[2] - 0.2 * tz;
    w[R_O + 3] = p3[3] - 0.2 * tx;
    w[R_O + 4] = p3[4];
    w[R_O + 5] = p3[6] - 0.6 * ty;
    w[R_O + 6] = p3[7] - 0.2 * tz;
    double2* o2 = reinterpret_cast<double2*>(out);
#pragma unroll
    for (int j = 0; j < NREC / 2; ++j) o2[j] = make_double2(w[2 * j], w[2 * j + 1]);
    com[0] = ox;
    com[NCELL] = oy;
    com[2 * NCELL] = oz;
}

// Sums of the 8 point masses mc[i][j][k] at offsets s a (s in {-1, 1}^3,
// component s_x = 2i - 1 etc., a = h/2) from their parent cell centre, as
// the contributions v of the upward step: with M, S_i = sum s_i m,
// S_ij = sum s_i s_j m (i != j), S_xyz, the first moments are a S_i, the
// second a^2 M (diagonal) and a^2 S_ij, the third a^3 S_i (xxx, xyy, xzz ...)
// and a^3 S_xyz (xyz).
__device__ __forceinline__ void leaf_octet(const double (&mc)[2][2][2], double hc, double (&v)[20]) {
    double p[2][2], d[2][2];  // along z: sum and difference
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            p[i][j] = mc[i][j][1] + mc[i][j][0];
            d[i][j] = mc[i][j][1] - mc[i][j][0];
        }
    double pp[2], pd[2], dp[2], dd[2];  // then along y
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        pp[i] = p[i][1] + p[i][0];
        pd[i] = p[i][1] - p[i][0];
        dp[i] = d[i][1] + d[i][0];
        dd[i] = d[i][1] - d[i][0];
    }
    const double M = pp[1] + pp[0], Sx = pp[1] - pp[0], Sy = pd[1] + pd[0], Sxy = pd[1] - pd[0];
    const double Sz = dp[1] + dp[0], Sxz = dp[1] - dp[0], Syz = dd[1] + dd[0], Sxyz = dd[1] - dd[0];
    const double a1 = 0.5 * hc, a2 = a1 * a1, a3 = a2 * a1;
    v[0] = M;
    v[1] = a1 * Sx;
    v[2] = a1 * Sy;
    v[3] = a1 * Sz;
    v[4] = v[5] = v[6] = a2 * M;
    v[7] = a2 * Sxy;
    v[8] = a2 * Sxz;
    v[9] = a2 * Syz;
    v[10] = v[13] = v[15] = a3 * Sx;  // xxx, xyy, xzz
    v[11] = v[16] = v[18] = a3 * Sy;  // xxy, yyy, yzz
    v[12] = v[17] = v[19] = a3 * Sz;  // xxz, yyz, zzz
    v[14] = a3 * Sxyz;
}

// One octant of a refined sub-grid's cells from the 512 cells of one child
// sub-grid (leaf: point masses m = rho h^3 at the cell centres, also stored
// for the same-level step; refined: their records).  The contribution of a
// child cell about the parent cell centre c (r0 = child COM - c) is
//   m, m r0, q + m r0 r0, o + sym(q r0) + m r0 r0 r0.
// Refined children: each thread takes one child cell and the 8 siblings of a
// parent cell are summed (lane shuffles across x and y parity, LDS across z
// parity).  Leaf children: one thread per parent cell sums its 8 point masses
// in closed form.  The sums are then moved to the parent COM
// offset d = S1/m (binomial shift with M1 = m d):
//   M2 = S2 - m d d,   M3 = S3 - sym(S2 d) + 2 m d d d,
// and stored trace-free (children's trace parts only feed trace parts).
// grid: (refined sub-grids of the level) x 8 octants, 512 threads.
__global__ __launch_bounds__(512) void k_m2m(Ctx cx, const M2MTask* __restrict__ list) {
    __shared__ double red[4][16][20];
    __shared__ double rin[NCELL + NCELL / 8];  // leaf densities, I/O order, one pad per z-row
    const M2MTask& tk = list[blockIdx.x >> 3];
    const int e = blockIdx.x & 7;
    const int cidx = tk.cidx[e], pidx = tk.pidx;
    const bool cref = ((tk.ckinds >> e) & 1) != 0;
    const int q = threadIdx.x;
    if (!cref) {
        const double v = cx.rho[size_t(cidx) * NCELL + q];  // coalesced
        check_rho(cx, v, size_t(cidx) * NCELL + q, true);
        rin[q + (q >> 3)] = v;
        __syncthreads();
    }
    const int x = q & 7, y = (q >> 3) & 7, z = q >> 6;
    const double hc = 0.5 * tk.ph;
    double v[20];
    if (!cref) {
        // leaf child: point masses at the cell centres, r0 = s a with sign
        // vector s in {-1, 1}^3 and a = h/2, so the sums need only the 8
        // signed mass sums M, S_i = sum s_i m, S_ij = sum s_i s_j m (i != j),
        // S_xyz; one thread per parent cell (the even-even-even child)
        const double h3 = hc * hc * hc;
        {
            const int io = io_index(q);
            cx.mass[size_t(cidx) * NCELL + q] = rin[io + (io >> 3)] * h3;
        }
        if ((x | y | z) & 1) return;
        double mc[2][2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int io = ((x + i) * NS + (y + j)) * NS + (z + k);
                    mc[i][j][k] = rin[io + (io >> 3)] * h3;
                }
        leaf_octet(mc, hc, v);
    } else {
        double r[NREC];
        load_rec(cx.rec, size_t(cidx) * NCELL + q, r);
        const double w = r[R_M];
        const double dx = r[R_DX], dy = r[R_DY], dz = r[R_DZ];
        const double qxx = r[R_Q + 0], qyy = r[R_Q + 1], qxy = r[R_Q + 2];
        const double qxz = r[R_Q + 3], qyz = r[R_Q + 4];
        const double o0 = r[R_O + 0], o1 = r[R_O + 1], o2 = r[R_O + 2];
        const double o3 = r[R_O + 3], o4 = r[R_O + 4], o5 = r[R_O + 5];
        const double o6 = r[R_O + 6];
        const double rx = ((x & 1) - 0.5) * hc + dx, ry = ((y & 1) - 0.5) * hc + dy, rz = ((z & 1) - 0.5) * hc + dz;
        const double qzz = -qxx - qyy;
        v[0] = w;
        v[1] = w * rx;
        v[2] = w * ry;
        v[3] = w * rz;
        v[4] = qxx + w * rx * rx;
        v[5] = qyy + w * ry * ry;
        v[6] = qzz + w * rz * rz;
        v[7] = qxy + w * rx * ry;
        v[8] = qxz + w * rx * rz;
        v[9] = qyz + w * ry * rz;
        v[10] = o0 + 3 * qxx * rx + w * rx * rx * rx;
        v[11] = o1 + qxx * ry + 2 * qxy * rx + w * rx * rx * ry;
        v[12] = o2 + qxx * rz + 2 * qxz * rx + w * rx * rx * rz;
        v[13] = o3 + 2 * qxy * ry + qyy * rx + w * rx * ry * ry;
        v[14] = o4 + qxy * rz + qxz * ry + qyz * rx + w * rx * ry * rz;
        v[15] = (-o0 - o3) + 2 * qxz * rz + qzz * rx + w * rx * rz * rz;
        v[16] = o5 + 3 * qyy * ry + w * ry * ry * ry;
        v[17] = o6 + qyy * rz + 2 * qyz * ry + w * ry * ry * rz;
        v[18] = (-o1 - o5) + 2 * qyz * rz + qzz * ry + w * ry * rz * rz;
        v[19] = (-o2 - o6) + 3 * qzz * rz + w * rz * rz * rz;
        // siblings across x parity (lane ^ 1: quad_perm [1, 0, 3, 2]) and y
        // parity (lane ^ 8: rotation by 8 within each row of 16 lanes), by
        // DPP moves (every lane of the block takes this branch)
#pragma unroll
        for (int k = 0; k < 20; ++k) {
            v[k] += dpp_f64<0xB1>(v[k]);
            v[k] += dpp_f64<0x128>(v[k]);
        }
        const bool leader = ((x | y) & 1) == 0;
        const int pc = (y >> 1) * 4 + (x >> 1);
        if (leader && (z & 1)) {
#pragma unroll
            for (int k = 0; k < 20; ++k) red[z >> 1][pc][k] = v[k];
        }
        __syncthreads();
        if (!leader || (z & 1)) return;
#pragma unroll
        for (int k = 0; k < 20; ++k) v[k] += red[z >> 1][pc][k];
    }
    const int ex = e >> 2, ey = (e >> 1) & 1, ez = e & 1;
    const int pq = ((4 * ez + (z >> 1)) * NS + (4 * ey + (y >> 1))) * NS + (4 * ex + (x >> 1));
    m2m_store(v, cx.rec + (size_t(pidx) * NCELL + pq) * NREC, cx.com + size_t(pidx) * 3 * NCELL + pq);
}

// A refined sub-grid whose 8 children are all leaves: one block per parent.
// The 8 children's densities are staged in LDS with coalesced loads (each
// thread issues its 8 loads at once), their masses written in the internal
// order, and each thread forms one parent cell from its 8 point masses, so
// that the record is written whole (coalesced per component).
// grid: (such parents of the level), 512 threads.
__global__ __launch_bounds__(512) void k_m2m_leafpar(Ctx cx, const M2MTask* __restrict__ list) {
    __shared__ double rin[8][NCELL + NCELL / 8];  // per child, I/O order, one pad per z-row
    const M2MTask& tk = list[blockIdx.x];
    const int q = threadIdx.x;
    double rv[8];
    size_t cb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        cb[e] = size_t(tk.cidx[e]) * NCELL;
        rv[e] = cx.rho[cb[e] + q];  // coalesced
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        check_rho(cx, rv[e], cb[e] + q, true);
        rin[e][q + (q >> 3)] = rv[e];
    }
    __syncthreads();
    const double hc = 0.5 * tk.ph, h3 = hc * hc * hc;
    const int io = io_index(q);
#pragma unroll
    for (int e = 0; e < 8; ++e) cx.mass[cb[e] + q] = rin[e][io + (io >> 3)] * h3;
    // parent cell q = (z*8 + y)*8 + x: child sub-grid e = (x/4, y/4, z/4),
    // children at (2 (x%4) + i, 2 (y%4) + j, 2 (z%4) + k) in it
    const int x = q & 7, y = (q >> 3) & 7, z = q >> 6;
    const int e = (x >> 2) * 4 + (y >> 2) * 2 + (z >> 2);
    const int cx0 = 2 * (x & 3), cy0 = 2 * (y & 3), cz0 = 2 * (z & 3);
    double mc[2][2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int ic = ((cx0 + i) * NS + (cy0 + j)) * NS + (cz0 + k);
                mc[i][j][k] = rin[e][ic + (ic >> 3)] * h3;
            }
    double v[20];
    leaf_octet(mc, hc, v);
    m2m_store(v, cx.rec + (size_t(tk.pidx) * NCELL + q) * NREC, cx.com + size_t(tk.pidx) * 3 * NCELL + q);
}

// ---------------------------------------------------------------------------
// step 2: same-level interactions as work items of 256 threads (4 waves)
// ---------------------------------------------------------------------------
// LDS of one item block: the largest of the multipole plane window (16
// record components x 18 x 18 cells + leaf flags), the monopole mass box (18
// planes x 18 rows of 20 cells), the class-4 source slab and totals, the
// 4-wave reduction buffer (doubles) and the top-level source tile, followed by
// the target's 27 neighbour codes.
template <typename P>
struct Smem {
    static constexpr int PLANE = NREC * MP_SLOTS * int(sizeof(P)) + MP_SLOTS;
    static constexpr int BOX = PW * PSLOTS * int(sizeof(P));
    static constexpr int RED = 4 * NLOC * 64 * 8;
    static constexpr int TOP = NREC * 256 * int(sizeof(P)) + 4 * 256 * 4;  // top-level source tile
    static constexpr int C4 = NREC * C4_SLAB * 8 * int(sizeof(P)) + NLEAF * NCELL * 8;  // class-4 slab + totals
    static constexpr int A0 = PLANE > BOX ? PLANE : BOX;
    static constexpr int A = A0 > C4 ? A0 : C4;
    static constexpr int B = RED > TOP ? RED : TOP;
    static constexpr int NBR_OFF = ((A > B ? A : B) + 15) & ~15;  // the target's 27 neighbour codes
    static constexpr int BYTES = NBR_OFF + 128;
};
// LDS layout of a block of precision form PR (the mixed form stages its
// multipole sources in FP64)
template <int PR>
using SmemPR = Smem<typename std::conditional<PR == PR_F32, float, double>::type>;

// Swap of the y and z axes in a record (mass, centre-of-mass offset,
// trace-free quadrupole xx yy xy xz yz, trace-free octupole xxx xxy xxz xyy
// xyz yyy yyz) or, with the same index pattern, in the 19 Taylor components
// (L0, L1, trace-free L2, trace-free L3, correction): dependent components
// (zz = -xx - yy, xzz = -xxx - xyy, zzz = -xxz - yyz, yzz = -xxy - yyy) take
// the place of the swapped ones.  The map is its own inverse.
template <typename T>
__device__ __forceinline__ void swap_yz(T& y, T& z) {
    const T t = y;
    y = z;
    z = t;
}
template <typename T>
__device__ __forceinline__ void swap_yz_q(T* q) {
    q[1] = -q[0] - q[1];
    swap_yz(q[2], q[3]);
}
template <typename T>
__device__ __forceinline__ void swap_yz_o(T* o) {
    const T o0 = o[0], o1 = o[1], o2 = o[2], o3 = o[3], o5 = o[5], o6 = o[6];
    o[1] = o2;
    o[2] = o1;
    o[3] = -o0 - o3;
    o[5] = -o2 - o6;
    o[6] = -o1 - o5;
}
// The same for a swap of the x and z axes (xx <- zz, xy <- yz, yz <- xy;
// xxx <- zzz, xxy <- yzz, xxz <- xzz, xyy <- yyz, yyz <- xyy).
template <typename T>
__device__ __forceinline__ void swap_xz_q(T* q) {
    const T q0 = q[0], q1 = q[1], q2 = q[2];
    q[0] = -q0 - q1;
    q[2] = q[4];
    q[4] = q2;
}
template <typename T>
__device__ __forceinline__ void swap_xz_o(T* o) {
    const T o0 = o[0], o1 = o[1], o2 = o[2], o3 = o[3], o5 = o[5], o6 = o[6];
    o[0] = -o2 - o6;
    o[1] = -o1 - o5;
    o[2] = -o0 - o3;
    o[3] = o6;
    o[6] = o3;
}

// Sweep frames (u, v, w): (x, y, z) for sweep 0, (x, z, y) for sweep 1,
// (z, y, x) for sweep 2; the cell-index strides of u, v and w and the
// neighbour-code strides of their sub-grid offsets (code (ox+1)*9 +
// (oy+1)*3 + (oz+1)), and the maps of a record or of the Taylor components
// into the frame and back (each its own inverse).
template <int SWEEP>
struct Frame {
    static constexpr int US = SWEEP == 2 ? 64 : 1, VS = SWEEP == 1 ? 64 : 8;
    static constexpr int WS = SWEEP == 0 ? 64 : (SWEEP == 1 ? 8 : 1);
    static constexpr int UN = SWEEP == 2 ? 1 : 9, VN = SWEEP == 1 ? 1 : 3;
    static constexpr int WN = SWEEP == 0 ? 1 : (SWEEP == 1 ? 3 : 9);
    template <typename T>
    __device__ static void vec(T& x, T& y, T& z) {
        if (SWEEP == 1) swap_yz(y, z);
        if (SWEEP == 2) swap_yz(x, z);
    }
    template <typename T>
    __device__ static void quad(T* q) {
        if (SWEEP == 1) swap_yz_q(q);
        if (SWEEP == 2) swap_xz_q(q);
    }
    template <typename T>
    __device__ static void oct(T* o) {
        if (SWEEP == 1) swap_yz_o(o);
        if (SWEEP == 2) swap_xz_o(o);
    }
};

// Refined-target item: target planes of refined sub-grid sid among the two
// planes 2 pz and 2 pz + 1 (the children of one plane of parent cells)
// against one group of their source planes.  The two planes have the same
// parent plane, so the interaction rule reaches the same 10 source planes
// from both (2 pz - 4 .. 2 pz + 5: staged plane j is canonical offset j - 4
// of the even plane and 5 - j of the odd one), and one staged window serves
// both.  An item of both planes gives waves 0 and 1 the 64 targets of the
// even plane and waves 2 and 3 those of the odd plane, the two waves of a
// plane splitting its entry list; an item of one plane gives all 4 waves its
// 64 targets, splitting the entry list four ways (twice the items, for
// workloads too small to fill the GPU otherwise).  The entries: every
// existing source over the far ones, leaf sources also over the near ones
// (classes 1 + 2).
// The sweep frame (u, v, w) puts the target planes at w = 2 pz, 2 pz + 1 and
// the lanes on (u, v): sweep 0 is (x, y, z); sweep 1 is (x, z, y) and sweep 2
// (z, y, x), chosen by the planner for targets whose sources lie mostly beside
// them in y or in x, so that whole source planes without sources are
// skipped.  A record is 16 contiguous values in any frame (staging stays
// coalesced per cell), and the stencil is symmetric under the axis swaps, so
// one set of tables serves all three: records are swapped into the frame when
// staged and the results swapped back before they are stored.
template <int PR, int SWEEP>
__device__ __forceinline__ void mp_item(const Ctx& cx, int sid, int planes, int group, unsigned char* smem) {
    // P: staged source data; PA: the pair terms' partial sums
    using P = typename std::conditional<PR == PR_F32, float, double>::type;
    using PA = typename std::conditional<PR == PR_F64, double, float>::type;
    // the window's records in 16-byte groups of V components: component k of
    // slot c is element k % V of group (k / V) * MP_SLOTS + c
    constexpr int V = 16 / int(sizeof(P));
    using PV = typename std::conditional<PR == PR_F32, float4, double2>::type;
    unsigned char* leafflag = smem + NREC * MP_SLOTS * sizeof(P);
    int* nb = reinterpret_cast<int*>(smem + SmemPR<PR>::NBR_OFF);

    const int t = item_tid(), lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index: uniform
    sid = __builtin_amdgcn_readfirstlane(sid);  // one item per block: uniform
    // planes: 2 pz in bits 0..3, the target planes in bits 4 (even) and 5
    // (odd).  The wave's target plane (0: even, 1: odd), the number of waves
    // on it and the wave's share of its entries
    const int zt0 = planes & 15, both = (planes >> 4) == 3;
    const int wp = both ? w >> 1 : (planes >> 5) & 1;
    const int nsplit = both ? 2 : 4, wi = both ? w & 1 : w;
    const int zt = zt0 + wp;
    // y runs fastest over the lanes: with the window row stride of 20 cells,
    // the 32 lanes of each LDS pass then hit distinct banks for every offset
    const int x = lane >> 3, y = lane & 7, cl = y * 8 + x;
    const SubDev& T = cx.subs[sid];
    // (visible to the staging loop after its barrier; no other use of this
    // LDS region, so no barrier is needed before the write)
    if (t < 27) nb[t] = T.nbr[t];
    const double h = T.h;
    const int tidx = T.idx;
    // cell-index strides of the frame's axes u, v, w and neighbour-code
    // strides of their sub-grid offsets
    using F = Frame<SWEEP>;
    constexpr int US = F::US, VS = F::VS, WS = F::WS, UN = F::UN, VN = F::VN, WN = F::WN;
    const int q = zt * WS + y * VS + x * US;
    const int sx = 1 - 2 * (x & 1), sy = 1 - 2 * (y & 1);

    // target data
    P oa[9];
    double rt[NREC];
    load_rec(cx.rec, size_t(tidx) * NCELL + q, rt);
    const double mA = rt[R_M];
    double dAx = rt[R_DX], dAy = rt[R_DY], dAz = rt[R_DZ];
    {
        const double os = mA > 0 ? 1.0 / (2.0 * mA) : 0.0;
#pragma unroll
        for (int k = 0; k < 7; ++k) oa[k] = P(rt[R_O + k] * os);
        F::vec(dAx, dAy, dAz);
        F::oct(oa);
        oa[7] = -oa[0] - oa[3];
        oa[8] = -oa[1] - oa[5];
    }
    const bool use_corr = cx.corr != 0;
    const bool do_near = (T.flags & 1) != 0;
    const int ng = cx.ngroups;
    const int j0 = group * NDZ / ng, j1 = (group + 1) * NDZ / ng;

    Acc<double> acc;
    acc.zero();
    // positions in the frame, relative to the centre of the target sub-grid's
    // first cell: the target's COM here, the sources' COM in the window, so
    // that a pair's separation is one subtraction per axis
    const P tu = P(fma(h, double(x), dAx)), tv = P(fma(h, double(y), dAy));
    const P tw = P(fma(h, double(zt), dAz));
    // byte offset of the source cell of canonical offset (dx, dy) in one
    // component group of the plane window:
    // lbase + sx * 16 dx + sy * (16 MP_PRS) dy  (mirror signs per lane)
    const int lbase = ((y + REACH) * MP_PRS + (x + REACH)) * 16;
    const short2_t sxy = {short(sx), short(sy)};

    static_assert(DZ0 + NDZ - 1 == 1 - DZ0, "the odd plane's canonical offsets mirror the even plane's");
    // the neighbour offsets along the sweep axis (-1, 0, 1) with at least one
    // existing sub-grid among their nine: a source plane at an offset without
    // any is skipped (uniform over the block)
    unsigned use_w = 0;
#pragma unroll
    for (int o = 0; o < 27; ++o)
        if (T.nbr[(o % 3) * UN + ((o / 3) % 3) * VN + (o / 9) * WN] >= 0) use_w |= 1u << (o / 9);
    const int32_t* tab = c_tab.mp_entry;
    for (int j = j0; j < j1; ++j) {
        // staged plane: canonical offset DZ0 + j of the even plane, mirrored
        // (sz = -1) DZ0 + NDZ - 1 - j of the odd one
        const int zs = zt0 + DZ0 + j;
        const int gi = wp ? NDZ - 1 - j : j;
        const int oz = zs < 0 ? -1 : (zs >= NS ? 1 : 0);
        if (!((use_w >> (oz + 1)) & 1)) continue;
        // the plane's entry ranges, read before the barrier so that their
        // latency overlaps it
        const int fb = c_tab.mp_far_begin[gi], fe = fb + c_tab.mp_far_count[gi];
        const int nbg = c_tab.mp_near_begin[gi], ne = nbg + c_tab.mp_near_count[gi];
        __syncthreads();
        // stage the 18x18 source window of plane zs: each thread takes up to
        // two cells and issues the loads of both at once (record and mass
        // loads are unconditional, from a valid address, and then selected)
        {
            const int lz = zs - NS * oz;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int cr = t + u * 256;
                if (cr < PCELLS) {
                    const int wx = cr % PW, wy = cr / PW;
                    const int c = wy * MP_PRS + wx;
                    const int lx = wx - REACH, ly = wy - REACH;
                    const int ox = lx < 0 ? -1 : (lx >= NS ? 1 : 0);
                    const int oy = ly < 0 ? -1 : (ly >= NS ? 1 : 0);
                    const int code = nb[(ox + 1) * UN + (oy + 1) * VN + (oz + 1) * WN];
                    const int cq = lz * WS + (ly - NS * oy) * VS + (lx - NS * ox) * US;
                    const int kind = code < 0 ? -1 : (code & 1), nidx = code >> 1;
                    // leaf and absent cells read the zero record; a leaf
                    // cell's mass then replaces its zero mass
                    const double* mp = cx.mass + (kind == 0 ? size_t(nidx) * NCELL + cq : size_t(0));
                    double v[NREC];
                    load_rec(cx.rec, kind == 1 ? size_t(nidx) * NCELL + cq : size_t(cx.rec_zero), v);
                    const double mm = *mp;
                    if (kind == 0) v[R_M] = mm;
                    F::vec(v[R_DX], v[R_DY], v[R_DZ]);
                    F::quad(v + R_Q);
                    F::oct(v + R_O);
                    // the COM offset becomes a position (frame coordinates of the
                    // cell centre plus the offset); moments scaled by stage_scale
                    const double pos[3] = {double(lx), double(ly), double(zs)};
                    P w[NREC];
#pragma unroll
                    for (int k = 0; k < NREC; ++k) {
                        double val = v[k];
                        if (k >= R_DX && k <= R_DZ) val = fma(h, pos[k - R_DX], val);
                        val *= stage_scale(k);
                        w[k] = P(val);
                    }
#pragma unroll
                    for (int j = 0; j < NREC / V; ++j) {
                        PV pv;
                        P* pp = reinterpret_cast<P*>(&pv);
#pragma unroll
                        for (int i = 0; i < V; ++i) pp[i] = w[j * V + i];
                        reinterpret_cast<PV*>(smem)[j * MP_SLOTS + c] = pv;
                    }
                    leafflag[c] = kind == 0;
                }
            }
        }
        __syncthreads();
        // FP32 forms: partial sums per source plane, flushed into the FP64
        // accumulators after the plane; FP64 form: accumulate directly
        Acc<PA> part_store;
        Acc<PA>& part = PR != PR_F64 ? part_store : *reinterpret_cast<Acc<PA>*>(&acc);
        if (PR != PR_F64) part.zero();
        // byte offset of an entry's source cell for this lane: the entry's
        // canonical offsets (dx, dy) scaled to bytes, in two signed 16-bit
        // halves, dotted with the lane's mirror signs (one instruction)
        auto addr = [&](int e) { return __builtin_amdgcn_sdot2(sxy, __builtin_bit_cast(short2_t, tab[e]), lbase, false); };
        auto one = [&](int e) {
            const unsigned char* cs = smem + addr(e);
            P src[NREC];
#pragma unroll
            for (int j = 0; j < NREC / V; ++j) {
                const PV pv = *reinterpret_cast<const PV*>(cs + j * (MP_SLOTS * 16));
                const P* pp = reinterpret_cast<const P*>(&pv);
#pragma unroll
                for (int i = 0; i < V; ++i) src[j * V + i] = pp[i];
            }
            const P X = tu - src[R_DX];
            const P Y = tv - src[R_DY];
            const P Z = tw - src[R_DZ];
            pair_any<true, PR>(X, Y, Z, src, oa, acc, part);
        };
        // the wave's far entries fb + wi + k nsplit, k < nk: two independent
        // pairs per iteration, two dependency chains per wave.  FP32 forms
        // with two waves on the plane flush the partial sums once more, after
        // about half of them, so that no partial sums more pairs than with
        // four waves on the plane
        const int nk = fe - fb > wi ? (fe - fb - wi + nsplit - 1) / nsplit : 0;
        const int kflush = (PR != PR_F64 && both) ? (nk >> 2) << 1 : -1;
        int k = 0;
        for (; k + 1 < nk; k += 2) {
            if (PR != PR_F64 && k == kflush && k > 0) {
                acc.add(part, true, PR == PR_F32);
                part.zero();
            }
            one(fb + wi + k * nsplit);
            one(fb + wi + (k + 1) * nsplit);
        }
        if (k < nk) one(fb + wi + k * nsplit);
        if (do_near) {
            for (int e = nbg + wi; e < ne; e += nsplit) {
                if (!leafflag[addr(e) >> 4]) continue;
                one(e);
            }
        }
        if (PR != PR_F64) acc.add(part, true, PR == PR_F32);
    }

    // combine the partial sums of each plane's waves in a fixed order
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);
    {
        double v[NLOC];
        // a target without mass gets no correction term (its descendants
        // carry no mass either, so no momentum is involved)
        if (!(mA > 0)) acc.s[0] = acc.s[1] = acc.s[2] = 0.0;
        acc.out(v);
        // back from the frame
        F::vec(v[T_L1], v[T_L1 + 1], v[T_L1 + 2]);
        F::quad(v + T_L2);
        F::oct(v + T_L3);
        F::vec(v[T_S], v[T_S + 1], v[T_S + 2]);
#pragma unroll
        for (int k = 0; k < NLOC; ++k) red[(w * NLOC + k) * 64 + cl] = v[k];
    }
    __syncthreads();
    const double G = cx.G;
    const double gs = use_corr ? 3.0 * G : 0.0;  // dg = 3G S
    // reduction slot l = v*8 + u of plane p holds target cell
    // (2 pz + p)*WS + v*VS + u*US
    double* out = cx.Lp + size_t(group) * size_t(cx.part_stride) + size_t(tidx) * NLOC * NCELL + zt0 * WS;
    if (both) {
        for (int i = t; i < 2 * NLOC * 64; i += 256) {
            const int p = i >= NLOC * 64, r = i - p * (NLOC * 64);
            const int k = r >> 6, l = r & 63;
            const double v = red[((2 * p) * NLOC + k) * 64 + l] + red[((2 * p + 1) * NLOC + k) * 64 + l];
            out[p * WS + k * NCELL + (l >> 3) * VS + (l & 7) * US] = (k >= T_S ? gs : -G) * v;
        }
    } else {
        for (int i = t; i < NLOC * 64; i += 256) {
            const int k = i >> 6, l = i & 63;
            const double v = red[(0 * NLOC + k) * 64 + l] + red[(1 * NLOC + k) * 64 + l] +
                             red[(2 * NLOC + k) * 64 + l] + red[(3 * NLOC + k) * 64 + l];
            out[wp * WS + k * NCELL + (l >> 3) * VS + (l & 7) * US] = (k >= T_S ? gs : -G) * v;
        }
    }
}

// Leaf-target item (class 4): the 512 leaf cells of sub-grid sid against the
// refined cells of its refined neighbours in slots [o0, o1), written to Lf3
// slot `slot`.  A leaf target takes every partner
// whose parent cell lies within |D|^2 <= 8 of its own parent, so the 8
// children of one target parent share one partner set: the 8 children of
// each partner parent.  A wave works on one target parent at a time with
// lane = target child * 8 + source child and one partner parent per step, so
// every lane of every step evaluates a real pair.  The partner parents in one
// refined neighbour (its slab, at most 32 parents) are staged in LDS, one
// neighbour at a time in slot order; the waves take the target parents of
// that neighbour in turn, add the 8 source-child sums of each target across
// lanes in a fixed order, and accumulate them into the item's LDS totals
// (one wave per target parent and neighbour, so the order is fixed).
template <int PR>
__device__ __forceinline__ void c4_item(const Ctx& cx, int sid, int o0, int o1, int slot, unsigned char* smem) {
    using P = typename std::conditional<PR == PR_F32, float, double>::type;
    using PA = typename std::conditional<PR == PR_F64, double, float>::type;
    constexpr int V = 16 / int(sizeof(P));
    using PV = typename std::conditional<PR == PR_F32, float4, double2>::type;
    constexpr int SLOTS = C4_SLAB * 8;
    // LDS: staged slab records [NREC / V groups][SLOTS] of 16 bytes, then the
    // totals [4][512] (L0, and L1 - S or L1)
    double* tot = reinterpret_cast<double*>(smem + NREC * SLOTS * sizeof(P));
    const int t = item_tid(), lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int c = lane & 7, tc = lane >> 3;
    sid = __builtin_amdgcn_readfirstlane(sid);  // one item per block: uniform
    const SubDev& T = cx.subs[sid];
    const double h = T.h;
    const double* tmass = cx.mass + size_t(T.idx) * NCELL;
    const double sfac = cx.corr ? 3.0 : 0.0;  // dg = 3G S
    for (int i = t; i < NLEAF * NCELL; i += 256) tot[i] = 0.0;
    const P oa[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // leaf targets carry no octupole
    // the 27 neighbour codes, one per lane, loaded once (not once per slot)
    const int nbc = lane < 27 ? T.nbr[lane] : -1;
    for (int o = o0; o < o1; ++o) {
        const int code = __builtin_amdgcn_readlane(nbc, o);
        if (o == 13 || code < 0 || !(code & 1)) continue;
        const int ox = o / 9 - 1, oy = (o / 3) % 3 - 1, oz = o % 3 - 1;
        const int sl = c_tab.c4_slab[o];
        const int ny = (sl >> 4) & 15, nz = (sl >> 8) & 15, nslab = (sl & 15) * ny * nz * 8;
        const int px0 = (sl >> 12) & 3, py0 = (sl >> 14) & 3, pz0 = (sl >> 16) & 3;
        __syncthreads();  // the previous neighbour's slab is no longer read
        // stage: thread t holds child t & 7 of slab parent t >> 3; its position
        // in the frame of the target sub-grid (centre of its cell (0,0,0)),
        // moments scaled by stage_scale
        if (t < nslab) {
            const int sp = t >> 3, ch = t & 7;
            const int ix = sp / (ny * nz), iy = (sp / nz) % ny, iz = sp % nz;
            const int lx = 2 * (px0 + ix) + (ch >> 2), ly = 2 * (py0 + iy) + ((ch >> 1) & 1);
            const int lz = 2 * (pz0 + iz) + (ch & 1);
            double v[NREC];
            load_rec(cx.rec, size_t(code >> 1) * NCELL + (lz * NS + ly) * NS + lx, v);
            v[R_DX] = fma(h, double(NS * ox + lx), v[R_DX]);
            v[R_DY] = fma(h, double(NS * oy + ly), v[R_DY]);
            v[R_DZ] = fma(h, double(NS * oz + lz), v[R_DZ]);
#pragma unroll
            for (int k = R_Q; k < NREC; ++k) v[k] *= stage_scale(k);
#pragma unroll
            for (int j = 0; j < NREC / V; ++j) {
                PV pv;
                P* pp = reinterpret_cast<P*>(&pv);
#pragma unroll
                for (int i = 0; i < V; ++i) pp[i] = P(v[j * V + i]);
                reinterpret_cast<PV*>(smem)[j * SLOTS + t] = pv;
            }
        }
        __syncthreads();
        const int gb = c_tab.c4_grp_begin[o], ge = c_tab.c4_grp_begin[o + 1];
        for (int g = gb + w; g < ge; g += 4) {
            const int gi = c_tab.c4_grp[g];
            const int pt = gi & 63, first = (gi >> 6) & 4095, cnt = gi >> 18;
            const int tx = 2 * (pt >> 4) + (tc >> 2), ty = 2 * ((pt >> 2) & 3) + ((tc >> 1) & 1);
            const int tz = 2 * (pt & 3) + (tc & 1);
            const P X0 = P(h * tx), Y0 = P(h * ty), Z0 = P(h * tz);
            // the target's mass, loaded before the steps (its latency hidden
            // by them) for the correction's switch after them
            const int q = (tz * NS + ty) * NS + tx;
            const double mq = tmass[q];
            // two steps per iteration, each into its own sums: two
            // independent dependency chains per wave
            Acc<double> acc, acc2;
            acc.zero();
            acc2.zero();
            Acc<PA> part_store, part2_store;
            Acc<PA>& part = PR != PR_F64 ? part_store : *reinterpret_cast<Acc<PA>*>(&acc);
            Acc<PA>& part2 = PR != PR_F64 ? part2_store : *reinterpret_cast<Acc<PA>*>(&acc2);
            if (PR != PR_F64) {
                part.zero();
                part2.zero();
            }
            auto step = [&](int sp, Acc<double>& ac, Acc<PA>& pa) {
                const unsigned char* cs = smem + (sp * 8 + c) * 16;
                P src[NREC];
#pragma unroll
                for (int j = 0; j < NREC / V; ++j) {
                    const PV pv = *reinterpret_cast<const PV*>(cs + j * (SLOTS * 16));
                    const P* pp = reinterpret_cast<const P*>(&pv);
#pragma unroll
                    for (int i = 0; i < V; ++i) src[j * V + i] = pp[i];
                }
                pair_any<false, PR>(X0 - src[R_DX], Y0 - src[R_DY], Z0 - src[R_DZ], src, oa, ac, pa);
            };
            const int kend = first + cnt;
            int k = first;
            for (; k + 1 < kend; k += 2) {
                const int sp0 = c_tab.c4_task[k], sp1 = c_tab.c4_task[k + 1];
                step(sp0, acc, part);
                step(sp1, acc2, part2);
            }
            if (k < kend) step(c_tab.c4_task[k], acc, part);
            if (PR != PR_F64) {
                acc.add(part, false, PR == PR_F32);
                acc.add(part2, false, PR == PR_F32);
            }
            acc.add(acc2, false);
            // the 8 source-child sums of each target, added across its 8 lanes
            double v[7] = {acc.l0, acc.l1[0], acc.l1[1], acc.l1[2], acc.s[0], acc.s[1], acc.s[2]};
#pragma unroll
            for (int k = 0; k < 7; ++k) v[k] = sum8_lanes(v[k]);
            if (c == 0) {
                // a target without mass gets no correction term
                const double sf = mq > 0 ? sfac : 0.0;
                tot[q] += v[0];
#pragma unroll
                for (int a = 0; a < 3; ++a) tot[(1 + a) * NCELL + q] += fma(sf, v[4 + a], v[1 + a]);
            }
        }
    }
    __syncthreads();
    // own terms from refined sources: phi = -G L0;  g = G (L1 - S)
    const double G = cx.G;
    double* out = cx.Lf3 + size_t(slot) * NLEAF * NCELL;
    for (int i = t; i < NLEAF * NCELL; i += 256) out[i] = (i < NCELL ? -G : G) * tot[i];
}

// Monopole item: leaf targets of one sub-grid against leaf sources (class 3).
// Cell pairs lie on the lattice: R = -h d, so phi = -(G/h) sum m/|d| and
// g = (G/h^2) sum m d/|d|^3 with per-offset kernel values from tables.  The
// 18^3 box of leaf masses around the sub-grid sits in LDS.  A lane owns the 8
// targets of its (x, y) column; wave w takes every fourth stencil column
// starting at w, and the four column parts are added pairwise in a fixed
// order.  Both z parities of a column read the same N + 6 source masses (the
// mirrored offsets of odd targets cover the same z range), so one column's
// LDS reads serve 8N pairs.

// kernel values {|d|^-1, |d|^-3} for |d|^2 = n (uniform: scalar loads)
template <typename P>
__device__ __forceinline__ void mono_r(int n, P& a, P& b);
template <>
__device__ __forceinline__ void mono_r<double>(int n, double& a, double& b) {
    a = c_tab.mono_r[n][0];
    b = c_tab.mono_r[n][1];
}
template <>
__device__ __forceinline__ void mono_r<float>(int n, float& a, float& b) {
    a = c_tab.mono_rf[n][0];
    b = c_tab.mono_rf[n][1];
}

template <int LO, int N, typename P>
__device__ __forceinline__ void mono_class(const P* __restrict__ box, int cbeg, int cend,
                                           int cstart, int cstep, int lbase, int sx, int syw, int sy,
                                           double (&phi)[8], double (&gx)[8], double (&gy)[8],
                                           double (&gz)[8]) {
    // source z of target z and canonical offset dzc: z + dzc (z even) or
    // z - dzc (z odd); over z = 0..7 and dzc in [LO, LO + N) it spans
    // [LO, LO + N + 5] for each of the three column classes
    constexpr int NSRC = N + 6;
    for (int c = cbeg + cstart; c < cend; c += cstep) {
        const int pk = c_tab.mono_col[c];
        const int dx = (pk & 255) - 8, dy = ((pk >> 8) & 255) - 8;
        const P* col = box + lbase + __mul24(sx, dx) + __mul24(syw, dy) + (LO + REACH) * PSLOTS;
        P m[NSRC];
#pragma unroll
        for (int j = 0; j < NSRC; ++j) m[j] = col[j * PSLOTS];
        const int rxy = dx * dx + dy * dy;
        // FP64: phi and gz accumulate straight into the totals (the sign of
        // odd targets' mirrored dz folded into the kernel value); the x and y
        // parts share one column sum, scaled by dx and dy once per column.
        // FP32: all three are column partial sums, flushed to FP64
        // The kernel values depend on dz^2 only, so canonical offsets +d and
        // -d (both in the column's range for d <= NP) share them: their masses
        // enter phi and the column sum as m(+d) + m(-d) and gz as
        // d (m(+d) - m(-d)), 5 operations for 2 pairs instead of 6.
        constexpr bool F64 = sizeof(P) == 8;
        constexpr int NP = -LO < LO + N - 1 ? -LO : LO + N - 1;
        P s0[8], s1[8], s2[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) s0[k] = s1[k] = s2[k] = 0;
        // mp: mass at canonical offset +d (mirrored for odd targets), mq at -d
        auto add = [&](int k, P a, P b, P cz, P mp, P mq, bool with_z) {
            s1[k] += mp * b;
            if (F64) {
                phi[k] = fmaP(double(mp), double(a), phi[k]);
                if (with_z) gz[k] = fmaP(double(mq), double((k & 1) ? -cz : cz), gz[k]);
            } else {
                s0[k] += mp * a;
                if (with_z) s2[k] += mq * cz;
            }
        };
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int dzc = LO + i;  // canonical dz
            if (dzc < 0 && -dzc <= NP) continue;  // taken with +|dzc|
            P a, b;
            mono_r<P>(rxy + dzc * dzc, a, b);
            const P cz = P(dzc) * b;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const P m1 = m[k + ((k & 1) ? -dzc : dzc) - LO];
                if (dzc > 0 && dzc <= NP) {
                    const P m2 = m[k + ((k & 1) ? dzc : -dzc) - LO];
                    add(k, a, b, cz, m1 + m2, m1 - m2, true);
                } else {
                    add(k, a, b, cz, m1, m1, dzc != 0);
                }
            }
        }
        const double fx = double(sx * dx), fy = double(sy * dy);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (!F64) {
                phi[k] += double(s0[k]);
                gz[k] += (k & 1) ? -double(s2[k]) : double(s2[k]);
            }
            gx[k] += fx * double(s1[k]);
            gy[k] += fy * double(s1[k]);
        }
    }
}

template <typename P>
__device__ __forceinline__ void mono_all(const P* box, int cstart, int cstep, int lbase, int sx,
                                         int syw, int sy, double (&phi)[8], double (&gx)[8],
                                         double (&gy)[8], double (&gz)[8]) {
    const int b0 = c_tab.mono_class_begin[0], b1 = c_tab.mono_class_begin[1];
    const int b2 = c_tab.mono_class_begin[2], b3 = c_tab.mono_class_begin[3];
    mono_class<-4, 10, P>(box, b0, b1, cstart, cstep, lbase, sx, syw, sy, phi, gx, gy, gz);
    mono_class<-2, 6, P>(box, b1, b2, cstart, cstep, lbase, sx, syw, sy, phi, gx, gy, gz);
    mono_class<0, 2, P>(box, b2, b3, cstart, cstep, lbase, sx, syw, sy, phi, gx, gy, gz);
}


// NB: byte offset of the neighbour codes in the block's LDS layout
template <int PR, int NB>
__device__ __forceinline__ void mono_item(const Ctx& cx, int sid, unsigned char* smem) {
    using P = typename std::conditional<PR == PR_F64, double, float>::type;
    P* box = reinterpret_cast<P*>(smem);
    int* nb = reinterpret_cast<int*>(smem + NB);
    const int t = item_tid();
    sid = __builtin_amdgcn_readfirstlane(sid);  // one item per block: uniform
    const SubDev& T = cx.subs[sid];
    if (t < 27) nb[t] = T.nbr[t];
    __syncthreads();
    // stage the 18^3 mass box by row segments: a window row (wy, wz) of 18
    // cells is three runs, 5 cells of the -x neighbour, 8 of the centre column,
    // 5 of the +x neighbour; a thread takes one run (up to 8 contiguous
    // masses) per unit, two units at a time with all their loads in flight
    // (unconditional, from a valid address, then selected)
    constexpr int NUNIT = PW * PW * 3, PER = (NUNIT + 255) / 256;
#pragma unroll
    for (int u0 = 0; u0 < PER; u0 += 2) {
        double v[2][NS];
        int dst[2], len[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            len[u] = 0;
            dst[u] = 0;
            if (u0 + u >= PER) continue;  // resolved at compile time
            const int un0 = t + (u0 + u) * 256;
            const bool ok = un0 < NUNIT;
            const int un = ok ? un0 : 0;
            const int part = un % 3, row = un / 3;
            const int wy = row % PW, wz = row / PW;
            const int ly = wy - REACH, lz = wz - REACH;
            const int ox = part - 1;
            const int oy = ly < 0 ? -1 : (ly >= NS ? 1 : 0);
            const int oz = lz < 0 ? -1 : (lz >= NS ? 1 : 0);
            const int code = nb[(ox + 1) * 9 + (oy + 1) * 3 + (oz + 1)];
            const bool leaf = code >= 0 && (code & 1) == 0;
            const int x0 = part == 0 ? NS - REACH : 0;  // first neighbour-local x of the run
            const double* src = cx.mass + (leaf ? size_t(code >> 1) * NCELL +
                                                      ((lz - NS * oz) * NS + (ly - NS * oy)) * NS + x0
                                                : size_t(0));
            const int n = part == 1 ? NS : REACH;
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                const double m = src[i < n ? i : 0];
                v[u][i] = leaf ? m : 0.0;
            }
            len[u] = ok ? n : 0;
            dst[u] = wz * PSLOTS + wy * PRS + (part == 0 ? 0 : part == 1 ? REACH : REACH + NS);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int i = 0; i < NS; ++i)
                if (i < len[u]) box[dst[u] + i] = P(v[u][i]);
    }
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63, x = lane >> 3, y = lane & 7;  // y fastest (LDS banks)
    const int sx = 1 - 2 * (x & 1), sy = 1 - 2 * (y & 1);
    const int lbase = (y + REACH) * PRS + (x + REACH);
    const int syw = sy * PRS;
    double phi[8], gx[8], gy[8], gz[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) phi[k] = gx[k] = gy[k] = gz[k] = 0;
    mono_all<P>(box, w, 4, lbase, sx, syw, sy, phi, gx, gy, gz);
    // column parts combined through LDS: w += w + 2 (waves 0, 1), then
    // 0 += 1
    double* red = reinterpret_cast<double*>(smem);
#pragma unroll
    for (int sh = 2; sh >= 1; sh /= 2) {
        __syncthreads();
        if (w >= sh && w < 2 * sh) {
            double* r = red + (w - sh) * 32 * 64 + lane;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                r[(4 * k + 0) * 64] = phi[k];
                r[(4 * k + 1) * 64] = gx[k];
                r[(4 * k + 2) * 64] = gy[k];
                r[(4 * k + 3) * 64] = gz[k];
            }
        }
        __syncthreads();
        if (w < sh) {
            const double* r = red + w * 32 * 64 + lane;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                phi[k] += r[(4 * k + 0) * 64];
                gx[k] += r[(4 * k + 1) * 64];
                gy[k] += r[(4 * k + 2) * 64];
                gz[k] += r[(4 * k + 3) * 64];
            }
        }
    }
    if (w == 0) {
        const double h = T.h, G = cx.G, gh = G / (h * h), gp = -G / h;
        double* out = cx.Lf + size_t(T.idx) * NLEAF * NCELL;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = k * 64 + y * 8 + x;
            out[0 * NCELL + q] = gp * phi[k];
            out[1 * NCELL + q] = gh * gx[k];
            out[2 * NCELL + q] = gh * gy[k];
            out[3 * NCELL + q] = gh * gz[k];
        }
    }
}

// Top-level tile (all-pairs rule): 64 targets (one plane of a top-level
// sub-grid) against a chunk of the tree's top-level cells; the sources are
// staged through LDS 256 at a time, the 4 waves take every fourth source
// (one LDS address per wave: broadcast reads) and their sums are added in a
// fixed order.
template <int PR>
__device__ __forceinline__ void top_item(const Ctx& cx, const TopItem& it, unsigned char* smem) {
    using P = typename std::conditional<PR == PR_F32, float, double>::type;
    using PA = typename std::conditional<PR == PR_F64, double, float>::type;
    const SubDev& T = cx.subs[it.target];
    const int t = item_tid(), lane = t & 63, x = lane & 7, y = lane >> 3;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int q = it.zt * 64 + lane;
    const bool tref = T.kind == 1;
    const double h = T.h;
    const int cax = NS * T.coord[0] + x, cay = NS * T.coord[1] + y, caz = NS * T.coord[2] + it.zt;
    double mA, dAx = 0, dAy = 0, dAz = 0;
    P oa[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (tref) {
        double r[NREC];
        load_rec(cx.rec, size_t(T.idx) * NCELL + q, r);
        mA = r[R_M];
        dAx = r[R_DX];
        dAy = r[R_DY];
        dAz = r[R_DZ];
        const double os = mA > 0 ? 1.0 / (2.0 * mA) : 0.0;
        for (int k = 0; k < 7; ++k) oa[k] = P(r[R_O + k] * os);
        oa[7] = -oa[0] - oa[3];
        oa[8] = -oa[1] - oa[5];
    } else {
        mA = cx.mass[size_t(T.idx) * NCELL + q];
    }
    Acc<double> acc;
    acc.zero();
    // sources staged through LDS, 256 per tile: 16 record values (moments
    // scaled by stage_scale, as the pair terms take them) and the
    // global integer cell coordinates (w = 1 for a refined sub-grid's cell)
    P* sv = reinterpret_cast<P*>(smem);
    int* sc = reinterpret_cast<int*>(smem + NREC * 256 * sizeof(P));
    for (int tb = it.src_begin; tb < it.src_end; tb += 256) {
        __syncthreads();
        const int j = tb + t;
        if (j < it.src_end) {
            const SubDev& S = cx.subs[cx.top_src[it.src_list + (j >> 9)]];
            const int cq = j & 511;
            sc[0 * 256 + t] = NS * S.coord[0] + (cq & 7);
            sc[1 * 256 + t] = NS * S.coord[1] + ((cq >> 3) & 7);
            sc[2 * 256 + t] = NS * S.coord[2] + (cq >> 6);
            sc[3 * 256 + t] = S.kind;
            if (S.kind == 1) {
                double r[NREC];
                load_rec(cx.rec, size_t(S.idx) * NCELL + cq, r);
#pragma unroll
                for (int k = 0; k < NREC; ++k) sv[k * 256 + t] = P(r[k] * stage_scale(k));
            } else {
                sv[t] = P(cx.mass[size_t(S.idx) * NCELL + cq]);
#pragma unroll
                for (int k = 1; k < NREC; ++k) sv[k * 256 + t] = P(0);
            }
        }
        __syncthreads();
        // FP32 forms: partial sums per tile, flushed into the FP64 sums
        Acc<PA> part_store;
        Acc<PA>& part = PR != PR_F64 ? part_store : *reinterpret_cast<Acc<PA>*>(&acc);
        if (PR != PR_F64) part.zero();
        const int nt = min(256, it.src_end - tb);
        for (int s = w; s < nt; s += 4) {
            const int dx = sc[0 * 256 + s] - cax;
            const int dy = sc[1 * 256 + s] - cay;
            const int dz = sc[2 * 256 + s] - caz;
            const int d2 = dx * dx + dy * dy + dz * dz;
            const bool sref = sc[3 * 256 + s] == 1;
            if (d2 == 0 || (d2 < 9 && tref && sref)) continue;
            P src[NREC];
#pragma unroll
            for (int k = 0; k < NREC; ++k) src[k] = sv[k * 256 + s];
            const P X = P(-h * dx) + (P(dAx) - src[R_DX]);
            const P Y = P(-h * dy) + (P(dAy) - src[R_DY]);
            const P Z = P(-h * dz) + (P(dAz) - src[R_DZ]);
            if (tref) pair_any<true, PR>(X, Y, Z, src, oa, acc, part);
            else pair_any<false, PR>(X, Y, Z, src, oa, acc, part);
        }
        if (PR != PR_F64) acc.add(part, tref, PR == PR_F32);
    }
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);
    {
        double v[NLOC];
        // a target without mass gets no correction term (its descendants
        // carry no mass either, so no momentum is involved)
        if (!(mA > 0)) acc.s[0] = acc.s[1] = acc.s[2] = 0.0;
        acc.out(v);
#pragma unroll
        for (int k = 0; k < NLOC; ++k) red[(w * NLOC + k) * 64 + lane] = v[k];
    }
    __syncthreads();
    double* out = cx.part + size_t(it.part) * NLOC * NCELL + it.zt * 64;
    for (int i = t; i < NLOC * 64; i += 256) {
        const int k = i >> 6, l = i & 63;
        out[k * NCELL + l] = red[(0 * NLOC + k) * 64 + l] + red[(1 * NLOC + k) * 64 + l] +
                             red[(2 * NLOC + k) * 64 + l] + red[(3 * NLOC + k) * 64 + l];
    }
}

template <int PR>
__device__ __forceinline__ void run_item(const Ctx& cx, const Item& it, unsigned char* smem) {
    switch (it.kind) {
        case IT_MP_REF:
            if ((it.b >> 3) == 1) mp_item<PR, 1>(cx, it.sub, it.a, it.b & 7, smem);
            else if ((it.b >> 3) == 2) mp_item<PR, 2>(cx, it.sub, it.a, it.b & 7, smem);
            else mp_item<PR, 0>(cx, it.sub, it.a, it.b & 7, smem);
            break;
        case IT_MP_LEAF: c4_item<PR>(cx, it.sub, it.a & 255, it.a >> 8, it.b, smem); break;
        case IT_MONO: mono_item<PR, SmemPR<PR>::NBR_OFF>(cx, it.sub, smem); break;
        default: top_item<PR>(cx, cx.top_items[it.sub], smem); break;
    }
}

// One launch per class: one block per item of that class.
template <int KIND, int PR>
__global__ __launch_bounds__(256) void k_class(Ctx cx, const Item* __restrict__ items) {
    // the monopole class of the mixed form uses FP32 masses, as PR_F32 does
    using L = SmemPR<(KIND == IT_MONO && PR == PR_MIX) ? PR_F32 : PR>;
    __shared__ __attribute__((aligned(16))) unsigned char smem[L::BYTES];
    const Item it = items[xcd_run_index()];
    if (KIND == IT_MP_REF) {
        if ((it.b >> 3) == 1) mp_item<PR, 1>(cx, it.sub, it.a, it.b & 7, smem);
        else if ((it.b >> 3) == 2) mp_item<PR, 2>(cx, it.sub, it.a, it.b & 7, smem);
        else mp_item<PR, 0>(cx, it.sub, it.a, it.b & 7, smem);
    }
    else if (KIND == IT_MP_LEAF) c4_item<PR>(cx, it.sub, it.a & 255, it.a >> 8, it.b, smem);
    else if (KIND == IT_MONO) mono_item<PR, L::NBR_OFF>(cx, it.sub, smem);
    else top_item<PR>(cx, cx.top_items[it.sub], smem);
}

// Persistent launch over NQUEUE item queues, one per XCD: the blocks of a
// launch are dealt to the XCDs in turn, so block b starts on queue b % NQUEUE
// (a compact region of the octree whose source records its XCD's L2 keeps),
// taking the next item from ctr[q] until the queue is exhausted, then helps
// with the other queues in turn (a single list is passed as queue 0 with the
// others empty).  Every block passes each queue once, so it exits once all
// items are taken; the last block to exit (counted in ctr[NQUEUE]) re-arms
// all NQUEUE + 1 counters (zero before the first launch) for the next launch.
template <int PR>
__global__ __launch_bounds__(256, 3) void k_persist(Ctx cx, const Item* __restrict__ items, Queues qs,
                                                    int* __restrict__ ctr) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[SmemPR<PR>::BYTES];
    __shared__ int s_it;
    const int home = int(blockIdx.x % NQUEUE);
    for (int r = 0; r < NQUEUE; ++r) {
        const int q = (home + r) % NQUEUE;
        const int b = qs.begin[q], e = qs.begin[q + 1];
        for (;;) {
            if (threadIdx.x == 0) s_it = b < e ? b + atomicAdd(&ctr[q], 1) : e;
            __syncthreads();
            const int it = s_it;
            __syncthreads();
            if (it >= e) break;
            run_item<PR>(cx, items[it], smem);
        }
    }
    if (threadIdx.x == 0 && atomicAdd(&ctr[NQUEUE], 1) == int(gridDim.x) - 1) {
        for (int q = 0; q <= NQUEUE; ++q) atomicExch(&ctr[q], 0);
    }
}

// ---------------------------------------------------------------------------
// step 3: downward pass
// ---------------------------------------------------------------------------
// Total expansion of a top-level target under the all-pairs rule: the sum of
// its partial slots in a fixed order, scaled by -G (the correction sums S
// by 3G).
__device__ __forceinline__ double top_total(const Ctx& cx, int red, int k, int q) {
    const TopReduce R = cx.top_reds[red];
    const double* base = cx.part + (size_t(R.part_begin) * NLOC + k) * NCELL + q;
    double v = 0;
#pragma unroll
    for (int p = 0; p < MAX_TOP_PARTS; ++p) {  // all loads issued together
        const double t = base[size_t(p < R.n_part ? p : R.n_part - 1) * (NLOC * NCELL)];
        v += p < R.n_part ? t : 0.0;
    }
    return (k >= T_S ? (cx.corr ? 3.0 * cx.G : 0.0) : -cx.G) * v;
}

// Parent expansion (L0, L1, trace-free L2, L3, correction dg) re-expanded at
// the child COM, r = X_child - X_parent:
//   o0 = L0 + L1.r + 1/2 r.L2.r + 1/6 L3:rrr,  o1 = L1 + L2.r + 1/2 L3:rr,
//   o2 = L2 + L3.r,  o3 = L3,  dg passed unchanged.
// The parent's total is formed from its top-level partial slots (level 0
// under the all-pairs rule), from its own plane-group sums (level 0 under the
// stencil rule), or as its inherited part Lr plus its own plane-group sums.
// Refined children: Lr = shifted parent (their own terms join when they act
// as parents, so this step does not wait for them).
// Leaf children: phi = own + o0,  g = own - o1 + dg.
// grid: one block of 512 per task (a child slot of a refined parent).
template <int NG>
__global__ __launch_bounds__(512) void k_l2l(Ctx cx, const L2LTask* __restrict__ tasks, int parent_mode,
                                             double* __restrict__ phi, double* __restrict__ gout) {
    __shared__ double obuf[4][NCELL];
    __shared__ double par[NLOC + 3][64];  // the octant's 64 parent cells: L (19), COM offset (3)
    rho_flag_out(cx);
    // (dealt to the XCDs in turn, not in runs: this bandwidth-bound pass is
    // 7 % faster with neighbouring tasks spread over all XCDs)
    const L2LTask tk = tasks[blockIdx.x];
    const int e = (tk.flags >> 1) & 7;
    const int q = threadIdx.x;
    const int x = q & 7, y = (q >> 3) & 7, z = q >> 6;
    const int ex = 4 * (e >> 2), ey = 4 * ((e >> 1) & 1), ez = 4 * (e & 1);
    // cooperative fetch of the parent octant: value i = comp * 64 + cell (the
    // component is uniform over a wave); every load of the three rounds (the
    // NG plane-group partials of each value included) is issued before the
    // first is used
    double v[3], t[3][NG];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int i = q + r * NCELL;
        const int k = i >> 6, c = i & 63;
        const int pq = ((ez + (c >> 4)) * NS + ey + ((c >> 2) & 3)) * NS + ex + (c & 3);
        v[r] = 0.0;
        if (i >= (NLOC + 3) * 64) continue;
        if (k >= NLOC) {
            v[r] = cx.com[(size_t(tk.pidx) * 3 + (k - NLOC)) * NCELL + pq];
        } else if (parent_mode == PARENT_TOP_PARTS) {
            v[r] = top_total(cx, tk.pred, k, pq);
        } else {
            const size_t base = (size_t(tk.pidx) * NLOC + k) * NCELL + pq;
            if (parent_mode == PARENT_TOTAL) v[r] = cx.Lr[base];
#pragma unroll
            for (int gg = 0; gg < NG; ++gg) t[r][gg] = cx.Lp[size_t(gg) * size_t(cx.part_stride) + base];
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int i = q + r * NCELL;
        if (i >= (NLOC + 3) * 64) continue;
        const int k = i >> 6;
        if (k < NLOC && parent_mode != PARENT_TOP_PARTS) {
#pragma unroll
            for (int gg = 0; gg < NG; ++gg) v[r] += t[r][gg];
        }
        par[k][i & 63] = v[r];
    }
    __syncthreads();
    const int pc = ((z >> 1) * 4 + (y >> 1)) * 4 + (x >> 1);
    double L[NLOC];
    for (int k = 0; k < NLOC; ++k) L[k] = par[k][pc];
    const double l0 = L[0], l1x = L[1], l1y = L[2], l1z = L[3];
    const double qxx = L[4], qyy = L[5], qxy = L[6], qxz = L[7], qyz = L[8];
    const double qzz = -qxx - qyy;
    double o[7];
    for (int k = 0; k < 7; ++k) o[k] = L[T_L3 + k];
    const double sgx = L[T_S], sgy = L[T_S + 1], sgz = L[T_S + 2];
    const double hc = tk.ch;
    double cdx = 0, cdy = 0, cdz = 0;
    const bool cref = (tk.flags & 1) != 0;
    if (cref) {
        const double* cr = cx.com + size_t(tk.cidx) * 3 * NCELL + q;
        cdx = cr[0];
        cdy = cr[NCELL];
        cdz = cr[2 * NCELL];
    }
    const double rx = ((x & 1) - 0.5) * hc + cdx - par[NLOC][pc];
    const double ry = ((y & 1) - 0.5) * hc + cdy - par[NLOC + 1][pc];
    const double rz = ((z & 1) - 0.5) * hc + cdz - par[NLOC + 2][pc];
    double w[3];
    oct_rr<double>(o, -o[0] - o[3], -o[1] - o[5], rx * rx - rz * rz, ry * ry - rz * rz, 2 * rx * ry,
                   2 * rx * rz, 2 * ry * rz, w);
    const double l3rrr = rx * w[0] + ry * w[1] + rz * w[2];
    const double vx = qxx * rx + qxy * ry + qxz * rz;
    const double vy = qxy * rx + qyy * ry + qyz * rz;
    const double vz = qxz * rx + qyz * ry + qzz * rz;
    const double rLr = rx * vx + ry * vy + rz * vz;
    const double o0 = l0 + l1x * rx + l1y * ry + l1z * rz + 0.5 * rLr + (1.0 / 6.0) * l3rrr;
    const double o1x = l1x + vx + 0.5 * w[0];
    const double o1y = l1y + vy + 0.5 * w[1];
    const double o1z = l1z + vz + 0.5 * w[2];
    if (cref) {
        const double oxzz = -o[0] - o[3], oyzz = -o[1] - o[5];
        double sh[NLOC];
        sh[0] = o0;
        sh[1] = o1x;
        sh[2] = o1y;
        sh[3] = o1z;
        sh[4] = qxx + o[0] * rx + o[1] * ry + o[2] * rz;
        sh[5] = qyy + o[3] * rx + o[5] * ry + o[6] * rz;
        sh[6] = qxy + o[1] * rx + o[3] * ry + o[4] * rz;
        sh[7] = qxz + o[2] * rx + o[4] * ry + oxzz * rz;
        sh[8] = qyz + o[4] * rx + o[6] * ry + oyzz * rz;
        for (int k = 0; k < 7; ++k) sh[T_L3 + k] = o[k];
        sh[T_S] = sgx;
        sh[T_S + 1] = sgy;
        sh[T_S + 2] = sgz;
        const size_t base = size_t(tk.cidx) * NLOC * NCELL + q;
#pragma unroll
        for (int k = 0; k < NLOC; ++k) cx.Lr[base + k * NCELL] = sh[k];
    } else {
        const double* F = cx.Lf + size_t(tk.cidx) * NLEAF * NCELL + q;
        double f0 = F[0], f1 = F[1 * NCELL], f2 = F[2 * NCELL], f3 = F[3 * NCELL];
        const int n3 = tk.flags >> 4;
        for (int j = 0; j < n3; ++j) {  // class-4 slots, in order
            const double* F3 = cx.Lf3 + size_t(tk.slot3 + j) * NLEAF * NCELL + q;
            f0 += F3[0];
            f1 += F3[1 * NCELL];
            f2 += F3[2 * NCELL];
            f3 += F3[3 * NCELL];
        }
        const int io = io_index(q);
        obuf[0][io] = f0 + o0;
        obuf[1][io] = f1 - o1x + sgx;
        obuf[2][io] = f2 - o1y + sgy;
        obuf[3][io] = f3 - o1z + sgz;
    }
    if (!cref) {
        __syncthreads();
        phi[size_t(tk.cidx) * NCELL + q] = obuf[0][q];
        double* g = gout + size_t(tk.cidx) * 3 * NCELL + q;
        g[0] = obuf[1][q];
        g[NCELL] = obuf[2][q];
        g[2 * NCELL] = obuf[3][q];
    }
}

// Leaves without a parent: output their own terms (from the top-level partial
// slots under the all-pairs rule, else from the stencil kernels).
// grid: one block per leaf.
__global__ __launch_bounds__(512) void k_leaf_out(Ctx cx, const int32_t* __restrict__ list,
                                                  double* __restrict__ phi, double* __restrict__ gout) {
    __shared__ double obuf[4][NCELL];
    rho_flag_out(cx);
    const SubDev& S = cx.subs[list[blockIdx.x]];
    const int q = threadIdx.x;
    const int io = io_index(q);
    if (S.red >= 0) {
        obuf[0][io] = top_total(cx, S.red, T_L0, q);
        for (int a = 0; a < 3; ++a)
            obuf[1 + a][io] = -top_total(cx, S.red, T_L1 + a, q) + top_total(cx, S.red, T_S + a, q);
    } else {
        const double* F = cx.Lf + size_t(S.idx) * NLEAF * NCELL + q;
        for (int k = 0; k < 4; ++k) {
            double v = F[k * NCELL];
            for (int j = 0; j < S.n3; ++j) v += cx.Lf3[size_t(S.slot3 + j) * NLEAF * NCELL + k * NCELL + q];
            obuf[k][io] = v;
        }
    }
    __syncthreads();
    phi[size_t(S.idx) * NCELL + q] = obuf[0][q];
    for (int a = 0; a < 3; ++a) gout[(size_t(S.idx) * 3 + a) * NCELL + q] = obuf[1 + a][q];
}

// Density check: records the smallest index of a negative or non-finite value.
__global__ void k_check_density(const double* __restrict__ rho, int64_t n,
                                unsigned long long* __restrict__ bad) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        double v = rho[i];
        if (!(v >= 0.0) || !(v < __builtin_inf())) atomicMin(bad, (unsigned long long)i);
    }
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}


// ---------------------------------------------------------------------------
// launchers (host)
// ---------------------------------------------------------------------------
hipError_t upload_tables(const StencilTables* t, hipStream_t st) {
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tab), t, sizeof(StencilTables), 0,
                                  hipMemcpyHostToDevice, st);
}

void launch_p2m_top(const Ctx& a, const int32_t* list, int n) {
    if (n > 0) hipLaunchKernelGGL(k_p2m_top, dim3(n), dim3(512), 0, a.st, a, list);
}

void launch_m2m(const Ctx& a, const M2MTask* list, int n) {
    if (n > 0) hipLaunchKernelGGL(k_m2m, dim3(n * 8), dim3(512), 0, a.st, a, list);
}

void launch_m2m_leafpar(const Ctx& a, const M2MTask* list, int n) {
    if (n > 0) hipLaunchKernelGGL(k_m2m_leafpar, dim3(n), dim3(512), 0, a.st, a, list);
}

template <int K>
static void launch_class_k(const Ctx& a, const Item* items, int n) {
    if (a.prec == PR_MIX) hipLaunchKernelGGL((k_class<K, PR_MIX>), dim3(n), dim3(256), 0, a.st, a, items);
    else if (a.prec == PR_F32) hipLaunchKernelGGL((k_class<K, PR_F32>), dim3(n), dim3(256), 0, a.st, a, items);
    else hipLaunchKernelGGL((k_class<K, PR_F64>), dim3(n), dim3(256), 0, a.st, a, items);
}

void launch_class(const Ctx& a, int kind, const Item* items, int n) {
    if (n <= 0) return;
    switch (kind) {
        case IT_MP_REF: launch_class_k<IT_MP_REF>(a, items, n); break;
        case IT_MP_LEAF: launch_class_k<IT_MP_LEAF>(a, items, n); break;
        case IT_MONO: launch_class_k<IT_MONO>(a, items, n); break;
        default: launch_class_k<IT_TOP>(a, items, n); break;
    }
}

void launch_persist(const Ctx& a, const Item* items, const Queues& qs, int grid, int* ctr) {
    const int n = qs.begin[NQUEUE];
    if (n <= 0 || grid <= 0) return;
    if (grid > n) grid = n;
    if (a.prec == PR_MIX)
        hipLaunchKernelGGL((k_persist<PR_MIX>), dim3(grid), dim3(256), 0, a.st, a, items, qs, ctr);
    else if (a.prec == PR_F32)
        hipLaunchKernelGGL((k_persist<PR_F32>), dim3(grid), dim3(256), 0, a.st, a, items, qs, ctr);
    else hipLaunchKernelGGL((k_persist<PR_F64>), dim3(grid), dim3(256), 0, a.st, a, items, qs, ctr);
}

int persist_blocks_per_cu(int prec) {
    int nb = 0;
    hipError_t e = prec == PR_MIX   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<PR_MIX>, 256, 0)
                   : prec == PR_F32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<PR_F32>, 256, 0)
                                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<PR_F64>, 256, 0);
    return e == hipSuccess ? nb : 0;
}

void launch_l2l(const Ctx& a, const L2LTask* tasks, int n, int parent_mode, double* phi, double* g) {
    if (n <= 0) return;
    switch (a.ngroups) {
        case 1: hipLaunchKernelGGL(k_l2l<1>, dim3(n), dim3(512), 0, a.st, a, tasks, parent_mode, phi, g); break;
        case 2: hipLaunchKernelGGL(k_l2l<2>, dim3(n), dim3(512), 0, a.st, a, tasks, parent_mode, phi, g); break;
        case 3: hipLaunchKernelGGL(k_l2l<3>, dim3(n), dim3(512), 0, a.st, a, tasks, parent_mode, phi, g); break;
        case 4: hipLaunchKernelGGL(k_l2l<4>, dim3(n), dim3(512), 0, a.st, a, tasks, parent_mode, phi, g); break;
        default: hipLaunchKernelGGL(k_l2l<5>, dim3(n), dim3(512), 0, a.st, a, tasks, parent_mode, phi, g); break;
    }
}

void launch_leaf_out(const Ctx& a, const int32_t* list, int n, double* phi, double* g) {
    if (n > 0) hipLaunchKernelGGL(k_leaf_out, dim3(n), dim3(512), 0, a.st, a, list, phi, g);
}

void launch_check_density(const double* rho, int64_t n, unsigned long long* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, bad, 1, ~0ull);
    if (n > 0) hipLaunchKernelGGL(k_check_density, dim3(1024), dim3(256), 0, st, rho, n, bad);
}

void launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
}

}  // namespace fmmg
