// kernels.hip -- gfx950 kernels of the octree FMM gravity solve
// (arXiv:1908.03121, Sec. 4.3: upward pass, same-level stencil interactions
// with order-3 multipoles and the angular-momentum correction, downward pass).
//
// Thread mapping of the same-level kernels: a wavefront holds one z-plane of
// 8x8 target cells (lane = y*8 + x).  Cells of different parity use mirror
// images of one canonical stencil, so every lane of a wave walks the same
// entry list (uniform control flow, scalar table loads) with its own signs.
// Sources are staged in LDS one z-plane window (18 x 18 cells) at a time.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fmmg_internal.h"
#include "launch.h"
#include <type_traits>

namespace fmmg {

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

// internal cell index (x fastest) -> I/O index (z fastest)
__device__ __forceinline__ int io_index(int q) {
    int x = q & 7, y = (q >> 3) & 7, z = q >> 6;
    return (x * 8 + y) * 8 + z;
}

// Accumulators of one target cell.  Refined targets carry all 19 components;
// leaf targets only L0, L1 and the correction sum S.
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
    __device__ __forceinline__ void add(const Acc<Q>& o, bool full) {
        l0 += P(o.l0);
        for (int i = 0; i < 3; ++i) l1[i] += P(o.l1[i]), s[i] += P(o.s[i]);
        if (full) {
            for (int i = 0; i < 5; ++i) l2[i] += P(o.l2[i]);
            for (int i = 0; i < 7; ++i) l3[i] += P(o.l3[i]);
        }
    }
};

// M3:RR for a trace-free rank-3 tensor stored as xxx xxy xxz xyy xyz yyy yyz
template <typename P>
__device__ __forceinline__ void oct_rr(const P o[7], P XX, P YY, P ZZ, P XY, P XZ, P YZ, P w[3]) {
    P oxzz = -o[0] - o[3], oyzz = -o[1] - o[5], ozzz = -o[2] - o[6];
    w[0] = o[0] * XX + o[3] * YY + oxzz * ZZ + P(2) * (o[1] * XY + o[2] * XZ + o[4] * YZ);
    w[1] = o[1] * XX + o[5] * YY + oyzz * ZZ + P(2) * (o[3] * XY + o[4] * XZ + o[6] * YZ);
    w[2] = o[2] * XX + o[6] * YY + ozzz * ZZ + P(2) * (o[4] * XY + oxzz * XZ + oyzz * YZ);
}

// One ordered pair: source B (mass mb, trace-free quadrupole q, octupole o)
// seen from target A at separation R = X_A - X_B.  Taylor coefficients of the
// potential truncated at (source order + target order) <= 3, without the
// factor -G (applied once per target):
//   L0 += mb D0 + 1/2 q:D2 - 1/6 o:D3,  L1 += mb D1 + 1/2 q:D3,
//   L2 += mb D2,  L3 += mb D3,
//   S  += D4:(o_B - (mb/mA) o_A)   (angular-momentum correction, times -G/6)
// With trace-free tensors and D^(n) = sum of R^k delta^j terms these reduce to
//   q:D2 = d2 RqR,  (q:D3)_i = d3 R_i RqR + 2 d2 (qR)_i,  o:D3 = d3 o:RRR,
//   (D4:Q)_i = d4 R_i Q:RRR + 3 d3 (Q:RR)_i,
// where d0 = 1/r, d1 = -1/r^3, d2 = 3/r^5, d3 = -15/r^7, d4 = 105/r^9.
// FULL: refined target (L2, L3 and its own octupole oa enter).
template <bool FULL, typename P>
__device__ __forceinline__ void pair_terms(P X, P Y, P Z, P mb, const P q[5], const P o[7],
                                           P inv_ma, const P oa[7], bool corr, Acc<P>& a) {
    P r2 = X * X + Y * Y + Z * Z;
    P d0 = rsqrt_full(r2);
    P ir2 = d0 * d0;
    P d1 = -d0 * ir2;
    P d2 = P(-3) * d1 * ir2;
    P d3 = P(-5) * d2 * ir2;
    P XX = X * X, YY = Y * Y, ZZ = Z * Z, XY = X * Y, XZ = X * Z, YZ = Y * Z;
    P qzz = -q[0] - q[1];
    P ux = q[0] * X + q[2] * Y + q[3] * Z;
    P uy = q[2] * X + q[1] * Y + q[4] * Z;
    P uz = q[3] * X + q[4] * Y + qzz * Z;
    P RqR = X * ux + Y * uy + Z * uz;
    P wb[3];
    oct_rr(o, XX, YY, ZZ, XY, XZ, YZ, wb);
    P BRRR = X * wb[0] + Y * wb[1] + Z * wb[2];
    a.l0 += mb * d0 + P(0.5) * d2 * RqR - P(1.0 / 6.0) * d3 * BRRR;
    P c1 = mb * d1 + P(0.5) * d3 * RqR;
    a.l1[0] += c1 * X + d2 * ux;
    a.l1[1] += c1 * Y + d2 * uy;
    a.l1[2] += c1 * Z + d2 * uz;
    if (FULL) {
        P md1 = mb * d1, md2 = mb * d2, md3 = mb * d3;
        a.l2[0] += md2 * XX + md1;
        a.l2[1] += md2 * YY + md1;
        a.l2[2] += md2 * XY;
        a.l2[3] += md2 * XZ;
        a.l2[4] += md2 * YZ;
        P tx = md3 * XX, ty = md3 * YY;
        a.l3[0] += X * (tx + P(3) * md2);
        a.l3[1] += Y * (tx + md2);
        a.l3[2] += Z * (tx + md2);
        a.l3[3] += X * (ty + md2);
        a.l3[4] += md3 * XY * Z;
        a.l3[5] += Y * (ty + P(3) * md2);
        a.l3[6] += Z * (ty + md2);
    }
    if (corr) {
        P d4 = P(-7) * d3 * ir2;
        P Qx = wb[0], Qy = wb[1], Qz = wb[2];
        if (FULL) {
            P wa[3];
            oct_rr(oa, XX, YY, ZZ, XY, XZ, YZ, wa);
            P rho = mb * inv_ma;
            Qx -= rho * wa[0];
            Qy -= rho * wa[1];
            Qz -= rho * wa[2];
        }
        P QRRR = X * Qx + Y * Qy + Z * Qz;
        P t4 = d4 * QRRR, t3 = P(3) * d3;
        a.s[0] += t4 * X + t3 * Qx;
        a.s[1] += t4 * Y + t3 * Qy;
        a.s[2] += t4 * Z + t3 * Qz;
    }
}

// ---------------------------------------------------------------------------
// step 1: leaf P2M and M2M
// ---------------------------------------------------------------------------
// m = rho h^3 in the internal cell order.  grid: one block of 512 per leaf.
__global__ __launch_bounds__(512) void k_p2m(const double* __restrict__ rho,
                                             const SubDev* __restrict__ subs,
                                             const int32_t* __restrict__ leaf_sub,
                                             double* __restrict__ mass) {
    __shared__ double buf[NCELL];
    int leaf = blockIdx.x, t = threadIdx.x;
    double h = subs[leaf_sub[leaf]].h;
    buf[t] = rho[size_t(leaf) * NCELL + t];
    __syncthreads();
    mass[size_t(leaf) * NCELL + t] = buf[io_index(t)] * (h * h * h);
}

// Moments of the refined cells of one level from their 8 children, in one
// pass about the parent cell centre c (r0 = child COM - c):
//   m = sum m_c,  S1 = sum m_c r0,  S2 = sum (q_c + m_c r0 r0),
//   S3 = sum (o_c + sym(q_c r0) + m_c r0 r0 r0),
// then moved to the COM offset d = S1/m (binomial shift, M1 = m d):
//   M2 = S2 - m d d,   M3 = S3 - sym(S2 d) + 2 m d d d,
// and stored trace-free (children's trace parts only feed trace parts).
// grid: one block of 512 (parent cells) per refined sub-grid of the level.
__global__ __launch_bounds__(512) void k_m2m(const SubDev* __restrict__ subs,
                                             const int32_t* __restrict__ list,
                                             const double* __restrict__ mass,
                                             double* __restrict__ rec) {
    const SubDev& Ps = subs[list[blockIdx.x]];
    const int q = threadIdx.x;
    const int x = q & 7, y = (q >> 3) & 7, z = q >> 6;
    const int oct = ((x >> 2) << 2) | ((y >> 2) << 1) | (z >> 2);
    const SubDev& Cs = subs[Ps.child[oct]];
    const bool cref = Cs.kind == 1;
    const double hc = Cs.h;
    const double* crec = rec + size_t(Cs.idx) * NREC * NCELL;
    const double* cmass = mass + size_t(Cs.idx) * NCELL;
    double m = 0, s1x = 0, s1y = 0, s1z = 0;
    // S2: xx yy zz xy xz yz;  S3: xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
    double p2[6] = {0, 0, 0, 0, 0, 0};
    double p3[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 2
    for (int e = 0; e < 8; ++e) {
        const int ex = e >> 2, ey = (e >> 1) & 1, ez = e & 1;
        const int cq = (((2 * z + ez) & 7) * 8 + ((2 * y + ey) & 7)) * 8 + ((2 * x + ex) & 7);
        double w, dx = 0, dy = 0, dz = 0;
        double qxx = 0, qyy = 0, qxy = 0, qxz = 0, qyz = 0;
        double o0 = 0, o1 = 0, o2 = 0, o3 = 0, o4 = 0, o5 = 0, o6 = 0;
        if (cref) {
            w = crec[R_M * NCELL + cq];
            dx = crec[R_DX * NCELL + cq];
            dy = crec[R_DY * NCELL + cq];
            dz = crec[R_DZ * NCELL + cq];
            qxx = crec[(R_Q + 0) * NCELL + cq];
            qyy = crec[(R_Q + 1) * NCELL + cq];
            qxy = crec[(R_Q + 2) * NCELL + cq];
            qxz = crec[(R_Q + 3) * NCELL + cq];
            qyz = crec[(R_Q + 4) * NCELL + cq];
            o0 = crec[(R_O + 0) * NCELL + cq];
            o1 = crec[(R_O + 1) * NCELL + cq];
            o2 = crec[(R_O + 2) * NCELL + cq];
            o3 = crec[(R_O + 3) * NCELL + cq];
            o4 = crec[(R_O + 4) * NCELL + cq];
            o5 = crec[(R_O + 5) * NCELL + cq];
            o6 = crec[(R_O + 6) * NCELL + cq];
        } else {
            w = cmass[cq];
        }
        const double rx = (ex - 0.5) * hc + dx, ry = (ey - 0.5) * hc + dy, rz = (ez - 0.5) * hc + dz;
        const double qzz = -qxx - qyy;
        m += w;
        s1x += w * rx;
        s1y += w * ry;
        s1z += w * rz;
        p2[0] += qxx + w * rx * rx;
        p2[1] += qyy + w * ry * ry;
        p2[2] += qzz + w * rz * rz;
        p2[3] += qxy + w * rx * ry;
        p2[4] += qxz + w * rx * rz;
        p2[5] += qyz + w * ry * rz;
        p3[0] += o0 + 3 * qxx * rx + w * rx * rx * rx;
        p3[1] += o1 + qxx * ry + 2 * qxy * rx + w * rx * rx * ry;
        p3[2] += o2 + qxx * rz + 2 * qxz * rx + w * rx * rx * rz;
        p3[3] += o3 + 2 * qxy * ry + qyy * rx + w * rx * ry * ry;
        p3[4] += o4 + qxy * rz + qxz * ry + qyz * rx + w * rx * ry * rz;
        p3[5] += (-o0 - o3) + 2 * qxz * rz + qzz * rx + w * rx * rz * rz;
        p3[6] += o5 + 3 * qyy * ry + w * ry * ry * ry;
        p3[7] += o6 + qyy * rz + 2 * qyz * ry + w * ry * ry * rz;
        p3[8] += (-o1 - o5) + 2 * qyz * rz + qzz * ry + w * ry * rz * rz;
        p3[9] += (-o2 - o6) + 3 * qzz * rz + w * rz * rz * rz;
    }
    double ox = 0, oy = 0, oz = 0;
    if (m > 0) {
        const double im = 1.0 / m;
        ox = s1x * im; oy = s1y * im; oz = s1z * im;
    }
    // shift about the COM: M3 = S3 - sym(S2 d) + 2 m d d d (uses S2 before its shift)
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
    double* out = rec + size_t(Ps.idx) * NREC * NCELL;
    out[R_M * NCELL + q] = m;
    out[R_DX * NCELL + q] = ox;
    out[R_DY * NCELL + q] = oy;
    out[R_DZ * NCELL + q] = oz;
    out[(R_Q + 0) * NCELL + q] = p2[0] - tr;
    out[(R_Q + 1) * NCELL + q] = p2[1] - tr;
    out[(R_Q + 2) * NCELL + q] = p2[3];
    out[(R_Q + 3) * NCELL + q] = p2[4];
    out[(R_Q + 4) * NCELL + q] = p2[5];
    out[(R_O + 0) * NCELL + q] = p3[0] - 0.6 * tx;
    out[(R_O + 1) * NCELL + q] = p3[1] - 0.2 * ty;
    out[(R_O + 2) * NCELL + q] = p3[2] - 0.2 * tz;
    out[(R_O + 3) * NCELL + q] = p3[3] - 0.2 * tx;
    out[(R_O + 4) * NCELL + q] = p3[4];
    out[(R_O + 5) * NCELL + q] = p3[6] - 0.6 * ty;
    out[(R_O + 6) * NCELL + q] = p3[7] - 0.2 * tz;
}

// ---------------------------------------------------------------------------
// step 2: same-level interactions as work items of 256 threads (4 waves)
// ---------------------------------------------------------------------------
// LDS of one item block: the largest of the multipole plane window (16
// records x 324 cells + leaf flags), the monopole mass box (18^3) and the
// 4-wave reduction buffer (doubles).
template <typename P>
struct Smem {
    static constexpr int PLANE = NREC * PCELLS * int(sizeof(P)) + PCELLS;
    static constexpr int BOX = PW * PW * PW * int(sizeof(P));
    static constexpr int RED = 4 * NLOC * 64 * 8;
    static constexpr int A = PLANE > BOX ? PLANE : BOX;
    static constexpr int BYTES = ((A > RED ? A : RED) + 15) & ~15;
};

// Multipole item: 64 target cells (plane zt of sub-grid sid) against the
// source planes of one group of canonical dz.  All 4 waves hold the same 64
// targets and split each plane's entry list.  Refined targets: every existing
// source over the far entries, leaf sources also over the near entries
// (classes 1 + 2).  Leaf targets: refined sources over all entries (class 4).
template <bool LEAF_T, bool MIXED>
__device__ __forceinline__ void mp_item(const Ctx& cx, int sid, int zt, int group,
                                        unsigned char* smem) {
    using P = typename std::conditional<MIXED, float, double>::type;
    P* sh = reinterpret_cast<P*>(smem);
    unsigned char* leafflag = smem + NREC * PCELLS * sizeof(P);

    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index: uniform
    const int x = lane & 7, y = lane >> 3;
    const SubDev& T = cx.subs[sid];
    const double h = T.h;
    const int tidx = T.idx;
    const int q = zt * 64 + lane;
    const int sx = 1 - 2 * (x & 1), sy = 1 - 2 * (y & 1), sz = 1 - 2 * (zt & 1);

    // target data
    double mA, dAx = 0, dAy = 0, dAz = 0;
    P oa[7] = {0, 0, 0, 0, 0, 0, 0};
    if (!LEAF_T) {
        const double* r = cx.rec + size_t(tidx) * NREC * NCELL;
        mA = r[R_M * NCELL + q];
        dAx = r[R_DX * NCELL + q];
        dAy = r[R_DY * NCELL + q];
        dAz = r[R_DZ * NCELL + q];
#pragma unroll
        for (int k = 0; k < 7; ++k) oa[k] = P(r[(R_O + k) * NCELL + q]);
    } else {
        mA = cx.mass[size_t(tidx) * NCELL + q];
    }
    const P inv_ma = mA > 0 ? P(1.0 / mA) : P(0);
    const bool use_corr = cx.corr != 0;
    const bool do_near = LEAF_T ? true : ((T.flags & 1) != 0);
    const int ng = LEAF_T ? 1 : cx.ngroups;
    const int i0 = group * NDZ / ng, i1 = (group + 1) * NDZ / ng;

    Acc<double> acc;
    acc.zero();
    const P hx = P(-h * sx), hy = P(-h * sy);
    // source cell of canonical offset (dx, dy) in the plane window:
    // c = lbase + sx*dx + (sy*PW)*dy  (mirror signs per lane)
    const int lbase = (y + REACH) * PW + (x + REACH);
    const int syw = sy * PW;

    for (int gi = i0; gi < i1; ++gi) {
        const int dz = sz * (DZ0 + gi);
        const int zs = zt + dz;
        __syncthreads();
        // stage the 18x18 source window of plane zs
        {
            const int oz = zs < 0 ? -1 : (zs >= NS ? 1 : 0);
            const int lz = zs - NS * oz;
            for (int c = t; c < PCELLS; c += 256) {
                const int wx = c % PW, wy = c / PW;
                const int lx = wx - REACH, ly = wy - REACH;
                const int ox = lx < 0 ? -1 : (lx >= NS ? 1 : 0);
                const int oy = ly < 0 ? -1 : (ly >= NS ? 1 : 0);
                const int code = T.nbr[(ox + 1) * 9 + (oy + 1) * 3 + (oz + 1)];
                const int cq = (lz * NS + (ly - NS * oy)) * NS + (lx - NS * ox);
                const int kind = code < 0 ? -1 : (code & 1), nidx = code >> 1;
                if (kind == 1) {
                    const double* r = cx.rec + size_t(nidx) * NREC * NCELL + cq;
#pragma unroll
                    for (int k = 0; k < NREC; ++k) sh[k * PCELLS + c] = P(r[k * NCELL]);
                } else {
                    P mm = (kind == 0 && !LEAF_T) ? P(cx.mass[size_t(nidx) * NCELL + cq]) : P(0);
                    sh[c] = mm;
#pragma unroll
                    for (int k = 1; k < NREC; ++k) sh[k * PCELLS + c] = P(0);
                }
                if (!LEAF_T) leafflag[c] = kind == 0;
            }
        }
        __syncthreads();
        const P zoff = P(-h * dz);
        // mixed form: FP32 partial sums per source plane, flushed into the FP64
        // accumulators after the plane; FP64 form: accumulate directly
        Acc<P> part_store;
        Acc<P>& part = MIXED ? part_store : *reinterpret_cast<Acc<P>*>(&acc);
        if (MIXED) part.zero();
        auto one = [&](int e) {
            const int ent = c_tab.mp_entry[e];
            const int dxc = (ent & 255) - 8, dyc = ((ent >> 8) & 255) - 8;
            const int c = lbase + __mul24(sx, dxc) + __mul24(syw, dyc);
            P src[NREC];
#pragma unroll
            for (int k = 0; k < NREC; ++k) src[k] = sh[k * PCELLS + c];
            const P X = hx * P(dxc) + (P(dAx) - src[R_DX]);
            const P Y = hy * P(dyc) + (P(dAy) - src[R_DY]);
            const P Z = zoff + (P(dAz) - src[R_DZ]);
            pair_terms<!LEAF_T, P>(X, Y, Z, src[R_M], &src[R_Q], &src[R_O], inv_ma, oa, use_corr, part);
        };
        const int fb = c_tab.mp_far_begin[gi], fe = fb + c_tab.mp_far_count[gi];
        for (int e = fb + w; e < fe; e += 4) one(e);
        if (do_near) {
            const int nbg = c_tab.mp_near_begin[gi], ne = nbg + c_tab.mp_near_count[gi];
            for (int e = nbg + w; e < ne; e += 4) {
                if (!LEAF_T) {
                    const int ent = c_tab.mp_entry[e];
                    const int dxc = (ent & 255) - 8, dyc = ((ent >> 8) & 255) - 8;
                    const int c = lbase + __mul24(sx, dxc) + __mul24(syw, dyc);
                    if (!leafflag[c]) continue;
                }
                one(e);
            }
        }
        if (MIXED) acc.add(part, !LEAF_T);
    }

    // combine the 4 waves' partial sums in a fixed order
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);
    {
        double v[NLOC];
        v[0] = acc.l0;
        for (int i = 0; i < 3; ++i) v[T_L1 + i] = acc.l1[i];
        for (int i = 0; i < 5; ++i) v[T_L2 + i] = acc.l2[i];
        for (int i = 0; i < 7; ++i) v[T_L3 + i] = acc.l3[i];
        for (int i = 0; i < 3; ++i) v[T_S + i] = acc.s[i];
#pragma unroll
        for (int k = 0; k < NLOC; ++k) red[(w * NLOC + k) * 64 + lane] = v[k];
    }
    __syncthreads();
    const double G = cx.G;
    const double gs = use_corr ? -G / 6.0 : 0.0;
    auto sum4 = [&](int k, int l) {
        return red[(0 * NLOC + k) * 64 + l] + red[(1 * NLOC + k) * 64 + l] +
               red[(2 * NLOC + k) * 64 + l] + red[(3 * NLOC + k) * 64 + l];
    };
    if (!LEAF_T) {
        double* out = cx.Lp + size_t(group) * size_t(cx.part_stride) + size_t(tidx) * NLOC * NCELL + zt * 64;
        for (int i = t; i < NLOC * 64; i += 256) {
            const int k = i >> 6, l = i & 63;
            out[k * NCELL + l] = (k >= T_S ? gs : -G) * sum4(k, l);
        }
    } else {
        // own terms from refined sources: phi = -G L0;  g = G L1 + (-G/6) S
        double* out = cx.Lf3 + size_t(T.slot3) * NLEAF * NCELL + zt * 64;
        if (t < 64) {
            out[0 * NCELL + t] = -G * sum4(0, t);
            for (int a = 0; a < 3; ++a) out[(1 + a) * NCELL + t] = G * sum4(T_L1 + a, t) + gs * sum4(T_S + a, t);
        }
    }
}

// Monopole item: leaf targets of one sub-grid against leaf sources (class 3).
// Cell pairs lie on the lattice: R = -h d, so phi = -(G/h) sum m/|d| and
// g = (G/h^2) sum m d/|d|^3 with per-offset kernel values from tables.  The
// 18^3 box of leaf masses around the sub-grid sits in LDS.  Wave w takes the
// targets of z parity pz = w & 1 (a lane owns the 4 targets z = pz + 2k of
// its (x, y) column) and every second stencil column (w >> 1); the two
// column halves are added in a fixed order.

template <typename P>
__device__ __forceinline__ P mono_tab(int i);
template <>
__device__ __forceinline__ double mono_tab<double>(int i) { return c_tab.mono_tab[i]; }
template <>
__device__ __forceinline__ float mono_tab<float>(int i) { return c_tab.mono_tabf[i]; }

template <int PZ, int LO, int N, typename P>
__device__ __forceinline__ void mono_class(const P* __restrict__ box, int cbeg, int cend, int tab0,
                                           int cstart, int cstep, int lbase, int sx, int syw, int sy,
                                           double (&phi)[4], double (&gx)[4], double (&gy)[4],
                                           double (&gz)[4]) {
    constexpr int SZ = 1 - 2 * PZ;
    constexpr int ZMIN = SZ > 0 ? PZ + LO : PZ - (LO + N - 1);  // lowest source z
    constexpr int NSRC = N + 6;
    for (int c = cbeg + cstart; c < cend; c += cstep) {
        const int pk = c_tab.mono_col[c];
        const int dx = (pk & 255) - 8, dy = ((pk >> 8) & 255) - 8;
        const P* col = box + lbase + __mul24(sx, dx) + __mul24(syw, dy)
                       + (ZMIN + REACH) * (PW * PW);
        P m[NSRC];
#pragma unroll
        for (int j = 0; j < NSRC; ++j) m[j] = col[j * (PW * PW)];
        const int t0 = tab0 + (c - cbeg) * (3 * N);
        P s0[4] = {0, 0, 0, 0}, s1[4] = {0, 0, 0, 0}, s2[4] = {0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const P a = mono_tab<P>(t0 + 3 * i), b = mono_tab<P>(t0 + 3 * i + 1),
                    cz = mono_tab<P>(t0 + 3 * i + 2);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // target z = PZ + 2k, source z = PZ + 2k + SZ*(LO + i)
                const P mm = m[PZ + 2 * k + SZ * (LO + i) - ZMIN];
                s0[k] += mm * a;
                s1[k] += mm * b;
                s2[k] += mm * cz;
            }
        }
        const double fx = double(sx * dx), fy = double(sy * dy);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            phi[k] += double(s0[k]);
            gx[k] += fx * double(s1[k]);
            gy[k] += fy * double(s1[k]);
            gz[k] += double(SZ) * double(s2[k]);
        }
    }
}

template <int PZ, typename P>
__device__ __forceinline__ void mono_all(const P* box, int cstart, int cstep, int lbase, int sx,
                                         int syw, int sy, double (&phi)[4], double (&gx)[4],
                                         double (&gy)[4], double (&gz)[4]) {
    const int b0 = c_tab.mono_class_begin[0], b1 = c_tab.mono_class_begin[1];
    const int b2 = c_tab.mono_class_begin[2], b3 = c_tab.mono_class_begin[3];
    const int t1 = (b1 - b0) * 30, t2 = t1 + (b2 - b1) * 18;
    mono_class<PZ, -4, 10, P>(box, b0, b1, 0, cstart, cstep, lbase, sx, syw, sy, phi, gx, gy, gz);
    mono_class<PZ, -2, 6, P>(box, b1, b2, t1, cstart, cstep, lbase, sx, syw, sy, phi, gx, gy, gz);
    mono_class<PZ, 0, 2, P>(box, b2, b3, t2, cstart, cstep, lbase, sx, syw, sy, phi, gx, gy, gz);
}


template <bool MIXED>
__device__ __forceinline__ void mono_item(const Ctx& cx, int sid, unsigned char* smem) {
    using P = typename std::conditional<MIXED, float, double>::type;
    P* box = reinterpret_cast<P*>(smem);
    const int t = threadIdx.x;
    const SubDev& T = cx.subs[sid];
    __syncthreads();
    for (int c = t; c < PW * PW * PW; c += 256) {
        const int wx = c % PW, wy = (c / PW) % PW, wz = c / (PW * PW);
        const int lx = wx - REACH, ly = wy - REACH, lz = wz - REACH;
        const int ox = lx < 0 ? -1 : (lx >= NS ? 1 : 0);
        const int oy = ly < 0 ? -1 : (ly >= NS ? 1 : 0);
        const int oz = lz < 0 ? -1 : (lz >= NS ? 1 : 0);
        const int code = T.nbr[(ox + 1) * 9 + (oy + 1) * 3 + (oz + 1)];
        P mm = 0;
        if (code >= 0 && (code & 1) == 0) {
            const int cq = ((lz - NS * oz) * NS + (ly - NS * oy)) * NS + (lx - NS * ox);
            mm = P(cx.mass[size_t(code >> 1) * NCELL + cq]);
        }
        box[c] = mm;
    }
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int pz = w & 1, half = w >> 1;
    const int lane = t & 63, x = lane & 7, y = lane >> 3;
    const int sx = 1 - 2 * (x & 1), sy = 1 - 2 * (y & 1);
    const int lbase = (y + REACH) * PW + (x + REACH);
    const int syw = sy * PW;
    double phi[4] = {0, 0, 0, 0}, gx[4] = {0, 0, 0, 0}, gy[4] = {0, 0, 0, 0}, gz[4] = {0, 0, 0, 0};
    if (pz == 0) mono_all<0, P>(box, half, 2, lbase, sx, syw, sy, phi, gx, gy, gz);
    else mono_all<1, P>(box, half, 2, lbase, sx, syw, sy, phi, gx, gy, gz);
    // column half 1 hands its partial sums to half 0 through LDS
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);
    if (half == 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            red[((pz * 16) + 4 * k + 0) * 64 + lane] = phi[k];
            red[((pz * 16) + 4 * k + 1) * 64 + lane] = gx[k];
            red[((pz * 16) + 4 * k + 2) * 64 + lane] = gy[k];
            red[((pz * 16) + 4 * k + 3) * 64 + lane] = gz[k];
        }
    }
    __syncthreads();
    if (half == 0) {
        const double h = T.h, G = cx.G, gh = G / (h * h), gp = -G / h;
        double* out = cx.Lf + size_t(T.idx) * NLEAF * NCELL;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int q = (pz + 2 * k) * 64 + lane;
            out[0 * NCELL + q] = gp * (phi[k] + red[((pz * 16) + 4 * k + 0) * 64 + lane]);
            out[1 * NCELL + q] = gh * (gx[k] + red[((pz * 16) + 4 * k + 1) * 64 + lane]);
            out[2 * NCELL + q] = gh * (gy[k] + red[((pz * 16) + 4 * k + 2) * 64 + lane]);
            out[3 * NCELL + q] = gh * (gz[k] + red[((pz * 16) + 4 * k + 3) * 64 + lane]);
        }
    }
}

// Top-level tile (all-pairs rule): 64 targets (one plane of a top-level
// sub-grid) against a chunk of the tree's top-level cells; the 4 waves take
// every fourth source and their sums are added in a fixed order.  The source
// index is uniform across a wave, so source data come through scalar loads.
template <bool MIXED>
__device__ __forceinline__ void top_item(const Ctx& cx, const TopItem& it, unsigned char* smem) {
    using P = typename std::conditional<MIXED, float, double>::type;
    const SubDev& T = cx.subs[it.target];
    const int t = threadIdx.x, lane = t & 63, x = lane & 7, y = lane >> 3;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int q = it.zt * 64 + lane;
    const bool tref = T.kind == 1;
    const double h = T.h;
    const int cax = NS * T.coord[0] + x, cay = NS * T.coord[1] + y, caz = NS * T.coord[2] + it.zt;
    double mA, dAx = 0, dAy = 0, dAz = 0;
    P oa[7] = {0, 0, 0, 0, 0, 0, 0};
    if (tref) {
        const double* r = cx.rec + size_t(T.idx) * NREC * NCELL;
        mA = r[R_M * NCELL + q];
        dAx = r[R_DX * NCELL + q];
        dAy = r[R_DY * NCELL + q];
        dAz = r[R_DZ * NCELL + q];
        for (int k = 0; k < 7; ++k) oa[k] = P(r[(R_O + k) * NCELL + q]);
    } else {
        mA = cx.mass[size_t(T.idx) * NCELL + q];
    }
    const P inv_ma = mA > 0 ? P(1.0 / mA) : P(0);
    const bool use_corr = cx.corr != 0;
    Acc<P> acc;
    acc.zero();
    for (int j = it.src_begin + w; j < it.src_end; j += 4) {
        const SubDev& S = cx.subs[cx.top_src[it.src_list + (j >> 9)]];
        const int cq = j & 511;
        const int dx = NS * S.coord[0] + (cq & 7) - cax;
        const int dy = NS * S.coord[1] + ((cq >> 3) & 7) - cay;
        const int dz = NS * S.coord[2] + (cq >> 6) - caz;
        const int d2 = dx * dx + dy * dy + dz * dz;
        const bool sref = S.kind == 1;
        if (d2 == 0 || (d2 < 9 && tref && sref)) continue;
        P src[NREC];
        if (sref) {
            const double* r = cx.rec + size_t(S.idx) * NREC * NCELL + cq;
            for (int k = 0; k < NREC; ++k) src[k] = P(r[k * NCELL]);
        } else {
            src[0] = P(cx.mass[size_t(S.idx) * NCELL + cq]);
            for (int k = 1; k < NREC; ++k) src[k] = P(0);
        }
        const P X = P(-h * dx) + (P(dAx) - src[R_DX]);
        const P Y = P(-h * dy) + (P(dAy) - src[R_DY]);
        const P Z = P(-h * dz) + (P(dAz) - src[R_DZ]);
        if (tref)
            pair_terms<true, P>(X, Y, Z, src[R_M], &src[R_Q], &src[R_O], inv_ma, oa, use_corr, acc);
        else
            pair_terms<false, P>(X, Y, Z, src[R_M], &src[R_Q], &src[R_O], inv_ma, oa, use_corr, acc);
    }
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);
    {
        double v[NLOC];
        v[0] = double(acc.l0);
        for (int i = 0; i < 3; ++i) v[T_L1 + i] = double(acc.l1[i]);
        for (int i = 0; i < 5; ++i) v[T_L2 + i] = double(acc.l2[i]);
        for (int i = 0; i < 7; ++i) v[T_L3 + i] = double(acc.l3[i]);
        for (int i = 0; i < 3; ++i) v[T_S + i] = double(acc.s[i]);
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

template <bool MIXED>
__device__ __forceinline__ void run_item(const Ctx& cx, const Item& it, unsigned char* smem) {
    switch (it.kind) {
        case IT_MP_REF: mp_item<false, MIXED>(cx, it.sub, it.a, it.b, smem); break;
        case IT_MP_LEAF: mp_item<true, MIXED>(cx, it.sub, it.a, 0, smem); break;
        case IT_MONO: mono_item<MIXED>(cx, it.sub, smem); break;
        default: top_item<MIXED>(cx, cx.top_items[it.sub], smem); break;
    }
}

// One launch per class: one block per item of that class.
template <int KIND, bool MIXED>
__global__ __launch_bounds__(256) void k_class(Ctx cx, const Item* __restrict__ items) {
    using P = typename std::conditional<MIXED, float, double>::type;
    __shared__ __attribute__((aligned(16))) unsigned char smem[Smem<P>::BYTES];
    const Item it = items[blockIdx.x];
    if (KIND == IT_MP_REF) mp_item<false, MIXED>(cx, it.sub, it.a, it.b, smem);
    else if (KIND == IT_MP_LEAF) mp_item<true, MIXED>(cx, it.sub, it.a, 0, smem);
    else if (KIND == IT_MONO) mono_item<MIXED>(cx, it.sub, smem);
    else top_item<MIXED>(cx, cx.top_items[it.sub], smem);
}

// Persistent launch of every class and tree: each block takes the next item
// of the (largest-first) list from a device counter until the list is
// exhausted, so every block exits once all items are taken.
template <bool MIXED>
__global__ __launch_bounds__(256) void k_persist(Ctx cx, const Item* __restrict__ items, int n,
                                                 int* __restrict__ counter) {
    using P = typename std::conditional<MIXED, float, double>::type;
    __shared__ __attribute__((aligned(16))) unsigned char smem[Smem<P>::BYTES];
    __shared__ int s_it;
    for (;;) {
        if (threadIdx.x == 0) s_it = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_it;
        __syncthreads();
        if (it >= n) break;
        run_item<MIXED>(cx, items[it], smem);
    }
}

__global__ void k_reset_counter(int* counter) { *counter = 0; }

// Sum a top-level target's partial slots in a fixed order and scale.
// grid: (reductions x 19 components), 512 threads (cells).
__global__ __launch_bounds__(512) void k_top_reduce(Ctx cx, const TopReduce* __restrict__ reds) {
    const TopReduce R = reds[blockIdx.x / NLOC];
    const int k = blockIdx.x % NLOC;
    const SubDev& T = cx.subs[R.target];
    const int q = threadIdx.x;
    double v = 0;
    for (int p = 0; p < R.n_part; ++p) v += cx.part[(size_t(R.part_begin + p) * NLOC + k) * NCELL + q];
    const double G = cx.G, gs = cx.corr ? -G / 6.0 : 0.0;
    if (T.kind == 1) {
        cx.Lr[(size_t(T.idx) * NLOC + k) * NCELL + q] = (k >= T_S ? gs : -G) * v;
    } else {
        // leaf target: phi from L0, g = G L1 + gs S, accumulated into Lf
        double* out = cx.Lf + size_t(T.idx) * NLEAF * NCELL + q;
        if (k == 0) out[0] = -G * v;
        else if (k >= T_L1 && k < T_L1 + 3) out[(1 + k - T_L1) * NCELL] = G * v;
    }
    (void)gs;
}

// The correction part of a top-level leaf target (kept apart from the L1
// part so that each output is written by one block).
__global__ __launch_bounds__(512) void k_top_reduce_leaf_dg(Ctx cx, const TopReduce* __restrict__ reds) {
    const TopReduce R = reds[blockIdx.x];
    const SubDev& T = cx.subs[R.target];
    if (T.kind == 1 || !cx.corr) return;
    const int q = threadIdx.x;
    const double gs = -cx.G / 6.0;
    double* out = cx.Lf + size_t(T.idx) * NLEAF * NCELL + q;
    for (int a = 0; a < 3; ++a) {
        double v = 0;
        for (int p = 0; p < R.n_part; ++p) v += cx.part[(size_t(R.part_begin + p) * NLOC + T_S + a) * NCELL + q];
        out[(1 + a) * NCELL] += gs * v;
    }
}

// Level-0 refined sub-grids in the stencil-only mode: total = own.
// grid: (sub-grids x 19 components), 512 threads.
__global__ __launch_bounds__(512) void k_sum_parts(Ctx cx, const int32_t* __restrict__ list) {
    const SubDev& T = cx.subs[list[blockIdx.x / NLOC]];
    const int k = blockIdx.x % NLOC, q = threadIdx.x;
    double v = 0;
    for (int g = 0; g < cx.ngroups; ++g)
        v += cx.Lp[size_t(g) * size_t(cx.part_stride) + (size_t(T.idx) * NLOC + k) * NCELL + q];
    cx.Lr[(size_t(T.idx) * NLOC + k) * NCELL + q] = v;
}

// ---------------------------------------------------------------------------
// step 3: downward pass
// ---------------------------------------------------------------------------
// Parent expansion (L0, L1, trace-free L2, L3, correction dg) re-expanded at
// the child COM, r = X_child - X_parent:
//   o0 = L0 + L1.r + 1/2 r.L2.r + 1/6 L3:rrr,  o1 = L1 + L2.r + 1/2 L3:rr,
//   o2 = L2 + L3.r,  o3 = L3,  dg passed unchanged.
// Refined children: total = own (sum of plane groups) + shifted parent.
// Leaf children: phi = own + o0,  g = own - o1 + dg.
// grid: (refined parents at level l) x 8 child sub-grids, 512 threads.
__global__ __launch_bounds__(512) void k_l2l(Ctx cx, const int32_t* __restrict__ list,
                                             double* __restrict__ phi, double* __restrict__ gout) {
    __shared__ double obuf[4][NCELL];
    const SubDev& Ps = cx.subs[list[blockIdx.x >> 3]];
    const int e = blockIdx.x & 7;
    const SubDev& Cs = cx.subs[Ps.child[e]];
    const int q = threadIdx.x;
    const int x = q & 7, y = (q >> 3) & 7, z = q >> 6;
    const int px = (x >> 1) + 4 * (e >> 2), py = (y >> 1) + 4 * ((e >> 1) & 1), pz = (z >> 1) + 4 * (e & 1);
    const int pq = (pz * NS + py) * NS + px;
    const double* L = cx.Lr + size_t(Ps.idx) * NLOC * NCELL + pq;
    const double* pr = cx.rec + size_t(Ps.idx) * NREC * NCELL + pq;
    double l0 = L[0];
    double l1x = L[1 * NCELL], l1y = L[2 * NCELL], l1z = L[3 * NCELL];
    double qxx = L[4 * NCELL], qyy = L[5 * NCELL], qxy = L[6 * NCELL], qxz = L[7 * NCELL], qyz = L[8 * NCELL];
    double qzz = -qxx - qyy;
    double o[7];
    for (int k = 0; k < 7; ++k) o[k] = L[(T_L3 + k) * NCELL];
    double sgx = L[16 * NCELL], sgy = L[17 * NCELL], sgz = L[18 * NCELL];
    const double hc = Cs.h;
    double cdx = 0, cdy = 0, cdz = 0;
    const bool cref = Cs.kind == 1;
    if (cref) {
        const double* cr = cx.rec + size_t(Cs.idx) * NREC * NCELL + q;
        cdx = cr[R_DX * NCELL];
        cdy = cr[R_DY * NCELL];
        cdz = cr[R_DZ * NCELL];
    }
    const double rx = ((x & 1) - 0.5) * hc + cdx - pr[R_DX * NCELL];
    const double ry = ((y & 1) - 0.5) * hc + cdy - pr[R_DY * NCELL];
    const double rz = ((z & 1) - 0.5) * hc + cdz - pr[R_DZ * NCELL];
    double w[3];
    oct_rr<double>(o, rx * rx, ry * ry, rz * rz, rx * ry, rx * rz, ry * rz, w);
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
        sh[16] = sgx;
        sh[17] = sgy;
        sh[18] = sgz;
        const size_t base = size_t(Cs.idx) * NLOC * NCELL + q;
        for (int k = 0; k < NLOC; ++k) {
            double own = 0;
            for (int g = 0; g < cx.ngroups; ++g) own += cx.Lp[size_t(g) * size_t(cx.part_stride) + base + k * NCELL];
            cx.Lr[base + k * NCELL] = own + sh[k];
        }
    } else {
        const double* F = cx.Lf + size_t(Cs.idx) * NLEAF * NCELL + q;
        double f0 = F[0], f1 = F[1 * NCELL], f2 = F[2 * NCELL], f3 = F[3 * NCELL];
        if (Cs.slot3 >= 0) {
            const double* F3 = cx.Lf3 + size_t(Cs.slot3) * NLEAF * NCELL + q;
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
        phi[size_t(Cs.idx) * NCELL + q] = obuf[0][q];
        double* g = gout + size_t(Cs.idx) * 3 * NCELL + q;
        g[0] = obuf[1][q];
        g[NCELL] = obuf[2][q];
        g[2 * NCELL] = obuf[3][q];
    }
}

// Leaves without a parent: output their own terms.  grid: one block per leaf.
__global__ __launch_bounds__(512) void k_leaf_out(Ctx cx, const int32_t* __restrict__ list,
                                                  double* __restrict__ phi, double* __restrict__ gout) {
    __shared__ double obuf[4][NCELL];
    const SubDev& S = cx.subs[list[blockIdx.x]];
    const int q = threadIdx.x;
    const double* F = cx.Lf + size_t(S.idx) * NLEAF * NCELL + q;
    const int io = io_index(q);
    for (int k = 0; k < 4; ++k) {
        double v = F[k * NCELL];
        if (S.slot3 >= 0) v += cx.Lf3[size_t(S.slot3) * NLEAF * NCELL + k * NCELL + q];
        obuf[k][io] = v;
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

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v) { *p = v; }

// ---------------------------------------------------------------------------
// launchers (host)
// ---------------------------------------------------------------------------
hipError_t upload_tables(const StencilTables* t, hipStream_t st) {
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tab), t, sizeof(StencilTables), 0,
                                  hipMemcpyHostToDevice, st);
}

void launch_p2m(const Ctx& a, const double* rho, int n_leaf) {
    if (n_leaf > 0) hipLaunchKernelGGL(k_p2m, dim3(n_leaf), dim3(512), 0, a.st, rho, a.subs, a.leaf_sub, a.mass);
}

void launch_m2m(const Ctx& a, const int32_t* list, int n) {
    if (n > 0) hipLaunchKernelGGL(k_m2m, dim3(n), dim3(512), 0, a.st, a.subs, list, a.mass, a.rec);
}

template <int K>
static void launch_class_k(const Ctx& a, const Item* items, int n) {
    if (a.mixed) hipLaunchKernelGGL((k_class<K, true>), dim3(n), dim3(256), 0, a.st, a, items);
    else hipLaunchKernelGGL((k_class<K, false>), dim3(n), dim3(256), 0, a.st, a, items);
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

void launch_persist(const Ctx& a, const Item* items, int n, int* counter, int grid) {
    if (n <= 0 || grid <= 0) return;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, a.st, counter);
    if (a.mixed) hipLaunchKernelGGL((k_persist<true>), dim3(grid), dim3(256), 0, a.st, a, items, n, counter);
    else hipLaunchKernelGGL((k_persist<false>), dim3(grid), dim3(256), 0, a.st, a, items, n, counter);
}

int persist_blocks_per_cu(int mixed) {
    int nb = 0;
    hipError_t e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<true>, 256, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<false>, 256, 0);
    return e == hipSuccess ? nb : 0;
}

void launch_top_reduce(const Ctx& a, const TopReduce* reds, int n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_top_reduce, dim3(n * NLOC), dim3(512), 0, a.st, a, reds);
    hipLaunchKernelGGL(k_top_reduce_leaf_dg, dim3(n), dim3(512), 0, a.st, a, reds);
}

void launch_sum_parts(const Ctx& a, const int32_t* list, int n) {
    if (n > 0) hipLaunchKernelGGL(k_sum_parts, dim3(n * NLOC), dim3(512), 0, a.st, a, list);
}

void launch_l2l(const Ctx& a, const int32_t* list, int n, double* phi, double* g) {
    if (n > 0) hipLaunchKernelGGL(k_l2l, dim3(n * 8), dim3(512), 0, a.st, a, list, phi, g);
}

void launch_leaf_out(const Ctx& a, const int32_t* list, int n, double* phi, double* g) {
    if (n > 0) hipLaunchKernelGGL(k_leaf_out, dim3(n), dim3(512), 0, a.st, a, list, phi, g);
}

void launch_check_density(const double* rho, int64_t n, unsigned long long* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, st, bad, ~0ull);
    if (n > 0) hipLaunchKernelGGL(k_check_density, dim3(1024), dim3(256), 0, st, rho, n, bad);
}

}  // namespace fmmg
