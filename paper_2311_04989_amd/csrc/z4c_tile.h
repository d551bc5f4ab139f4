// z4c_tile.h -- device templates of the tile kernels (included by the
// per-variant translation units z4c_variants_*.hip).
#pragma once
// Tile kernels (one workgroup = one tile of TX*TY*TZ interior points of a
// MeshBlock, one point per thread).  The state fields are staged one at a
// time into LDS as a (TX+2R)(TY+2R)(TZ+2R) halo tile, R = p/2 + 1 (the
// Kreiss-Oliger half width); while a field is being differentiated the next
// field's halo tile is already in flight from HBM into registers.  Each
// field's derivatives are consumed at once in a fixed order (stage kernel:
// shift -> conformal metric -> Gamma-tilde -> chi -> lapse -> Khat, Theta ->
// At) so that the 66 first and 66 second derivatives of the Z4c right-hand
// side are never all live together, and each field's Runge-Kutta update is
// applied as soon as its right-hand side is complete.
//
// Stencils are centred, of order p = 4 or 6 (Sec. 4 uses 6), applied in
// centre-subtracted form (u_m - u_-m, u_m - u_0), mixed second derivatives
// as the first-derivative stencil applied along one axis to first
// differences along the other; Kreiss-Oliger dissipation of order p + 2 on
// every field (Sec. 4, sigma_KO).  The pointwise algebra is the standard
// Z4c system with constraint damping kappa1, kappa2 and the moving-puncture
// gauge (Sec. 2, Sec. 4), with the perfect-fluid ADM sources rho, S_i,
// S_ij (Sec. 2.1) as inputs.
//
// Arithmetic type R: double, or float with every stencil difference formed
// in double first (storage, Runge-Kutta combination and floors stay double).
#include <cmath>
#include <type_traits>
#include <utility>

#include "z4c_internal.h"

namespace z4c {
namespace tile {

constexpr double PI = 3.14159265358979323846;
constexpr int LDS_PER_CU = 163840;   // gfx950

// Symmetric 3x3 index: xx 0, xy 1, xz 2, yy 3, yz 4, zz 5.
__host__ __device__ constexpr int S(int i, int j)
{
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? b : (a == 1 ? 2 + b : 5);
}
// Weight of a symmetric component in a full double contraction.
__host__ __device__ constexpr int SW(int a) { return (a == 1 || a == 2 || a == 4) ? 2 : 1; }
__host__ __device__ constexpr int SI(int a) { return a < 3 ? 0 : (a < 5 ? 1 : 2); }
__host__ __device__ constexpr int SJ(int a) { return a == 0 ? 0 : (a == 1 ? 1 : (a == 2 ? 2 : (a == 3 ? 1 : 2))); }

// LDS x pitch: the smallest value >= lx that is 8 mod 16 doubles, so that
// neighbouring rows of a wave's 8x8 footprint fall into disjoint banks.
constexpr int pad_pitch(int lx)
{
    int p = lx;
    while (p % 16 != 8)
        ++p;
    return p;
}

// ---------------------------------------------------------------------------
// 1-D stencils on LDS (centre pointer c, compile-time stride ST), unscaled
// ---------------------------------------------------------------------------
template <int P, typename R, int ST>
__device__ __forceinline__ R d1raw(const double *c)
{
    if constexpr (P == 4) {
        return R(8) * R(c[ST] - c[-ST]) - R(c[2 * ST] - c[-2 * ST]);
    } else {
        return R(45) * R(c[ST] - c[-ST]) - R(9) * R(c[2 * ST] - c[-2 * ST])
               + R(c[3 * ST] - c[-3 * ST]);
    }
}

template <int P, typename R, int ST>
__device__ __forceinline__ R d2raw(const double *c)
{
    const double c0 = c[0];
    if constexpr (P == 4) {
        return R(16) * R((c[ST] - c0) + (c[-ST] - c0))
               - R((c[2 * ST] - c0) + (c[-2 * ST] - c0));
    } else {
        return R(270) * R((c[ST] - c0) + (c[-ST] - c0))
               - R(27) * R((c[2 * ST] - c0) + (c[-2 * ST] - c0))
               + R(2) * R((c[3 * ST] - c0) + (c[-3 * ST] - c0));
    }
}

template <int P>
__device__ __forceinline__ constexpr double w1(int m)
{
    return P == 4 ? (m == 1 ? 8.0 : -1.0) : (m == 1 ? 45.0 : (m == 2 ? -9.0 : 1.0));
}

// d_a d_b: first-derivative stencil along a applied to first differences
// along b; each second difference is formed in double.
template <int P, typename R, int SA, int SB, typename C>
__device__ __forceinline__ R dmixraw(const C &c)
{
    constexpr int Q = P / 2;
    R acc = R(0);
#pragma unroll
    for (int a = 1; a <= Q; ++a) {
        R inner = R(0);
#pragma unroll
        for (int b = 1; b <= Q; ++b) {
            const double d = (c[a * SA + b * SB] - c[a * SA - b * SB])
                           - (c[-a * SA + b * SB] - c[-a * SA - b * SB]);
            inner += R(w1<P>(b)) * R(d);
        }
        acc += R(w1<P>(a)) * inner;
    }
    return acc;
}

// Undivided difference Delta^(2r) in centre-subtracted form.
template <int P, typename R, int ST>
__device__ __forceinline__ R koraw(const double *c)
{
    const double c0 = c[0];
    if constexpr (P == 4) {
        return R(15) * R((c[ST] - c0) + (c[-ST] - c0))
               - R(6) * R((c[2 * ST] - c0) + (c[-2 * ST] - c0))
               + R((c[3 * ST] - c0) + (c[-3 * ST] - c0));
    } else {
        return -R(56) * R((c[ST] - c0) + (c[-ST] - c0))
               + R(28) * R((c[2 * ST] - c0) + (c[-2 * ST] - c0))
               - R(8) * R((c[3 * ST] - c0) + (c[-3 * ST] - c0))
               + R((c[4 * ST] - c0) + (c[-4 * ST] - c0));
    }
}

template <typename R>
struct Fac {
    R d1[3], d2[3], mix[3], ko[3];   // mix: xy, xz, yz
};


// All three operators along one axis from one set of samples: first and
// second derivative and the dissipation term.
template <int P, typename R, int ST, typename C>
__device__ __forceinline__ void axis3(const C &c, R f1, R f2, R fk, R &d1, R &d2, R &ko)
{
    const double c0 = c[0];
    double p[5], m[5];
#pragma unroll
    for (int q = 1; q <= P / 2 + 1; ++q) {
        p[q] = c[q * ST];
        m[q] = c[-q * ST];
    }
    if constexpr (P == 4) {
        d1 = (R(8) * R(p[1] - m[1]) - R(p[2] - m[2])) * f1;
        const double s1 = (p[1] - c0) + (m[1] - c0), s2 = (p[2] - c0) + (m[2] - c0),
                     s3 = (p[3] - c0) + (m[3] - c0);
        d2 = (R(16) * R(s1) - R(s2)) * f2;
        ko = (R(15) * R(s1) - R(6) * R(s2) + R(s3)) * fk;
    } else {
        d1 = (R(45) * R(p[1] - m[1]) - R(9) * R(p[2] - m[2]) + R(p[3] - m[3])) * f1;
        const double s1 = (p[1] - c0) + (m[1] - c0), s2 = (p[2] - c0) + (m[2] - c0),
                     s3 = (p[3] - c0) + (m[3] - c0), s4 = (p[4] - c0) + (m[4] - c0);
        d2 = (R(270) * R(s1) - R(27) * R(s2) + R(2) * R(s3)) * f2;
        ko = (-R(56) * R(s1) + R(28) * R(s2) - R(8) * R(s3) + R(s4)) * fk;
    }
}

// Lopsided first derivative along one axis, unscaled (same 1/(c1 h) factor
// as the centred one): the order-P stencil on the points shifted by one
// towards the side `pos` (offsets -P/2+1 .. P/2+1 when pos, mirrored
// otherwise), in differences from the centre.  Weights, exact on
// polynomials of degree <= P: order 6 (2, -24, -35, 80, -30, 8, -1) / 60 at
// offsets -2 .. 4; order 4 (-3, -10, 18, -6, 1) / 12 at offsets -1 .. 3.
template <int P, typename R, int ST, typename C>
__device__ __forceinline__ R lop1(const C &c, bool pos)
{
    const double c0 = c[0];
    double a[P / 2 + 2], b[P / 2 + 2];   // a: the shifted side, b: the other
#pragma unroll
    for (int q = 1; q <= P / 2 + 1; ++q) {
        const double pq = c[q * ST], mq = c[-q * ST];
        a[q] = pos ? pq : mq;
        b[q] = pos ? mq : pq;
    }
    R v;
    if constexpr (P == 4)
        v = -R(3) * R(b[1] - c0) + R(18) * R(a[1] - c0) - R(6) * R(a[2] - c0) + R(a[3] - c0);
    else
        v = R(2) * R(b[2] - c0) - R(24) * R(b[1] - c0) + R(80) * R(a[1] - c0)
            - R(30) * R(a[2] - c0) + R(8) * R(a[3] - c0) - R(a[4] - c0);
    return pos ? v : -v;
}

// Stencil taps addressed from the lower corner of the halo box (CO elements
// before the centre), so that every tap is a non-negative constant offset
// from one base address.
__device__ __forceinline__ int corner(int o)
{
    asm volatile("" : "+v"(o));   // keeps the rebased offset from being folded back
    return o;
}
template <int CO>
struct Corner {
    const double *b;
    __device__ __forceinline__ double operator[](int x) const { return b[CO + x]; }
};

// Ordering of LDS reads.  The backend issues every LDS read of a field at
// once unless the address of a group of reads depends on the results of the
// previous group; passing the LDS offset through an empty asm that consumes
// those results creates that dependency (no instruction is emitted), so at
// most one group of samples is live at a time.
template <typename A>
__device__ __forceinline__ int after(int off, A x)
{
    asm volatile("" : "+v"(off) : "v"(x));
    return off;
}
template <typename A, typename B, typename C, typename D>
__device__ __forceinline__ int after(int off, A x, B y, C z, D w)
{
    asm volatile("" : "+v"(off) : "v"(x), "v"(y), "v"(z), "v"(w));
    return off;
}

// First derivatives and dissipation of the field staged in L; `off` is the
// thread's stencil centre in L and is re-ordered after the reads.
// CHAIN: order the groups of LDS reads through `after` (register budget of
// two or more waves per SIMD); otherwise the compiler may issue them freely.
template <int P, typename R, int PX, int PXY, bool CHAIN = true>
__device__ __forceinline__ void first_ko(const double *L, int &off, const Fac<R> &F, R d[3], R &ko)
{
    constexpr int CO = (P / 2 + 1) * (1 + PX + PXY);
    const Corner<CO> c{L + corner(off - CO)};
    R d2x, d2y, d2z, kx, ky, kz;
    axis3<P, R, 1>(c, F.d1[0], F.d2[0], F.ko[0], d[0], d2x, kx);
    axis3<P, R, PX>(c, F.d1[1], F.d2[1], F.ko[1], d[1], d2y, ky);
    axis3<P, R, PXY>(c, F.d1[2], F.d2[2], F.ko[2], d[2], d2z, kz);
    ko = kx + ky + kz;
    if constexpr (CHAIN)
        off = after(off, d[0], d[1], d[2], ko);
}

// First and second derivatives and dissipation of the field staged in L.
template <int P, typename R, int PX, int PXY, bool CHAIN = true>
__device__ __forceinline__ void all_ko(const double *L, int &off, const Fac<R> &F, R d[3], R dd[6],
                                       R &ko)
{
    constexpr int CO = (P / 2 + 1) * (1 + PX + PXY);
    Corner<CO> c{L + corner(off - CO)};
    R kx, ky, kz;
    axis3<P, R, 1>(c, F.d1[0], F.d2[0], F.ko[0], d[0], dd[0], kx);
    axis3<P, R, PX>(c, F.d1[1], F.d2[1], F.ko[1], d[1], dd[3], ky);
    axis3<P, R, PXY>(c, F.d1[2], F.d2[2], F.ko[2], d[2], dd[5], kz);
    ko = kx + ky + kz;
    if constexpr (CHAIN) {
        off = after(off, d[0], d[1], d[2], ko);
        c.b = L + corner(off - CO);
    }
    dd[1] = dmixraw<P, R, 1, PX>(c) * F.mix[0];
    off = after(off, dd[1], ko, d[0], d[2]);   // at most two groups in flight
    c.b = L + corner(off - CO);
    dd[2] = dmixraw<P, R, 1, PXY>(c) * F.mix[1];
    if constexpr (CHAIN) {
        off = after(off, dd[2]);
        c.b = L + corner(off - CO);
    }
    dd[4] = dmixraw<P, R, PX, PXY>(c) * F.mix[2];
    if constexpr (CHAIN)
        off = after(off, dd[4]);
}

// Mixed second derivatives in two passes, x/y first (the constraint
// kernel's form; the stage kernel's z-first form follows): every
// thread first writes unscaled x- and y-first-derivative sums of the staged
// field over the tile extended by the stencil half width in the other
// directions (x sums: y and z extended; y sums: z extended); after a
// barrier, d_x d_y, d_x d_z and d_y d_z are first-derivative stencils on
// those sums (the same tensor-product stencil as dmixraw).
template <int P, int TX, int TY, int TZ>
struct MixDims {
    static constexpr int Q = P / 2;
    static constexpr int DY = TY + 2 * Q, DZ = TZ + 2 * Q;
    static constexpr int NXS = TX * DY * DZ;   // x sums
    static constexpr int NYS = TX * TY * DZ;   // y sums
};

template <int P, typename R, int TX, int TY, int TZ, int PX, int PXY>
__device__ __forceinline__ void mix_prep(const double *L, R *dxb, R *dyb, int t)
{
    using M = MixDims<P, TX, TY, TZ>;
    constexpr int NT = TX * TY * TZ, RAD = P / 2 + 1, Q = M::Q;
#pragma unroll
    for (int q = 0; q < (M::NXS + NT - 1) / NT; ++q) {
        const int e = t + q * NT;
        if ((q + 1) * NT <= M::NXS || e < M::NXS) {
            const int ex = e % TX, r = e / TX, ey = r % M::DY, ez = r / M::DY;
            dxb[e] = d1raw<P, R, 1>(L + (ez - Q + RAD) * PXY + (ey - Q + RAD) * PX + (ex + RAD));
        }
    }
#pragma unroll
    for (int q = 0; q < (M::NYS + NT - 1) / NT; ++q) {
        const int e = t + q * NT;
        if ((q + 1) * NT <= M::NYS || e < M::NYS) {
            const int ex = e % TX, r = e / TX, ey = r % TY, ez = r / TY;
            dyb[e] = d1raw<P, R, PX>(L + (ez - Q + RAD) * PXY + (ey + RAD) * PX + (ex + RAD));
        }
    }
}

template <int P, typename R, int ST>
__device__ __forceinline__ R d1sum(const R *c)
{
    if constexpr (P == 4)
        return R(8) * (c[ST] - c[-ST]) - (c[2 * ST] - c[-2 * ST]);
    else
        return R(45) * (c[ST] - c[-ST]) - R(9) * (c[2 * ST] - c[-2 * ST]) + (c[3 * ST] - c[-3 * ST]);
}

// Two-pass mixed derivatives of the stage kernel, z-pass first: zs = D_z u
// over the tile extended by Q in x and y, ys = D_y u over the tile extended
// by Q in x (unscaled sums); then xz = D_x(zs), yz = D_y(zs), xy = D_x(ys).
// A z plane of NR rows of at most 16 sums: even rows 16 apart from the
// plane's start, odd rows 16 apart from an offset of 8 mod 16, so that for
// double sums any run of two to four consecutive rows, each read at 8
// consecutive x (the 8x8 footprint of a wave), falls in distinct LDS banks
// (rows r..r+3 start at 0, 8, 16, 24 mod 32 doubles in some order);
// consecutive rows at a pitch of 14 or 12 sums would share banks.
template <int NR>
struct SumRows {
    static constexpr int OFF = 16 * ((NR + 1) / 2) + 8;
    static constexpr int PLANE = OFF + 16 * (NR / 2);
    __host__ __device__ static constexpr int row(int r) { return (r & 1) * OFF + (r >> 1) * 16; }
};

template <int P, int TX, int TY, int TZ>
struct MixDimsZ {
    static constexpr int Q = P / 2;
    static constexpr int EX = TX + 2 * Q, EY = TY + 2 * Q;
    static_assert(EX <= 16, "a row of sums spans at most 16 x");
    using ZR = SumRows<EY>;                          // z sums: EY rows per plane
    using YR = SumRows<TY>;                          // y sums: TY rows per plane
    static constexpr int NZS = ZR::PLANE * TZ;       // storage, in sums
    static constexpr int NYS = YR::PLANE * TZ;
};

// The sums from the staged tile L; ZPASS: the z sums too (else they were
// formed from the stager's registers).
template <int P, typename R, int TX, int TY, int TZ, int PX, int PXY, bool ZPASS>
__device__ __forceinline__ void mix_prep_z(const double *L, R *zs, R *ys, int t)
{
    using M = MixDimsZ<P, TX, TY, TZ>;
    constexpr int NT = TX * TY * TZ, RAD = P / 2 + 1, Q = M::Q;
    // 16 threads per row (those past EX idle): one row per 16 lanes
    if constexpr (ZPASS) {
        constexpr int NE = 16 * M::EY * TZ;
#pragma unroll
        for (int q = 0; q < (NE + NT - 1) / NT; ++q) {
            const int e = t + q * NT;
            const int ex = e % 16, r = e / 16, ey = r % M::EY, ez = r / M::EY;
            if (((q + 1) * NT <= NE || e < NE) && ex < M::EX)
                zs[ez * M::ZR::PLANE + M::ZR::row(ey) + ex] =
                    d1raw<P, R, PXY>(L + (ez + RAD) * PXY + (ey - Q + RAD) * PX + (ex - Q + RAD));
        }
    }
    constexpr int NE = 16 * TY * TZ;
#pragma unroll
    for (int q = 0; q < (NE + NT - 1) / NT; ++q) {
        const int e = t + q * NT;
        const int ex = e % 16, r = e / 16, ey = r % TY, ez = r / TY;
        if (((q + 1) * NT <= NE || e < NE) && ex < M::EX)
            ys[ez * M::YR::PLANE + M::YR::row(ey) + ex] =
                d1raw<P, R, PX>(L + (ez + RAD) * PXY + (ey + RAD) * PX + (ex - Q + RAD));
    }
}

// First derivative along y of the z sums at row r of a plane, from pe = the
// sum at row r and po = the same x at row r + 1 (rows r + k: pe + 8k for even
// k, po + 8(k - 1) for odd k); the terms as in d1sum.
template <int P, typename R>
__device__ __forceinline__ R d1sum_rows(const R *pe, const R *po)
{
    if constexpr (P == 4)
        return R(8) * (po[0] - po[-16]) - (pe[16] - pe[-16]);
    else
        return R(45) * (po[0] - po[-16]) - R(9) * (pe[16] - pe[-16]) + (po[16] - po[-32]);
}

// As all_ko (pure derivatives and dissipation from the staged tile), with
// the mixed derivatives from the z-first two-pass sums.
template <int P, typename R, int PX, int PXY, int TX, int TY, int TZ>
__device__ __forceinline__ void all_ko_sums_z(const double *L, int off, const Fac<R> &F, R d[3],
                                              R dd[6], R &ko, const R *zs, const R *ys, int tx,
                                              int ty, int tz)
{
    using M = MixDimsZ<P, TX, TY, TZ>;
    constexpr int CO = (P / 2 + 1) * (1 + PX + PXY);
    const Corner<CO> c{L + corner(off - CO)};
    R kx, ky, kz;
    axis3<P, R, 1>(c, F.d1[0], F.d2[0], F.ko[0], d[0], dd[0], kx);
    axis3<P, R, PX>(c, F.d1[1], F.d2[1], F.ko[1], d[1], dd[3], ky);
    axis3<P, R, PXY>(c, F.d1[2], F.d2[2], F.ko[2], d[2], dd[5], kz);
    ko = kx + ky + kz;
    const R *pz = zs + tz * M::ZR::PLANE + M::ZR::row(ty + M::Q) + (tx + M::Q);
    const R *pz1 = zs + tz * M::ZR::PLANE + M::ZR::row(ty + M::Q + 1) + (tx + M::Q);
    const R *py = ys + tz * M::YR::PLANE + M::YR::row(ty) + (tx + M::Q);
    dd[1] = d1sum<P, R, 1>(py) * F.mix[0];
    dd[2] = d1sum<P, R, 1>(pz) * F.mix[1];
    dd[4] = d1sum_rows<P, R>(pz, pz1) * F.mix[2];
}

// beta^k d_k of the field staged in L with lopsided derivatives.
template <int P, typename R, int PX, int PXY>
__device__ __forceinline__ R lop_adv(const double *L, int off, const Fac<R> &F, const R beta[3])
{
    constexpr int CO = (P / 2 + 1) * (1 + PX + PXY);
    const Corner<CO> c{L + corner(off - CO)};
    return beta[0] * (lop1<P, R, 1>(c, beta[0] > R(0)) * F.d1[0])
         + beta[1] * (lop1<P, R, PX>(c, beta[1] > R(0)) * F.d1[1])
         + beta[2] * (lop1<P, R, PXY>(c, beta[2] > R(0)) * F.d1[2]);
}

// Unfused helpers used by the constraint kernel.
template <int P, typename R, int PX, int PXY>
__device__ __forceinline__ void first(const double *c, const Fac<R> &F, R d[3])
{
    d[0] = d1raw<P, R, 1>(c) * F.d1[0];
    d[1] = d1raw<P, R, PX>(c) * F.d1[1];
    d[2] = d1raw<P, R, PXY>(c) * F.d1[2];
}

template <int P, typename R, int PX, int PXY>
__device__ __forceinline__ void second(const double *c, const Fac<R> &F, R dd[6])
{
    dd[0] = d2raw<P, R, 1>(c) * F.d2[0];
    dd[3] = d2raw<P, R, PX>(c) * F.d2[1];
    dd[5] = d2raw<P, R, PXY>(c) * F.d2[2];
    dd[1] = dmixraw<P, R, 1, PX>(c) * F.mix[0];
    dd[2] = dmixraw<P, R, 1, PXY>(c) * F.mix[1];
    dd[4] = dmixraw<P, R, PX, PXY>(c) * F.mix[2];
}

// As second, with the mixed derivatives from the two-pass sums of mix_prep
// (dxb, dyb) instead of the tensor-product stencil.
template <int P, typename R, int PX, int PXY, int TX, int TY, int TZ>
__device__ __forceinline__ void second_sums(const double *c, const Fac<R> &F, R dd[6],
                                            const R *dxb, const R *dyb, int tx, int ty, int tz)
{
    using M = MixDims<P, TX, TY, TZ>;
    dd[0] = d2raw<P, R, 1>(c) * F.d2[0];
    dd[3] = d2raw<P, R, PX>(c) * F.d2[1];
    dd[5] = d2raw<P, R, PXY>(c) * F.d2[2];
    const R *px = dxb + ((tz + M::Q) * M::DY + (ty + M::Q)) * TX + tx;
    const R *py = dyb + ((tz + M::Q) * TY + ty) * TX + tx;
    dd[1] = d1sum<P, R, TX>(px) * F.mix[0];
    dd[2] = d1sum<P, R, TX * M::DY>(px) * F.mix[1];
    dd[4] = d1sum<P, R, TX * TY>(py) * F.mix[2];
}

template <int P, typename R, int PX, int PXY>
__device__ __forceinline__ R dissipation(const double *c, const Fac<R> &F)
{
    return koraw<P, R, 1>(c) * F.ko[0] + koraw<P, R, PX>(c) * F.ko[1]
           + koraw<P, R, PXY>(c) * F.ko[2];
}

template <typename R>
__device__ __forceinline__ R symtrace(const R gi[6], const R t[6])
{
    return gi[0] * t[0] + gi[3] * t[3] + gi[5] * t[5]
           + R(2) * (gi[1] * t[1] + gi[2] * t[2] + gi[4] * t[4]);
}

// Logical workgroup index: consecutive logical indices on the same XCD
// (the dispatcher places workgroup w on XCD w % 8).
__device__ __forceinline__ int xcd_logical(int w, int G)
{
    const int q = G >> 3, r = G & 7;
    const int x = w & 7, k = w >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Work distribution of a tile launch.  Grid launch (a.persistent == 0): one
// workgroup per tile, workgroup w taking the tile of logical index
// xcd_logical(w), so that consecutive tiles (neighbours in one block, which
// share halo points) run on one XCD and meet in its L2.  Persistent launch: the
// tiles are cut into 8 contiguous ranges, one per XCD; a workgroup takes the
// next tile of its XCD's range from that range's counter in a.queue (zeroed
// before the launch), and once the range is exhausted the next tiles of the
// other ranges in turn, so that no XCD idles while another has tiles left.
// Every workgroup ends when all counters are exhausted.
__device__ __forceinline__ int grab_tile(const StageArgs &a)
{
    const int x0 = blockIdx.x & 7;
    for (int d = 0; d < 8; ++d) {
        const int x = (x0 + d) & 7;
        const int lo = (int)(((long long)x * a.ntiles) >> 3);
        const int hi = (int)(((long long)(x + 1) * a.ntiles) >> 3);
        if (lo >= hi)
            continue;
        const int k = atomicAdd(a.queue + x, 1);
        if (k < hi - lo)
            return lo + k;
    }
    return -1;
}

__device__ __forceinline__ int first_tile(const StageArgs &a, int t, int *slot)
{
    if (!a.persistent)
        return xcd_logical(blockIdx.x, gridDim.x);
    if (t == 0)
        *slot = grab_tile(a);
    __syncthreads();
    return *slot;
}

// Called by every thread at the end of a tile.  Every thread read the slot
// right after the barrier that published it, before the tile's staging
// barriers, so thread 0 cannot overwrite it early.
__device__ __forceinline__ int next_tile(const StageArgs &a, int t, int *slot)
{
    if (!a.persistent)
        return -1;
    if (t == 0)
        *slot = grab_tile(a);
    __syncthreads();
    return *slot;
}

// Algebraic enforcement after a stage (double): det(gt) = 1, tr(At) = 0, floors.
__device__ __forceinline__ void enforce(double v[NFIELD], double chi_floor, double alpha_floor)
{
    double g[6];
#pragma unroll
    for (int a = 0; a < 6; ++a)
        g[a] = v[GXX + a];
    double det = g[0] * (g[3] * g[5] - g[4] * g[4]) - g[1] * (g[1] * g[5] - g[4] * g[2])
               + g[2] * (g[1] * g[4] - g[3] * g[2]);
    const double f = 1.0 / cbrt(det);
#pragma unroll
    for (int a = 0; a < 6; ++a)
        g[a] *= f;
    det = g[0] * (g[3] * g[5] - g[4] * g[4]) - g[1] * (g[1] * g[5] - g[4] * g[2])
        + g[2] * (g[1] * g[4] - g[3] * g[2]);
    const double id = 1.0 / det;
    double gi[6];
    gi[0] = (g[3] * g[5] - g[4] * g[4]) * id;
    gi[1] = (g[2] * g[4] - g[1] * g[5]) * id;
    gi[2] = (g[1] * g[4] - g[2] * g[3]) * id;
    gi[3] = (g[0] * g[5] - g[2] * g[2]) * id;
    gi[4] = (g[2] * g[1] - g[0] * g[4]) * id;
    gi[5] = (g[0] * g[3] - g[1] * g[1]) * id;
    double A[6];
#pragma unroll
    for (int a = 0; a < 6; ++a)
        A[a] = v[AXX + a];
    const double tr = gi[0] * A[0] + gi[3] * A[3] + gi[5] * A[5]
                    + 2.0 * (gi[1] * A[1] + gi[2] * A[2] + gi[4] * A[4]);
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        v[GXX + a] = g[a];
        v[AXX + a] = A[a] - g[a] * tr * (1.0 / 3.0);
    }
    v[CHI] = v[CHI] > chi_floor ? v[CHI] : chi_floor;
    v[ALPHA] = v[ALPHA] > alpha_floor ? v[ALPHA] : alpha_floor;
}

// ---------------------------------------------------------------------------
// The tile kernel
// ---------------------------------------------------------------------------
template <typename Fn, int... Is>
__device__ __forceinline__ void sfor_impl(Fn &&f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
// Compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1.
template <int N, typename Fn>
__device__ __forceinline__ void sfor(Fn &&f)
{
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// Field staged after field f (-1: none).
// Field staged after field f (-1: none).  Constraints: gt, Gt, chi, Khat,
// Theta, At.  Right-hand side / stage: beta, gt, Gt, chi, alpha, Khat,
// Theta, At.
template <int MODE>
__host__ __device__ constexpr int next_field(int f)
{
    if (MODE != MODE_CONS) {
        if (f == BETAX || f == BETAY)
            return f + 1;
        if (f == BETAZ)
            return GXX;
    }
    if (f >= GXX && f < GZZ)
        return f + 1;
    if (f == GZZ)
        return GAMX;
    if (f == GAMX || f == GAMY)
        return f + 1;
    if (f == GAMZ)
        return CHI;
    if (f == CHI)
        return MODE == MODE_CONS ? KHAT : ALPHA;
    if (f == ALPHA)
        return KHAT;
    if (f == KHAT)
        return THETA;
    if (f == THETA)
        return AXX;
    if (f >= AXX && f < AZZ)
        return f + 1;
    return -1;
}

// Position of field f in the staging order (0 for the first field).
template <int MODE>
__host__ __device__ constexpr int stage_pos(int f)
{
    int g = MODE == MODE_CONS ? GXX : BETAX, p = 0;
    while (g >= 0 && g != f) {
        g = next_field<MODE>(g);
        ++p;
    }
    return p;
}

// Fields whose u1/u2 values the one-wave stage kernel requests one stage
// early: every field completed in its own stage (not Gamma-tilde, which is
// completed after Theta).
__host__ __device__ constexpr bool early_old(int f)
{
    return f >= 0 && !(f >= GAMX && f <= GAMZ);
}

template <typename R>
__device__ __forceinline__ Fac<R> load_fac(const StageArgs &a, int block)
{
    Fac<R> F;
    if constexpr (sizeof(R) == sizeof(double)) {
        const double *f = a.fac64 + 12 * block;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            F.d1[q] = f[q];
            F.d2[q] = f[3 + q];
            F.mix[q] = f[6 + q];
            F.ko[q] = f[9 + q];
        }
    } else {
        const float *f = a.fac32 + 12 * block;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            F.d1[q] = f[q];
            F.d2[q] = f[3 + q];
            F.mix[q] = f[6 + q];
            F.ko[q] = f[9 + q];
        }
    }
    return F;
}

// Halo-tile staging of one field at a time: registers <- HBM (prefetch of
// the next field), LDS <- registers (between two barriers).  Each halo
// element has a 32-bit element offset found once per tile: from the block's
// own base of field 0 for its own points and stored ghosts, the periodic
// image and the same point of `frozen`; from the state array base for
// another block's point under the neighbour rule (the plan refuses that rule
// unless such offsets stay below 2^32).  Blocks of the first kind may lie
// anywhere in the state array.
template <int NLD>
struct Stager {
    int ldo[NLD];
    unsigned src[NLD];
    unsigned valid, frz, far;   // bit q: element q is loaded / from `frozen` / from another block
    double pf[NLD];
    const double *own, *own_frozen, *all;   // u + offset, frozen + offset, u
    long long fs;

    __device__ __forceinline__ void prefetch(int f)
    {
        const long long e = (long long)f * fs;   // uniform
#pragma unroll
        for (int q = 0; q < NLD; ++q)
            pf[q] = (valid >> q) & 1u
                        ? ((far >> q) & 1u ? all + e : (frz >> q) & 1u ? own_frozen + e : own + e)[src[q]]
                        : 0.0;
    }
    __device__ __forceinline__ void store(double *lds)
    {
#pragma unroll
        for (int q = 0; q < NLD; ++q)
            if (ldo[q] >= 0)
                lds[ldo[q]] = pf[q];
    }
};

template <int NLD, int NT, int RAD, int LX, int LY, int LZ, int PX, int PXY>
__device__ __forceinline__ void setup_stager(Stager<NLD> &st, const StageArgs &a, const Tile &T,
                                             const z4c_block &B, int t)
{
    constexpr int LVOL = LX * LY * LZ;
    const int ng = B.ng;
    const int sy = B.nx + 2 * ng;
    const int sz = sy * (B.ny + 2 * ng);
    st.own = a.u + B.offset;
    st.own_frozen = a.frozen ? a.frozen + B.offset : nullptr;
    st.all = a.u;
    st.fs = B.field_stride;
    st.valid = 0u;
    st.frz = 0u;
    st.far = 0u;
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        const int e = t + q * NT;
        st.ldo[q] = -1;
        st.src[q] = 0u;
        if (e < LVOL) {
            const int lx = e % LX, r1 = e / LX, ly = r1 % LY, lz = r1 / LY;
            const int gi = T.i0 - RAD + lx, gj = T.j0 - RAD + ly, gk = T.k0 - RAD + lz;
            st.ldo[q] = lz * PXY + ly * PX + lx;
            if (gi >= -ng && gi < B.nx + ng && gj >= -ng && gj < B.ny + ng && gk >= -ng
                && gk < B.nz + ng) {
                const int ox = gi < 0 ? -1 : (gi >= B.nx ? 1 : 0);
                const int oy = gj < 0 ? -1 : (gj >= B.ny ? 1 : 0);
                const int oz = gk < 0 ? -1 : (gk >= B.nz ? 1 : 0);
                unsigned idx = (unsigned)((gk + ng) * sz + (gj + ng) * sy + (gi + ng));
                if ((ox | oy | oz) != 0 && a.halo != Z4C_GHOST_NONE) {
                    int sb = -1;
                    if (a.halo == Z4C_GHOST_PERIODIC)
                        sb = T.block;
                    else if (a.halo == Z4C_GHOST_NEIGHBOUR)
                        sb = a.nbr[T.block * 27 + (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)];
                    if (sb >= 0) {
                        // same nx, ny, nz, ng and field stride as this block
                        const int si = gi - ox * B.nx, sj = gj - oy * B.ny, sk = gk - oz * B.nz;
                        idx = (unsigned)((sk + ng) * sz + (sj + ng) * sy + (si + ng));
                        if (sb != T.block) {
                            idx += (unsigned)a.blocks[sb].offset;
                            st.far |= 1u << q;
                        }
                    } else if (a.frozen) {
                        st.frz |= 1u << q;
                    }   // else: the stored ghost, which a refresh leaves as it is
                }
                st.src[q] = idx;
                st.valid |= 1u << q;
            }
        }
    }
}

// Element at byte offset `boff` from a (wave-uniform) base: a 32-bit offset
// added to a scalar base, the addressing form that needs no 64-bit per-lane
// address.
__device__ __forceinline__ const double &at(const double *b, unsigned boff)
{
    return *(const double *)((const char *)b + boff);
}
__device__ __forceinline__ double &at(double *b, unsigned boff)
{
    return *(double *)((char *)b + boff);
}

// Halo-tile staging for the stage kernel: as Stager, with the per-element
// sources kept in LDS (one 32-bit word per element and thread) and the LDS
// destination recomputed from the thread index, so that only the prefetched
// values occupy registers across the kernel.  A source word is the byte
// offset of the element from the block's own base (its own points and
// stored ghosts, a periodic image, or the same point of the frozen array);
// for a point of another block (neighbour rule) it is the element offset
// from the array base.  Elements beyond the stored region of the block
// (ragged tiles) are clamped to an in-bounds point: no active point's
// stencil reaches them.
template <int NLD, int NT, int LX, int LY, int LZ, int PX, int PXY, bool GEN>
struct LStager {
    static constexpr int LVOL = LX * LY * LZ;
    double pf[NLD];
    const double *own, *own_frozen, *all;   // u + offset, frozen + offset, u (uniform)
    long long fs;
    const unsigned *src;                    // LDS, src[q * NT + t]
    unsigned frz, far;                      // bit q: from `frozen` / from another block

    __device__ __forceinline__ void prefetch(int f, int t)
    {
        const double *bo = own + (long long)f * fs;
        const unsigned sp = frz | far;
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            if ((q + 1) * NT <= LVOL || t + q * NT < LVOL) {
                const unsigned o = src[q * NT + t];
                if (GEN && ((sp >> q) & 1u)) {
                    pf[q] = (far >> q) & 1u ? (all + (long long)f * fs)[o]
                                            : at(own_frozen + (long long)f * fs, o);
                    asm volatile("");   // keeps the two loads apart (uniform base below)
                } else {
                    pf[q] = at(bo, o);
                }
            }
        }
    }
    // NAIVE: the values are rounded to float on their way into the tile, so
    // that every stencil difference is one of float samples (the naive
    // FP32 form, kept for precision comparisons).
    template <bool NAIVE = false>
    __device__ __forceinline__ void store(double *lds, int t)
    {
        if constexpr (LX * LY == NT && NLD == LZ) {
            // one z-column per thread: element q at z = q, PXY apart
            double *col = lds + (t / LX) * PX + t % LX;
#pragma unroll
            for (int q = 0; q < NLD; ++q)
                col[q * PXY] = NAIVE ? double(float(pf[q])) : pf[q];
            return;
        }
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = t + q * NT;
            if ((q + 1) * NT <= LVOL || e < LVOL) {
                const int lx = e % LX, r1 = e / LX, ly = r1 % LY, lz = r1 / LY;
                lds[lz * PXY + ly * PX + lx] = NAIVE ? double(float(pf[q])) : pf[q];
            }
        }
    }
};

// GEN: sources may be frozen or other blocks' points (frozen and neighbour
// rules); otherwise every source is a point of the block itself.
template <int NLD, int NT, int RAD, int LX, int LY, int LZ, int PX, int PXY, bool GEN>
__device__ __forceinline__ void setup_lstager(LStager<NLD, NT, LX, LY, LZ, PX, PXY, GEN> &st,
                                              unsigned *src, const StageArgs &a, const Tile &T,
                                              const z4c_block &B, int t)
{
    constexpr int LVOL = LX * LY * LZ;
    const int ng = B.ng;
    const int sy = B.nx + 2 * ng;
    const int sz = sy * (B.ny + 2 * ng);
    const bool rule = a.halo != Z4C_GHOST_NONE;
    st.own = a.u + B.offset;
    st.own_frozen = a.frozen ? a.frozen + B.offset : nullptr;
    st.all = a.u;
    st.fs = B.field_stride;
    st.src = src;
    st.frz = 0u;
    st.far = 0u;
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        const int e = t + q * NT;
        if ((q + 1) * NT <= LVOL || e < LVOL) {
            const int lx = e % LX, r1 = e / LX, ly = r1 % LY, lz = r1 / LY;
            int gi = T.i0 - RAD + lx, gj = T.j0 - RAD + ly, gk = T.k0 - RAD + lz;
            gi = gi < B.nx + ng ? gi : B.nx + ng - 1;
            gj = gj < B.ny + ng ? gj : B.ny + ng - 1;
            gk = gk < B.nz + ng ? gk : B.nz + ng - 1;
            const int ox = gi < 0 ? -1 : (gi >= B.nx ? 1 : 0);
            const int oy = gj < 0 ? -1 : (gj >= B.ny ? 1 : 0);
            const int oz = gk < 0 ? -1 : (gk >= B.nz ? 1 : 0);
            unsigned w = 8u * (unsigned)((gk + ng) * sz + (gj + ng) * sy + (gi + ng));
            if ((ox | oy | oz) != 0 && rule) {
                int sb = -1;
                if (a.halo == Z4C_GHOST_PERIODIC)
                    sb = T.block;
                else if (GEN && a.halo == Z4C_GHOST_NEIGHBOUR)
                    sb = a.nbr[T.block * 27 + (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)];
                if (sb >= 0) {
                    // same nx, ny, nz, ng and field stride as this block
                    const int si = gi - ox * B.nx, sj = gj - oy * B.ny, sk = gk - oz * B.nz;
                    const unsigned loc = (unsigned)((sk + ng) * sz + (sj + ng) * sy + (si + ng));
                    if (sb == T.block) {
                        w = 8u * loc;
                    } else {
                        w = (unsigned)a.blocks[sb].offset + loc;
                        st.far |= 1u << q;
                    }
                } else if (GEN && a.frozen) {
                    st.frz |= 1u << q;
                }   // else: the stored ghost, which a refresh leaves as it is
            }
            src[q * NT + t] = w;
        }
    }
}

template <int P, int TX, int TY, int TZ, typename R, int MODE>
__global__ void __launch_bounds__(TX *TY *TZ) cons_kernel(const StageArgs a)
{
    constexpr int RAD = P / 2 + 1;
    constexpr int NT = TX * TY * TZ;
    constexpr int LX = TX + 2 * RAD, LY = TY + 2 * RAD, LZ = TZ + 2 * RAD;
    constexpr int PX = pad_pitch(LX);
    constexpr int PXY = PX * LY;
    constexpr int LVOL = LX * LY * LZ;
    constexpr int NLD = (LVOL + NT - 1) / NT;
    constexpr bool CONS = MODE == MODE_CONS;
    __shared__ double lds[PXY * LZ];
    __shared__ double red[(NT / 64) * 16];
    // mixed second derivatives of chi and gt in two passes (as the stage
    // kernel at one wave per SIMD): x and y first-derivative sums here
    using MD = MixDims<P, TX, TY, TZ>;
    __shared__ R dxb[MD::NXS];
    __shared__ R dyb[MD::NYS];

    const int t = threadIdx.x;
    const int tx = t % TX, ty = (t / TX) % TY, tz = t / (TX * TY);
    const double *lc = lds + (tz + RAD) * PXY + (ty + RAD) * PX + (tx + RAD);

    __shared__ int tile_slot;
    for (int tile = first_tile(a, t, &tile_slot); tile >= 0; tile = next_tile(a, t, &tile_slot)) {
        const Tile T = a.tiles[tile];
        const z4c_block B = a.blocks[T.block];
        const int ng = B.ng;
        const int sy = B.nx + 2 * ng;
        const int sz = sy * (B.ny + 2 * ng);
        const int i = T.i0 + tx, j = T.j0 + ty, k = T.k0 + tz;
        const bool active = i < B.nx && j < B.ny && k < B.nz;
        const int pt = (k + ng) * sz + (j + ng) * sy + (i + ng);
        const double *ub = a.u + B.offset;
        const long long fs = B.field_stride;

        Stager<NLD> st;
        setup_stager<NLD, NT, RAD, LX, LY, LZ, PX, PXY>(st, a, T, B, t);
        auto stage = [&](auto FC) __attribute__((always_inline)) {
            constexpr int FF = decltype(FC)::value;
            constexpr int NX = next_field<MODE>(FF);
            __syncthreads();
            st.store(lds);
            if constexpr (NX >= 0)
                st.prefetch(NX);
            __syncthreads();
            if constexpr (FF == CHI || (FF >= GXX && FF <= GZZ)) {
                mix_prep<P, R, TX, TY, TZ, PX, PXY>(lds, dxb, dyb, t);
                __syncthreads();
            }
        };

        st.prefetch(GXX);

        const Fac<R> F = load_fac<R>(a, T.block);
        auto centre = [&](int f) __attribute__((always_inline)) { return active ? R(ub[f * fs + pt]) : R(0); };

        // Conformal metric, its inverse; shift, conformal factor, lapse.
        R g[6];
        sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { g[q] = active ? R(ub[(GXX + q) * fs + pt]) : ((q == 0 || q == 3 || q == 5) ? R(1) : R(0)); } });
        R gi[6];
        {
            const R det = g[0] * (g[3] * g[5] - g[4] * g[4]) - g[1] * (g[1] * g[5] - g[4] * g[2])
                        + g[2] * (g[1] * g[4] - g[3] * g[2]);
            const R id = R(1) / det;
            gi[0] = (g[3] * g[5] - g[4] * g[4]) * id;
            gi[1] = (g[2] * g[4] - g[1] * g[5]) * id;
            gi[2] = (g[1] * g[4] - g[2] * g[3]) * id;
            gi[3] = (g[0] * g[5] - g[2] * g[2]) * id;
            gi[4] = (g[2] * g[1] - g[0] * g[4]) * id;
            gi[5] = (g[0] * g[3] - g[1] * g[1]) * id;
        }
        const R beta[3] = {centre(BETAX), centre(BETAY), centre(BETAZ)};
        const R chi = active ? R(ub[CHI * fs + pt]) : R(1);
        const R alpha = active ? R(ub[ALPHA * fs + pt]) : R(1);
        const R chis = chi > R(a.chi_floor) ? chi : R(a.chi_floor);
        const R ichi2 = R(0.5) / chis;          // 1 / (2 chi)
        const R kap1 = R(a.kappa1), kap2 = R(a.kappa2);

        R rhs[NFIELD];
        sfor<NFIELD>([&](auto f_c) __attribute__((always_inline)) { constexpr int f = decltype(f_c)::value; { rhs[f] = R(0); } });
        R cons[NCONS];
        sfor<NCONS>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { cons[q] = R(0); } });

        auto adv = [&](const R d[3]) __attribute__((always_inline)) { return beta[0] * d[0] + beta[1] * d[1] + beta[2] * d[2]; };

        // ---- conformal metric: d gt, d d gt -> Rt_ij (second-derivative part)
        R dg[3][6];
        R Rij[6];
        sfor<6>([&](auto Q) __attribute__((always_inline)) {
            constexpr int q = decltype(Q)::value;
            stage(std::integral_constant<int, GXX + q>{});
            if (active) {
                R d[3], dd[6];
                first<P, R, PX, PXY>(lc, F, d);
                second_sums<P, R, PX, PXY, TX, TY, TZ>(lc, F, dd, dxb, dyb, tx, ty, tz);
                sfor<3>([&](auto kk_c) __attribute__((always_inline)) { constexpr int kk = decltype(kk_c)::value; { dg[kk][q] = d[kk]; } });
                Rij[q] = R(-0.5) * symtrace(gi, dd);
                if constexpr (!CONS)
                    rhs[GXX + q] += adv(d) + dissipation<P, R, PX, PXY>(lc, F);
            }
        });

        // Christoffel symbols: Gl[k][ij] = Gt_{k ij}, Gu[k][ij] = Gt^k_{ij}, Gd^i.
        R Gu[3][6], Gd[3];
        if (active) {
            R Gl[3][6];
            sfor<3>([&](auto kk_c) __attribute__((always_inline)) { constexpr int kk = decltype(kk_c)::value; {                 sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
                    const int ii = SI(q), jj = SJ(q);
                    Gl[kk][q] = R(0.5) * (dg[ii][S(jj, kk)] + dg[jj][S(ii, kk)] - dg[kk][q]);
                } }); } });
            sfor<3>([&](auto kk_c) __attribute__((always_inline)) { constexpr int kk = decltype(kk_c)::value; {                 sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { Gu[kk][q] = gi[S(kk, 0)] * Gl[0][q] + gi[S(kk, 1)] * Gl[1][q]
                              + gi[S(kk, 2)] * Gl[2][q]; } }); } });
            sfor<3>([&](auto ii_c) __attribute__((always_inline)) { constexpr int ii = decltype(ii_c)::value; { Gd[ii] = symtrace(gi, Gu[ii]); } });
            // Rt_ij += 1/2 Gd^k (Gt_{ijk} + Gt_{jik})
            //        + sum_kl (Gu^k_{li} T_{jk}^l + Gu^k_{lj} T_{ik}^l + Gu^k_{il} T_{kj}^l),
            // T_{ab}^c = gt^{cm} Gt_{a bm}
            sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
                const int ii = SI(q), jj = SJ(q);
                R s = R(0);
                sfor<3>([&](auto kk_c) __attribute__((always_inline)) { constexpr int kk = decltype(kk_c)::value; { s += R(0.5) * Gd[kk] * (Gl[ii][S(jj, kk)] + Gl[jj][S(ii, kk)]); } });
                Rij[q] += s;
            } });
            sfor<3>([&](auto p0_c) __attribute__((always_inline)) { constexpr int p0 = decltype(p0_c)::value; {                 sfor<3>([&](auto p1_c) __attribute__((always_inline)) { constexpr int p1 = decltype(p1_c)::value; {
                    R Tc[3];
                    sfor<3>([&](auto p2_c) __attribute__((always_inline)) { constexpr int p2 = decltype(p2_c)::value; { Tc[p2] = gi[S(p2, 0)] * Gl[p0][S(p1, 0)] + gi[S(p2, 1)] * Gl[p0][S(p1, 1)]
                               + gi[S(p2, 2)] * Gl[p0][S(p1, 2)]; } });
                    // T_{p0 p1}^{l}: contributes as T_{jk}^l (j=p0, k=p1),
                    // T_{ik}^l (i=p0, k=p1) and T_{kj}^l (k=p0, j=p1)
                    sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
                        const int ii = SI(q), jj = SJ(q);
                        R s = R(0);
                        sfor<3>([&](auto l_c) __attribute__((always_inline)) { constexpr int l = decltype(l_c)::value; {
                            if (jj == p0)
                                s += Gu[p1][S(l, ii)] * Tc[l];
                            if (ii == p0)
                                s += Gu[p1][S(l, jj)] * Tc[l];
                            if (jj == p1)
                                s += Gu[p0][S(ii, l)] * Tc[l];
                        } });
                        Rij[q] += s;
                    } });
                } }); } });
        }

        // ---- Gamma-tilde: d_j Gt^k -> Rt_ij; damping; Z^i
        sfor<3>([&](auto KK) __attribute__((always_inline)) {
            constexpr int kk = decltype(KK)::value;
            stage(std::integral_constant<int, GAMX + kk>{});
            if (active) {
                R d[3];
                first<P, R, PX, PXY>(lc, F, d);
                sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
                    const int ii = SI(q), jj = SJ(q);
                    Rij[q] += R(0.5) * (g[S(kk, ii)] * d[jj] + g[S(kk, jj)] * d[ii]);
                } });
                const R Gam = R(lc[0]);
                if constexpr (!CONS) {
                    rhs[GAMX + kk] += adv(d) + dissipation<P, R, PX, PXY>(lc, F)
                                    - R(2) * alpha * kap1 * (Gam - Gd[kk]);
                    rhs[BETAX + kk] += (a.shift == Z4C_SHIFT_GAMMADRIVER ? Gam : R(0));
                } else {
                    cons[C_ZX + kk] = R(0.5) * (Gam - Gd[kk]);
                }
            }
        });

        // ---- chi: R^chi_ij
        R dchi[3];
        stage(std::integral_constant<int, CHI>{});
        if (active) {
            R dd[6];
            first<P, R, PX, PXY>(lc, F, dchi);
            second_sums<P, R, PX, PXY, TX, TY, TZ>(lc, F, dd, dxb, dyb, tx, ty, tz);
            R DD[6];
            sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { DD[q] = dd[q] - (Gu[0][q] * dchi[0] + Gu[1][q] * dchi[1] + Gu[2][q] * dchi[2]); } });
            const R trDD = symtrace(gi, DD);
            R dc2[6];
            sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { dc2[q] = dchi[SI(q)] * dchi[SJ(q)]; } });
            const R dchi2 = symtrace(gi, dc2);
            const R i4c2 = ichi2 * ichi2;   // 1 / (4 chi^2)
            sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { Rij[q] += (DD[q] + g[q] * trDD) * ichi2 - (dc2[q] + R(3) * g[q] * dchi2) * i4c2; } });
            if constexpr (!CONS)
                rhs[CHI] += adv(dchi) + dissipation<P, R, PX, PXY>(lc, F);
        }

        // ---- lapse: D_i D_j alpha (RHS / stage only)
        R dal[3], DDa[6];
        R D2a = R(0);
        if constexpr (!CONS) {
            stage(std::integral_constant<int, ALPHA>{});
            if (active) {
                R dd[6];
                first<P, R, PX, PXY>(lc, F, dal);
                second<P, R, PX, PXY>(lc, F, dd);
                R ca = R(0);   // gt^{kl} d_k chi d_l alpha
                sfor<3>([&](auto p0_c) __attribute__((always_inline)) { constexpr int p0 = decltype(p0_c)::value; {                     sfor<3>([&](auto p1_c) __attribute__((always_inline)) { constexpr int p1 = decltype(p1_c)::value; { ca += gi[S(p0, p1)] * dchi[p0] * dal[p1]; } }); } });
                sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
                    const int ii = SI(q), jj = SJ(q);
                    DDa[q] = dd[q] - (Gu[0][q] * dal[0] + Gu[1][q] * dal[1] + Gu[2][q] * dal[2])
                           + (dchi[ii] * dal[jj] + dchi[jj] * dal[ii] - g[q] * ca) * ichi2;
                } });
                D2a = chi * symtrace(gi, DDa);
                rhs[ALPHA] += (a.advect_gauge ? adv(dal) : R(0))
                            + dissipation<P, R, PX, PXY>(lc, F);
            }
        }

        // ---- Khat, Theta (their Gamma-tilde source terms)
        R KT[2];
        sfor<2>([&](auto Q) __attribute__((always_inline)) {
            constexpr int q = decltype(Q)::value;
            stage(std::integral_constant<int, q == 0 ? KHAT : THETA>{});
            if (active) {
                R d[3];
                first<P, R, PX, PXY>(lc, F, d);
                KT[q] = R(lc[0]);
                if constexpr (!CONS) {
                    const R c = q == 0 ? R(-4.0 / 3.0) * alpha : R(-2.0 / 3.0) * alpha;
                    sfor<3>([&](auto ii_c) __attribute__((always_inline)) { constexpr int ii = decltype(ii_c)::value; { rhs[GAMX + ii] += c * (gi[S(ii, 0)] * d[0] + gi[S(ii, 1)] * d[1]
                                               + gi[S(ii, 2)] * d[2]); } });
                    rhs[q == 0 ? KHAT : THETA] += adv(d) + dissipation<P, R, PX, PXY>(lc, F);
                } else {
                    const R c = q == 0 ? R(-2.0 / 3.0) : R(-4.0 / 3.0);
                    sfor<3>([&](auto ii_c) __attribute__((always_inline)) { constexpr int ii = decltype(ii_c)::value; { cons[C_MX + ii] += c * d[ii]; } });
                }
            }
        });

        // ---- pointwise algebra
        R A[6];
        if (active) {
            const R Khat = KT[0], Theta = KT[1];
            sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { A[q] = R(ub[(AXX + q) * fs + pt]); } });
            R rho = R(0), Si[3] = {R(0), R(0), R(0)}, Sij[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
            if (a.matter) {
                const double *mb = a.matter + B.moffset;
                rho = R(mb[pt]);
                sfor<3>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { Si[q] = R(mb[(1 + q) * fs + pt]); } });
                sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { Sij[q] = R(mb[(4 + q) * fs + pt]); } });
            }
            // At^i_j and At^{ij}
            R Amix[3][3];
            sfor<3>([&](auto ii_c) __attribute__((always_inline)) { constexpr int ii = decltype(ii_c)::value; {                 sfor<3>([&](auto jj_c) __attribute__((always_inline)) { constexpr int jj = decltype(jj_c)::value; { Amix[ii][jj] = gi[S(ii, 0)] * A[S(0, jj)] + gi[S(ii, 1)] * A[S(1, jj)]
                                 + gi[S(ii, 2)] * A[S(2, jj)]; } }); } });
            R Aup[6];
            sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
                const int ii = SI(q), jj = SJ(q);
                Aup[q] = Amix[ii][0] * gi[S(0, jj)] + Amix[ii][1] * gi[S(1, jj)]
                       + Amix[ii][2] * gi[S(2, jj)];
            } });
            R AA = R(0);
            sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { AA += R(SW(q)) * A[q] * Aup[q]; } });
            const R K = Khat + R(2) * Theta;
            const R Rs = chi * symtrace(gi, Rij);
            const R pi = R(PI);
            if constexpr (!CONS) {
                const R trS = chi * symtrace(gi, Sij);
                R X[6];
                sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { X[q] = -DDa[q] + alpha * (Rij[q] - R(8) * pi * Sij[q]); } });
                const R trX = symtrace(gi, X);
                rhs[CHI] += R(2.0 / 3.0) * chi * alpha * K;
                sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
                    const int ii = SI(q), jj = SJ(q);
                    rhs[GXX + q] += R(-2) * alpha * A[q];
                    const R AAm = A[S(ii, 0)] * Amix[0][jj] + A[S(ii, 1)] * Amix[1][jj]
                                + A[S(ii, 2)] * Amix[2][jj];
                    rhs[AXX + q] += chi * (X[q] - g[q] * trX * R(1.0 / 3.0))
                                  + alpha * (K * A[q] - R(2) * AAm);
                } });
                rhs[KHAT] += -D2a + alpha * (AA + K * K * R(1.0 / 3.0))
                           + R(4) * pi * alpha * (trS + rho) + alpha * kap1 * (R(1) - kap2) * Theta;
                rhs[THETA] += R(0.5) * alpha * (Rs - AA + R(2.0 / 3.0) * K * K)
                            - alpha * (R(8) * pi * rho + kap1 * (R(2) + kap2) * Theta);
                sfor<3>([&](auto ii_c) __attribute__((always_inline)) { constexpr int ii = decltype(ii_c)::value; {
                    R gA = R(0);
                    sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { gA += R(SW(q)) * Gu[ii][q] * Aup[q]; } });
                    const R Ad = Aup[S(ii, 0)] * dal[0] + Aup[S(ii, 1)] * dal[1]
                               + Aup[S(ii, 2)] * dal[2];
                    const R Ac = Aup[S(ii, 0)] * dchi[0] + Aup[S(ii, 1)] * dchi[1]
                               + Aup[S(ii, 2)] * dchi[2];
                    const R gS = gi[S(ii, 0)] * Si[0] + gi[S(ii, 1)] * Si[1] + gi[S(ii, 2)] * Si[2];
                    rhs[GAMX + ii] += R(-2) * Ad
                                    + R(2) * alpha * (gA - R(1.5) / chis * Ac - R(8) * pi * gS);
                } });
                R muL = R(0);
                if (a.lapse == Z4C_LAPSE_1PLUSLOG)
                    muL = R(2) * alpha;
                else if (a.lapse == Z4C_LAPSE_HARMONIC)
                    muL = alpha * alpha;
                rhs[ALPHA] += -muL * Khat;
                const R eta = R(a.eta);
                sfor<3>([&](auto ii_c) __attribute__((always_inline)) { constexpr int ii = decltype(ii_c)::value; { rhs[BETAX + ii] += -eta * beta[ii]; } });
            } else {
                cons[C_H] = Rs + R(2.0 / 3.0) * K * K - AA - R(16) * pi * rho;
                cons[C_THETA] = Theta;
                sfor<3>([&](auto ii_c) __attribute__((always_inline)) { constexpr int ii = decltype(ii_c)::value; {
                    R s = R(0);
                    sfor<3>([&](auto jj_c) __attribute__((always_inline)) { constexpr int jj = decltype(jj_c)::value; {                         sfor<3>([&](auto kk_c) __attribute__((always_inline)) { constexpr int kk = decltype(kk_c)::value; {
                            R c2 = R(0);
                            sfor<3>([&](auto l_c) __attribute__((always_inline)) { constexpr int l = decltype(l_c)::value; { c2 += Gu[l][S(jj, kk)] * A[S(l, ii)] + Gu[l][S(jj, ii)] * A[S(kk, l)]; } });
                            s += gi[S(jj, kk)] * c2;
                        } }); } });
                    const R Ac = Amix[0][ii] * dchi[0] + Amix[1][ii] * dchi[1]
                               + Amix[2][ii] * dchi[2];
                    cons[C_MX + ii] += -s - R(1.5) / chis * Ac - R(8) * pi * Si[ii];
                } });
            }
        }

        // ---- At_ij
        sfor<6>([&](auto Q) __attribute__((always_inline)) {
            constexpr int q = decltype(Q)::value;
            stage(std::integral_constant<int, AXX + q>{});
            if (active) {
                R d[3];
                first<P, R, PX, PXY>(lc, F, d);
                if constexpr (!CONS) {
                    rhs[AXX + q] += adv(d) + dissipation<P, R, PX, PXY>(lc, F);
                } else {
                    constexpr int ii = SI(q), jj = SJ(q);
                    cons[C_MX + ii] += gi[S(jj, 0)] * d[0] + gi[S(jj, 1)] * d[1] + gi[S(jj, 2)] * d[2];
                    if constexpr (ii != jj)
                        cons[C_MX + jj] += gi[S(ii, 0)] * d[0] + gi[S(ii, 1)] * d[1]
                                         + gi[S(ii, 2)] * d[2];
                }
            }
        });

        // ---- shift: d d beta terms of Gamma-tilde, Lie derivative terms
        if constexpr (!CONS) {
            R db[3][3];   // db[k][j] = d_j beta^k
            sfor<3>([&](auto KK) __attribute__((always_inline)) {
                constexpr int kk = decltype(KK)::value;
                stage(std::integral_constant<int, BETAX + kk>{});
                if (active) {
                    R d[3], dd[6];
                    first<P, R, PX, PXY>(lc, F, d);
                    second<P, R, PX, PXY>(lc, F, dd);
                    sfor<3>([&](auto jj_c) __attribute__((always_inline)) { constexpr int jj = decltype(jj_c)::value; { db[kk][jj] = d[jj]; } });
                    rhs[GAMX + kk] += symtrace(gi, dd);
                    sfor<3>([&](auto ii_c) __attribute__((always_inline)) { constexpr int ii = decltype(ii_c)::value; { rhs[GAMX + ii] += R(1.0 / 3.0) * (gi[S(ii, 0)] * dd[S(0, kk)]
                                                          + gi[S(ii, 1)] * dd[S(1, kk)]
                                                          + gi[S(ii, 2)] * dd[S(2, kk)]); } });
                    rhs[BETAX + kk] += (a.advect_gauge ? adv(d) : R(0))
                                     + dissipation<P, R, PX, PXY>(lc, F);
                }
            });
            if (active) {
                const R divb = db[0][0] + db[1][1] + db[2][2];
                rhs[CHI] += R(-2.0 / 3.0) * chi * divb;
                sfor<6>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
                    const int ii = SI(q), jj = SJ(q);
                    R lg = R(0), la = R(0);
                    sfor<3>([&](auto kk_c) __attribute__((always_inline)) { constexpr int kk = decltype(kk_c)::value; {
                        lg += g[S(ii, kk)] * db[kk][jj] + g[S(jj, kk)] * db[kk][ii];
                        la += A[S(ii, kk)] * db[kk][jj] + A[S(jj, kk)] * db[kk][ii];
                    } });
                    rhs[GXX + q] += lg - R(2.0 / 3.0) * g[q] * divb;
                    rhs[AXX + q] += la - R(2.0 / 3.0) * A[q] * divb;
                } });
                sfor<3>([&](auto ii_c) __attribute__((always_inline)) { constexpr int ii = decltype(ii_c)::value; { rhs[GAMX + ii] += -(Gd[0] * db[ii][0] + Gd[1] * db[ii][1] + Gd[2] * db[ii][2])
                                    + R(2.0 / 3.0) * Gd[ii] * divb; } });
            }
        }

        // ---- output
        if constexpr (MODE == MODE_RHS) {
            if (active) {
                double *ob = a.out + B.offset;
                sfor<NFIELD>([&](auto f_c) __attribute__((always_inline)) { constexpr int f = decltype(f_c)::value; { ob[f * fs + pt] = double(rhs[f]); } });
            }
        } else if constexpr (MODE == MODE_RK) {
            if (active) {
                double v[NFIELD];
                double *u1b = a.u1 ? a.u1 + B.offset : nullptr;
                const double *u2b = a.u2 ? a.u2 + B.offset : nullptr;
                sfor<NFIELD>([&](auto f_c) __attribute__((always_inline)) { constexpr int f = decltype(f_c)::value; {
                    const long long e = f * fs + pt;
                    const double u0 = ub[e];
                    const double kf = double(rhs[f]);
                    const double n1 = (a.read_u1 ? u1b[e] : 0.0) + a.delta * u0 + a.eps_dt * kf;
                    double w = a.g1 * u0 + a.g2 * n1;
                    if (a.use_u2)
                        w += a.g3 * (a.u2_is_u0 ? u0 : u2b[e]);
                    v[f] = w + a.beta_dt * kf;
                    if (a.write_u1)
                        u1b[e] = n1;
                } });
                enforce(v, a.chi_floor, a.alpha_floor);
                double *ob = a.out + B.offset;
                sfor<NFIELD>([&](auto f_c) __attribute__((always_inline)) { constexpr int f = decltype(f_c)::value; { ob[f * fs + pt] = v[f]; } });
            }
        } else {
            if (active && a.out) {
                double *cb = a.out + B.coffset;
                sfor<NCONS>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { cb[q * fs + pt] = double(cons[q]); } });
            }
            // Per-tile sums of |c| and c^2 in a fixed order: wave reduction,
            // then the waves in order.
            double v[16];
            sfor<NCONS>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
                const double c = active ? double(cons[q]) : 0.0;
                v[2 * q] = fabs(c);
                v[2 * q + 1] = c * c;
            } });
            sfor<16>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; {
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1)
                    v[q] += __shfl_xor(v[q], off, 64);
            } });
            const int wave = t >> 6, lane = t & 63;
            __syncthreads();
            if (lane == 0)
                sfor<16>([&](auto q_c) __attribute__((always_inline)) { constexpr int q = decltype(q_c)::value; { red[wave * 16 + q] = v[q]; } });
            __syncthreads();
            if (t < 16) {
                double s = 0.0;
                for (int w = 0; w < NT / 64; ++w)
                    s += red[w * 16 + t];
                a.partial[(a.tile_base + tile) * 16 + t] = s;
            }
        }
        __syncthreads();   // LDS reuse by the next tile of a persistent workgroup
    }
}

// Fused right-hand side (+ Runge-Kutta stage) kernel.  Field order:
// shift, conformal metric, Gamma-tilde, chi, lapse, Khat, Theta, At.  Each
// field's right-hand side is finished as soon as its last contribution is
// known and, in a stage, combined with u1/u2 and stored at once; only the new
// conformal metric and At are held back for the det/trace enforcement.
// MON: the constraint monitor of the stage's input state (Sec. 4.1): H,
// M_i, Theta and Z^i formed from the derivatives the stage takes anyway,
// written to a.cons (when not null) and summed per tile into a.partial as
// the constraint kernel does (same per-tile order).
// LOP: lopsided stencils in the advection terms beta^k d_k u (re-read from
// the staged field in LDS); every other derivative stays centred.
// NAIVE (right-hand side, float arithmetic only): every staged value is
// rounded to float before the stencil differences (the naive FP32 form).
template <int P, int TX, int TY, int TZ, int WPE, typename R, int MODE, bool GEN, bool MON = false,
          bool LOP = false, bool NAIVE = false>
__global__ void __launch_bounds__(TX *TY *TZ) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
stage_kernel(const StageArgs a)
{
    constexpr int RAD = P / 2 + 1;
    constexpr int NT = TX * TY * TZ;
    constexpr int LX = TX + 2 * RAD, LY = TY + 2 * RAD, LZ = TZ + 2 * RAD;
    constexpr int PX = pad_pitch(LX);
    constexpr int PXY = PX * LY;
    constexpr int LVOL = LX * LY * LZ;
    constexpr int NLD = (LVOL + NT - 1) / NT;
    constexpr bool RK = MODE == MODE_RK;
    constexpr bool CHAIN = WPE > 1;
    constexpr bool EARLY_OLD = WPE == 1;
    // one workgroup per CU: LDS for the two-pass mixed derivatives
    constexpr bool MIX2 = WPE == 1;
    using MZ = MixDimsZ<P, TX, TY, TZ>;
    // One wave per SIMD leaves LDS room for a second halo tile: consecutive
    // stagings alternate between the two, so a staging need not wait for
    // every thread to finish with the previous field (the barrier after the
    // staging before last has seen to that).  In the monitor form it takes
    // the LDS that would hold the per-thread constraint values (MSTORE);
    // not in the lopsided form nor in the monitor form on 8x4x8 tiles, where
    // it would push values to scratch memory (measured slower).
    constexpr bool DBUF = MIX2 && !LOP && !(MON && TY == 4);
    constexpr int TILE = PXY * LZ;
    __shared__ double lds[(DBUF ? 2 : 1) * TILE];
    // The stager gives each thread one z-column of the halo box when the box
    // has as many columns as the tile has points (8x8x4 tiles): the z sums
    // of the mixed derivatives are then formed from its registers while the
    // field is stored, into one of two alternating buffers (they are written
    // before the staging barrier, so the buffer the previous mixed field
    // reads must be the other one).
    constexpr bool COLZ = MIX2 && LX * LY == NT && NLD == LZ && !NAIVE;
    constexpr int NZB = COLZ ? 2 : 1;
    __shared__ R zsb[MIX2 ? NZB * MZ::NZS : 1];
    __shared__ R ysb[MIX2 ? MZ::NYS : 1];
    // Per-thread LDS slots for long-lived values where the LDS that the halo
    // tile leaves at this occupancy allows: the Christoffel symbols (from the
    // conformal metric stage to the lapse stage) and the shift gradient (from
    // the shift stage to the At stage).  Each slot is one R per thread,
    // consecutive threads adjacent.
    constexpr int WG_PER_CU = (4 * WPE * 64 + NT - 1) / NT;
    __shared__ unsigned src_lds[NLD * NT];
    // monitor: per-wave sums of |c| and c^2 of the 8 constraints
    __shared__ double mred[MON ? (NT / 64) * 16 : 1];
    constexpr int SLOT_BUDGET =
        (LDS_PER_CU / WG_PER_CU - (DBUF ? 2 : 1) * TILE * (int)sizeof(double) - NLD * NT * 4
         - (MIX2 ? (NZB * MZ::NZS + MZ::NYS) * (int)sizeof(R) : 0)
         - (MON ? (NT / 64) * 16 * (int)sizeof(double) : 0)) / (NT * (int)sizeof(R));
    constexpr bool GU_SLOT = SLOT_BUDGET >= 18;
    constexpr bool DB_SLOT = SLOT_BUDGET >= (GU_SLOT ? 27 : 9);
    constexpr int GU0 = 0, DB0 = GU_SLOT ? 18 : 0;
    constexpr int NSLOT = (GU_SLOT ? 18 : 0) + (DB_SLOT ? 9 : 0);
    __shared__ R slots[NSLOT > 0 ? NSLOT * NT : 1];
    // Monitor: where the LDS left after the slots holds 8 doubles per thread,
    // each constraint value waits there and the 16 wave sums run together at
    // the end of the tile (independent chains) instead of one pair at a time.
    constexpr bool MSTORE = MON && (SLOT_BUDGET - NSLOT) * (int)sizeof(R) >= 8 * (int)sizeof(double);
    __shared__ double mval[MSTORE ? 8 * NT : 1];

    const int t = threadIdx.x;
    const int tx = t % TX, ty = (t / TX) % TY, tz = t / (TX * TY);
    R *const sl = slots + t;
    // Stencil centre of this thread in the LDS tile.  The offset is passed
    // through an opaque move after every staging barrier so that the
    // compiler recomputes the stencil addresses per field instead of
    // keeping dozens of them live across the whole kernel.
    constexpr int CO = RAD * (1 + PX + PXY);
    const int tofs = tz * PXY + ty * PX + tx + CO;
    int loff = tofs;

    __shared__ int tile_slot;
    for (int tile = first_tile(a, t, &tile_slot); tile >= 0; tile = next_tile(a, t, &tile_slot)) {
        const Tile T = a.tiles[tile];
        const z4c_block B = a.blocks[T.block];
        const int ng = B.ng;
        const int sy = B.nx + 2 * ng;
        const int sz = sy * (B.ny + 2 * ng);
        const int i = T.i0 + tx, j = T.j0 + ty, k = T.k0 + tz;
        const bool active = i < B.nx && j < B.ny && k < B.nz;
        const int pt = (k + ng) * sz + (j + ng) * sy + (i + ng);
        const unsigned upt8 = 8u * (unsigned)pt;   // byte offset from a uniform field base
        const double *ub = a.u + B.offset;
        const long long fs = B.field_stride;

        double *ob = a.out + B.offset;
        double *u1b = a.u1 ? a.u1 + B.offset : nullptr;
        const double *u2b = a.u2 ? a.u2 + B.offset : nullptr;
        // Values of field f at this point in the u1 and u2 registers, loaded
        // at the start of the stage that completes f so that the stage's LDS
        // work covers their latency; with one wave per SIMD (no other wave to
        // cover it), one stage before, with the halo prefetch of f.
        struct Old {
            double u1, u2;
        };
        auto old = [&](int f) __attribute__((always_inline)) {
            Old o{0.0, 0.0};
            if constexpr (RK) {
                const long long e = f * fs;
                if (a.read_u1)
                    o.u1 = at(u1b + e, upt8);
                if (a.use_u2 && !a.u2_is_u0)
                    o.u2 = at(u2b + e, upt8);
            }
            return o;
        };
        Old pending{0.0, 0.0};

        LStager<NLD, NT, LX, LY, LZ, PX, PXY, GEN> st;
        setup_lstager<NLD, NT, RAD, LX, LY, LZ, PX, PXY, GEN>(st, src_lds, a, T, B, t);
        // z sums of the mixed derivatives of the field staged last
        const R *zcur = zsb;
        // Stages field FF; returns the early-loaded u1/u2 values of FF.
        auto stage = [&](auto FC) __attribute__((always_inline)) {
            constexpr int FF = decltype(FC)::value;
            constexpr int NX = next_field<MODE>(FF);
            constexpr int BUF = DBUF ? (stage_pos<MODE>(FF) & 1) * TILE : 0;
            constexpr bool MIXF = MIX2 && (FF == CHI || FF == ALPHA || (FF >= GXX && FF <= GZZ)
                                           || (FF >= BETAX && FF <= BETAZ));
            constexpr int ZB = COLZ ? (stage_pos<MODE>(FF) & 1) * MZ::NZS : 0;
            if constexpr (!DBUF)
                __syncthreads();
            st.template store<NAIVE>(lds + BUF, t);
            if constexpr (MIXF && COLZ) {
                // this thread's column: (x, y) = (t mod LX, t / LX), z = q
                constexpr int X0 = RAD - MZ::Q;
                const int cx = t % LX - X0, cy = t / LX - X0;
                if (cx >= 0 && cx < MZ::EX && cy >= 0 && cy < MZ::EY) {
                    double col[LZ];
#pragma unroll
                    for (int q = 0; q < LZ; ++q)
                        col[q] = st.pf[q];
#pragma unroll
                    for (int z = 0; z < TZ; ++z)
                        zsb[ZB + z * MZ::ZR::PLANE + MZ::ZR::row(cy) + cx] =
                            d1raw<P, R, 1>(col + z + RAD);
                }
            }
            if constexpr (NX >= 0)
                st.prefetch(NX, t);
            const Old mine = pending;
            if constexpr (RK && EARLY_OLD && early_old(NX)) {
                if (active)
                    pending = old(NX);
            }
            __syncthreads();
            if constexpr (MIXF) {
                mix_prep_z<P, R, TX, TY, TZ, PX, PXY, !COLZ>(lds + BUF, zsb + ZB, ysb, t);
                __syncthreads();
                zcur = zsb + ZB;
            }
            loff = tofs + BUF;
            asm volatile("" : "+v"(loff));
            return mine;
        };
        st.prefetch(BETAX, t);
        if constexpr (RK && EARLY_OLD && early_old(BETAX)) {
            if (active)
                pending = old(BETAX);
        }

        const Fac<R> F = load_fac<R>(a, T.block);
        // first and second derivatives and dissipation of the staged field
        auto derivs2 = [&](R d[3], R dd[6], R &ko) __attribute__((always_inline)) {
            if constexpr (MIX2)
                all_ko_sums_z<P, R, PX, PXY, TX, TY, TZ>(lds, loff, F, d, dd, ko, zcur, ysb, tx,
                                                         ty, tz);
            else
                all_ko<P, R, PX, PXY, CHAIN>(lds, loff, F, d, dd, ko);
        };
        auto centre = [&](int f) __attribute__((always_inline)) {
            return active ? R(at(ub + f * fs, upt8)) : R(0);
        };
        // State value of the field staged in LDS at this thread's point.
        auto staged = [&]() __attribute__((always_inline)) { return lds[loff]; };
        // Runge-Kutta combination of field f (state u0) with right-hand side kf (FP64).
        auto combine = [&](int f, R kf_r, double u0, const Old &o) __attribute__((always_inline)) {
            const double kf = double(kf_r);
            const double n1 = o.u1 + a.delta * u0 + a.eps_dt * kf;
            double w = a.g1 * u0 + a.g2 * n1;
            if (a.use_u2)
                w += a.g3 * (a.u2_is_u0 ? u0 : o.u2);
            if (a.write_u1)
                at(u1b + f * fs, upt8) = n1;
            return w + a.beta_dt * kf;
        };
        // Finish a field that needs no enforcement.
        auto finish = [&](int f, R kf, double u0, const Old &o) __attribute__((always_inline)) {
            if constexpr (RK)
                at(ob + f * fs, upt8) = combine(f, kf, u0, o);
            else
                at(ob + f * fs, upt8) = double(kf);
        };
        // Shift gradient d_j beta^k and Christoffel symbols Gt^k_q: LDS slots
        // or registers.
        R db_r[3][3], Gu[3][6];
        auto DBw = [&](int kk, int jj, R v) __attribute__((always_inline)) {
            if constexpr (DB_SLOT)
                sl[(DB0 + 3 * kk + jj) * NT] = v;
            else
                db_r[kk][jj] = v;
        };
        auto DB = [&](int kk, int jj) __attribute__((always_inline)) -> R {
            if constexpr (DB_SLOT)
                return sl[(DB0 + 3 * kk + jj) * NT];
            else
                return db_r[kk][jj];
        };
        auto GU = [&](int kk, int q) __attribute__((always_inline)) -> R {
            if constexpr (GU_SLOT)
                return sl[(GU0 + 6 * kk + q) * NT];
            else
                return Gu[kk][q];
        };

        R g[6];
        sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
            constexpr int q = decltype(Q_c)::value;
            g[q] = active ? R(at(ub + (GXX + q) * fs, upt8)) : ((q == 0 || q == 3 || q == 5) ? R(1) : R(0));
        });
        R gi[6];
        {
            const R det = g[0] * (g[3] * g[5] - g[4] * g[4]) - g[1] * (g[1] * g[5] - g[4] * g[2])
                        + g[2] * (g[1] * g[4] - g[3] * g[2]);
            const R id = R(1) / det;
            gi[0] = (g[3] * g[5] - g[4] * g[4]) * id;
            gi[1] = (g[2] * g[4] - g[1] * g[5]) * id;
            gi[2] = (g[1] * g[4] - g[2] * g[3]) * id;
            gi[3] = (g[0] * g[5] - g[2] * g[2]) * id;
            gi[4] = (g[2] * g[1] - g[0] * g[4]) * id;
            gi[5] = (g[0] * g[3] - g[1] * g[1]) * id;
        }
        const R beta[3] = {centre(BETAX), centre(BETAY), centre(BETAZ)};
        const R chi = active ? R(at(ub + CHI * fs, upt8)) : R(1);
        const R alpha = active ? R(at(ub + ALPHA * fs, upt8)) : R(1);
        const R Khat = centre(KHAT), Theta = centre(THETA);
        const R K = Khat + R(2) * Theta;
        const R chis = chi > R(a.chi_floor) ? chi : R(a.chi_floor);
        const R ichi2 = R(0.5) / chis;          // 1 / (2 chi)
        const R kap1 = R(a.kappa1), kap2 = R(a.kappa2);
        const R pi = R(PI);

        auto adv = [&](const R d[3]) __attribute__((always_inline)) {
            if constexpr (LOP)
                return lop_adv<P, R, PX, PXY>(lds, loff, F, beta);
            else
                return beta[0] * d[0] + beta[1] * d[1] + beta[2] * d[2];
        };
        // Monitor: constraint q at this point (0 where inactive) to a.cons,
        // and its |c|, c^2 summed over the wave (butterfly) into mred.
        // Called by every lane of the workgroup.
        double *cb = MON && a.cons ? a.cons + B.coffset : nullptr;
        R Mc[3] = {R(0), R(0), R(0)};   // M_i accumulated over the stages
        auto mon = [&](auto QC, R c_r) __attribute__((always_inline)) {
            constexpr int q = decltype(QC)::value;
            const double c = active ? double(c_r) : 0.0;
            if (active && cb)
                at(cb + q * fs, upt8) = c;
            if constexpr (MSTORE) {
                mval[q * NT + t] = c;
            } else {
                double v1 = fabs(c), v2 = c * c;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    v1 += __shfl_xor(v1, off, 64);
                    v2 += __shfl_xor(v2, off, 64);
                }
                if ((t & 63) == 0) {
                    mred[(t >> 6) * 16 + 2 * q] = v1;
                    mred[(t >> 6) * 16 + 2 * q + 1] = v2;
                }
            }
        };

        // ---- shift: d beta (kept for the Lie-derivative terms), d d beta -> Gt
        R rG[3] = {R(0), R(0), R(0)};
        R divb = R(0);
        sfor<3>([&](auto K_c) __attribute__((always_inline)) {
            constexpr int kk = decltype(K_c)::value;
            const Old oe = stage(std::integral_constant<int, BETAX + kk>{});
            if (active) {
                const Old o = EARLY_OLD && early_old(BETAX + kk) ? oe : old(BETAX + kk);
                const R Gam = R(at(ub + (GAMX + kk) * fs, upt8));
                R d[3], dd[6], ko;
                derivs2(d, dd, ko);
                sfor<3>([&](auto J_c) __attribute__((always_inline)) {
                    constexpr int jj = decltype(J_c)::value;
                    DBw(kk, jj, d[jj]);
                });
                divb += d[kk];
                rG[kk] += symtrace(gi, dd);
                sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                    constexpr int ii = decltype(I_c)::value;
                    rG[ii] += R(1.0 / 3.0) * (gi[S(ii, 0)] * dd[S(0, kk)] + gi[S(ii, 1)] * dd[S(1, kk)]
                                              + gi[S(ii, 2)] * dd[S(2, kk)]);
                });
                const R kb = (a.advect_gauge ? adv(d) : R(0)) + ko
                           + (a.shift == Z4C_SHIFT_GAMMADRIVER ? Gam : R(0)) - R(a.eta) * beta[kk];
                finish(BETAX + kk, kb, staged(), o);
            }
        });

        // ---- conformal metric
        R dg[3][6];
        R Rij[6];
        double vg[6];   // new conformal metric (stage), held for the det enforcement
        sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
            constexpr int q = decltype(Q_c)::value;
            constexpr int ii = SI(q), jj = SJ(q);
            const Old oe = stage(std::integral_constant<int, GXX + q>{});
            if (active) {
                const Old o = EARLY_OLD && early_old(GXX + q) ? oe : old(GXX + q);
                const R Aq = R(at(ub + (AXX + q) * fs, upt8));
                R d[3], dd[6], ko;
                derivs2(d, dd, ko);
                sfor<3>([&](auto K_c) __attribute__((always_inline)) {
                    constexpr int kk = decltype(K_c)::value;
                    dg[kk][q] = d[kk];
                });
                Rij[q] = R(-0.5) * symtrace(gi, dd);
                R lie = R(0);
                sfor<3>([&](auto K_c) __attribute__((always_inline)) {
                    constexpr int kk = decltype(K_c)::value;
                    lie += g[S(ii, kk)] * DB(kk, jj) + g[S(jj, kk)] * DB(kk, ii);
                });
                const R kg = adv(d) + ko - R(2) * alpha * Aq + lie
                           - R(2.0 / 3.0) * g[q] * divb;
                if constexpr (RK)
                    vg[q] = combine(GXX + q, kg, staged(), o);
                else
                    at(ob + (GXX + q) * fs, upt8) = double(kg);
            }
        });
        if constexpr (RK) {
            if (active) {
                // det(gt) = 1
                const double det = vg[0] * (vg[3] * vg[5] - vg[4] * vg[4])
                                 - vg[1] * (vg[1] * vg[5] - vg[4] * vg[2])
                                 + vg[2] * (vg[1] * vg[4] - vg[3] * vg[2]);
                const double f = 1.0 / cbrt(det);
                sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    vg[q] *= f;
                    at(ob + (GXX + q) * fs, upt8) = vg[q];
                });
            }
        }

        // Christoffel symbols and the first-derivative part of the Ricci tensor.
        R Gd[3];
        if (active) {
            R Gl[3][6];
            sfor<3>([&](auto K_c) __attribute__((always_inline)) {
                constexpr int kk = decltype(K_c)::value;
                sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    constexpr int ii = SI(q), jj = SJ(q);
                    Gl[kk][q] = R(0.5) * (dg[ii][S(jj, kk)] + dg[jj][S(ii, kk)] - dg[kk][q]);
                });
            });
            sfor<3>([&](auto K_c) __attribute__((always_inline)) {
                constexpr int kk = decltype(K_c)::value;
                sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    Gu[kk][q] = gi[S(kk, 0)] * Gl[0][q] + gi[S(kk, 1)] * Gl[1][q]
                              + gi[S(kk, 2)] * Gl[2][q];
                });
                Gd[kk] = symtrace(gi, Gu[kk]);
            });
            sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                constexpr int q = decltype(Q_c)::value;
                constexpr int ii = SI(q), jj = SJ(q);
                R s = R(0);
                sfor<3>([&](auto K_c) __attribute__((always_inline)) {
                    constexpr int kk = decltype(K_c)::value;
                    s += R(0.5) * Gd[kk] * (Gl[ii][S(jj, kk)] + Gl[jj][S(ii, kk)]);
                });
                Rij[q] += s;
            });
            // + sum_kl (Gu^k_{li} T_{jk}^l + Gu^k_{lj} T_{ik}^l + Gu^k_{il} T_{kj}^l),
            //   T_{ab}^c = gt^{cm} Gt_{a bm}
            sfor<3>([&](auto P0_c) __attribute__((always_inline)) {
                constexpr int p0 = decltype(P0_c)::value;
                sfor<3>([&](auto P1_c) __attribute__((always_inline)) {
                    constexpr int p1 = decltype(P1_c)::value;
                    R Tc[3];
                    sfor<3>([&](auto P2_c) __attribute__((always_inline)) {
                        constexpr int p2 = decltype(P2_c)::value;
                        Tc[p2] = gi[S(p2, 0)] * Gl[p0][S(p1, 0)] + gi[S(p2, 1)] * Gl[p0][S(p1, 1)]
                               + gi[S(p2, 2)] * Gl[p0][S(p1, 2)];
                    });
                    sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                        constexpr int q = decltype(Q_c)::value;
                        constexpr int ii = SI(q), jj = SJ(q);
                        R s = R(0);
                        sfor<3>([&](auto L_c) __attribute__((always_inline)) {
                            constexpr int l = decltype(L_c)::value;
                            if constexpr (jj == p0)
                                s += Gu[p1][S(l, ii)] * Tc[l];
                            if constexpr (ii == p0)
                                s += Gu[p1][S(l, jj)] * Tc[l];
                            if constexpr (jj == p1)
                                s += Gu[p0][S(ii, l)] * Tc[l];
                        });
                        Rij[q] += s;
                    });
                });
            });
            // Lie-derivative terms of Gamma-tilde
            sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                constexpr int ii = decltype(I_c)::value;
                rG[ii] += -(Gd[0] * DB(ii, 0) + Gd[1] * DB(ii, 1) + Gd[2] * DB(ii, 2))
                        + R(2.0 / 3.0) * Gd[ii] * divb;
            });
            if constexpr (GU_SLOT) {
                sfor<3>([&](auto K_c) __attribute__((always_inline)) {
                    constexpr int kk = decltype(K_c)::value;
                    sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                        constexpr int q = decltype(Q_c)::value;
                        sl[(GU0 + 6 * kk + q) * NT] = Gu[kk][q];
                    });
                });
            }
        }

        // ---- Gamma-tilde: d_j Gt^k -> Ricci; damping
        sfor<3>([&](auto K_c) __attribute__((always_inline)) {
            constexpr int kk = decltype(K_c)::value;
            stage(std::integral_constant<int, GAMX + kk>{});
            R Zk = R(0);
            if (active) {
                R d[3], ko;
                first_ko<P, R, PX, PXY, CHAIN>(lds, loff, F, d, ko);
                sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    constexpr int ii = SI(q), jj = SJ(q);
                    Rij[q] += R(0.5) * (g[S(kk, ii)] * d[jj] + g[S(kk, jj)] * d[ii]);
                });
                const R Gam = R(lds[loff]);
                rG[kk] += adv(d) + ko
                        - R(2) * alpha * kap1 * (Gam - Gd[kk]);
                if constexpr (MON)
                    Zk = R(0.5) * (Gam - Gd[kk]);
            }
            if constexpr (MON)
                mon(std::integral_constant<int, C_ZX + kk>{}, Zk);
        });

        // ---- chi: R^chi_ij; chi is complete.  With the Ricci tensor and At
        // known, everything in the sources of Khat, Theta and At except the
        // lapse second derivatives is formed here.
        R Aup[6];
        R dchi[3];
        R PA[6];                      // At source without the D_i D_j alpha term
        R Kpart = R(0), Tpart = R(0); // pointwise sources of Khat (without D^2 alpha), Theta
        R Hc = R(0);                  // monitor: Hamiltonian constraint
        const Old oe_chi = stage(std::integral_constant<int, CHI>{});
        if (active) {
            const Old o = EARLY_OLD && early_old(CHI) ? oe_chi : old(CHI);
            R A[6];
            sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                constexpr int q = decltype(Q_c)::value;
                A[q] = R(at(ub + (AXX + q) * fs, upt8));
            });
            R dd[6], ko;
            derivs2(dchi, dd, ko);
            {
                R DD[6], dc2[6];
                sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    DD[q] = dd[q] - (GU(0, q) * dchi[0] + GU(1, q) * dchi[1] + GU(2, q) * dchi[2]);
                    dc2[q] = dchi[SI(q)] * dchi[SJ(q)];
                });
                const R trDD = symtrace(gi, DD);
                const R dchi2 = symtrace(gi, dc2);
                const R i4c2 = ichi2 * ichi2;   // 1 / (4 chi^2)
                sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    Rij[q] += (DD[q] + g[q] * trDD) * ichi2 - (dc2[q] + R(3) * g[q] * dchi2) * i4c2;
                });
            }
            const R kc = adv(dchi) + ko
                       + R(2.0 / 3.0) * chi * (alpha * K - divb);
            if constexpr (RK) {
                const double v = combine(CHI, kc, staged(), o);
                at(ob + CHI * fs, upt8) = v > a.chi_floor ? v : a.chi_floor;
            } else {
                at(ob + CHI * fs, upt8) = double(kc);
            }
            // At^i_j, At^{ij}, At.At
            R Amix[3][3];
            sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                constexpr int ii = decltype(I_c)::value;
                sfor<3>([&](auto J_c) __attribute__((always_inline)) {
                    constexpr int jj = decltype(J_c)::value;
                    Amix[ii][jj] = gi[S(ii, 0)] * A[S(0, jj)] + gi[S(ii, 1)] * A[S(1, jj)]
                                 + gi[S(ii, 2)] * A[S(2, jj)];
                });
            });
            R AA = R(0);
            sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                constexpr int q = decltype(Q_c)::value;
                constexpr int ii = SI(q), jj = SJ(q);
                Aup[q] = Amix[ii][0] * gi[S(0, jj)] + Amix[ii][1] * gi[S(1, jj)]
                       + Amix[ii][2] * gi[S(2, jj)];
                AA += R(SW(q)) * A[q] * Aup[q];
            });
            // 2 alpha (Gt^i_jk At^jk - 3/(2 chi) At^ij d_j chi)
            sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                constexpr int ii = decltype(I_c)::value;
                R gA = R(0);
                sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    gA += R(SW(q)) * GU(ii, q) * Aup[q];
                });
                const R Ac = Aup[S(ii, 0)] * dchi[0] + Aup[S(ii, 1)] * dchi[1]
                           + Aup[S(ii, 2)] * dchi[2];
                rG[ii] += R(2) * alpha * (gA - R(1.5) / chis * Ac);
            });
            // matter
            R rho = R(0), Si[3] = {R(0), R(0), R(0)}, Sij[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
            if (a.matter) {
                const double *mb = a.matter + B.moffset;
                rho = R(at(mb, upt8));
                sfor<3>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    Si[q] = R(at(mb + (1 + q) * fs, upt8));
                });
                sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    Sij[q] = R(at(mb + (4 + q) * fs, upt8));
                });
            }
            const R trS = chi * symtrace(gi, Sij);
            sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                constexpr int ii = decltype(I_c)::value;
                rG[ii] += R(-16) * pi * alpha
                        * (gi[S(ii, 0)] * Si[0] + gi[S(ii, 1)] * Si[1] + gi[S(ii, 2)] * Si[2]);
            });
            const R Rs = chi * symtrace(gi, Rij);
            Kpart = alpha * (AA + K * K * R(1.0 / 3.0)) + R(4) * pi * alpha * (trS + rho)
                  + alpha * kap1 * (R(1) - kap2) * Theta;
            Tpart = R(0.5) * alpha * (Rs - AA + R(2.0 / 3.0) * K * K)
                  - alpha * (R(8) * pi * rho + kap1 * (R(2) + kap2) * Theta);
            if constexpr (MON) {
                Hc = Rs + R(2.0 / 3.0) * K * K - AA - R(16) * pi * rho;
                // M_i: -Gt_d^l At_li - Gt^l_ji At^j_l - 3/(2 chi) At^j_i d_j chi
                // - 8 pi S_i here; the At and K derivative terms in their stages
                sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                    constexpr int ii = decltype(I_c)::value;
                    R m = -(Gd[0] * A[S(0, ii)] + Gd[1] * A[S(1, ii)] + Gd[2] * A[S(2, ii)]);
                    sfor<3>([&](auto J_c) __attribute__((always_inline)) {
                        constexpr int jj = decltype(J_c)::value;
                        m -= GU(0, S(jj, ii)) * Amix[jj][0] + GU(1, S(jj, ii)) * Amix[jj][1]
                           + GU(2, S(jj, ii)) * Amix[jj][2];
                    });
                    m -= R(1.5) / chis * (Amix[0][ii] * dchi[0] + Amix[1][ii] * dchi[1]
                                          + Amix[2][ii] * dchi[2]);
                    Mc[ii] += m - R(8) * pi * Si[ii];
                });
            }
            // At: chi [alpha (R - 8 pi S)]^tf + alpha (K At - 2 At At) + Lie
            // (the -chi [D D alpha]^tf part follows in the lapse stage)
            R Y[6];
            sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                constexpr int q = decltype(Q_c)::value;
                Y[q] = alpha * (Rij[q] - R(8) * pi * Sij[q]);
            });
            const R trY = symtrace(gi, Y);
            sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                constexpr int q = decltype(Q_c)::value;
                constexpr int ii = SI(q), jj = SJ(q);
                const R AAm = A[S(ii, 0)] * Amix[0][jj] + A[S(ii, 1)] * Amix[1][jj]
                            + A[S(ii, 2)] * Amix[2][jj];
                R la = R(0);
                sfor<3>([&](auto K_c) __attribute__((always_inline)) {
                    constexpr int kk = decltype(K_c)::value;
                    la += A[S(ii, kk)] * DB(kk, jj) + A[S(jj, kk)] * DB(kk, ii);
                });
                PA[q] = chi * (Y[q] - g[q] * trY * R(1.0 / 3.0)) + alpha * (K * A[q] - R(2) * AAm)
                      + la - R(2.0 / 3.0) * A[q] * divb;
            });
        }

        if constexpr (MON) {
            mon(std::integral_constant<int, C_H>{}, Hc);
            mon(std::integral_constant<int, C_THETA>{}, Theta);
        }

        // ---- lapse: D_i D_j alpha; alpha is complete; the lapse terms of
        // the Khat and At sources
        const Old oe_alpha = stage(std::integral_constant<int, ALPHA>{});
        if (active) {
            const Old o = EARLY_OLD && early_old(ALPHA) ? oe_alpha : old(ALPHA);
            R dal[3], dd[6], ko;
            derivs2(dal, dd, ko);
            R ca = R(0);   // gt^{kl} d_k chi d_l alpha
            sfor<3>([&](auto P0_c) __attribute__((always_inline)) {
                constexpr int p0 = decltype(P0_c)::value;
                sfor<3>([&](auto P1_c) __attribute__((always_inline)) {
                    constexpr int p1 = decltype(P1_c)::value;
                    ca += gi[S(p0, p1)] * dchi[p0] * dal[p1];
                });
            });
            R DDa[6];
            sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                constexpr int q = decltype(Q_c)::value;
                constexpr int ii = SI(q), jj = SJ(q);
                DDa[q] = dd[q] - (GU(0, q) * dal[0] + GU(1, q) * dal[1] + GU(2, q) * dal[2])
                       + (dchi[ii] * dal[jj] + dchi[jj] * dal[ii] - g[q] * ca) * ichi2;
            });
            const R trDDa = symtrace(gi, DDa);
            R muL = R(0);
            if (a.lapse == Z4C_LAPSE_1PLUSLOG)
                muL = R(2) * alpha;
            else if (a.lapse == Z4C_LAPSE_HARMONIC)
                muL = alpha * alpha;
            const R ka = (a.advect_gauge ? adv(dal) : R(0)) + ko
                       - muL * Khat;
            if constexpr (RK) {
                const double v = combine(ALPHA, ka, staged(), o);
                at(ob + ALPHA * fs, upt8) = v > a.alpha_floor ? v : a.alpha_floor;
            } else {
                at(ob + ALPHA * fs, upt8) = double(ka);
            }
            // -2 At^ij d_j alpha
            sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                constexpr int ii = decltype(I_c)::value;
                rG[ii] += R(-2) * (Aup[S(ii, 0)] * dal[0] + Aup[S(ii, 1)] * dal[1]
                                   + Aup[S(ii, 2)] * dal[2]);
            });
            Kpart -= chi * trDDa;
            sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                constexpr int q = decltype(Q_c)::value;
                PA[q] -= chi * (DDa[q] - g[q] * trDDa * R(1.0 / 3.0));
            });
        }

        // ---- Khat, Theta (their Gamma-tilde source terms); both complete
        double gam0[3] = {0.0, 0.0, 0.0};   // state of Gamma-tilde, completed after Theta
        Old gamo[3];
        sfor<2>([&](auto Q_c) __attribute__((always_inline)) {
            constexpr int q = decltype(Q_c)::value;
            const Old oe = stage(std::integral_constant<int, q == 0 ? KHAT : THETA>{});
            if (active) {
                const Old o = EARLY_OLD && early_old(q == 0 ? KHAT : THETA) ? oe
                                                                             : old(q == 0 ? KHAT : THETA);
                if constexpr (q == 1 && RK) {
                    sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                        constexpr int ii = decltype(I_c)::value;
                        gam0[ii] = at(ub + (GAMX + ii) * fs, upt8);
                        gamo[ii] = old(GAMX + ii);
                    });
                }
                R d[3], ko;
                first_ko<P, R, PX, PXY, CHAIN>(lds, loff, F, d, ko);
                const R c = q == 0 ? R(-4.0 / 3.0) * alpha : R(-2.0 / 3.0) * alpha;
                sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                    constexpr int ii = decltype(I_c)::value;
                    rG[ii] += c * (gi[S(ii, 0)] * d[0] + gi[S(ii, 1)] * d[1] + gi[S(ii, 2)] * d[2]);
                });
                if constexpr (MON) {   // -2/3 d_i K, K = Khat + 2 Theta
                    sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                        constexpr int ii = decltype(I_c)::value;
                        Mc[ii] -= R(q == 0 ? 2.0 / 3.0 : 4.0 / 3.0) * d[ii];
                    });
                }
                const R kq = adv(d) + ko + (q == 0 ? Kpart : Tpart);
                finish(q == 0 ? KHAT : THETA, kq, staged(), o);
            }
        });
        // Gamma-tilde is complete
        if (active) {
            sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                constexpr int ii = decltype(I_c)::value;
                finish(GAMX + ii, rG[ii], gam0[ii], gamo[ii]);
            });
        }

        // ---- At_ij; then tr(At) = 0 with the new conformal metric
        double vA[6], vn[6];
        sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
            constexpr int q = decltype(Q_c)::value;
            const Old oe = stage(std::integral_constant<int, AXX + q>{});
            if (active) {
                const Old o = EARLY_OLD && early_old(AXX + q) ? oe : old(AXX + q);
                if constexpr (q == 5 && RK) {
                    // the new conformal metric, as stored by this thread
                    unsigned upr = upt8;
                    asm volatile("" : "+v"(upr));
                    sfor<6>([&](auto P_c) __attribute__((always_inline)) {
                        constexpr int p = decltype(P_c)::value;
                        vn[p] = at(ob + (GXX + p) * fs, upr);
                    });
                }
                R d[3], ko;
                first_ko<P, R, PX, PXY, CHAIN>(lds, loff, F, d, ko);
                if constexpr (MON) {   // gt^{jk} d_k At_ij, At_ij = At_ji
                    constexpr int ii = SI(q), jj = SJ(q);
                    Mc[ii] += gi[S(jj, 0)] * d[0] + gi[S(jj, 1)] * d[1] + gi[S(jj, 2)] * d[2];
                    if constexpr (ii != jj)
                        Mc[jj] += gi[S(ii, 0)] * d[0] + gi[S(ii, 1)] * d[1] + gi[S(ii, 2)] * d[2];
                }
                const R kA = adv(d) + ko + PA[q];
                if constexpr (RK)
                    vA[q] = combine(AXX + q, kA, staged(), o);
                else
                    at(ob + (AXX + q) * fs, upt8) = double(kA);
            }
        });
        if constexpr (RK) {
            if (active) {
                const double det = vn[0] * (vn[3] * vn[5] - vn[4] * vn[4])
                                 - vn[1] * (vn[1] * vn[5] - vn[4] * vn[2])
                                 + vn[2] * (vn[1] * vn[4] - vn[3] * vn[2]);
                const double id = 1.0 / det;
                const double gn[6] = {(vn[3] * vn[5] - vn[4] * vn[4]) * id,
                                      (vn[2] * vn[4] - vn[1] * vn[5]) * id,
                                      (vn[1] * vn[4] - vn[2] * vn[3]) * id,
                                      (vn[0] * vn[5] - vn[2] * vn[2]) * id,
                                      (vn[2] * vn[1] - vn[0] * vn[4]) * id,
                                      (vn[0] * vn[3] - vn[1] * vn[1]) * id};
                const double tr = gn[0] * vA[0] + gn[3] * vA[3] + gn[5] * vA[5]
                                + 2.0 * (gn[1] * vA[1] + gn[2] * vA[2] + gn[4] * vA[4]);
                sfor<6>([&](auto Q_c) __attribute__((always_inline)) {
                    constexpr int q = decltype(Q_c)::value;
                    at(ob + (AXX + q) * fs, upt8) = vA[q] - vn[q] * tr * (1.0 / 3.0);
                });
            }
        }
        if constexpr (MON) {
            sfor<3>([&](auto I_c) __attribute__((always_inline)) {
                constexpr int ii = decltype(I_c)::value;
                mon(std::integral_constant<int, C_MX + ii>{}, Mc[ii]);
            });
            if constexpr (MSTORE) {   // the values this thread parked, summed per wave
                double v[16];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const double c = mval[q * NT + t];
                    v[2 * q] = fabs(c);
                    v[2 * q + 1] = c * c;
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
                    for (int q = 0; q < 16; ++q)
                        v[q] += __shfl_xor(v[q], off, 64);
                }
                if ((t & 63) == 0) {
#pragma unroll
                    for (int q = 0; q < 16; ++q)
                        mred[(t >> 6) * 16 + q] = v[q];
                }
            }
            __syncthreads();
            // per-tile sums, the waves in order (as the constraint kernel)
            if (t < 16) {
                double sum = 0.0;
                for (int w = 0; w < NT / 64; ++w)
                    sum += mred[w * 16 + t];
                a.partial[(a.tile_base + tile) * 16 + t] = sum;
            }
        }
        __syncthreads();   // LDS reuse by the next tile of a persistent workgroup
    }
}

}  // namespace tile

// Launch of one tile-kernel variant (grid: one workgroup per tile, or
// `persistent` workgroups each taking a contiguous run of tiles).
inline int grid_size(const StageArgs &a)
{
    return a.persistent ? (a.persistent < a.ntiles ? a.persistent : a.ntiles) : a.ntiles;
}

template <int P, int TX, int TY, int TZ, int WPE, typename R>
hipError_t launch_variant(int mode, const StageArgs &a, hipStream_t s)
{
    const int grid = grid_size(a);
    if (grid <= 0)
        return hipSuccess;
    const dim3 blk(TX * TY * TZ);
    // halo sources beyond the block itself only under the frozen and neighbour rules
    const bool gen = a.halo == Z4C_GHOST_FROZEN || a.halo == Z4C_GHOST_NEIGHBOUR;
    if (mode == MODE_RHS) {
        if (gen)
            tile::stage_kernel<P, TX, TY, TZ, WPE, R, MODE_RHS, true><<<grid, blk, 0, s>>>(a);
        else
            tile::stage_kernel<P, TX, TY, TZ, WPE, R, MODE_RHS, false><<<grid, blk, 0, s>>>(a);
    } else {
        if (gen)
            tile::stage_kernel<P, TX, TY, TZ, WPE, R, MODE_RK, true><<<grid, blk, 0, s>>>(a);
        else
            tile::stage_kernel<P, TX, TY, TZ, WPE, R, MODE_RK, false><<<grid, blk, 0, s>>>(a);
    }
    return hipGetLastError();
}

// Right-hand side with the naive FP32 form (samples rounded to float before
// the stencil differences).
template <int P, int TX, int TY, int TZ, int WPE>
hipError_t launch_variant_naive(const StageArgs &a, hipStream_t s)
{
    const int grid = grid_size(a);
    if (grid <= 0)
        return hipSuccess;
    const dim3 blk(TX * TY * TZ);
    const bool gen = a.halo == Z4C_GHOST_FROZEN || a.halo == Z4C_GHOST_NEIGHBOUR;
    if (gen)
        tile::stage_kernel<P, TX, TY, TZ, WPE, float, MODE_RHS, true, false, false, true>
            <<<grid, blk, 0, s>>>(a);
    else
        tile::stage_kernel<P, TX, TY, TZ, WPE, float, MODE_RHS, false, false, false, true>
            <<<grid, blk, 0, s>>>(a);
    return hipGetLastError();
}

// Right-hand side or stage with lopsided advection (FP64 arithmetic).
template <int P, int TX, int TY, int TZ, int WPE>
hipError_t launch_variant_lop(int mode, const StageArgs &a, hipStream_t s)
{
    const int grid = grid_size(a);
    if (grid <= 0)
        return hipSuccess;
    const dim3 blk(TX * TY * TZ);
    const bool gen = a.halo == Z4C_GHOST_FROZEN || a.halo == Z4C_GHOST_NEIGHBOUR;
    if (mode == MODE_RHS) {
        if (gen)
            tile::stage_kernel<P, TX, TY, TZ, WPE, double, MODE_RHS, true, false, true>
                <<<grid, blk, 0, s>>>(a);
        else
            tile::stage_kernel<P, TX, TY, TZ, WPE, double, MODE_RHS, false, false, true>
                <<<grid, blk, 0, s>>>(a);
    } else {
        if (gen)
            tile::stage_kernel<P, TX, TY, TZ, WPE, double, MODE_RK, true, false, true>
                <<<grid, blk, 0, s>>>(a);
        else
            tile::stage_kernel<P, TX, TY, TZ, WPE, double, MODE_RK, false, false, true>
                <<<grid, blk, 0, s>>>(a);
    }
    return hipGetLastError();
}

// Stage with the constraint monitor (FP64 arithmetic).
template <int P, int TX, int TY, int TZ, int WPE>
hipError_t launch_variant_mon(const StageArgs &a, hipStream_t s)
{
    const int grid = grid_size(a);
    if (grid <= 0)
        return hipSuccess;
    const dim3 blk(TX * TY * TZ);
    const bool gen = a.halo == Z4C_GHOST_FROZEN || a.halo == Z4C_GHOST_NEIGHBOUR;
    if (gen)
        tile::stage_kernel<P, TX, TY, TZ, WPE, double, MODE_RK, true, true><<<grid, blk, 0, s>>>(a);
    else
        tile::stage_kernel<P, TX, TY, TZ, WPE, double, MODE_RK, false, true><<<grid, blk, 0, s>>>(a);
    return hipGetLastError();
}

template <int P, int TX, int TY, int TZ>
hipError_t launch_cons(const StageArgs &a, hipStream_t s)
{
    const int grid = grid_size(a);
    if (grid <= 0)
        return hipSuccess;
    tile::cons_kernel<P, TX, TY, TZ, double, MODE_CONS><<<grid, dim3(TX * TY * TZ), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace z4c
