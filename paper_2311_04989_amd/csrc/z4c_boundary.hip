// z4c_boundary.hip -- radiative (Sommerfeld) outer boundary of a level set.
//
// The paper states no outer boundary condition for Z4c (its static-star
// test moves the outer boundary further out instead of treating it); this is
// the usual radiative law of moving-puncture codes, taken as a reading.  The
// outer ghost points of a block (those in a direction whose neighbour entry
// is -1) advance, in every Runge-Kutta stage, by
//     d_t u = -(x^a / r) D_a u - (u - u_inf) / r,      r = |x|,
// for each of the 22 fields, u_inf its flat-space value (1 for chi, gt_xx,
// gt_yy, gt_zz and alpha, 0 otherwise), D_a the second-order difference
// along a: centred where the point's index along a lies inside the interior
// range, one-sided towards the interior outside it (it reads only stored
// points; samples at ghost points that have a neighbour are read through
// the neighbour rule when the stage reads its halo that way, so that both
// see the same values).  The stage combination and the enforcement (det gt = 1, tr At = 0,
// floors) are those of the interior points; there is no dissipation.  The
// stage kernel writes interior points and this one the outer ghost points,
// and both read only the stage input, so the two run in either order.
#include "z4c_tile.h"

namespace z4c {
namespace {

__device__ __forceinline__ double flat_value(int f)
{
    return (f == CHI || f == GXX || f == GYY || f == GZZ || f == ALPHA) ? 1.0 : 0.0;
}

// Second-order difference along one direction at index i of n interior
// points, from the centre value c0 and the two samples the stencil takes
// (s1, s2: the next two towards the interior outside the interior range,
// else the neighbours at -1 and +1), in differences from the centre.
__device__ __forceinline__ double d1_radiative(double c0, double s1, double s2, int i, int n,
                                               double h)
{
    if (i < 0)
        return (4.0 * (s1 - c0) - (s2 - c0)) / (2.0 * h);
    if (i >= n)
        return (-4.0 * (s1 - c0) + (s2 - c0)) / (2.0 * h);
    return (s2 - s1) / (2.0 * h);
}

// One thread per outer point, all 22 fields.
__global__ void __launch_bounds__(256) radiative_kernel(const RadiativeArgs a)
{
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.total)
        return;
    int lo = 0, hi = a.nregions;   // region by binary search over the prefix sums
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.start[mid] <= gid)
            lo = mid;
        else
            hi = mid;
    }
    const OuterRegion R = a.regions[lo];
    const z4c_block B = a.blocks[R.block];
    long long q = gid - a.start[lo];
    const int i = R.lo[0] + (int)(q % R.n[0]);
    q /= R.n[0];
    const int j = R.lo[1] + (int)(q % R.n[1]);
    const int k = R.lo[2] + (int)(q / R.n[1]);
    const int ng = B.ng;
    const long long sy = B.nx + 2 * ng, sz = sy * (B.ny + 2 * ng);
    // Element offset (field 0) of stored point (ii, jj, kk) of this block, or,
    // under the neighbour rule, of the point a neighbour copy would bring
    // there (neighbours share nx, ny, nz, ng and the field stride).
    auto locate = [&](int ii, int jj, int kk) {
        long long base = B.offset;
        if (a.nbr) {
            const int ox = ii < 0 ? -1 : (ii >= B.nx ? 1 : 0);
            const int oy = jj < 0 ? -1 : (jj >= B.ny ? 1 : 0);
            const int oz = kk < 0 ? -1 : (kk >= B.nz ? 1 : 0);
            if (ox | oy | oz) {
                const int sb = a.nbr[R.block * 27 + (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)];
                if (sb >= 0) {
                    base = a.blocks[sb].offset;
                    ii -= ox * B.nx;
                    jj -= oy * B.ny;
                    kk -= oz * B.nz;
                }
            }
        }
        return base + (long long)(kk + ng) * sz + (long long)(jj + ng) * sy + (ii + ng);
    };
    const int idx[3] = {i, j, k};
    const int n[3] = {B.nx, B.ny, B.nz};
    const double h[3] = {B.dx, B.dy, B.dz};
    // the two stencil samples per direction
    long long smp[3][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int s1 = idx[d] < 0 ? 1 : -1;                 // towards the interior / centred -1
        const int s2 = idx[d] < 0 ? 2 : (idx[d] >= n[d] ? -2 : 1);
        int p1[3] = {i, j, k}, p2[3] = {i, j, k};
        p1[d] += s1;
        p2[d] += s2;
        smp[d][0] = locate(p1[0], p1[1], p1[2]);
        smp[d][1] = locate(p2[0], p2[1], p2[2]);
    }
    const long long e0 = B.offset + (long long)(k + ng) * sz + (long long)(j + ng) * sy + (i + ng);
    double X[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        X[d] = a.origins[3 * R.block + d] + idx[d] * h[d];
    const double r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    const long long fs = B.field_stride;
    double kf[NFIELD];
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) {
        const double c0 = a.u[e0 + f * fs];
        double adv = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            adv += X[d] * d1_radiative(c0, a.u[smp[d][0] + f * fs], a.u[smp[d][1] + f * fs],
                                       idx[d], n[d], h[d]);
        kf[f] = -adv / r - (c0 - flat_value(f)) / r;
    }
    if (a.rhs) {
#pragma unroll
        for (int f = 0; f < NFIELD; ++f)
            a.rhs[e0 + f * fs] = kf[f];
        return;
    }
    double v[NFIELD];
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) {
        const long long e = e0 + f * fs;
        const double u0 = a.u[e];
        const double n1 = (a.read_u1 ? a.u1[e] : 0.0) + a.delta * u0 + a.eps_dt * kf[f];
        double w = a.g1 * u0 + a.g2 * n1;
        if (a.use_u2)
            w += a.g3 * a.u2[e];
        v[f] = w + a.beta_dt * kf[f];
        if (a.write_u1)
            a.u1[e] = n1;
    }
    tile::enforce(v, a.chi_floor, a.alpha_floor);
#pragma unroll
    for (int f = 0; f < NFIELD; ++f)
        a.out[e0 + f * fs] = v[f];
}

}  // namespace

hipError_t launch_radiative(const RadiativeArgs &a, hipStream_t s)
{
    if (a.total <= 0)
        return hipSuccess;
    const long long nb = (a.total + 255) / 256;
    radiative_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace z4c
