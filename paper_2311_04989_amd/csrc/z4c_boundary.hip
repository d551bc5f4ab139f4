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
// see the same values).  The stage combination and the enforcement (det gt
// = 1, tr At = 0, floors) are those of the interior points; there is no
// dissipation.  The stage kernel writes interior points and this one the
// outer ghost points, and both read only the stage input, so the two run in
// either order.
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

// Fields the enforcement couples (the conformal metric, At, chi, alpha);
// the others are finished by their own thread.
__device__ __forceinline__ bool coupled(int f)
{
    return f == CHI || (f >= GXX && f <= GZZ) || (f >= AXX && f <= AZZ) || f == ALPHA;
}

// Where the samples of one outer point sit.
struct PointGeom {
    long long e0;        // element offset of field 0 of the point
    long long smp[3][2]; // element offsets of the two samples per direction
    double X[3];         // coordinates
    double r, h[3];
    int idx[3], n[3];
    long long fs;
};

// A workgroup takes chunks of RAD_PTS consecutive outer points in turn (a
// workgroup lives for many chunks: short-lived workgroups left the SIMDs
// nearly empty) with one thread per (field, point): consecutive threads are
// consecutive points of one field (coalesced), and a thread holds one field,
// so the loads of the stencil are in flight together.  Per chunk the first
// RAD_PTS threads locate the points (outer box, samples through the
// neighbour rule) into LDS; after the combination the enforced fields meet
// in LDS and the first RAD_PTS threads enforce and store them.
constexpr int RAD_PTS = 32;
constexpr int RAD_THREADS = RAD_PTS * NFIELD;   // 704: 11 waves

// One chunk of RAD_PTS outer points (called by every thread of the
// workgroup; the barriers inside are reached by all of them).
__device__ __forceinline__ void radiative_chunk(const RadiativeArgs &a, long long chunk,
                                                PointGeom *geo, double (*vv)[RAD_PTS], int t)
{
    const int f = t / RAD_PTS, lp = t % RAD_PTS;
    const long long gid = chunk * RAD_PTS + lp;
    const bool live = gid < a.total;
    if (f == 0 && live) {
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
        // Element offset (field 0) of stored point (ii, jj, kk) of this block,
        // or, under the neighbour rule, of the point a neighbour copy would
        // bring there (neighbours share nx, ny, nz, ng and the field stride).
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
        PointGeom G;
        G.idx[0] = i;
        G.idx[1] = j;
        G.idx[2] = k;
        G.n[0] = B.nx;
        G.n[1] = B.ny;
        G.n[2] = B.nz;
        G.h[0] = B.dx;
        G.h[1] = B.dy;
        G.h[2] = B.dz;
        G.fs = B.field_stride;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            // samples: the next two towards the interior, else -1 and +1
            const int s1 = G.idx[d] < 0 ? 1 : -1;
            const int s2 = G.idx[d] < 0 ? 2 : (G.idx[d] >= G.n[d] ? -2 : 1);
            int p1[3] = {i, j, k}, p2[3] = {i, j, k};
            p1[d] += s1;
            p2[d] += s2;
            G.smp[d][0] = locate(p1[0], p1[1], p1[2]);
            G.smp[d][1] = locate(p2[0], p2[1], p2[2]);
            G.X[d] = a.origins[3 * R.block + d] + G.idx[d] * G.h[d];
        }
        G.e0 = B.offset + (long long)(k + ng) * sz + (long long)(j + ng) * sy + (i + ng);
        G.r = sqrt(G.X[0] * G.X[0] + G.X[1] * G.X[1] + G.X[2] * G.X[2]);
        geo[lp] = G;
    }
    __syncthreads();
    double v = 0.0;
    long long e = 0;
    if (live) {
        const PointGeom &G = geo[lp];
        const long long fo = f * G.fs;
        e = G.e0 + fo;
        const double c0 = a.u[e];
        double adv = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            adv += G.X[d] * d1_radiative(c0, a.u[G.smp[d][0] + fo], a.u[G.smp[d][1] + fo],
                                         G.idx[d], G.n[d], G.h[d]);
        const double kf = -adv / G.r - (c0 - flat_value(f)) / G.r;
        if (a.rhs) {
            a.rhs[e] = kf;
        } else {
            const double n1 = (a.read_u1 ? a.u1[e] : 0.0) + a.delta * c0 + a.eps_dt * kf;
            double w = a.g1 * c0 + a.g2 * n1;
            if (a.use_u2)
                w += a.g3 * a.u2[e];
            v = w + a.beta_dt * kf;
            if (a.write_u1)
                a.u1[e] = n1;
        }
    }
    if (!a.rhs) {   // uniform
        if (live) {
            if (coupled(f))
                vv[f][lp] = v;
            else
                a.out[e] = v;
        }
        __syncthreads();
        if (f == 0 && live) {
            const PointGeom &G = geo[lp];
            double w[NFIELD];
#pragma unroll
            for (int q = 0; q < NFIELD; ++q)
                w[q] = coupled(q) ? vv[q][lp] : 0.0;
            tile::enforce(w, a.chi_floor, a.alpha_floor);
#pragma unroll
            for (int q = 0; q < NFIELD; ++q)
                if (coupled(q))
                    a.out[G.e0 + q * G.fs] = w[q];
        }
    }
    __syncthreads();   // geo and vv are rewritten by the next chunk
}

__global__ void __launch_bounds__(RAD_THREADS) radiative_kernel(const RadiativeArgs a)
{
    __shared__ PointGeom geo[RAD_PTS];
    __shared__ double vv[NFIELD][RAD_PTS];
    const long long nchunks = (a.total + RAD_PTS - 1) / RAD_PTS;
    for (long long chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x)
        radiative_chunk(a, chunk, geo, vv, threadIdx.x);
}

}  // namespace

hipError_t launch_radiative(const RadiativeArgs &a, hipStream_t s)
{
    if (a.total <= 0)
        return hipSuccess;
    // two resident workgroups of 11 waves per CU, twice over
    const long long nchunks = (a.total + RAD_PTS - 1) / RAD_PTS;
    const long long nb = nchunks < 1024 ? nchunks : 1024;
    radiative_kernel<<<dim3((unsigned)nb), dim3(RAD_THREADS), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace z4c
