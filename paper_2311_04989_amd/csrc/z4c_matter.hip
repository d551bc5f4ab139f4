// z4c_matter.hip -- matter coupling of the Z4c right-hand side: Lagrange
// interpolation between the vertex-centred Z4c grid and the cell-centred
// fluid grid (Sec. 3.2, intergrid communication) and the ADM projections of
// the perfect-fluid / ideal-GRMHD stress-energy tensor (Sec. 2.1, 2.2).
//
// Interpolation is separable and marches along z: a workgroup of 256
// threads owns an ITX x ITY column of outputs and ITZ output planes; for each
// input plane it stages the (ITX + order - 1)(ITY + order - 1) inputs in LDS
// (the next planes already in flight in registers), reduces them along x and
// then y, and each
// thread keeps the y-reduced values of the last `order` planes in registers
// for the z reduction, so every input plane is read once per column and the
// z halo costs (order - 1) / ITZ extra planes.  The ADM projections are
// pointwise, one cell per thread over contiguous chunks of stored cells.
// Both kernels are HBM-bound.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "z4c_internal.h"
#include "z4c_matter.h"

struct z4c_mplan {
    std::vector<z4c_mblock> blocks;
    bool device = false;
    z4c_mblock *blocks_d = nullptr;
    void *cc_tiles_d = nullptr;   // MTile[n_cc]: interpolation columns over every stored cell
    void *vc_tiles_d = nullptr;   // MTile[n_vc]: interpolation columns over vertices [0, nc]
    void *pt_tiles_d = nullptr;   // MTile[n_pt]: point tiles over every stored cell
    int n_cc = 0, n_vc = 0, n_pt = 0;
};

namespace z4c {
namespace {

// interpolation columns: ITX x ITY outputs per plane, ITZ planes, one thread per (x, y)
// (32 x 8 x 16 and four planes in flight measured best on the 8 x 128^3-cell
// level set among 16 x 16, 32 x 16 and 32 x 8 columns of 16 or 32 planes and
// one to six planes in flight)
constexpr int ITX = 32, ITY = 8, ITZ = 16, INT_ = ITX * ITY;
constexpr int PD = 4;   // input planes in flight per workgroup
// ADM projections: chunks of PNT consecutive stored cells, one per thread
constexpr int PNT = 512;

struct MTile {
    int block, i0, j0, k0;   // tile origin (stored CC index, or vertex index)
};

// Weight k of the Lagrange polynomial through O equally spaced nodes,
// evaluated midway between the two central nodes.
template <int O>
__device__ __forceinline__ constexpr double midw(int k)
{
    if constexpr (O == 2)
        return 0.5;
    else if constexpr (O == 4)
        return (k == 0 || k == 3) ? -1.0 / 16.0 : 9.0 / 16.0;
    else
        return (k == 0 || k == 5) ? 3.0 / 256.0 : ((k == 1 || k == 4) ? -25.0 / 256.0 : 150.0 / 256.0);
}

template <int O>
__device__ __forceinline__ double midsum(const double *c, int st)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < O; ++k)
        s += midw<O>(k) * c[k * st];
    return s;
}

// TO_CC: the 7 conformal-geometry fields of the VC state to cells (stored CC
// index in [ngc - ext, ngc + nc + ext)); otherwise the 10 ADM fields from the
// CC sources to vertices [0, nc].
template <int O, bool TO_CC>
__global__ void __launch_bounds__(INT_)
interp_kernel(const z4c_mblock *blocks, const MTile *tiles, int ext, const double *in, double *out)
{
    constexpr int LX = ITX + O - 1, LY = ITY + O - 1;
    constexpr int NPL = LX * LY;                      // one input plane
    constexpr int NLD = (NPL + INT_ - 1) / INT_;      // its values per thread
    constexpr int NP = ITZ + O - 1;                   // input planes per column
    __shared__ double s_pl[NPL];
    __shared__ double s_x[ITX * LY];
    const MTile T = tiles[blockIdx.x];
    const z4c_mblock B = blocks[T.block];
    const int n[3] = {B.ncx, B.ncy, B.ncz};
    const int o[3] = {T.i0, T.j0, T.k0};
    constexpr int TD[3] = {ITX, ITY, ITZ};
    // per direction: the first valid tile-local output index and one past
    // the last, and the stored input index of the first stencil point of
    // tile-local output 0
    int lo[3], hi[3], in0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if constexpr (TO_CC) {
            lo[d] = B.ngc - ext - o[d];
            hi[d] = B.ngc + n[d] + ext - o[d];
            in0[d] = o[d] - B.ngc - O / 2 + 1 + B.ngv;
        } else {
            lo[d] = -o[d];
            hi[d] = n[d] + 1 - o[d];
            in0[d] = o[d] - O / 2 + B.ngc;
        }
    }
    if (hi[0] <= 0 || hi[1] <= 0 || hi[2] <= 0 || lo[0] >= TD[0] || lo[1] >= TD[1]
        || lo[2] >= TD[2])
        return;   // the whole column lies outside this call's range (uniform)
    const int isx = TO_CC ? B.ncx + 1 + 2 * B.ngv : B.ncx + 2 * B.ngc;
    const int isy = TO_CC ? B.ncy + 1 + 2 * B.ngv : B.ncy + 2 * B.ngc;
    const int isz = TO_CC ? B.ncz + 1 + 2 * B.ngv : B.ncz + 2 * B.ngc;
    const int osx = TO_CC ? B.ncx + 2 * B.ngc : B.ncx + 1 + 2 * B.ngv;
    const int osy = TO_CC ? B.ncy + 2 * B.ngc : B.ncy + 1 + 2 * B.ngv;
    const long long ibase = TO_CC ? B.vs_offset : B.ca_offset;
    const long long ifs = TO_CC ? B.vc_stride : B.cc_stride;
    const long long obase = TO_CC ? B.cg_offset : B.vm_offset;
    const long long ofs = TO_CC ? B.cc_stride : B.vc_stride;
    const int og = TO_CC ? 0 : B.ngv;   // stored output index = tile origin + local + og
    const int t = threadIdx.x, tx = t % ITX, ty = t / ITX;
    const bool col_ok = tx >= lo[0] && tx < hi[0] && ty >= lo[1] && ty < hi[1];
    // plane element q of this thread: input offset within a plane (positions
    // outside the stored array are clamped into it; they feed only outputs
    // outside the call's range)
    long long eoff[NLD];
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        const int e = t + q * INT_;
        const int lx = e % LX, ly = e / LX;
        const int gx = min(max(in0[0] + lx, 0), isx - 1);
        const int gy = min(max(in0[1] + ly, 0), isy - 1);
        eoff[q] = gx + (long long)isx * gy;
    }
    const long long pstride = (long long)isx * isy;
    constexpr int NF = TO_CC ? 7 : 10;
    for (int f = 0; f < NF; ++f) {
        const double *src = in + ibase + f * ifs;
        double *dst = out + obase + f * ofs;
        double r[PD][NLD];   // planes p .. p + PD - 1 in flight
        auto load = [&](int p) __attribute__((always_inline)) {
            const long long zo = min(max(in0[2] + p, 0), isz - 1) * pstride;
#pragma unroll
            for (int q = 0; q < NLD; ++q)
                if ((q + 1) * INT_ <= NPL || t + q * INT_ < NPL)
                    r[p % PD][q] = src[zo + eoff[q]];
        };
#pragma unroll
        for (int p = 0; p < PD; ++p)
            load(p);
        double col[O];   // y-reduced values of the last O input planes
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int q = 0; q < NLD; ++q)
                if ((q + 1) * INT_ <= NPL || t + q * INT_ < NPL)
                    s_pl[t + q * INT_] = r[p % PD][q];
            if (p + PD < NP)
                load(p + PD);
            __syncthreads();
            for (int e = t; e < ITX * LY; e += INT_) {
                const int x = e % ITX, ly = e / ITX;
                s_x[e] = midsum<O>(s_pl + ly * LX + x, 1);
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k + 1 < O; ++k)
                col[k] = col[k + 1];
            col[O - 1] = midsum<O>(s_x + ty * ITX + tx, ITX);
            if (p >= O - 1) {
                const int z = p - (O - 1);
                if (col_ok && z >= lo[2] && z < hi[2]) {
                    double v = 0.0;
#pragma unroll
                    for (int k = 0; k < O; ++k)
                        v += midw<O>(k) * col[k];
                    dst[(o[0] + og + tx) + (long long)osx * ((o[1] + og + ty)
                        + (long long)osy * (o[2] + og + z))] = v;
                }
            }
        }
    }
}

// ADM projections at the cells of one tile (stored CC index in
// [ngc - ext, ngc + nc + ext)).
template <bool MHD>
__global__ void __launch_bounds__(PNT)
adm_kernel(const z4c_mblock *blocks, const MTile *tiles, int ext, double gfac, double chi_floor,
           const double *geom, const double *prim, double *adm)
{
    const MTile T = tiles[blockIdx.x];
    const z4c_mblock B = blocks[T.block];
    const int sx = B.ncx + 2 * B.ngc, sy = B.ncy + 2 * B.ngc;
    const long long fs = B.cc_stride;
    const int a0 = B.ngc - ext;
    const int ax = B.ngc + B.ncx + ext, ay = B.ngc + B.ncy + ext, az = B.ngc + B.ncz + ext;
    {
        // T.i0: first stored cell (linear index) of the chunk
        const long long lin = (long long)T.i0 + threadIdx.x;
        if (lin >= (long long)sx * sy * (B.ncz + 2 * B.ngc))
            return;
        const int x = (int)(lin % sx), r = (int)(lin / sx), y = r % sy, z = r / sy;
        if (x < a0 || y < a0 || z < a0 || x >= ax || y >= ay || z >= az)
            return;
        const long long p = lin;
        const double *g = geom + B.cg_offset + p;
        const double *w = prim + B.cp_offset + p;
        const double chi = g[0];
        const double ic = 1.0 / (chi > chi_floor ? chi : chi_floor);
        double gam[6];
#pragma unroll
        for (int q = 0; q < 6; ++q)
            gam[q] = g[(1 + q) * fs] * ic;
        const double rho = w[0], ux = w[fs], uy = w[2 * fs], uz = w[3 * fs], pr = w[4 * fs];
        // ut_i = gamma_ij ut^j
        const double lx = gam[0] * ux + gam[1] * uy + gam[2] * uz;
        const double ly = gam[1] * ux + gam[3] * uy + gam[4] * uz;
        const double lz = gam[2] * ux + gam[4] * uy + gam[5] * uz;
        const double W = sqrt(1.0 + lx * ux + ly * uy + lz * uz);
        const double iW = 1.0 / W;
        const double v[3] = {lx * iW, ly * iW, lz * iW};   // v_i
        const double rhoh = rho + gfac * pr;
        double E, P, ab0 = 0.0, b[3] = {0.0, 0.0, 0.0};
        if constexpr (MHD) {
            const double Bx = w[5 * fs], By = w[6 * fs], Bz = w[7 * fs];
            const double Blx = gam[0] * Bx + gam[1] * By + gam[2] * Bz;
            const double Bly = gam[1] * Bx + gam[3] * By + gam[4] * Bz;
            const double Blz = gam[2] * Bx + gam[4] * By + gam[5] * Bz;
            ab0 = W * (Bx * v[0] + By * v[1] + Bz * v[2]);           // alpha b^0
            const double B2 = Blx * Bx + Bly * By + Blz * Bz;
            const double b2 = (ab0 * ab0 + B2) * iW * iW;
            b[0] = Blx * iW + ab0 * v[0];                             // b_i
            b[1] = Bly * iW + ab0 * v[1];
            b[2] = Blz * iW + ab0 * v[2];
            E = (rhoh + b2) * W * W;
            P = pr + 0.5 * b2;
        } else {
            E = rhoh * W * W;
            P = pr;
        }
        double *o = adm + B.ca_offset + p;
        o[0] = E - P - ab0 * ab0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            o[(1 + i) * fs] = E * v[i] - ab0 * b[i];
        constexpr int QI[6] = {0, 0, 0, 1, 1, 2}, QJ[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int q = 0; q < 6; ++q)
            o[(4 + q) * fs] = E * v[QI[q]] * v[QJ[q]] + P * gam[q] - b[QI[q]] * b[QJ[q]];
    }
}

// ---- primitive <-> conservative maps (ideal gas, Sec. 2.2; Appendix A) ----

struct C2PArgs {
    const z4c_mblock *blocks;
    const MTile *tiles;
    int ext, mhd, max_iter;
    double gm1, chi_floor, rho_atm, p_atm, eps_atm, rho_thr, vmax2, ut_max2, tol;
    const double *geom;
    const double *prim_in;    // p2c
    double *cons;
    double *prim;             // c2p
    int *status;
};

// Cell of one thread (chunk of consecutive stored cells) or -1 when it lies
// outside [ngc - ext, ngc + nc + ext) per direction.
__device__ __forceinline__ long long chunk_cell(const z4c_mblock &B, const MTile &T, int ext)
{
    const int sx = B.ncx + 2 * B.ngc, sy = B.ncy + 2 * B.ngc;
    const long long lin = (long long)T.i0 + threadIdx.x;
    if (lin >= (long long)sx * sy * (B.ncz + 2 * B.ngc))
        return -1;
    const int x = (int)(lin % sx), r = (int)(lin / sx), y = r % sy, z = r / sy;
    const int a0 = B.ngc - ext;
    if (x < a0 || y < a0 || z < a0 || x >= B.ngc + B.ncx + ext || y >= B.ngc + B.ncy + ext
        || z >= B.ngc + B.ncz + ext)
        return -1;
    return lin;
}

// gamma_ij (6, symmetric storage) from the CC geometry, its determinant.
__device__ __forceinline__ double cell_metric(const double *g, long long fs, double chi_floor,
                                              double gam[6])
{
    const double chi = g[0];
    const double ic = 1.0 / (chi > chi_floor ? chi : chi_floor);
#pragma unroll
    for (int q = 0; q < 6; ++q)
        gam[q] = g[(1 + q) * fs] * ic;
    return gam[0] * (gam[3] * gam[5] - gam[4] * gam[4]) - gam[1] * (gam[1] * gam[5] - gam[4] * gam[2])
         + gam[2] * (gam[1] * gam[4] - gam[3] * gam[2]);
}

__device__ __forceinline__ void lower(const double gam[6], const double u[3], double l[3])
{
    l[0] = gam[0] * u[0] + gam[1] * u[1] + gam[2] * u[2];
    l[1] = gam[1] * u[0] + gam[3] * u[1] + gam[4] * u[2];
    l[2] = gam[2] * u[0] + gam[4] * u[1] + gam[5] * u[2];
}

// Conservatives (densitised) of rho, ut^i, p, B^i.  With W^2 = 1 + ut.ut,
// v_i = ut_i / W, alpha b^0 = W B.v, b_i = B_i / W + alpha b^0 v_i,
// b^2 = ((alpha b^0)^2 + B^2) / W^2 (the lapse cancels):
//   D = sg rho W,  S_j = sg ((rho h + b^2) W ut_j - alpha b^0 b_j),
//   tau = sg ((rho h + b^2) W^2 - rho W - (p + b^2/2) - (alpha b^0)^2).
template <bool MHD>
__device__ __forceinline__ void p2c_point(const double gam[6], double sg, double gm1, double rho,
                                          const double ut[3], double p, const double Bu[3],
                                          double q[8])
{
    double ul[3];
    lower(gam, ut, ul);
    const double W2 = 1.0 + ul[0] * ut[0] + ul[1] * ut[1] + ul[2] * ut[2];
    const double W = sqrt(W2);
    const double rhoh = rho + (1.0 + 1.0 / gm1) * p;   // rho (1 + eps) + p
    double ab0 = 0.0, b2 = 0.0, bl[3] = {0.0, 0.0, 0.0};
    if constexpr (MHD) {
        double Bl[3];
        lower(gam, Bu, Bl);
        const double iW = 1.0 / W;
        ab0 = (Bu[0] * ul[0] + Bu[1] * ul[1] + Bu[2] * ul[2]);         // W B.v = B.ut
        b2 = (ab0 * ab0 + Bl[0] * Bu[0] + Bl[1] * Bu[1] + Bl[2] * Bu[2]) * iW * iW;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            bl[i] = Bl[i] * iW + ab0 * ul[i] * iW;                        // v_i = ut_i / W
    }
    const double e = rhoh + b2;
    q[0] = sg * rho * W;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        q[1 + i] = sg * (e * W * ul[i] - ab0 * bl[i]);
    q[4] = sg * (e * W2 - rho * W - (p + 0.5 * b2) - ab0 * ab0);
    if constexpr (MHD) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
            q[5 + i] = sg * Bu[i];
    }
}

template <bool MHD>
__global__ void __launch_bounds__(PNT) p2c_kernel(const C2PArgs a)
{
    const MTile T = a.tiles[blockIdx.x];
    const z4c_mblock B = a.blocks[T.block];
    const long long p = chunk_cell(B, T, a.ext);
    if (p < 0)
        return;
    const long long fs = B.cc_stride;
    double gam[6];
    const double sg = sqrt(cell_metric(a.geom + B.cg_offset + p, fs, a.chi_floor, gam));
    const double *w = a.prim_in + B.cp_offset + p;
    const double ut[3] = {w[fs], w[2 * fs], w[3 * fs]};
    double Bu[3] = {0.0, 0.0, 0.0};
    if constexpr (MHD) {
        Bu[0] = w[5 * fs];
        Bu[1] = w[6 * fs];
        Bu[2] = w[7 * fs];
    }
    double q[8];
    p2c_point<MHD>(gam, sg, a.gm1, w[0], ut, w[4 * fs], Bu, q);
    double *o = a.cons + B.cq_offset + p;
    constexpr int NQ = MHD ? 8 : 5;
#pragma unroll
    for (int i = 0; i < NQ; ++i)
        o[i * fs] = q[i];
}

// Primitive recovery of one cell: the master function of Kastaun, Kalinani &
// Ciolfi in mu = 1 / (h W), with the normalised conservatives q = tau / D,
// r_i = S_i / D, b^i = B^i / sqrt(D) (all undensitised):
//   x = 1 / (1 + mu b^2),  rbar^2 = x^2 r^2 + mu x (1 + x) (r.b)^2,
//   qbar = q - b^2/2 - mu^2 x^2 (b^2 r^2 - (r.b)^2) / 2,
//   v^2 = min(mu^2 rbar^2, vmax^2),  W = 1 / sqrt(1 - v^2),  rho = D / W,
//   eps = max(W (qbar - mu rbar^2) + v^2 W^2 / (1 + W), 0),
//   a = p / (rho (1 + eps)),  h = (1 + eps)(1 + a),
//   nu = max(h / W, (1 + a)(1 + qbar - mu rbar^2)),  mu_hat = 1 / (nu + mu rbar^2),
//   f(mu) = mu - mu_hat(mu).
// For the ideal gas p = (Gamma - 1) rho eps this reduces exactly to
//   eps = max(W (qbar - mu rbar^2 + 1) - 1, 0)   (v^2 W^2 / (1 + W) = W - 1),
//   h = 1 + Gamma eps,  nu = h / W            (the two branches of the max
//   coincide unless eps is clamped, when h / W is the larger),
// and, nu + mu rbar^2 being positive, the root and the sign of f are those
// of g(mu) = mu (nu + mu rbar^2) - 1, which needs no division.
struct Master {
    double q, r2, b2, rb2, gam, vmax2;
    __device__ __forceinline__ double x(double mu) const { return 1.0 / (1.0 + mu * b2); }
    __device__ __forceinline__ double rbar2(double mu) const
    {
        const double xx = x(mu);
        return r2 * xx * xx + mu * xx * (1.0 + xx) * rb2;
    }
    // g(mu); W and eps of the estimate
    __device__ __forceinline__ double f(double mu, double &W, double &eps) const
    {
        const double xx = x(mu);
        const double rb = r2 * xx * xx + mu * xx * (1.0 + xx) * rb2;
        const double qb = q - 0.5 * b2 - 0.5 * mu * mu * xx * xx * (b2 * r2 - rb2);
        const double v2 = fmin(mu * mu * rb, vmax2);
        const double iW = sqrt(1.0 - v2);
        W = 1.0 / iW;
        const double e = W * (qb - mu * rb + 1.0) - 1.0;
        eps = e > 0.0 ? e : 0.0;
        const double nu = (1.0 + gam * eps) * iW;
        return mu * (nu + mu * rb) - 1.0;
    }
};

// Illinois iterations for a sign change of fn on [lo, hi] (fn(lo) < 0 <=
// fn(hi)), every eighth step a bisection (the bracket shrinks whatever fn
// does); converged when the bracket is narrower than tol * hi or one ulp;
// returns false after max_iter steps without convergence.  An end where fn
// is exactly zero is the root: cold gas puts the master function's root on
// the bracket end mu+, where the secant step cannot move and only
// bisections would remain.
template <typename Fn>
__device__ __forceinline__ bool illinois(Fn fn, double lo, double hi, double flo, double fhi,
                                         double tol, int max_iter, double &root)
{
    if (fhi == 0.0 || flo == 0.0) {
        root = fhi == 0.0 ? hi : lo;
        return true;
    }
    int side = 0;
    for (int it = 0; it < max_iter; ++it) {
        double m = (lo * fhi - hi * flo) / (fhi - flo);
        if (!(m > lo && m < hi) || (it & 7) == 7)
            m = 0.5 * (lo + hi);
        if (!(m > lo && m < hi)) {
            root = m;
            return true;
        }
        const double fm = fn(m);
        if (fm == 0.0) {
            root = m;
            return true;
        }
        if (fm < 0.0) {
            lo = m;
            flo = fm;
            if (side == -1)
                fhi *= 0.5;
            side = -1;
        } else {
            hi = m;
            fhi = fm;
            if (side == 1)
                flo *= 0.5;
            side = 1;
        }
        if (hi - lo <= tol * hi) {
            root = 0.5 * (lo + hi);
            return true;
        }
    }
    return false;
}

template <bool MHD>
__global__ void __launch_bounds__(PNT) c2p_kernel(const C2PArgs a)
{
    const MTile T = a.tiles[blockIdx.x];
    const z4c_mblock B = a.blocks[T.block];
    const long long p = chunk_cell(B, T, a.ext);
    if (p < 0)
        return;
    const long long fs = B.cc_stride;
    double gam[6];
    const double det = cell_metric(a.geom + B.cg_offset + p, fs, a.chi_floor, gam);
    const double sg = sqrt(det), isg = 1.0 / sg;
    double *c = a.cons + B.cq_offset + p;
    const double D = c[0] * isg;
    const double Sl[3] = {c[fs] * isg, c[2 * fs] * isg, c[3 * fs] * isg};
    const double tau = c[4 * fs] * isg;
    double Bu[3] = {0.0, 0.0, 0.0};
    if constexpr (MHD) {
        Bu[0] = c[5 * fs] * isg;
        Bu[1] = c[6 * fs] * isg;
        Bu[2] = c[7 * fs] * isg;
    }
    int st = 0;
    double rho = 0.0, pr = 0.0, ut[3] = {0.0, 0.0, 0.0};
    if (!(D >= a.rho_thr)) {
        st = 1;
    } else {
        // inverse metric
        const double id = 1.0 / det;
        const double gi[6] = {(gam[3] * gam[5] - gam[4] * gam[4]) * id,
                              (gam[2] * gam[4] - gam[1] * gam[5]) * id,
                              (gam[1] * gam[4] - gam[2] * gam[3]) * id,
                              (gam[0] * gam[5] - gam[2] * gam[2]) * id,
                              (gam[2] * gam[1] - gam[0] * gam[4]) * id,
                              (gam[0] * gam[3] - gam[1] * gam[1]) * id};
        const double iD = 1.0 / D;
        const double rl[3] = {Sl[0] * iD, Sl[1] * iD, Sl[2] * iD};
        double ru[3];
        lower(gi, rl, ru);                                    // r^i = gamma^ij r_j
        const double sD = 1.0 / sqrt(D);
        const double bu[3] = {Bu[0] * sD, Bu[1] * sD, Bu[2] * sD};
        double bl[3];
        lower(gam, bu, bl);
        Master M;
        M.q = tau * iD;
        M.r2 = rl[0] * ru[0] + rl[1] * ru[1] + rl[2] * ru[2];
        M.b2 = bl[0] * bu[0] + bl[1] * bu[1] + bl[2] * bu[2];
        const double rb = rl[0] * bu[0] + rl[1] * bu[1] + rl[2] * bu[2];
        M.rb2 = rb * rb;
        M.gam = a.gm1 + 1.0;
        M.vmax2 = a.vmax2;
        // bracket [0, mu+]: mu+ is the root of mu sqrt(1 + rbar^2(mu)) - 1
        // (minimum enthalpy 1) when it lies below 1
        double mup = 1.0;
        const double fa1 = sqrt(1.0 + M.rbar2(1.0)) - 1.0;
        bool ok = true;
        if (fa1 > 0.0) {
            auto fa = [&](double mu) { return mu * sqrt(1.0 + M.rbar2(mu)) - 1.0; };
            ok = illinois(fa, 0.0, 1.0, -1.0, fa1, a.tol, a.max_iter, mup);
        }
        double W = 1.0, eps = 0.0, mu = 0.0;
        if (ok) {
            double Wd, ed;
            auto fm = [&](double m) { return M.f(m, Wd, ed); };
            const double f0 = fm(0.0), f1 = fm(mup);
            if (f0 < 0.0 && f1 >= 0.0)
                ok = illinois(fm, 0.0, mup, f0, f1, a.tol, a.max_iter, mu);
            else if (f0 < 0.0 && f1 >= -1e-12)
                mu = mup;   // cold gas (h = 1): the root is mu+ itself, g(mu+) = 0 up to rounding
            else
                ok = false;
        }
        if (!ok) {
            st = 3;
        } else {
            M.f(mu, W, eps);
            const double xx = M.x(mu);
            const double s = mu * xx;
            ut[0] = W * s * (ru[0] + mu * rb * bu[0]);
            ut[1] = W * s * (ru[1] + mu * rb * bu[1]);
            ut[2] = W * s * (ru[2] + mu * rb * bu[2]);
            rho = D / W;
            pr = a.gm1 * rho * eps;
            if (mu * mu * M.rbar2(mu) >= a.vmax2 || W * W - 1.0 > a.ut_max2)
                st = 2;
            else if (!(rho >= a.rho_thr))
                st = 1;
        }
    }
    double *w = a.prim + B.cp_offset + p;
    if (st != 0) {
        rho = a.rho_atm;
        pr = a.p_atm;
        ut[0] = ut[1] = ut[2] = 0.0;
        double q[8];
        p2c_point<MHD>(gam, sg, a.gm1, rho, ut, pr, Bu, q);
#pragma unroll
        for (int i = 0; i < 5; ++i)
            c[i * fs] = q[i];
    }
    w[0] = rho;
    w[fs] = ut[0];
    w[2 * fs] = ut[1];
    w[3 * fs] = ut[2];
    w[4 * fs] = pr;
    if constexpr (MHD) {
        w[5 * fs] = Bu[0];
        w[6 * fs] = Bu[1];
        w[7 * fs] = Bu[2];
    }
    if (a.status)
        a.status[B.cf_offset + p] = st;
}

template <bool TO_CC>
hipError_t launch_interp(int order, const z4c_mplan *P, int ext, const double *in, double *out,
                         hipStream_t s)
{
    const MTile *tiles = (const MTile *)(TO_CC ? P->cc_tiles_d : P->vc_tiles_d);
    const int n = TO_CC ? P->n_cc : P->n_vc;
    if (n == 0)
        return hipSuccess;
    if (order == 2)
        interp_kernel<2, TO_CC><<<n, INT_, 0, s>>>(P->blocks_d, tiles, ext, in, out);
    else if (order == 4)
        interp_kernel<4, TO_CC><<<n, INT_, 0, s>>>(P->blocks_d, tiles, ext, in, out);
    else
        interp_kernel<6, TO_CC><<<n, INT_, 0, s>>>(P->blocks_d, tiles, ext, in, out);
    return hipGetLastError();
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

z4c_status check_plan(const z4c_mplan *P)
{
    if (!P)
        return set_error(Z4C_EINVAL, "mplan is NULL");
    if (!P->device)
        return set_error(Z4C_ENODEV, "mplan was created without a device");
    return Z4C_OK;
}

z4c_status check_order(int order)
{
    if (order != 2 && order != 4 && order != 6)
        return set_error(Z4C_EINVAL, "interpolation order must be 2, 4 or 6");
    return Z4C_OK;
}

}  // namespace
}  // namespace z4c

using namespace z4c;

extern "C" {

z4c_status z4c_mplan_create(const z4c_mblock *blocks, int nblocks, int flags, z4c_mplan **out)
{
    if (!out)
        return set_error(Z4C_EINVAL, "out is NULL");
    *out = nullptr;
    if (!blocks || nblocks < 1)
        return set_error(Z4C_EINVAL, "blocks is NULL or nblocks < 1");
    if (flags & ~Z4C_PLAN_NO_DEVICE)
        return set_error(Z4C_EINVAL, "unknown flags");
    std::vector<MTile> cc, vc, pt;
    for (int b = 0; b < nblocks; ++b) {
        const z4c_mblock &B = blocks[b];
        char buf[160];
        if (B.ncx < 1 || B.ncy < 1 || B.ncz < 1 || B.ngv < 0 || B.ngc < 0) {
            snprintf(buf, sizeof buf, "block %d: cells must be >= 1 and ghosts >= 0", b);
            return set_error(Z4C_EINVAL, buf);
        }
        if (B.vs_offset < 0 || B.vm_offset < 0 || B.cg_offset < 0 || B.cp_offset < 0
            || B.ca_offset < 0 || B.cq_offset < 0 || B.cf_offset < 0 || B.vc_stride < 0
            || B.cc_stride < 0) {
            snprintf(buf, sizeof buf, "block %d: offsets and strides must be >= 0", b);
            return set_error(Z4C_EINVAL, buf);
        }
        const long long nv = (long long)(B.ncx + 1 + 2 * B.ngv) * (B.ncy + 1 + 2 * B.ngv)
                           * (B.ncz + 1 + 2 * B.ngv);
        const long long nc = (long long)(B.ncx + 2 * B.ngc) * (B.ncy + 2 * B.ngc)
                           * (B.ncz + 2 * B.ngc);
        if (B.vc_stride < nv || B.cc_stride < nc) {
            snprintf(buf, sizeof buf, "block %d: a field stride is smaller than the stored field", b);
            return set_error(Z4C_EINVAL, buf);
        }
        const int sc[3] = {B.ncx + 2 * B.ngc, B.ncy + 2 * B.ngc, B.ncz + 2 * B.ngc};
        for (int k = 0; k < sc[2]; k += ITZ)
            for (int j = 0; j < sc[1]; j += ITY)
                for (int i = 0; i < sc[0]; i += ITX)
                    cc.push_back({b, i, j, k});
        for (int k = 0; k <= B.ncz; k += ITZ)
            for (int j = 0; j <= B.ncy; j += ITY)
                for (int i = 0; i <= B.ncx; i += ITX)
                    vc.push_back({b, i, j, k});
        const long long ncs = (long long)sc[0] * sc[1] * sc[2];
        if (ncs > INT32_MAX) {
            snprintf(buf, sizeof buf, "block %d: more than 2^31 stored cells", b);
            return set_error(Z4C_EINVAL, buf);
        }
        for (long long c = 0; c < ncs; c += PNT)
            pt.push_back({b, (int)c, 0, 0});
    }
    if (cc.size() > (size_t)INT32_MAX || vc.size() > (size_t)INT32_MAX
        || pt.size() > (size_t)INT32_MAX)
        return set_error(Z4C_EINVAL, "too many tiles");
    z4c_mplan *P = new z4c_mplan;
    P->blocks.assign(blocks, blocks + nblocks);
    P->n_cc = (int)cc.size();
    P->n_vc = (int)vc.size();
    P->n_pt = (int)pt.size();
    if (!(flags & Z4C_PLAN_NO_DEVICE)) {
        hipError_t e = hipMalloc(&P->blocks_d, sizeof(z4c_mblock) * nblocks);
        if (e == hipSuccess)
            e = hipMalloc(&P->cc_tiles_d, sizeof(MTile) * cc.size());
        if (e == hipSuccess)
            e = hipMalloc(&P->vc_tiles_d, sizeof(MTile) * vc.size());
        if (e == hipSuccess)
            e = hipMalloc(&P->pt_tiles_d, sizeof(MTile) * pt.size());
        if (e == hipSuccess)
            e = hipMemcpy(P->blocks_d, blocks, sizeof(z4c_mblock) * nblocks,
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(P->cc_tiles_d, cc.data(), sizeof(MTile) * cc.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(P->vc_tiles_d, vc.data(), sizeof(MTile) * vc.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(P->pt_tiles_d, pt.data(), sizeof(MTile) * pt.size(),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            z4c_mplan_destroy(P);
            return e == hipErrorOutOfMemory ? set_error(Z4C_ENOMEM, "hipMalloc(mplan tables)")
                                            : set_hip_error(e, "mplan tables");
        }
        P->device = true;
    }
    *out = P;
    return Z4C_OK;
}

z4c_status z4c_mplan_destroy(z4c_mplan *P)
{
    if (!P)
        return Z4C_OK;
    if (P->blocks_d)
        (void)hipFree(P->blocks_d);
    if (P->cc_tiles_d)
        (void)hipFree(P->cc_tiles_d);
    if (P->vc_tiles_d)
        (void)hipFree(P->vc_tiles_d);
    if (P->pt_tiles_d)
        (void)hipFree(P->pt_tiles_d);
    delete P;
    return Z4C_OK;
}

z4c_status z4c_metric_to_cc(const z4c_mplan *P, int order, int ext, const double *u,
                            double *geom, void *stream)
{
    z4c_status st;
    if (!P)
        return set_error(Z4C_EINVAL, "mplan is NULL");
    if ((st = check_order(order)) != Z4C_OK)
        return st;
    if (!u || !geom)
        return set_error(Z4C_EINVAL, "u and geom must not be NULL");
    if ((const void *)u == (const void *)geom)
        return set_error(Z4C_EINVAL, "geom must not alias u");
    if (!aligned8(u) || !aligned8(geom))
        return set_error(Z4C_EALIGN, "arrays must be 8-byte aligned");
    if (ext < 0)
        return set_error(Z4C_EINVAL, "ext must be >= 0");
    for (size_t b = 0; b < P->blocks.size(); ++b) {
        const z4c_mblock &B = P->blocks[b];
        char buf[160];
        if (ext > B.ngc) {
            snprintf(buf, sizeof buf, "block %zu: ext %d exceeds the %d stored ghost cells", b, ext,
                     B.ngc);
            return set_error(Z4C_EINVAL, buf);
        }
        if (B.ngv < order / 2 - 1 + ext) {
            snprintf(buf, sizeof buf, "block %zu: order %d to %d ghost cells needs %d ghost "
                     "vertices, %d stored", b, order, ext, order / 2 - 1 + ext, B.ngv);
            return set_error(Z4C_ENOGHOST, buf);
        }
    }
    if ((st = check_plan(P)) != Z4C_OK)
        return st;
    const hipError_t e = launch_interp<true>(order, P, ext, u, geom, (hipStream_t)stream);
    return e == hipSuccess ? Z4C_OK : set_hip_error(e, "interpolation kernel launch");
}

z4c_status z4c_sources_to_vc(const z4c_mplan *P, int order, const double *adm, double *matter,
                             void *stream)
{
    z4c_status st;
    if (!P)
        return set_error(Z4C_EINVAL, "mplan is NULL");
    if ((st = check_order(order)) != Z4C_OK)
        return st;
    if (!adm || !matter)
        return set_error(Z4C_EINVAL, "adm and matter must not be NULL");
    if ((const void *)adm == (const void *)matter)
        return set_error(Z4C_EINVAL, "matter must not alias adm");
    if (!aligned8(adm) || !aligned8(matter))
        return set_error(Z4C_EALIGN, "arrays must be 8-byte aligned");
    for (size_t b = 0; b < P->blocks.size(); ++b) {
        const z4c_mblock &B = P->blocks[b];
        if (B.ngc < order / 2) {
            char buf[160];
            snprintf(buf, sizeof buf, "block %zu: order %d needs %d ghost cells, %d stored", b,
                     order, order / 2, B.ngc);
            return set_error(Z4C_ENOGHOST, buf);
        }
    }
    if ((st = check_plan(P)) != Z4C_OK)
        return st;
    const hipError_t e = launch_interp<false>(order, P, 0, adm, matter, (hipStream_t)stream);
    return e == hipSuccess ? Z4C_OK : set_hip_error(e, "interpolation kernel launch");
}

z4c_status z4c_adm_sources(const z4c_mplan *P, const z4c_fluid *fluid, int ext,
                           const double *geom, const double *prim, double *adm, void *stream)
{
    z4c_status st;
    if (!P)
        return set_error(Z4C_EINVAL, "mplan is NULL");
    if (!fluid || !geom || !prim || !adm)
        return set_error(Z4C_EINVAL, "fluid, geom, prim and adm must not be NULL");
    if (fluid->mhd != 0 && fluid->mhd != 1)
        return set_error(Z4C_EINVAL, "mhd must be 0 or 1");
    if (!(fluid->gamma_ad > 1.0) || !std::isfinite(fluid->gamma_ad))
        return set_error(Z4C_EINVAL, "gamma_ad must be finite and > 1");
    if (!(fluid->chi_floor > 0.0) || !std::isfinite(fluid->chi_floor))
        return set_error(Z4C_EINVAL, "chi_floor must be finite and > 0");
    if ((const void *)adm == (const void *)geom || (const void *)adm == (const void *)prim)
        return set_error(Z4C_EINVAL, "adm must not alias geom or prim");
    if (!aligned8(geom) || !aligned8(prim) || !aligned8(adm))
        return set_error(Z4C_EALIGN, "arrays must be 8-byte aligned");
    if (ext < 0)
        return set_error(Z4C_EINVAL, "ext must be >= 0");
    for (size_t b = 0; b < P->blocks.size(); ++b)
        if (ext > P->blocks[b].ngc) {
            char buf[160];
            snprintf(buf, sizeof buf, "block %zu: ext %d exceeds the %d stored ghost cells", b,
                     ext, P->blocks[b].ngc);
            return set_error(Z4C_EINVAL, buf);
        }
    if ((st = check_plan(P)) != Z4C_OK)
        return st;
    if (P->n_pt == 0)
        return Z4C_OK;
    const double gfac = fluid->gamma_ad / (fluid->gamma_ad - 1.0);
    const MTile *tiles = (const MTile *)P->pt_tiles_d;
    if (fluid->mhd)
        adm_kernel<true><<<P->n_pt, PNT, 0, (hipStream_t)stream>>>(
            P->blocks_d, tiles, ext, gfac, fluid->chi_floor, geom, prim, adm);
    else
        adm_kernel<false><<<P->n_pt, PNT, 0, (hipStream_t)stream>>>(
            P->blocks_d, tiles, ext, gfac, fluid->chi_floor, geom, prim, adm);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? Z4C_OK : set_hip_error(e, "ADM source kernel launch");
}

static z4c_status c2p_common(const z4c_mplan *P, const z4c_c2p_params *c, int ext,
                             const void *geom, const void *a, const void *b, C2PArgs &A)
{
    if (!P)
        return set_error(Z4C_EINVAL, "mplan is NULL");
    if (!c || !geom || !a || !b)
        return set_error(Z4C_EINVAL, "params and arrays must not be NULL");
    if (c->mhd != 0 && c->mhd != 1)
        return set_error(Z4C_EINVAL, "mhd must be 0 or 1");
    if (!(c->gamma_ad > 1.0) || !std::isfinite(c->gamma_ad))
        return set_error(Z4C_EINVAL, "gamma_ad must be finite and > 1");
    if (!(c->chi_floor > 0.0) || !std::isfinite(c->chi_floor))
        return set_error(Z4C_EINVAL, "chi_floor must be finite and > 0");
    if (!(c->rho_atm > 0.0) || !(c->p_atm >= 0.0) || !(c->f_thr >= 0.0)
        || !std::isfinite(c->rho_atm) || !std::isfinite(c->p_atm) || !std::isfinite(c->f_thr))
        return set_error(Z4C_EINVAL, "rho_atm > 0, p_atm >= 0 and f_thr >= 0 must be finite");
    if (!(c->ut_max > 0.0) || !std::isfinite(c->ut_max) || !(c->tol > 0.0) || c->max_iter < 1)
        return set_error(Z4C_EINVAL, "ut_max and tol must be > 0, max_iter >= 1");
    if (a == b || a == geom || b == geom)
        return set_error(Z4C_EINVAL, "geom, input and output arrays must not alias");
    if (!aligned8(geom) || !aligned8(a) || !aligned8(b))
        return set_error(Z4C_EALIGN, "arrays must be 8-byte aligned");
    if (ext < 0)
        return set_error(Z4C_EINVAL, "ext must be >= 0");
    for (size_t k = 0; k < P->blocks.size(); ++k)
        if (ext > P->blocks[k].ngc) {
            char buf[160];
            snprintf(buf, sizeof buf, "block %zu: ext %d exceeds the %d stored ghost cells", k,
                     ext, P->blocks[k].ngc);
            return set_error(Z4C_EINVAL, buf);
        }
    z4c_status st = check_plan(P);
    if (st != Z4C_OK)
        return st;
    A = C2PArgs{};
    A.blocks = P->blocks_d;
    A.tiles = (const MTile *)P->pt_tiles_d;
    A.ext = ext;
    A.mhd = c->mhd;
    A.max_iter = c->max_iter;
    A.gm1 = c->gamma_ad - 1.0;
    A.chi_floor = c->chi_floor;
    A.rho_atm = c->rho_atm;
    A.p_atm = c->p_atm;
    A.eps_atm = c->p_atm / ((c->gamma_ad - 1.0) * c->rho_atm);
    A.rho_thr = c->f_thr * c->rho_atm;
    A.ut_max2 = c->ut_max * c->ut_max;
    A.vmax2 = A.ut_max2 / (1.0 + A.ut_max2);
    A.tol = c->tol;
    A.geom = (const double *)geom;
    return Z4C_OK;
}

z4c_status z4c_p2c(const z4c_mplan *P, const z4c_c2p_params *c, int ext, const double *geom,
                   const double *prim, double *cons, void *stream)
{
    C2PArgs A;
    const z4c_status st = c2p_common(P, c, ext, geom, prim, cons, A);
    if (st != Z4C_OK)
        return st;
    if (P->n_pt == 0)
        return Z4C_OK;
    A.prim_in = prim;
    A.cons = cons;
    if (c->mhd)
        p2c_kernel<true><<<P->n_pt, PNT, 0, (hipStream_t)stream>>>(A);
    else
        p2c_kernel<false><<<P->n_pt, PNT, 0, (hipStream_t)stream>>>(A);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? Z4C_OK : set_hip_error(e, "p2c kernel launch");
}

z4c_status z4c_c2p(const z4c_mplan *P, const z4c_c2p_params *c, int ext, const double *geom,
                   double *cons, double *prim, int *status, void *stream)
{
    C2PArgs A;
    const z4c_status st = c2p_common(P, c, ext, geom, cons, prim, A);
    if (st != Z4C_OK)
        return st;
    if (status && (((uintptr_t)status & 3u) != 0))
        return set_error(Z4C_EALIGN, "status must be 4-byte aligned");
    if (P->n_pt == 0)
        return Z4C_OK;
    A.cons = cons;
    A.prim = prim;
    A.status = status;
    if (c->mhd)
        c2p_kernel<true><<<P->n_pt, PNT, 0, (hipStream_t)stream>>>(A);
    else
        c2p_kernel<false><<<P->n_pt, PNT, 0, (hipStream_t)stream>>>(A);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? Z4C_OK : set_hip_error(e, "c2p kernel launch");
}

}  // extern "C"
