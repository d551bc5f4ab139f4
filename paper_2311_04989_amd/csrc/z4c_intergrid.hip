// z4c_intergrid.hip -- transfers between refinement levels of the
// vertex-centred Z4c grid (ratio 2): prolongation coarse -> fine by
// Lagrange interpolation and restriction fine -> coarse by injection
// (Sec. 3.2: vertex-centred variables keep these operators simple at high
// order).
// Prolongation: the host cuts every destination box into tiles of at most
// 16 x 16 x 4 fine points and records the coarse index range (footprint)
// each tile reads; one workgroup per (tile, field) stages the footprint in
// LDS and applies the three direction rules one after the other (x, then
// y, then z; an even fine index copies, an odd one takes `order` taps), the
// z pass writing the fine points to HBM.  Restriction: one thread per
// (destination point, field), the transfer found by a binary search over the
// prefix sums of the box sizes.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "z4c_internal.h"

namespace z4c {
namespace {

// A tile of a prolongation box: fine points lo .. lo + n - 1 per direction
// (index of the fine block, ghosts negative), the coarse points s0 ..
// s0 + sn - 1 their stencils reach, and the order of the three direction
// passes (dir[0] first).
struct XTile {
    int t;
    int lo[3], n[3], s0[3], sn[3];
    int dir[3];
};
static_assert(sizeof(XTile) == 64, "XTile layout");

// LDS of a tile (doubles): A holds the footprint, then the second pass's
// result; B the first pass's result.
constexpr int XA = 2048, XB = 2048;

}  // namespace
}  // namespace z4c

struct z4c_xplan {
    const z4c_plan *plan = nullptr;
    int order = 0;
    bool device = false;
    std::vector<z4c_transfer> pro, res;
    std::vector<z4c::XTile> tiles;
    long long lds_a = 0, lds_b = 0;   // LDS (doubles) of the largest tile
    z4c_transfer *pro_d = nullptr, *res_d = nullptr;
    z4c::XTile *tiles_d = nullptr;
    long long *res_start_d = nullptr;   // prefix sums of the restriction boxes, n + 1
    long long res_total = 0;
};

namespace z4c {
namespace {

template <int O>
__device__ __forceinline__ double mid_weight(int k)
{
    if constexpr (O == 2)
        return 0.5;
    else if constexpr (O == 4)
        return (k == 0 || k == 3) ? -1.0 / 16.0 : 9.0 / 16.0;
    else
        return (k == 0 || k == 5) ? 3.0 / 256.0 : ((k == 1 || k == 4) ? -25.0 / 256.0 : 150.0 / 256.0);
}

// transfer of global destination point r, and r's index within it
__device__ __forceinline__ int find_transfer(const long long *start, int n, long long r)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ long long point_index(const z4c_block &B, int i, int j, int k)
{
    const long long sx = B.nx + 2LL * B.ng, sy = B.ny + 2LL * B.ng;
    return (i + B.ng) + sx * ((j + B.ng) + sy * (long long)(k + B.ng));
}

// first coarse tap of fine index i (c0: coarse index of fine index 0)
template <int O>
__device__ __forceinline__ int first_tap(int i, int c0)
{
    return (i & 1) == 0 ? c0 + (i >> 1) : c0 + ((i - 1) >> 1) - (O / 2 - 1);
}

// one direction rule at fine index i over values p[first * stride], ...
template <int O>
__device__ __forceinline__ double rule(const double *p, int first, int i, int stride)
{
    if ((i & 1) == 0)
        return p[first * stride];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < O; ++k)
        s += mid_weight<O>(k) * p[(first + k) * stride];
    return s;
}

// e / d and e % d for e * d < 2^20 (every index and extent of a tile):
// e * ceil(2^20 / d) / 2^20 errs by less than e / 2^20 < 1 / d.
struct SmallDiv {
    unsigned m, d;
    __device__ explicit SmallDiv(unsigned d_) : m(((1u << 20) + d_ - 1) / d_), d(d_) {}
    __device__ unsigned q(unsigned e) const { return (e * m) >> 20; }
};

// One direction pass (direction D) of a tile: `in` holds i0 x i1 x i2
// values (x fastest); the result has T.n[D] points in direction D, written
// to `out` (x fastest) or, for the last pass, to the fine block's points.
// D is a template argument so that every index into the tile stays in
// registers.
template <int O, int D, bool LAST>
__device__ __forceinline__ void dir_pass(const double *in, double *out, int i0, int i1, int i2,
                                         const XTile &T, const z4c_transfer &R,
                                         const z4c_block &F, double *dst)
{
    const int o0 = D == 0 ? T.n[0] : i0, o1 = D == 1 ? T.n[1] : i1, o2 = D == 2 ? T.n[2] : i2;
    const int st1 = i0, st2 = i0 * i1;
    const int std_ = D == 0 ? 1 : (D == 1 ? st1 : st2);
    const SmallDiv d0(o0), d1(o1);
    const unsigned total = o0 * o1 * o2;
    constexpr int NK = (LAST ? 1024 : XA) / 256;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const unsigned e = threadIdx.x + 256u * k;
        if (e < total) {
            const unsigned r = d0.q(e), x = e - r * o0;
            const unsigned z = d1.q(r), y = r - z * o1;
            const int c = D == 0 ? (int)x : (D == 1 ? (int)y : (int)z);
            const int i = T.lo[D] + c;
            const int first = first_tap<O>(i, R.c0[D]) - T.s0[D];
            const int base = (int)x + st1 * (int)y + st2 * (int)z + (first - c) * std_;
            const double v = rule<O>(in + base, 0, i, std_);
            if constexpr (LAST)
                dst[point_index(F, T.lo[0] + (int)x, T.lo[1] + (int)y, T.lo[2] + (int)z)] = v;
            else
                out[e] = v;
        }
    }
}

template <int O, bool LAST>
__device__ __forceinline__ void any_pass(int d, const double *in, double *out, int &i0, int &i1,
                                         int &i2, const XTile &T, const z4c_transfer &R,
                                         const z4c_block &F, double *dst)
{
    if (d == 0) {
        dir_pass<O, 0, LAST>(in, out, i0, i1, i2, T, R, F, dst);
        i0 = T.n[0];
    } else if (d == 1) {
        dir_pass<O, 1, LAST>(in, out, i0, i1, i2, T, R, F, dst);
        i1 = T.n[1];
    } else {
        dir_pass<O, 2, LAST>(in, out, i0, i1, i2, T, R, F, dst);
        i2 = T.n[2];
    }
}

template <int O>
__global__ void __launch_bounds__(256)
prolong_kernel(const z4c_block *blocks, const z4c_transfer *tr, const XTile *tiles, int a_size,
               double *u)
{
    extern __shared__ double lds[];
    double *A = lds, *Bx = lds + a_size;
    const XTile T = tiles[blockIdx.x];
    const int f = blockIdx.y;
    const z4c_transfer R = tr[T.t];
    const z4c_block C = blocks[R.coarse];
    const z4c_block F = blocks[R.fine];
    const unsigned tid = threadIdx.x;
    int i0 = T.sn[0], i1 = T.sn[1], i2 = T.sn[2];
    // footprint -> A (x fastest): every load issued before the first LDS write
    {
        const SmallDiv ds0(i0), ds1(i1);
        const long long csx = C.nx + 2LL * C.ng, csy = C.ny + 2LL * C.ng;
        const double *src = u + C.offset + (long long)f * C.field_stride
                          + point_index(C, T.s0[0], T.s0[1], T.s0[2]);
        const unsigned ns = i0 * i1 * i2;
        double v[XA / 256];
#pragma unroll
        for (int k = 0; k < XA / 256; ++k) {
            const unsigned e = tid + 256u * k;
            if (e < ns) {
                const unsigned r = ds0.q(e), x = e - r * i0;
                const unsigned z = ds1.q(r), y = r - z * i1;
                v[k] = src[x + csx * (y + csy * (long long)z)];
            }
        }
#pragma unroll
        for (int k = 0; k < XA / 256; ++k) {
            const unsigned e = tid + 256u * k;
            if (e < ns)
                A[e] = v[k];
        }
    }
    __syncthreads();
    double *dst = u + F.offset + (long long)f * F.field_stride;
    any_pass<O, false>(T.dir[0], A, Bx, i0, i1, i2, T, R, F, dst);
    __syncthreads();
    any_pass<O, false>(T.dir[1], Bx, A, i0, i1, i2, T, R, F, dst);
    __syncthreads();
    any_pass<O, true>(T.dir[2], A, nullptr, i0, i1, i2, T, R, F, dst);
}

__global__ void __launch_bounds__(256)
restrict_kernel(const z4c_block *blocks, const z4c_transfer *tr, const long long *start, int n,
                long long total, double *u)
{
    for (long long r = blockIdx.x * 256LL + threadIdx.x; r < total;
         r += (long long)gridDim.x * 256) {
        const int t = find_transfer(start, n, r);
        const z4c_transfer T = tr[t];
        const long long loc = r - start[t];
        const int bx = T.hi[0] - T.lo[0], by = T.hi[1] - T.lo[1];
        const int cj[3] = {T.lo[0] + (int)(loc % bx), T.lo[1] + (int)((loc / bx) % by),
                           T.lo[2] + (int)(loc / ((long long)bx * by))};
        const z4c_block C = blocks[T.coarse];
        const z4c_block F = blocks[T.fine];
        const long long src = F.offset + point_index(F, 2 * (cj[0] - T.c0[0]),
                                                     2 * (cj[1] - T.c0[1]), 2 * (cj[2] - T.c0[2]));
        const long long dst = C.offset + point_index(C, cj[0], cj[1], cj[2]);
        double v[NFIELD];   // every load issued before the first store
#pragma unroll
        for (int f = 0; f < NFIELD; ++f)
            v[f] = u[src + f * F.field_stride];
#pragma unroll
        for (int f = 0; f < NFIELD; ++f)
            u[dst + f * C.field_stride] = v[f];
    }
}

bool same_ratio(double c, double f) { return std::fabs(c - 2.0 * f) <= 1e-12 * c; }

// Validates one transfer; the source index range of its destination box.
z4c_status check_transfer(const std::vector<z4c_block> &B, const z4c_transfer &T, bool pro,
                          int order, int idx)
{
    char buf[200];
    const int nb = (int)B.size();
    if (T.coarse < 0 || T.coarse >= nb || T.fine < 0 || T.fine >= nb || T.coarse == T.fine) {
        snprintf(buf, sizeof buf, "transfer %d: bad block indices", idx);
        return set_error(Z4C_EINVAL, buf);
    }
    const z4c_block &C = B[T.coarse], &F = B[T.fine];
    if (!same_ratio(C.dx, F.dx) || !same_ratio(C.dy, F.dy) || !same_ratio(C.dz, F.dz)) {
        snprintf(buf, sizeof buf, "transfer %d: coarse spacing is not twice the fine spacing", idx);
        return set_error(Z4C_EINVAL, buf);
    }
    const z4c_block &D = pro ? F : C, &S = pro ? C : F;
    const int dn[3] = {D.nx, D.ny, D.nz}, sn[3] = {S.nx, S.ny, S.nz};
    for (int d = 0; d < 3; ++d) {
        if (T.lo[d] > T.hi[d] || T.lo[d] < -D.ng || T.hi[d] > dn[d] + D.ng) {
            snprintf(buf, sizeof buf, "transfer %d: destination box outside the stored points",
                     idx);
            return set_error(Z4C_EINVAL, buf);
        }
        if (T.lo[d] == T.hi[d])
            continue;
        int smin = INT32_MAX, smax = INT32_MIN;
        for (int i = T.lo[d]; i < T.hi[d]; ++i) {
            int a, b;
            if (pro) {
                if (i % 2 == 0) {
                    a = b = T.c0[d] + i / 2;
                } else {
                    const int left = T.c0[d] + (i - 1) / 2;   // i - 1 even
                    a = left - (order / 2 - 1);
                    b = left + order / 2;
                }
            } else {
                a = b = 2 * (i - T.c0[d]);
            }
            smin = std::min(smin, a);
            smax = std::max(smax, b);
        }
        if (smin < -S.ng || smax >= sn[d] + S.ng) {
            snprintf(buf, sizeof buf, "transfer %d: source points [%d, %d] of direction %d "
                     "outside the stored [%d, %d)", idx, smin, smax, d, -S.ng, sn[d] + S.ng);
            return set_error(Z4C_ENOGHOST, buf);
        }
    }
    return Z4C_OK;
}

bool boxes_overlap(const z4c_transfer &a, const z4c_transfer &b)
{
    for (int d = 0; d < 3; ++d)
        if (a.hi[d] <= b.lo[d] || b.hi[d] <= a.lo[d])
            return false;
    return true;
}

// Writes of one kind never reach what the same kind reads, nor each other.
z4c_status check_set(const std::vector<z4c_transfer> &v, bool pro)
{
    for (size_t a = 0; a < v.size(); ++a) {
        const int wa = pro ? v[a].fine : v[a].coarse;
        for (size_t b = 0; b < v.size(); ++b) {
            const int rb = pro ? v[b].coarse : v[b].fine;
            if (wa == rb)
                return set_error(Z4C_EINVAL, "a block is written by one transfer and read by "
                                             "another of the same kind");
            if (b > a && wa == (pro ? v[b].fine : v[b].coarse) && boxes_overlap(v[a], v[b]))
                return set_error(Z4C_EINVAL, "two transfers write the same points");
        }
    }
    return Z4C_OK;
}

std::vector<long long> prefix(const std::vector<z4c_transfer> &v)
{
    std::vector<long long> s(v.size() + 1, 0);
    for (size_t t = 0; t < v.size(); ++t) {
        const long long n = (long long)(v[t].hi[0] - v[t].lo[0]) * (v[t].hi[1] - v[t].lo[1])
                          * (v[t].hi[2] - v[t].lo[2]);
        s[t + 1] = s[t] + n;
    }
    return s;
}

// coarse index range [s0, s0 + sn) the rule reaches from fine indices
// lo .. lo + n - 1 (c0: coarse index of fine index 0)
void footprint(int lo, int n, int c0, int order, int &s0, int &sn)
{
    int a = INT32_MAX, b = INT32_MIN;
    for (int i = lo; i < lo + n; ++i) {
        int first, last;
        if (i % 2 == 0) {
            first = last = c0 + i / 2;
        } else {
            const int left = c0 + (i - 1) / 2;   // i - 1 even
            first = left - (order / 2 - 1);
            last = left + order / 2;
        }
        a = std::min(a, first);
        b = std::max(b, last);
    }
    s0 = a;
    sn = b - a + 1;
}

// LDS (doubles) of a tile: a = footprint and second pass, b = first pass.
void tile_lds(const XTile &T, long long &a, long long &b)
{
    long long dims[3] = {T.sn[0], T.sn[1], T.sn[2]};
    const long long S = dims[0] * dims[1] * dims[2];
    dims[T.dir[0]] = T.n[T.dir[0]];
    b = dims[0] * dims[1] * dims[2];
    dims[T.dir[1]] = T.n[T.dir[1]];
    a = std::max(S, dims[0] * dims[1] * dims[2]);
}

// Cuts every prolongation box into tiles whose LDS needs fit XA and XB.
std::vector<XTile> make_tiles(const std::vector<z4c_transfer> &v, int order)
{
    // footprint bound of n fine points: ceil(n / 2) - 1 + order
    auto sb = [order](int n) { return (n + 1) / 2 + order; };
    std::vector<XTile> out;
    for (size_t t = 0; t < v.size(); ++t) {
        const z4c_transfer &R = v[t];
        const int bx = R.hi[0] - R.lo[0], by = R.hi[1] - R.lo[1], bz = R.hi[2] - R.lo[2];
        if (bx == 0 || by == 0 || bz == 0)
            continue;
        int tx = std::min(bx, 16), ty = std::min(by, 16);
        int tz = std::min({bz, 16, std::max(1, 1024 / (tx * ty))});
        for (;;) {
            const long long S = (long long)sb(tx) * sb(ty) * sb(tz);
            const long long Xs = (long long)sb(tz) * sb(ty) * tx, Ys = (long long)sb(tz) * ty * tx;
            if (std::max(S, Ys) <= XA && Xs <= XB)
                break;
            if (tz > 1)
                --tz;
            else if (ty > 1)
                --ty;
            else
                --tx;
        }
        for (int z = R.lo[2]; z < R.hi[2]; z += tz)
            for (int y = R.lo[1]; y < R.hi[1]; y += ty)
                for (int x = R.lo[0]; x < R.hi[0]; x += tx) {
                    XTile T{};
                    T.t = (int)t;
                    const int lo[3] = {x, y, z}, tn[3] = {tx, ty, tz};
                    for (int d = 0; d < 3; ++d) {
                        T.lo[d] = lo[d];
                        T.n[d] = std::min(tn[d], R.hi[d] - lo[d]);
                        footprint(T.lo[d], T.n[d], R.c0[d], order, T.s0[d], T.sn[d]);
                        T.dir[d] = d;
                    }
                    // the most shrinking direction first keeps the
                    // intermediate results small
                    std::stable_sort(T.dir, T.dir + 3, [&T](int p, int q) {
                        return (long long)T.n[p] * T.sn[q] < (long long)T.n[q] * T.sn[p];
                    });
                    long long a, b;
                    tile_lds(T, a, b);
                    if (std::max(a, b) > XA) {   // fall back to x, y, z (fits by the bound)
                        for (int d = 0; d < 3; ++d)
                            T.dir[d] = d;
                    }
                    out.push_back(T);
                }
    }
    return out;
}

int grid_for(long long total)
{
    const long long g = (total + 255) / 256;
    return (int)std::min<long long>(std::max<long long>(g, 1), 65536);
}

}  // namespace
}  // namespace z4c

using namespace z4c;

extern "C" {

z4c_status z4c_xplan_create(const z4c_plan *plan, const z4c_transfer *prolong, int nprolong,
                            const z4c_transfer *restrict_, int nrestrict, int order, int flags,
                            z4c_xplan **out)
{
    if (!out)
        return set_error(Z4C_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plan)
        return set_error(Z4C_EINVAL, "plan is NULL");
    if (nprolong < 0 || nrestrict < 0 || (nprolong > 0 && !prolong)
        || (nrestrict > 0 && !restrict_))
        return set_error(Z4C_EINVAL, "bad transfer arrays");
    if (order != 2 && order != 4 && order != 6)
        return set_error(Z4C_EINVAL, "interpolation order must be 2, 4 or 6");
    if (flags & ~Z4C_PLAN_NO_DEVICE)
        return set_error(Z4C_EINVAL, "unknown flags");
    const std::vector<z4c_block> &B = plan_blocks(plan);
    z4c_status st;
    for (int t = 0; t < nprolong; ++t)
        if ((st = check_transfer(B, prolong[t], true, order, t)) != Z4C_OK)
            return st;
    for (int t = 0; t < nrestrict; ++t)
        if ((st = check_transfer(B, restrict_[t], false, order, t)) != Z4C_OK)
            return st;
    z4c_xplan *X = new z4c_xplan;
    X->plan = plan;
    X->order = order;
    X->pro.assign(prolong, prolong + nprolong);
    X->res.assign(restrict_, restrict_ + nrestrict);
    if ((st = check_set(X->pro, true)) != Z4C_OK || (st = check_set(X->res, false)) != Z4C_OK) {
        delete X;
        return st;
    }
    const std::vector<long long> rs = prefix(X->res);
    X->res_total = rs.back();
    X->tiles = make_tiles(X->pro, order);
    for (const XTile &T : X->tiles) {
        long long a, b;
        tile_lds(T, a, b);
        X->lds_a = std::max<long long>(X->lds_a, a);
        X->lds_b = std::max<long long>(X->lds_b, b);
        bool small = T.n[0] * T.n[1] * T.n[2] <= 1024;   // the kernel's index arithmetic
        bool perm = T.dir[0] + T.dir[1] + T.dir[2] == 3 && T.dir[0] != T.dir[1]
                 && T.dir[1] != T.dir[2] && T.dir[0] != T.dir[2];
        for (int d = 0; d < 3; ++d)
            small = small && T.n[d] <= 16 && T.sn[d] <= 16 && T.dir[d] >= 0 && T.dir[d] < 3;
        if (a > XA || b > XB || !small || !perm) {   // the bound of make_tiles failed
            delete X;
            return set_error(Z4C_ENOTSUP, "prolongation tile exceeds its LDS");
        }
    }
    if (X->tiles.size() > (size_t)INT32_MAX) {
        delete X;
        return set_error(Z4C_ENOTSUP, "too many prolongation tiles");
    }
    if (!(flags & Z4C_PLAN_NO_DEVICE)) {
        if (!plan_blocks_device(plan)) {
            delete X;
            return set_error(Z4C_ENODEV, "plan was created without a device");
        }
        hipError_t e = hipSuccess;
        auto up = [&](void **dst, const void *src, size_t bytes) {
            if (e == hipSuccess)
                e = hipMalloc(dst, std::max<size_t>(bytes, 8));
            if (e == hipSuccess && bytes)
                e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        };
        up((void **)&X->pro_d, X->pro.data(), sizeof(z4c_transfer) * X->pro.size());
        up((void **)&X->res_d, X->res.data(), sizeof(z4c_transfer) * X->res.size());
        up((void **)&X->tiles_d, X->tiles.data(), sizeof(XTile) * X->tiles.size());
        up((void **)&X->res_start_d, rs.data(), sizeof(long long) * rs.size());
        if (e != hipSuccess) {
            z4c_xplan_destroy(X);
            return e == hipErrorOutOfMemory ? set_error(Z4C_ENOMEM, "hipMalloc(xplan tables)")
                                            : set_hip_error(e, "xplan tables");
        }
        X->device = true;
    }
    *out = X;
    return Z4C_OK;
}

z4c_status z4c_xplan_destroy(z4c_xplan *X)
{
    if (!X)
        return Z4C_OK;
    for (void *p : {(void *)X->pro_d, (void *)X->res_d, (void *)X->tiles_d,
                    (void *)X->res_start_d})
        if (p)
            (void)hipFree(p);
    delete X;
    return Z4C_OK;
}

static z4c_status xcall(const z4c_xplan *X, double *u, bool pro, hipStream_t s)
{
    if (!X)
        return set_error(Z4C_EINVAL, "xplan is NULL");
    if (!u)
        return set_error(Z4C_EINVAL, "u is NULL");
    if (((uintptr_t)u & 7u) != 0)
        return set_error(Z4C_EALIGN, "arrays must be 8-byte aligned");
    if (!X->device)
        return set_error(Z4C_ENODEV, "xplan was created without a device");
    const z4c_block *blocks = plan_blocks_device(X->plan);
    if (pro) {
        const unsigned nt = (unsigned)X->tiles.size();
        if (nt == 0)
            return Z4C_OK;
        const dim3 grid(nt, NFIELD);
        const int a = (int)X->lds_a;
        const size_t bytes = sizeof(double) * (size_t)(X->lds_a + X->lds_b);
        if (X->order == 2)
            prolong_kernel<2><<<grid, 256, bytes, s>>>(blocks, X->pro_d, X->tiles_d, a, u);
        else if (X->order == 4)
            prolong_kernel<4><<<grid, 256, bytes, s>>>(blocks, X->pro_d, X->tiles_d, a, u);
        else
            prolong_kernel<6><<<grid, 256, bytes, s>>>(blocks, X->pro_d, X->tiles_d, a, u);
    } else {
        if (X->res_total == 0)
            return Z4C_OK;
        restrict_kernel<<<grid_for(X->res_total), 256, 0, s>>>(blocks, X->res_d, X->res_start_d,
                                             (int)X->res.size(), X->res_total, u);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? Z4C_OK : set_hip_error(e, "intergrid kernel launch");
}

z4c_status z4c_level_transfers(const z4c_plan *plan, const z4c_loc *locs, int coarse_level,
                               z4c_transfer *prolong, int max_prolong, int *nprolong,
                               z4c_transfer *restrict_, int max_restrict, int *nrestrict)
{
    if (!plan || !locs || !nprolong || !nrestrict)
        return set_error(Z4C_EINVAL, "plan, locs and the counts must not be NULL");
    if (max_prolong < 0 || max_restrict < 0 || (max_prolong > 0 && !prolong)
        || (max_restrict > 0 && !restrict_))
        return set_error(Z4C_EINVAL, "bad output arrays");
    *nprolong = *nrestrict = 0;
    const std::vector<z4c_block> &B = plan_blocks(plan);
    const int nb = (int)B.size();
    int lmax = 0;
    for (int b = 0; b < nb; ++b) {
        if (locs[b].level < 0 || locs[b].level > 30)
            return set_error(Z4C_EINVAL, "levels must be in 0..30");
        lmax = std::max(lmax, locs[b].level);
    }
    if (coarse_level < 0 || coarse_level + 1 > lmax)
        return set_error(Z4C_EINVAL, "coarse_level + 1 must be a level of the set");
    // lattice step of a level, and the checks of the pairs used
    auto step = [lmax](int L) { return 1LL << (lmax - L); };
    std::vector<int> cs, fs;
    for (int b = 0; b < nb; ++b) {
        if (locs[b].level == coarse_level)
            cs.push_back(b);
        else if (locs[b].level == coarse_level + 1)
            fs.push_back(b);
    }
    const long long sc = step(coarse_level), sf = step(coarse_level + 1);
    for (int c : cs)
        for (int f : fs) {
            if (!same_ratio(B[c].dx, B[f].dx) || !same_ratio(B[c].dy, B[f].dy)
                || !same_ratio(B[c].dz, B[f].dz))
                return set_error(Z4C_EINVAL, "block spacings do not halve from the coarse to "
                                             "the fine level");
            for (int d = 0; d < 3; ++d)
                if (((long long)locs[f].o[d] - locs[c].o[d]) % sc != 0)
                    return set_error(Z4C_EINVAL, "a fine block's vertex 0 is not a coarse "
                                                 "lattice vertex");
        }
    // ghost region r of a block (26, no interior): per direction -1, 0, +1
    auto region = [](const z4c_block &K, int r, int lo[3], int hi[3]) {
        const int n[3] = {K.nx, K.ny, K.nz};
        const int q[3] = {r % 3 - 1, (r / 3) % 3 - 1, r / 9 - 1};
        for (int d = 0; d < 3; ++d) {
            lo[d] = q[d] < 0 ? -K.ng : (q[d] == 0 ? 0 : n[d]);
            hi[d] = q[d] < 0 ? 0 : (q[d] == 0 ? n[d] : n[d] + K.ng);
        }
        return !(q[0] == 0 && q[1] == 0 && q[2] == 0);
    };
    // floor and ceiling of a / b, b > 0
    auto fdiv = [](long long a, long long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    auto cdiv = [&fdiv](long long a, long long b) { return -fdiv(-a, b); };
    int np = 0, nr = 0;
    for (int f : fs)
        for (int c : cs) {
            const z4c_block &F = B[f], &C = B[c];
            const int nC[3] = {C.nx, C.ny, C.nz}, nF[3] = {F.nx, F.ny, F.nz};
            int c0[3];
            for (int d = 0; d < 3; ++d)
                c0[d] = (int)(((long long)locs[f].o[d] - locs[c].o[d]) / sc);
            for (int r = 0; r < 27; ++r) {
                int lo[3], hi[3];
                // prolongation: ghost points of F in C's span [o, o + n step)
                if (region(F, r, lo, hi)) {
                    bool ok = true;
                    z4c_transfer T{c, f, {c0[0], c0[1], c0[2]}, {0, 0, 0}, {0, 0, 0}};
                    for (int d = 0; d < 3 && ok; ++d) {
                        const long long a = locs[c].o[d] - (long long)locs[f].o[d];
                        const long long i0 = std::max<long long>(lo[d], cdiv(a, sf));
                        const long long i1 = std::min<long long>(
                            hi[d], fdiv(a + (long long)nC[d] * sc - 1, sf) + 1);
                        ok = i0 < i1;
                        T.lo[d] = (int)i0;
                        T.hi[d] = (int)i1;
                    }
                    if (ok) {
                        if (np < max_prolong)
                            prolong[np] = T;
                        ++np;
                    }
                }
                // restriction: ghost points of C in F's span (all its vertices)
                if (region(C, r, lo, hi)) {
                    bool ok = true;
                    z4c_transfer T{c, f, {c0[0], c0[1], c0[2]}, {0, 0, 0}, {0, 0, 0}};
                    for (int d = 0; d < 3 && ok; ++d) {
                        const long long a = locs[f].o[d] - (long long)locs[c].o[d];
                        const long long j0 = std::max<long long>(lo[d], cdiv(a, sc));
                        const long long j1 = std::min<long long>(
                            hi[d], fdiv(a + (long long)(nF[d] - 1) * sf, sc) + 1);
                        ok = j0 < j1;
                        T.lo[d] = (int)j0;
                        T.hi[d] = (int)j1;
                    }
                    if (ok) {
                        if (nr < max_restrict)
                            restrict_[nr] = T;
                        ++nr;
                    }
                }
            }
        }
    *nprolong = np;
    *nrestrict = nr;
    if (np > max_prolong || nr > max_restrict)
        return (max_prolong == 0 && max_restrict == 0)
                   ? Z4C_OK
                   : set_error(Z4C_EINVAL, "output arrays too small (counts in *nprolong, "
                                           "*nrestrict)");
    return Z4C_OK;
}

}  // extern "C"

const z4c_plan *z4c::xplan_plan(const z4c_xplan *X) { return X ? X->plan : nullptr; }

extern "C" {

z4c_status z4c_prolongate(const z4c_xplan *X, double *u, void *stream)
{
    return xcall(X, u, true, (hipStream_t)stream);
}

z4c_status z4c_restrict(const z4c_xplan *X, double *u, void *stream)
{
    return xcall(X, u, false, (hipStream_t)stream);
}

}  // extern "C"
