// z4c_intergrid.hip -- transfers between refinement levels of the
// vertex-centred Z4c grid (ratio 2): prolongation coarse -> fine by
// Lagrange interpolation and restriction fine -> coarse by injection
// (Sec. 3.2: vertex-centred variables keep these operators simple at high
// order).  One thread per destination point; transfers are located by a
// binary search over the prefix sums of their box sizes; each point
// gathers its 1 or `order` source points per direction (1 for an even fine
// index, `order` for an odd one) for all 22 fields.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "z4c_internal.h"

struct z4c_xplan {
    const z4c_plan *plan = nullptr;
    int order = 0;
    bool device = false;
    std::vector<z4c_transfer> pro, res;
    z4c_transfer *pro_d = nullptr, *res_d = nullptr;
    long long *pro_start_d = nullptr, *res_start_d = nullptr;   // prefix sums, n + 1
    long long pro_total = 0, res_total = 0;
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

template <int O>
__global__ void __launch_bounds__(256)
prolong_kernel(const z4c_block *blocks, const z4c_transfer *tr, const long long *start, int n,
               long long total, double *u)
{
    for (long long r = blockIdx.x * 256LL + threadIdx.x; r < total;
         r += (long long)gridDim.x * 256) {
        const int t = find_transfer(start, n, r);
        const z4c_transfer T = tr[t];
        const long long loc = r - start[t];
        const int bx = T.hi[0] - T.lo[0], by = T.hi[1] - T.lo[1];
        const int fi[3] = {T.lo[0] + (int)(loc % bx), T.lo[1] + (int)((loc / bx) % by),
                           T.lo[2] + (int)(loc / ((long long)bx * by))};
        // per direction: first coarse index, number of taps (1 or O)
        int c[3], nt[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if ((fi[d] & 1) == 0) {
                c[d] = T.c0[d] + (fi[d] >> 1);
                nt[d] = 1;
            } else {
                c[d] = T.c0[d] + ((fi[d] - 1) >> 1) - (O / 2 - 1);
                nt[d] = O;
            }
        }
        const z4c_block C = blocks[T.coarse];
        const z4c_block F = blocks[T.fine];
        const long long csx = C.nx + 2LL * C.ng, csy = C.ny + 2LL * C.ng;
        const long long cbase = C.offset + point_index(C, c[0], c[1], c[2]);
        const long long dst = F.offset + point_index(F, fi[0], fi[1], fi[2]);
        for (int f = 0; f < NFIELD; ++f) {
            const double *src = u + cbase + f * C.field_stride;
            double s = 0.0;
            for (int kz = 0; kz < nt[2]; ++kz) {
                const double wz = nt[2] == 1 ? 1.0 : mid_weight<O>(kz);
                for (int ky = 0; ky < nt[1]; ++ky) {
                    const double wy = nt[1] == 1 ? 1.0 : mid_weight<O>(ky);
                    const double *row = src + csx * (ky + csy * (long long)kz);
                    double sx = 0.0;
                    for (int kx = 0; kx < nt[0]; ++kx)
                        sx += (nt[0] == 1 ? 1.0 : mid_weight<O>(kx)) * row[kx];
                    s += wz * wy * sx;
                }
            }
            u[dst + f * F.field_stride] = s;
        }
    }
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
        for (int f = 0; f < NFIELD; ++f)
            u[dst + f * C.field_stride] = u[src + f * F.field_stride];
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
    const std::vector<long long> ps = prefix(X->pro), rs = prefix(X->res);
    X->pro_total = ps.back();
    X->res_total = rs.back();
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
        up((void **)&X->pro_start_d, ps.data(), sizeof(long long) * ps.size());
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
    for (void *p : {(void *)X->pro_d, (void *)X->res_d, (void *)X->pro_start_d,
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
    const long long total = pro ? X->pro_total : X->res_total;
    if (total == 0)
        return Z4C_OK;
    const z4c_block *blocks = plan_blocks_device(X->plan);
    const int n = (int)(pro ? X->pro.size() : X->res.size());
    const int g = grid_for(total);
    if (!pro)
        restrict_kernel<<<g, 256, 0, s>>>(blocks, X->res_d, X->res_start_d, n, total, u);
    else if (X->order == 2)
        prolong_kernel<2><<<g, 256, 0, s>>>(blocks, X->pro_d, X->pro_start_d, n, total, u);
    else if (X->order == 4)
        prolong_kernel<4><<<g, 256, 0, s>>>(blocks, X->pro_d, X->pro_start_d, n, total, u);
    else
        prolong_kernel<6><<<g, 256, 0, s>>>(blocks, X->pro_d, X->pro_start_d, n, total, u);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? Z4C_OK : set_hip_error(e, "intergrid kernel launch");
}

z4c_status z4c_prolongate(const z4c_xplan *X, double *u, void *stream)
{
    return xcall(X, u, true, (hipStream_t)stream);
}

z4c_status z4c_restrict(const z4c_xplan *X, double *u, void *stream)
{
    return xcall(X, u, false, (hipStream_t)stream);
}

}  // extern "C"
