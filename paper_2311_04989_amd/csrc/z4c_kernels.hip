// z4c_kernels.hip -- gfx950 kernels of the Z4c hot path other than the tile
// kernels (those live in z4c_tile.h, instantiated in z4c_variants_*.hip):
// ghost refresh, per-block norm reduction, non-finite scan, and the dispatch
// to the tile-kernel variants.
#include <cmath>
#include <type_traits>
#include <utility>

#include "z4c_internal.h"

namespace z4c {
namespace {

// ---------------------------------------------------------------------------
// Ghost refresh: one thread per ghost point, all 22 fields
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) ghost_kernel(const GhostArgs g, long long total)
{
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total)
        return;
    // block by binary search over the prefix sums
    int lo = 0, hi = g.nblocks;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (g.ghost_start[mid] <= gid)
            lo = mid;
        else
            hi = mid;
    }
    const int b = lo;
    const z4c_block B = g.blocks[b];
    long long r = gid - g.ghost_start[b];
    const int ng = B.ng;
    const int ex = B.nx + 2 * ng, ey = B.ny + 2 * ng, ez = B.nz + 2 * ng;
    int i, j, k;
    // z slabs (full planes), then y slabs (interior z), then x slabs
    const long long zslab = (long long)ng * ey * ex;
    const long long yslab = (long long)ng * B.nz * ex;
    if (r < 2 * zslab) {
        const int side = r >= zslab;
        r -= side * zslab;
        const int kk = (int)(r / ((long long)ey * ex));
        const int rem = (int)(r % ((long long)ey * ex));
        k = side ? B.nz + kk : kk - ng;
        j = rem / ex - ng;
        i = rem % ex - ng;
    } else if ((r -= 2 * zslab) < 2 * yslab) {
        const int side = r >= yslab;
        r -= side * yslab;
        const int kk = (int)(r / ((long long)ng * ex));
        const int rem = (int)(r % ((long long)ng * ex));
        k = kk;
        const int jj = rem / ex;
        j = side ? B.ny + jj : jj - ng;
        i = rem % ex - ng;
    } else {
        r -= 2 * yslab;
        const long long xslab = (long long)ng * B.nz * B.ny;
        const int side = r >= xslab;
        r -= side * xslab;
        const int kk = (int)(r / ((long long)B.ny * ng));
        const int rem = (int)(r % ((long long)B.ny * ng));
        k = kk;
        j = rem / ng;
        const int ii = rem % ng;
        i = side ? B.nx + ii : ii - ng;
    }
    const int ox = i < 0 ? -1 : (i >= B.nx ? 1 : 0);
    const int oy = j < 0 ? -1 : (j >= B.ny ? 1 : 0);
    const int oz = k < 0 ? -1 : (k >= B.nz ? 1 : 0);
    const long long dst = (long long)(k + ng) * ey * ex + (long long)(j + ng) * ex + (i + ng);
    int src_b = -1;
    if (g.policy == Z4C_GHOST_PERIODIC)
        src_b = b;
    else if (g.policy == Z4C_GHOST_NEIGHBOUR)
        src_b = g.neighbours[b * 27 + (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)];
    double *ub = g.u + B.offset;
    if (src_b < 0) {
        if (g.frozen) {
            const double *fb = g.frozen + B.offset;
            for (int f = 0; f < NFIELD; ++f)
                ub[f * B.field_stride + dst] = fb[f * B.field_stride + dst];
        }
        return;
    }
    const z4c_block Sb = g.blocks[src_b];
    const int si = i - ox * B.nx, sj = j - oy * B.ny, sk = k - oz * B.nz;
    const int sex = Sb.nx + 2 * Sb.ng, sey = Sb.ny + 2 * Sb.ng;
    const long long src = (long long)(sk + Sb.ng) * sey * sex + (long long)(sj + Sb.ng) * sex
                        + (si + Sb.ng);
    const double *sbp = g.u + Sb.offset;
    for (int f = 0; f < NFIELD; ++f)
        ub[f * B.field_stride + dst] = sbp[f * Sb.field_stride + src];
}

// Per-block norms from per-tile partial sums, fixed summation order.
__global__ void norm_reduce_kernel(const z4c_block *blocks, int nblocks, const long long *tile_start,
                                   const int *tile_count, const double *partial, double *norms)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nblocks * 16)
        return;
    const int b = id / 16, q = id % 16;
    double s = 0.0;
    const long long t0 = tile_start[b];
    for (int t = 0; t < tile_count[b]; ++t)
        s += partial[(t0 + t) * 16 + q];
    const z4c_block B = blocks[b];
    norms[id] = s * (B.dx * B.dy * B.dz);
}

__global__ void finite_count_kernel(const z4c_block *blocks, int nblocks, const long long *pt_start,
                                    long long total, const double *u, unsigned long long *count)
{
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long bad = 0;
    if (gid < total) {
        int lo = 0, hi = nblocks;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pt_start[mid] <= gid)
                lo = mid;
            else
                hi = mid;
        }
        const z4c_block B = blocks[lo];
        const long long r = gid - pt_start[lo];
        const int i = (int)(r % B.nx), j = (int)((r / B.nx) % B.ny), k = (int)(r / ((long long)B.nx * B.ny));
        const int ex = B.nx + 2 * B.ng, ey = B.ny + 2 * B.ng;
        const long long pt = (long long)(k + B.ng) * ey * ex + (long long)(j + B.ng) * ex + (i + B.ng);
        for (int f = 0; f < NFIELD; ++f) {
            const double v = u[B.offset + f * B.field_stride + pt];
            bad += isfinite(v) ? 0ull : 1ull;
        }
    }
    // wave-level sum, one atomic per wave
    for (int off = 32; off >= 1; off >>= 1)
        bad += __shfl_xor(bad, off, 64);
    if ((threadIdx.x & 63) == 0 && bad)
        atomicAdd(count, bad);
}

__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0ull; }

__global__ void zero_queue_kernel(int *q)
{
    if (threadIdx.x < 8)
        q[threadIdx.x] = 0;
}

}  // namespace

bool stage_shape_supported(int fd_order, int tx, int ty, int tz, int waves)
{
    // one wave per SIMD (a 256-register budget plus as many accumulation
    // registers): 256-point tiles 8x8x4 and 8x4x8 of the order-6 kernels
    if (tx == 8 && ty == 4 && tz == 8)
        return waves == 1 && fd_order == 6;
    if (tx != 8 || ty != 8 || (tz != 8 && tz != 4))
        return false;
    return waves == 2 || (waves == 1 && tz == 4 && fd_order == 6);
}

hipError_t launch_stage(int mode, int fd_order, int arith, int tx, int ty, int tz, int waves,
                        const StageArgs &a, hipStream_t s)
{
    if (mode == MODE_RK_MON)
        return launch_monitor(fd_order, tx, ty, tz, waves, a, s);
    if (arith == Z4C_ARITH_FP32_NAIVE && mode != MODE_CONS)
        return mode == MODE_RHS ? launch_naive(fd_order, tx, ty, tz, waves, a, s)
                                : hipErrorInvalidValue;
    if (fd_order == 4)
        return launch_p4(mode, arith, tx, ty, tz, waves, a, s);
    if (mode == MODE_CONS || arith != Z4C_ARITH_FP32)
        return launch_p6_f64(mode, tx, ty, tz, waves, a, s);
    return launch_p6_f32(mode, tx, ty, tz, waves, a, s);
}

hipError_t launch_ghost(const GhostArgs &g, long long total_ghost, hipStream_t s)
{
    if (total_ghost <= 0)
        return hipSuccess;
    const long long nb = (total_ghost + 255) / 256;
    ghost_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(g, total_ghost);
    return hipGetLastError();
}

hipError_t launch_norm_reduce(const z4c_block *blocks, int nblocks, const long long *tile_start,
                              const int *tile_count, const double *partial, double *norms,
                              hipStream_t s)
{
    const int n = nblocks * 16;
    norm_reduce_kernel<<<dim3((n + 255) / 256), dim3(256), 0, s>>>(blocks, nblocks, tile_start,
                                                                  tile_count, partial, norms);
    return hipGetLastError();
}

hipError_t launch_finite_count(const z4c_block *blocks, int nblocks, const long long *pt_start,
                               long long total_pts, const double *u, unsigned long long *count,
                               hipStream_t s)
{
    if (total_pts <= 0)
        return hipSuccess;
    const long long nb = (total_pts + 255) / 256;
    finite_count_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(blocks, nblocks, pt_start,
                                                                total_pts, u, count);
    return hipGetLastError();
}

hipError_t launch_zero_queue(int *q, hipStream_t s)
{
    zero_queue_kernel<<<1, 64, 0, s>>>(q);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s)
{
    zero_u64_kernel<<<1, 1, 0, s>>>(p);
    return hipGetLastError();
}

}  // namespace z4c
