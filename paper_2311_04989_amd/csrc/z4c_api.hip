// z4c_api.hip -- host side of libz4c.so: argument validation, plans (block
// tables and tile lists in device memory), launches, Runge-Kutta steps,
// graph capture of whole steps, launch-shape autotuning.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "z4c_internal.h"

using namespace z4c;

// Scratch of z4c_constraints_noalloc (partial sums, 16 doubles per tile).
constexpr int NOALLOC_MAX_TILES = 65536;   // 8 MiB per device
static __device__ __align__(256) double scratch[NOALLOC_MAX_TILES * 16];

namespace {

thread_local std::string g_last_error;

z4c_status fail(z4c_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

z4c_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return Z4C_EHIP;
}

#define HIP_TRY(call, what)                        \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess)                      \
            return hip_fail(e_, what);             \
    } while (0)

struct LaunchGroup {
    int tx, ty, tz, persistent, waves;
    std::vector<Tile> tiles;
    Tile *tiles_d = nullptr;
    int *queue_d = nullptr;   // persistent launches: 8 tile counters
    long long tile_base = 0;
};

struct SizeClass {
    int nx, ny, nz;
    z4c_launch launch;
    std::vector<int> blocks;
};

struct StepKey {
    double *regs[4];
    const double *matter;
    const double *frozen;
    double dt;
    int nstages, ghost_policy, flags;
    double *cons, *norms;
    z4c_rk_coeffs table[8];
    int version;
    bool operator==(const StepKey &o) const { return std::memcmp(this, &o, sizeof(StepKey)) == 0; }
};

struct GraphEntry {
    StepKey key;
    hipGraphExec_t exec;
    int result;
};

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

z4c_status check_params(const z4c_params *p)
{
    if (!p)
        return fail(Z4C_EINVAL, "params is NULL");
    if (p->fd_order != 4 && p->fd_order != 6)
        return fail(Z4C_EINVAL, "fd_order must be 4 or 6");
    if (!(std::isfinite(p->ko_sigma) && p->ko_sigma >= 0.0))
        return fail(Z4C_EINVAL, "ko_sigma must be finite and >= 0");
    if (!std::isfinite(p->kappa1) || !std::isfinite(p->kappa2) || !std::isfinite(p->eta))
        return fail(Z4C_EINVAL, "kappa1, kappa2, eta must be finite");
    if (p->lapse < 0 || p->lapse > 2 || p->shift < 0 || p->shift > 1)
        return fail(Z4C_EINVAL, "unknown lapse or shift condition");
    if (p->advect_gauge != 0 && p->advect_gauge != 1)
        return fail(Z4C_EINVAL, "advect_gauge must be 0 or 1");
    if (!(p->chi_floor > 0.0) || !(p->alpha_floor >= 0.0) || !std::isfinite(p->chi_floor)
        || !std::isfinite(p->alpha_floor))
        return fail(Z4C_EINVAL, "chi_floor must be > 0 and alpha_floor >= 0");
    if (p->arith != Z4C_ARITH_FP64 && p->arith != Z4C_ARITH_FP32
        && p->arith != Z4C_ARITH_FP32_NAIVE)
        return fail(Z4C_EINVAL, "arith must be FP64, FP32 or FP32_NAIVE");
    if (p->arith == Z4C_ARITH_FP32_NAIVE && p->fd_order != 6)
        return fail(Z4C_ENOTSUP, "the naive FP32 form is built for order 6 only");
    if (p->advection != Z4C_ADVECT_CENTRED && p->advection != Z4C_ADVECT_LOPSIDED)
        return fail(Z4C_EINVAL, "advection must be CENTRED or LOPSIDED");
    if (p->advection == Z4C_ADVECT_LOPSIDED && p->arith != Z4C_ARITH_FP64)
        return fail(Z4C_ENOTSUP, "lopsided advection runs with FP64 arithmetic only");
    return Z4C_OK;
}

z4c_status check_block(const z4c_block &b, int idx, int fd_order)
{
    char buf[160];
    if (b.nx < 1 || b.ny < 1 || b.nz < 1) {
        std::snprintf(buf, sizeof buf, "block %d: nx, ny, nz must be >= 1", idx);
        return fail(Z4C_EINVAL, buf);
    }
    if (b.ng < fd_order / 2 + 1) {
        std::snprintf(buf, sizeof buf, "block %d: ng = %d < fd_order/2 + 1 = %d", idx, b.ng,
                      fd_order / 2 + 1);
        return fail(Z4C_ENOGHOST, buf);
    }
    if (!(b.dx > 0.0 && b.dy > 0.0 && b.dz > 0.0) || !std::isfinite(b.dx) || !std::isfinite(b.dy)
        || !std::isfinite(b.dz)) {
        std::snprintf(buf, sizeof buf, "block %d: grid spacings must be finite and > 0", idx);
        return fail(Z4C_EINVAL, buf);
    }
    const long long ex = b.nx + 2LL * b.ng, ey = b.ny + 2LL * b.ng, ez = b.nz + 2LL * b.ng;
    const long long npts = ex * ey * ez;
    if (npts >= (1LL << 29)) {
        // the kernels address a block's points as 32-bit byte offsets from
        // the block's field base
        std::snprintf(buf, sizeof buf, "block %d: %lld stored points; at most 2^29 - 1 are "
                      "supported", idx, npts);
        return fail(Z4C_ENOTSUP, buf);
    }
    if (b.offset < 0 || b.moffset < 0 || b.coffset < 0 || b.field_stride < npts) {
        std::snprintf(buf, sizeof buf,
                      "block %d: offsets must be >= 0 and field_stride >= stored points", idx);
        return fail(Z4C_EINVAL, buf);
    }
    return Z4C_OK;
}

}  // namespace

namespace z4c {
void block_factors(const z4c_block &b, int fd_order, double sigma, double out[12])
{
    const double h[3] = {b.dx, b.dy, b.dz};
    const double c1 = fd_order == 4 ? 12.0 : 60.0;
    const double c2 = fd_order == 4 ? 12.0 : 180.0;
    const double cko = fd_order == 4 ? sigma / 64.0 : -sigma / 256.0;
    double i1[3];
    for (int a = 0; a < 3; ++a) {
        i1[a] = 1.0 / (c1 * h[a]);
        out[a] = i1[a];
        out[3 + a] = 1.0 / (c2 * h[a] * h[a]);
        out[9 + a] = cko / h[a];
    }
    out[6] = i1[0] * i1[1];
    out[7] = i1[0] * i1[2];
    out[8] = i1[1] * i1[2];
}
}  // namespace z4c

struct z4c_plan {
    z4c_params params{};
    bool device = false;
    int nblocks = 0;
    std::vector<z4c_block> blocks;
    z4c_block *blocks_d = nullptr;
    double *fac64_d = nullptr;
    float *fac32_d = nullptr;
    std::vector<SizeClass> classes;
    std::vector<LaunchGroup> groups;
    long long total_tiles = 0;
    long long *tile_start_d = nullptr;
    int *tile_count_d = nullptr;
    double *partial_d = nullptr;
    long long *ghost_start_d = nullptr;
    long long total_ghost = 0;
    int *nbr_d = nullptr;
    bool has_nbr = false;
    bool periodic_ok = true;   // every block has nx, ny, nz >= ng
    // every block the neighbour table names for another block ends within
    // 2^32 elements of the array base (halo reads address such points with
    // 32-bit element offsets from the base)
    bool nbr32 = true;
    int halo = Z4C_GHOST_NONE; // halo reads of z4c_rhs / z4c_rk_stage / z4c_constraints
    // level-jump exchange of Z4C_STEP_LEVEL_EXCHANGE: one transfer plan per
    // pair of adjacent levels, coarsest pair first
    std::vector<const z4c_xplan *> levels;
    const double *halo_frozen = nullptr;
    long long *pt_start_d = nullptr;
    long long total_pts = 0;
    unsigned long long *count_d = nullptr;
    hipStream_t capture_stream = nullptr;
    std::vector<GraphEntry> graphs;
    int version = 0;
    int num_cus = 256;
    // host copy of the neighbour table (nblocks*27) once set
    std::vector<int> nbr_h;
    // radiative outer boundary (z4c_plan_set_sommerfeld): block origins and
    // the boxes of outer ghost points, with prefix sums of their sizes
    bool radiative = false;
    std::vector<double> origins;
    std::vector<OuterRegion> outer;
    double *origins_d = nullptr;
    OuterRegion *outer_d = nullptr;
    long long *outer_start_d = nullptr;
    long long total_outer = 0;

    void free_outer()
    {
        if (origins_d)
            (void)hipFree(origins_d);
        if (outer_d)
            (void)hipFree(outer_d);
        if (outer_start_d)
            (void)hipFree(outer_start_d);
        origins_d = nullptr;
        outer_d = nullptr;
        outer_start_d = nullptr;
    }

    void free_groups()
    {
        for (auto &g : groups) {
            if (g.tiles_d)
                (void)hipFree(g.tiles_d);
            if (g.queue_d)
                (void)hipFree(g.queue_d);
        }
        groups.clear();
        if (tile_start_d)
            (void)hipFree(tile_start_d);
        if (tile_count_d)
            (void)hipFree(tile_count_d);
        if (partial_d)
            (void)hipFree(partial_d);
        tile_start_d = nullptr;
        tile_count_d = nullptr;
        partial_d = nullptr;
    }
    void clear_graphs()
    {
        for (auto &g : graphs)
            (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
};

namespace {

// Boxes of outer ghost points of every block under the neighbour table
// `nbr`: the ghost region of each direction whose entry is -1.  Fails when
// a box comes within half a grid spacing of the coordinate origin (the
// radiative law divides by r).
z4c_status outer_regions(const z4c_plan *P, const int *nbr, const double *origins,
                         std::vector<OuterRegion> &out)
{
    out.clear();
    for (int b = 0; b < P->nblocks; ++b) {
        const z4c_block &B = P->blocks[b];
        const int n[3] = {B.nx, B.ny, B.nz};
        const double h[3] = {B.dx, B.dy, B.dz};
        for (int d = 0; d < 27; ++d) {
            if (d == 13 || nbr[b * 27 + d] >= 0)
                continue;
            const int o[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
            OuterRegion R{};
            R.block = b;
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                R.lo[a] = o[a] < 0 ? -B.ng : (o[a] > 0 ? n[a] : 0);
                R.n[a] = o[a] != 0 ? B.ng : n[a];
                const double x_lo = origins[3 * b + a] + R.lo[a] * h[a];
                const double x_hi = origins[3 * b + a] + (R.lo[a] + R.n[a] - 1) * h[a];
                const double c = x_lo > 0.0 ? x_lo : (x_hi < 0.0 ? x_hi : 0.0);
                d2 += c * c;
            }
            const double hmin = std::min(h[0], std::min(h[1], h[2]));
            if (!(std::sqrt(d2) >= 0.5 * hmin)) {
                char buf[200];
                std::snprintf(buf, sizeof buf, "block %d: outer ghost points within half a grid "
                              "spacing of the coordinate origin (the radiative law divides by "
                              "r)", b);
                return fail(Z4C_EINVAL, buf);
            }
            out.push_back(R);
        }
    }
    return Z4C_OK;
}

// Upload the radiative boundary's tables (origins, boxes, prefix sums).  On
// a failure the boundary is removed (no half-built tables stay in use).
z4c_status upload_outer(z4c_plan *P)
{
    std::vector<long long> start(P->outer.size() + 1, 0);
    for (size_t q = 0; q < P->outer.size(); ++q) {
        const OuterRegion &R = P->outer[q];
        start[q + 1] = start[q] + (long long)R.n[0] * R.n[1] * R.n[2];
    }
    P->total_outer = start.back();
    if (!P->device)
        return Z4C_OK;
    P->clear_graphs();
    P->free_outer();
    const char *what = nullptr;
    hipError_t e = hipMalloc(&P->origins_d, sizeof(double) * 3 * P->nblocks);
    if (e != hipSuccess)
        what = "hipMalloc(origins)";
    if (!what && (e = hipMemcpy(P->origins_d, P->origins.data(), sizeof(double) * 3 * P->nblocks,
                                hipMemcpyHostToDevice)) != hipSuccess)
        what = "hipMemcpy(origins)";
    if (!what && (e = hipMalloc(&P->outer_start_d, sizeof(long long) * start.size()))
                     != hipSuccess)
        what = "hipMalloc(outer prefix sums)";
    if (!what && (e = hipMemcpy(P->outer_start_d, start.data(), sizeof(long long) * start.size(),
                                hipMemcpyHostToDevice)) != hipSuccess)
        what = "hipMemcpy(outer prefix sums)";
    if (!what && !P->outer.empty()) {
        if ((e = hipMalloc(&P->outer_d, sizeof(OuterRegion) * P->outer.size())) != hipSuccess)
            what = "hipMalloc(outer boxes)";
        else if ((e = hipMemcpy(P->outer_d, P->outer.data(), sizeof(OuterRegion) * P->outer.size(),
                                hipMemcpyHostToDevice)) != hipSuccess)
            what = "hipMemcpy(outer boxes)";
    }
    if (what) {
        P->free_outer();
        P->radiative = false;
        P->outer.clear();
        P->total_outer = 0;
        return hip_fail(e, what);
    }
    return Z4C_OK;
}

// One radiative stage (c != nullptr) or right-hand side (rhs != nullptr) of
// the outer ghost points; rule: samples at ghost points with a neighbour are
// read from the neighbour (as the stage's neighbour-rule halo reads).
z4c_status enqueue_radiative(z4c_plan *P, const double *u0_in, double *u0_out, double *u1,
                             const double *u2, const z4c_rk_coeffs *c, double dt, double *rhs,
                             bool rule, hipStream_t s)
{
    RadiativeArgs a{};
    a.nbr = rule ? P->nbr_d : nullptr;
    a.blocks = P->blocks_d;
    a.origins = P->origins_d;
    a.regions = P->outer_d;
    a.start = P->outer_start_d;
    a.nregions = (int)P->outer.size();
    a.total = P->total_outer;
    a.u = u0_in;
    a.rhs = rhs;
    a.chi_floor = P->params.chi_floor;
    a.alpha_floor = P->params.alpha_floor;
    if (c) {
        a.out = u0_out;
        a.u1 = u1;
        a.u2 = u2;
        a.delta = c->delta;
        a.eps_dt = c->eps * dt;
        a.g1 = c->g1;
        a.g2 = c->g2;
        a.g3 = c->g3;
        a.beta_dt = c->beta * dt;
        a.read_u1 = c->read_u1;
        a.write_u1 = c->write_u1;
        a.use_u2 = c->g3 != 0.0;
    }
    const hipError_t e = launch_radiative(a, s);
    if (e != hipSuccess)
        return hip_fail(e, "radiative boundary launch");
    return Z4C_OK;
}

z4c_status upload_factors(z4c_plan *P)
{
    if (!P->device)
        return Z4C_OK;
    std::vector<double> f64(12 * (size_t)P->nblocks);
    std::vector<float> f32(12 * (size_t)P->nblocks);
    for (int b = 0; b < P->nblocks; ++b) {
        block_factors(P->blocks[b], P->params.fd_order, P->params.ko_sigma, &f64[12 * (size_t)b]);
        for (int q = 0; q < 12; ++q)
            f32[12 * (size_t)b + q] = (float)f64[12 * (size_t)b + q];
    }
    if (!P->fac64_d)
        HIP_TRY(hipMalloc(&P->fac64_d, sizeof(double) * f64.size()), "hipMalloc(factors)");
    if (!P->fac32_d)
        HIP_TRY(hipMalloc(&P->fac32_d, sizeof(float) * f32.size()), "hipMalloc(factors)");
    HIP_TRY(hipMemcpy(P->fac64_d, f64.data(), sizeof(double) * f64.size(), hipMemcpyHostToDevice),
            "hipMemcpy(factors)");
    HIP_TRY(hipMemcpy(P->fac32_d, f32.data(), sizeof(float) * f32.size(), hipMemcpyHostToDevice),
            "hipMemcpy(factors)");
    return Z4C_OK;
}

// Build launch groups from the size classes and upload tile lists.
z4c_status build_groups(z4c_plan *P)
{
    P->free_groups();
    P->clear_graphs();
    ++P->version;
    std::map<std::vector<int>, int> gidx;
    std::vector<long long> tstart(P->nblocks, 0);
    std::vector<int> tcount(P->nblocks, 0);
    for (const SizeClass &c : P->classes) {
        const std::vector<int> key = {c.launch.tile_x, c.launch.tile_y, c.launch.tile_z,
                                      c.launch.persistent, c.launch.waves};
        auto it = gidx.find(key);
        int gi;
        if (it == gidx.end()) {
            gi = (int)P->groups.size();
            gidx[key] = gi;
            LaunchGroup g;
            g.tx = c.launch.tile_x;
            g.ty = c.launch.tile_y;
            g.tz = c.launch.tile_z;
            g.persistent = c.launch.persistent;
            g.waves = c.launch.waves;
            P->groups.push_back(g);
        } else {
            gi = it->second;
        }
        LaunchGroup &g = P->groups[gi];
        for (int b : c.blocks) {
            const z4c_block &B = P->blocks[b];
            tstart[b] = (long long)g.tiles.size();   // relative for now
            int n = 0;
            for (int k0 = 0; k0 < B.nz; k0 += g.tz)
                for (int j0 = 0; j0 < B.ny; j0 += g.ty)
                    for (int i0 = 0; i0 < B.nx; i0 += g.tx) {
                        g.tiles.push_back(Tile{b, i0, j0, k0});
                        ++n;
                    }
            tcount[b] = n;
        }
    }
    long long base = 0;
    std::vector<int> block_group(P->nblocks, 0);
    for (size_t gi = 0; gi < P->groups.size(); ++gi) {
        P->groups[gi].tile_base = base;
        base += (long long)P->groups[gi].tiles.size();
    }
    for (size_t ci = 0; ci < P->classes.size(); ++ci) {
        const SizeClass &c = P->classes[ci];
        const std::vector<int> key = {c.launch.tile_x, c.launch.tile_y, c.launch.tile_z,
                                      c.launch.persistent, c.launch.waves};
        const int gi = gidx[key];
        for (int b : c.blocks)
            tstart[b] += P->groups[gi].tile_base;
    }
    P->total_tiles = base;
    if (!P->device)
        return Z4C_OK;
    for (auto &g : P->groups) {
        HIP_TRY(hipMalloc(&g.tiles_d, sizeof(Tile) * std::max<size_t>(1, g.tiles.size())),
                "hipMalloc(tiles)");
        if (g.persistent)
            HIP_TRY(hipMalloc(&g.queue_d, sizeof(int) * 16), "hipMalloc(queue)");
        HIP_TRY(hipMemcpy(g.tiles_d, g.tiles.data(), sizeof(Tile) * g.tiles.size(),
                          hipMemcpyHostToDevice),
                "hipMemcpy(tiles)");
    }
    HIP_TRY(hipMalloc(&P->tile_start_d, sizeof(long long) * P->nblocks), "hipMalloc");
    HIP_TRY(hipMalloc(&P->tile_count_d, sizeof(int) * P->nblocks), "hipMalloc");
    HIP_TRY(hipMemcpy(P->tile_start_d, tstart.data(), sizeof(long long) * P->nblocks,
                      hipMemcpyHostToDevice),
            "hipMemcpy");
    HIP_TRY(hipMemcpy(P->tile_count_d, tcount.data(), sizeof(int) * P->nblocks,
                      hipMemcpyHostToDevice),
            "hipMemcpy");
    HIP_TRY(hipMalloc(&P->partial_d, sizeof(double) * 16 * std::max<long long>(1, base)),
            "hipMalloc(partial)");
    return Z4C_OK;
}

StageArgs base_args(const z4c_plan *P)
{
    StageArgs a{};
    a.blocks = P->blocks_d;
    a.fac64 = P->fac64_d;
    a.fac32 = P->fac32_d;
    a.ko_sigma = P->params.ko_sigma;
    a.kappa1 = P->params.kappa1;
    a.kappa2 = P->params.kappa2;
    a.eta = P->params.eta;
    a.chi_floor = P->params.chi_floor;
    a.alpha_floor = P->params.alpha_floor;
    a.lapse = P->params.lapse;
    a.shift = P->params.shift;
    a.advect_gauge = P->params.advect_gauge;
    a.halo = P->halo;
    a.nbr = P->nbr_d;
    a.frozen = P->halo_frozen;
    return a;
}

z4c_status run_groups(z4c_plan *P, int mode, int arith, StageArgs a, hipStream_t s)
{
    for (const auto &g : P->groups) {
        a.tiles = g.tiles_d;
        a.ntiles = (int)g.tiles.size();
        a.persistent = g.persistent;
        a.queue = g.queue_d;
        a.tile_base = g.tile_base;
        if (g.persistent && !g.tiles.empty()) {
            const hipError_t ez = launch_zero_queue(g.queue_d, s);
            if (ez != hipSuccess)
                return hip_fail(ez, "tile-queue reset launch");
        }
        const bool lop = P->params.advection == Z4C_ADVECT_LOPSIDED
                      && (mode == MODE_RHS || mode == MODE_RK);
        const hipError_t e = lop ? launch_lopsided(mode, P->params.fd_order, g.tx, g.ty, g.tz,
                                                   g.waves, a, s)
                                 : launch_stage(mode, P->params.fd_order, arith, g.tx, g.ty,
                                                g.tz, g.waves, a, s);
        if (e != hipSuccess)
            return hip_fail(e, "tile kernel launch");
    }
    return Z4C_OK;
}

z4c_status need_device(const z4c_plan *P)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    if (!P->device)
        return fail(Z4C_ENODEV, "plan was created without a device");
    return Z4C_OK;
}

z4c_status validate_stage(const z4c_plan *P, const double *u0_in, const double *u0_out,
                          const double *u1, const double *u2, const double *matter,
                          const z4c_rk_coeffs *c, double dt)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    if (!u0_in || !u0_out || !c)
        return fail(Z4C_EINVAL, "u0_in, u0_out and coefficients must not be NULL");
    if (u0_in == u0_out)
        return fail(Z4C_EINVAL, "u0_out must not alias u0_in (neighbouring tiles read u0_in)");
    if ((c->read_u1 || c->write_u1 || c->g2 != 0.0) && !u1)
        return fail(Z4C_EINVAL, "u1 is NULL but the stage reads or writes it");
    if (c->g3 != 0.0 && !u2)
        return fail(Z4C_EINVAL, "u2 is NULL but g3 != 0");
    if (u1 && (u1 == u0_in || u1 == u0_out))
        return fail(Z4C_EINVAL, "u1 must not alias u0_in or u0_out");
    if (c->g3 != 0.0 && u2 == u0_out)
        return fail(Z4C_EINVAL, "u2 must not alias u0_out when the stage reads it");
    if (!aligned8(u0_in) || !aligned8(u0_out) || !aligned8(u1) || !aligned8(u2)
        || !aligned8(matter))
        return fail(Z4C_EALIGN, "arrays must be 8-byte aligned");
    if (!std::isfinite(dt))
        return fail(Z4C_EINVAL, "dt must be finite");
    if (P->params.arith == Z4C_ARITH_FP32_NAIVE)
        return fail(Z4C_ENOTSUP, "the naive FP32 form is a right-hand side only");
    if (c->read_u1 < 0 || c->read_u1 > 1 || c->write_u1 < 0 || c->write_u1 > 1)
        return fail(Z4C_EINVAL, "read_u1/write_u1 must be 0 or 1");
    return Z4C_OK;
}

z4c_status enqueue_stage(z4c_plan *P, const double *u0_in, double *u0_out, double *u1,
                         const double *u2, const double *matter, const z4c_rk_coeffs *c,
                         double dt, hipStream_t s, int halo = -1, const double *frozen = nullptr,
                         bool monitor = false, double *cons = nullptr)
{
    StageArgs a = base_args(P);
    if (monitor) {
        a.cons = cons;
        a.partial = P->partial_d;
    }
    if (halo >= 0) {
        a.halo = halo;
        a.frozen = frozen;
    }
    a.u = u0_in;
    a.matter = matter;
    a.out = u0_out;
    a.u1 = u1;
    a.u2 = u2;
    a.delta = c->delta;
    a.eps_dt = c->eps * dt;
    a.g1 = c->g1;
    a.g2 = c->g2;
    a.g3 = c->g3;
    a.beta_dt = c->beta * dt;
    a.read_u1 = c->read_u1;
    a.write_u1 = c->write_u1;
    a.use_u2 = c->g3 != 0.0;
    a.u2_is_u0 = u2 == u0_in;
    if (!a.use_u2)
        a.u2 = nullptr;
    return run_groups(P, monitor ? MODE_RK_MON : MODE_RK, P->params.arith, a, s);
}

z4c_status enqueue_ghost(z4c_plan *P, int policy, double *u, const double *frozen, hipStream_t s)
{
    if (policy == Z4C_GHOST_NONE)
        return Z4C_OK;
    GhostArgs g{};
    g.blocks = P->blocks_d;
    g.nblocks = P->nblocks;
    g.ghost_start = P->ghost_start_d;
    g.neighbours = P->nbr_d;
    g.frozen = frozen;
    g.u = u;
    g.policy = policy;
    const hipError_t e = launch_ghost(g, P->total_ghost, s);
    if (e != hipSuccess)
        return hip_fail(e, "ghost kernel launch");
    return Z4C_OK;
}

z4c_status validate_ghost(const z4c_plan *P, int policy, const double *u, const double *frozen)
{
    if (policy < 0 || policy > 3)
        return fail(Z4C_EINVAL, "unknown ghost policy");
    if (policy != Z4C_GHOST_NONE && !u)
        return fail(Z4C_EINVAL, "u is NULL");
    if (policy == Z4C_GHOST_FROZEN && !frozen)
        return fail(Z4C_EINVAL, "frozen policy needs the frozen array");
    if (policy == Z4C_GHOST_NEIGHBOUR && !P->has_nbr)
        return fail(Z4C_EINVAL, "neighbour policy needs z4c_plan_set_neighbours first");
    if (policy == Z4C_GHOST_PERIODIC && !P->periodic_ok)
        return fail(Z4C_EINVAL, "periodic refresh needs nx, ny, nz >= ng for every block");
    if (frozen && frozen == u)
        return fail(Z4C_EINVAL, "frozen must not alias u");
    if (!aligned8(u) || !aligned8(frozen))
        return fail(Z4C_EALIGN, "arrays must be 8-byte aligned");
    return Z4C_OK;
}

z4c_status validate_halo(const z4c_plan *P, int policy, const double *frozen)
{
    if (policy < 0 || policy > 3)
        return fail(Z4C_EINVAL, "unknown ghost policy");
    if (policy == Z4C_GHOST_NONE)
        return Z4C_OK;
    if (policy == Z4C_GHOST_NEIGHBOUR && !P->has_nbr)
        return fail(Z4C_EINVAL, "neighbour policy needs z4c_plan_set_neighbours first");
    if (policy == Z4C_GHOST_NEIGHBOUR && !P->nbr32)
        return fail(Z4C_ENOTSUP, "neighbour-rule halo reads need offset + stored points <= 2^32 "
                                 "for every block that is another block's neighbour");
    if (policy == Z4C_GHOST_PERIODIC && !P->periodic_ok)
        return fail(Z4C_EINVAL, "periodic refresh needs nx, ny, nz >= ng for every block");
    if ((policy == Z4C_GHOST_FROZEN || policy == Z4C_GHOST_NEIGHBOUR) && !frozen) {
        if (policy == Z4C_GHOST_FROZEN)
            return fail(Z4C_EINVAL, "frozen policy needs the frozen array");
    }
    if (!aligned8(frozen))
        return fail(Z4C_EALIGN, "arrays must be 8-byte aligned");
    return Z4C_OK;
}

// Buffer schedule of a step: stage s reads regs[in_s]; every stage but the
// last writes the first of {1, 2} it does not read; the last stage writes
// regs[0] when it does not read u2 (= regs[0]), so that the step leaves the
// new state where the old one was.
z4c_status step_schedule(const z4c_step_desc *d, int in[8], int out[8], int *result)
{
    int cur = 0;
    for (int s = 0; s < d->nstages; ++s) {
        const bool last = s + 1 == d->nstages;
        int o = cur == 1 ? 2 : 1;
        if (last && d->table[s].g3 == 0.0)
            o = 0;
        in[s] = cur;
        out[s] = o;
        cur = o;
    }
    *result = cur;
    return Z4C_OK;
}

z4c_status validate_step(const z4c_plan *P, const z4c_step_desc *d)
{
    if (!d)
        return fail(Z4C_EINVAL, "step descriptor is NULL");
    if (d->nstages < 1 || d->nstages > 8 || !d->table)
        return fail(Z4C_EINVAL, "nstages must be in 1..8 with a coefficient table");
    for (int r = 0; r < 4; ++r)
        for (int q = r + 1; q < 4; ++q)
            if (d->regs[r] && d->regs[r] == d->regs[q])
                return fail(Z4C_EINVAL, "step registers must be distinct");
    if (!d->regs[0] || !d->regs[1] || !d->regs[2])
        return fail(Z4C_EINVAL, "regs[0..2] must not be NULL");
    for (int s = 0; s < d->nstages; ++s) {
        const z4c_rk_coeffs &c = d->table[s];
        if ((c.read_u1 || c.write_u1 || c.g2 != 0.0) && !d->regs[3])
            return fail(Z4C_EINVAL, "regs[3] (accumulator) is NULL but a stage uses it");
    }
    if (d->flags & ~(Z4C_STEP_STORED_GHOSTS | Z4C_STEP_NO_FINAL_FILL | Z4C_STEP_MONITOR
                     | Z4C_STEP_LEVEL_EXCHANGE | Z4C_STEP_SOMMERFELD))
        return fail(Z4C_EINVAL, "unknown step flags");
    if (d->flags & Z4C_STEP_SOMMERFELD) {
        if (!P || !P->radiative)
            return fail(Z4C_EINVAL, "Z4C_STEP_SOMMERFELD needs z4c_plan_set_sommerfeld");
        if (d->ghost_policy != Z4C_GHOST_NEIGHBOUR || d->frozen)
            return fail(Z4C_EINVAL, "Z4C_STEP_SOMMERFELD needs the neighbour policy without a "
                                    "frozen array (the outer ghosts are evolved)");
    }
    if (d->flags & Z4C_STEP_LEVEL_EXCHANGE) {
        if (!P || P->levels.empty())
            return fail(Z4C_EINVAL, "Z4C_STEP_LEVEL_EXCHANGE needs z4c_plan_set_level_exchange");
        if (d->ghost_policy == Z4C_GHOST_NONE)
            return fail(Z4C_EINVAL, "Z4C_STEP_LEVEL_EXCHANGE needs a same-level ghost policy");
    }
    if (d->flags & Z4C_STEP_MONITOR) {
        if (!d->norms)
            return fail(Z4C_EINVAL, "Z4C_STEP_MONITOR needs norms");
        if (d->cons && d->cons == d->norms)
            return fail(Z4C_EINVAL, "cons must not alias norms");
        for (const double *x : {(const double *)d->regs[0], (const double *)d->regs[1],
                                (const double *)d->regs[2], (const double *)d->regs[3],
                                d->matter, d->frozen})
            if (x && (x == d->cons || x == d->norms))
                return fail(Z4C_EINVAL, "cons and norms must not alias a register, matter or "
                                        "frozen");
        if (!aligned8(d->cons) || !aligned8(d->norms))
            return fail(Z4C_EALIGN, "arrays must be 8-byte aligned");
        if (P && P->params.arith != Z4C_ARITH_FP64)
            return fail(Z4C_ENOTSUP, "the constraint monitor runs with FP64 arithmetic only");
        if (P && P->params.advection != Z4C_ADVECT_CENTRED)
            return fail(Z4C_ENOTSUP, "the constraint monitor has centred advection only");
    }
    return validate_ghost(P, d->ghost_policy, d->regs[0], d->frozen);
}

// Ghost exchange across level jumps after the same-level fill: restrictions
// (coarse ghosts in fine spans, from fine interiors) finest pair first, then
// prolongations (fine ghosts in coarse spans, from coarse points whose ghosts
// are now current) coarsest pair first.
z4c_status enqueue_level_exchange(z4c_plan *P, double *u, hipStream_t s)
{
    for (size_t q = P->levels.size(); q-- > 0;) {
        const z4c_status st = z4c_restrict(P->levels[q], u, s);
        if (st != Z4C_OK)
            return st;
    }
    for (const z4c_xplan *X : P->levels) {
        const z4c_status st = z4c_prolongate(X, u, s);
        if (st != Z4C_OK)
            return st;
    }
    return Z4C_OK;
}

z4c_status enqueue_step(z4c_plan *P, const z4c_step_desc *d, int *result, hipStream_t s)
{
    int in[8], out[8], res;
    z4c_status st = step_schedule(d, in, out, &res);
    if (st != Z4C_OK)
        return st;
    // Ghost data of every stage input are read through the refresh rule
    // (no refresh pass) unless stored ghosts are asked for or unavailable;
    // a level-jump exchange works on stored ghosts.
    const bool levels = (d->flags & Z4C_STEP_LEVEL_EXCHANGE) != 0;
    // Neighbour-rule halo reads beyond their offset limit: stored ghosts
    // instead, those of y_n refreshed first (halo reads would ignore them),
    // so that both forms read the same values.
    const bool fallback = !(d->flags & Z4C_STEP_STORED_GHOSTS) && !levels
                          && d->ghost_policy == Z4C_GHOST_NEIGHBOUR && !P->nbr32;
    const bool stored = (d->flags & Z4C_STEP_STORED_GHOSTS) || d->ghost_policy == Z4C_GHOST_NONE
                        || fallback || levels;
    if (fallback) {
        st = enqueue_ghost(P, d->ghost_policy, d->regs[0], d->frozen, s);
        if (st != Z4C_OK)
            return st;
    }
    // radiative outer ghosts: advanced beside every stage (both read only
    // the stage input; the stage writes interior points, this the ghost
    // points without a same-level neighbour, which the same-level refresh
    // leaves alone; with a level exchange, the exchange then overwrites
    // those that a block of another level owns)
    const bool som = (d->flags & Z4C_STEP_SOMMERFELD) != 0;
    for (int k = 0; k < d->nstages; ++k) {
        const double *y = d->regs[0];
        const bool mon = k == 0 && (d->flags & Z4C_STEP_MONITOR);
        if (som) {
            st = enqueue_radiative(P, d->regs[in[k]], d->regs[out[k]], d->regs[3], y,
                                   &d->table[k], d->dt, nullptr, !stored, s);
            if (st != Z4C_OK)
                return st;
        }
        if (stored) {
            st = enqueue_stage(P, d->regs[in[k]], d->regs[out[k]], d->regs[3], y, d->matter,
                               &d->table[k], d->dt, s, Z4C_GHOST_NONE, nullptr, mon, d->cons);
            if (st == Z4C_OK)
                st = enqueue_ghost(P, d->ghost_policy, d->regs[out[k]], d->frozen, s);
            if (st == Z4C_OK && levels)
                st = enqueue_level_exchange(P, d->regs[out[k]], s);
        } else {
            st = enqueue_stage(P, d->regs[in[k]], d->regs[out[k]], d->regs[3], y, d->matter,
                               &d->table[k], d->dt, s, d->ghost_policy, d->frozen, mon,
                               d->cons);
        }
        if (st == Z4C_OK && mon) {
            const hipError_t e = launch_norm_reduce(P->blocks_d, P->nblocks, P->tile_start_d,
                                                    P->tile_count_d, P->partial_d, d->norms, s);
            if (e != hipSuccess)
                st = hip_fail(e, "norm reduction launch");
        }
        if (st != Z4C_OK)
            return st;
    }
    if (!stored && !(d->flags & Z4C_STEP_NO_FINAL_FILL)) {
        st = enqueue_ghost(P, d->ghost_policy, d->regs[res], d->frozen, s);
        if (st != Z4C_OK)
            return st;
    }
    if (result)
        *result = res;
    return Z4C_OK;
}

z4c_status validate_constraints(const z4c_plan *P, const double *u, const double *matter,
                                const double *cons, const double *norms)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    if (!u || !norms)
        return fail(Z4C_EINVAL, "u and norms must not be NULL");
    if (cons == u || norms == u || (cons && cons == norms))
        return fail(Z4C_EINVAL, "outputs must not alias u or each other");
    if (!aligned8(u) || !aligned8(cons) || !aligned8(norms) || !aligned8(matter))
        return fail(Z4C_EALIGN, "arrays must be 8-byte aligned");
    return need_device(P);
}

// Constraint kernel + per-block norm reduction, with the per-tile partial
// sums in `partial` (16 doubles per tile of the plan).
z4c_status enqueue_constraints(z4c_plan *P, const double *u, const double *matter, double *cons,
                               double *norms, double *partial, hipStream_t s)
{
    StageArgs a = base_args(P);
    a.u = u;
    a.matter = matter;
    a.out = cons;
    a.partial = partial;
    z4c_status st = run_groups(P, MODE_CONS, Z4C_ARITH_FP64, a, s);
    if (st != Z4C_OK)
        return st;
    const hipError_t e = launch_norm_reduce(P->blocks_d, P->nblocks, P->tile_start_d,
                                            P->tile_count_d, partial, norms, s);
    if (e != hipSuccess)
        return hip_fail(e, "norm reduction launch");
    return Z4C_OK;
}

// Autotuning cache: one line per size class and scheme,
//   <key> <tile_x> <tile_y> <tile_z> <persistent> <waves> <ms per launch>
// keyed by the device architecture, order, arithmetic, advection, halo rule
// and the block's interior and ghost sizes; the time is that of the launch
// that made the choice (the class alone, or the merged set it joined).  The
// path is set with z4c_set_tune_cache (empty: no cache).
struct TuneEntry {
    z4c_launch launch;
    float ms;
};
struct TuneCache {
    std::map<std::string, TuneEntry> entries;
};
std::mutex g_tune_mutex;
std::string g_tune_path;

std::string tune_key(const z4c_plan *P, const SizeClass &c)
{
    std::string arch = "unknown";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');   // drop feature suffixes
        if (colon != std::string::npos)
            arch.resize(colon);
    }
    const z4c_block &B = P->blocks[c.blocks.front()];
    char buf[192];
    std::snprintf(buf, sizeof buf, "%s:p%d:arith%d:adv%d:halo%d:n%dx%dx%d:ng%d", arch.c_str(),
                  P->params.fd_order, P->params.arith, P->params.advection, P->halo, c.nx, c.ny,
                  c.nz, B.ng);
    return buf;
}

TuneCache tune_cache_load()
{
    TuneCache c;
    std::string path;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        path = g_tune_path;
    }
    if (path.empty())
        return c;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f)
        return c;
    char key[192];
    z4c_launch L{};
    float ms = 0.f;
    while (std::fscanf(f, "%191s %d %d %d %d %d %f", key, &L.tile_x, &L.tile_y, &L.tile_z,
                       &L.persistent, &L.waves, &ms) == 7)
        c.entries[key] = TuneEntry{L, ms};
    std::fclose(f);
    return c;
}

void tune_cache_store(const TuneCache &c)
{
    std::string path;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        path = g_tune_path;
    }
    if (path.empty())
        return;
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f)
        return;
    for (const auto &e : c.entries)
        std::fprintf(f, "%s %d %d %d %d %d %.6f\n", e.first.c_str(), e.second.launch.tile_x,
                     e.second.launch.tile_y, e.second.launch.tile_z, e.second.launch.persistent,
                     e.second.launch.waves, e.second.ms);
    std::fclose(f);
    (void)std::rename(tmp.c_str(), path.c_str());
}

// Scratch of z4c_constraints_noalloc: the per-tile partial sums live in this
// file-scope device array instead of the plan's buffer, so that the call
// allocates nothing.  Each device holds its own copy; in host code the name
// is only a stand-in, and the device address comes from hipGetSymbolAddress,
// looked up once per device (at plan creation, or on the first call on that
// device) and kept in noalloc_ptr.
constexpr int NOALLOC_MAX_DEVICES = 64;
double *noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
std::mutex noalloc_mutex;

// Device address of this device's scratch array (looked up on first use).
z4c_status noalloc_scratch(double **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(Z4C_ENOTSUP, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(noalloc_mutex);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p)
            return fail(Z4C_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        noalloc_ptr[dev] = static_cast<double *>(p);
    }
    *out = noalloc_ptr[dev];
    return Z4C_OK;
}

}  // namespace

z4c_status z4c::set_error(z4c_status s, const char *msg) { return fail(s, msg); }
const std::vector<z4c_block> &z4c::plan_blocks(const z4c_plan *P) { return P->blocks; }
const z4c_block *z4c::plan_blocks_device(const z4c_plan *P)
{
    return P->device ? P->blocks_d : nullptr;
}
z4c_status z4c::set_hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }

extern "C" {

const char *z4c_strerror(z4c_status s)
{
    switch (s) {
    case Z4C_OK: return "success";
    case Z4C_EINVAL: return "invalid argument";
    case Z4C_ENOGHOST: return "not enough ghost points for the stencil";
    case Z4C_EALIGN: return "misaligned array";
    case Z4C_EHIP: return "HIP runtime error";
    case Z4C_ENOTSUP: return "not supported";
    case Z4C_ENOMEM: return "device allocation failed";
    case Z4C_ENODEV: return "plan has no device";
    }
    return "unknown status";
}

const char *z4c_last_error(void) { return g_last_error.c_str(); }

z4c_status z4c_plan_create(const z4c_params *params, const z4c_block *blocks, int nblocks,
                           int flags, z4c_plan **out)
{
    if (!out)
        return fail(Z4C_EINVAL, "out is NULL");
    *out = nullptr;
    z4c_status st = check_params(params);
    if (st != Z4C_OK)
        return st;
    if (!blocks || nblocks < 1)
        return fail(Z4C_EINVAL, "need at least one block");
    for (int b = 0; b < nblocks; ++b) {
        st = check_block(blocks[b], b, params->fd_order);
        if (st != Z4C_OK)
            return st;
    }
    z4c_plan *P = new z4c_plan();
    P->params = *params;
    P->device = !(flags & Z4C_PLAN_NO_DEVICE);
    P->nblocks = nblocks;
    P->blocks.assign(blocks, blocks + nblocks);
    std::map<std::vector<int>, int> cls;
    for (int b = 0; b < nblocks; ++b) {
        const std::vector<int> key = {blocks[b].nx, blocks[b].ny, blocks[b].nz};
        auto it = cls.find(key);
        if (it == cls.end()) {
            SizeClass c;
            c.nx = blocks[b].nx;
            c.ny = blocks[b].ny;
            c.nz = blocks[b].nz;
            c.launch = z4c_launch{8, 8, 8, 0, 2};
            c.blocks.push_back(b);
            cls[key] = (int)P->classes.size();
            P->classes.push_back(c);
        } else {
            P->classes[it->second].blocks.push_back(b);
        }
    }
    // ghost-point and interior-point prefix sums
    std::vector<long long> gs(nblocks + 1, 0), ps(nblocks + 1, 0);
    for (int b = 0; b < nblocks; ++b) {
        const z4c_block &B = blocks[b];
        const long long ex = B.nx + 2LL * B.ng, ey = B.ny + 2LL * B.ng, ez = B.nz + 2LL * B.ng;
        const long long interior = (long long)B.nx * B.ny * B.nz;
        gs[b + 1] = gs[b] + ex * ey * ez - interior;
        if (B.nx < B.ng || B.ny < B.ng || B.nz < B.ng)
            P->periodic_ok = false;
        ps[b + 1] = ps[b] + interior;
    }
    P->total_ghost = gs[nblocks];
    P->total_pts = ps[nblocks];
    if (P->device) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&P->num_cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipMalloc(&P->blocks_d, sizeof(z4c_block) * nblocks);
        if (e == hipSuccess)
            e = hipMemcpy(P->blocks_d, blocks, sizeof(z4c_block) * nblocks, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMalloc(&P->ghost_start_d, sizeof(long long) * (nblocks + 1));
        if (e == hipSuccess)
            e = hipMemcpy(P->ghost_start_d, gs.data(), sizeof(long long) * (nblocks + 1),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMalloc(&P->pt_start_d, sizeof(long long) * (nblocks + 1));
        if (e == hipSuccess)
            e = hipMemcpy(P->pt_start_d, ps.data(), sizeof(long long) * (nblocks + 1),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMalloc(&P->count_d, sizeof(unsigned long long));
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            z4c_plan_destroy(P);
            return hip_fail(e, "plan device set-up");
        }
        double *scratch_d = nullptr;   // z4c_constraints_noalloc's scratch on this device
        st = noalloc_scratch(&scratch_d);
        if (st != Z4C_OK) {
            z4c_plan_destroy(P);
            return st;
        }
    }
    st = build_groups(P);
    if (st == Z4C_OK)
        st = upload_factors(P);
    if (st != Z4C_OK) {
        z4c_plan_destroy(P);
        return st;
    }
    *out = P;
    return Z4C_OK;
}

z4c_status z4c_plan_destroy(z4c_plan *P)
{
    if (!P)
        return Z4C_OK;
    if (P->device) {
        P->clear_graphs();
        P->free_groups();
        if (P->blocks_d)
            (void)hipFree(P->blocks_d);
        if (P->fac64_d)
            (void)hipFree(P->fac64_d);
        if (P->fac32_d)
            (void)hipFree(P->fac32_d);
        if (P->ghost_start_d)
            (void)hipFree(P->ghost_start_d);
        if (P->pt_start_d)
            (void)hipFree(P->pt_start_d);
        if (P->nbr_d)
            (void)hipFree(P->nbr_d);
        P->free_outer();
        if (P->count_d)
            (void)hipFree(P->count_d);
        if (P->capture_stream)
            (void)hipStreamDestroy(P->capture_stream);
    }
    delete P;
    return Z4C_OK;
}

z4c_status z4c_plan_set_params(z4c_plan *P, const z4c_params *params)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    z4c_status st = check_params(params);
    if (st != Z4C_OK)
        return st;
    for (int b = 0; b < P->nblocks; ++b) {
        st = check_block(P->blocks[b], b, params->fd_order);
        if (st != Z4C_OK)
            return st;
    }
    const bool order_changed = P->params.fd_order != params->fd_order;
    P->params = *params;
    if (P->device)
        P->clear_graphs();
    ++P->version;
    if (order_changed) {
        bool reset = false;
        for (auto &c : P->classes)
            if (!stage_shape_supported(params->fd_order, c.launch.tile_x, c.launch.tile_y,
                                       c.launch.tile_z, c.launch.waves)) {
                c.launch = z4c_launch{8, 8, 8, 0, 2};
                reset = true;
            }
        if (reset) {
            st = build_groups(P);
            if (st != Z4C_OK)
                return st;
        }
    }
    return upload_factors(P);
}

z4c_status z4c_plan_set_neighbours(z4c_plan *P, const int *nbr)
{
    if (!P || !nbr)
        return fail(Z4C_EINVAL, "plan and neighbour table must not be NULL");
    bool far32 = true;
    for (int b = 0; b < P->nblocks; ++b)
        for (int d = 0; d < 27; ++d) {
            const int n = nbr[b * 27 + d];
            if (n < -1 || n >= P->nblocks)
                return fail(Z4C_EINVAL, "neighbour index out of range");
            if (n >= 0 && n != b) {
                const z4c_block &N = P->blocks[n];
                const long long npts = (N.nx + 2LL * N.ng) * (N.ny + 2LL * N.ng) * (N.nz + 2LL * N.ng);
                if (N.offset + npts > (1LL << 32))
                    far32 = false;
            }
            if (n >= 0) {
                const z4c_block &A = P->blocks[b], &B = P->blocks[n];
                if (A.nx != B.nx || A.ny != B.ny || A.nz != B.nz || A.ng != B.ng
                    || A.field_stride != B.field_stride)
                    return fail(Z4C_EINVAL,
                                "neighbours must have equal nx, ny, nz, ng and field_stride");
                const int ox = d % 3 - 1, oy = (d / 3) % 3 - 1, oz = d / 9 - 1;
                if ((ox && A.nx < A.ng) || (oy && A.ny < A.ng) || (oz && A.nz < A.ng))
                    return fail(Z4C_EINVAL, "a neighbour copy needs n >= ng along its direction");
            }
        }
    if (!far32 && P->halo == Z4C_GHOST_NEIGHBOUR)
        return fail(Z4C_ENOTSUP, "the plan reads halos through the neighbour rule, which needs "
                                 "offset + stored points <= 2^32 for every block that is another "
                                 "block's neighbour");
    std::vector<OuterRegion> outer;
    if (P->radiative) {
        const z4c_status so = outer_regions(P, nbr, P->origins.data(), outer);
        if (so != Z4C_OK)
            return so;
    }
    if (P->device) {
        if (!P->nbr_d)
            HIP_TRY(hipMalloc(&P->nbr_d, sizeof(int) * 27 * P->nblocks), "hipMalloc(neighbours)");
        HIP_TRY(hipMemcpy(P->nbr_d, nbr, sizeof(int) * 27 * P->nblocks, hipMemcpyHostToDevice),
                "hipMemcpy(neighbours)");
        P->clear_graphs();
    }
    P->has_nbr = true;
    P->nbr32 = far32;
    P->nbr_h.assign(nbr, nbr + 27 * (size_t)P->nblocks);
    ++P->version;
    if (P->radiative) {
        P->outer.swap(outer);
        return upload_outer(P);
    }
    return Z4C_OK;
}

z4c_status z4c_plan_set_sommerfeld(z4c_plan *P, const double *origins)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    if (!origins) {
        P->radiative = false;
        P->outer.clear();
        P->total_outer = 0;
        if (P->device) {
            P->clear_graphs();
            P->free_outer();
        }
        ++P->version;
        return Z4C_OK;
    }
    if (!P->has_nbr)
        return fail(Z4C_EINVAL, "the radiative boundary needs z4c_plan_set_neighbours first");
    for (int q = 0; q < 3 * P->nblocks; ++q)
        if (!std::isfinite(origins[q]))
            return fail(Z4C_EINVAL, "origins must be finite");
    std::vector<OuterRegion> outer;
    const z4c_status st = outer_regions(P, P->nbr_h.data(), origins, outer);
    if (st != Z4C_OK)
        return st;
    P->origins.assign(origins, origins + 3 * (size_t)P->nblocks);
    P->outer.swap(outer);
    P->radiative = true;
    ++P->version;
    return upload_outer(P);
}

z4c_status z4c_plan_set_halo(z4c_plan *P, int policy, const double *frozen)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    z4c_status st = validate_halo(P, policy, frozen);
    if (st != Z4C_OK)
        return st;
    P->halo = policy;
    P->halo_frozen = frozen;
    if (P->device)
        P->clear_graphs();
    ++P->version;
    return Z4C_OK;
}

z4c_status z4c_plan_set_level_exchange(z4c_plan *P, const z4c_xplan *const *xplans, int n)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    if (n < 0 || (n > 0 && !xplans))
        return fail(Z4C_EINVAL, "need n >= 0 transfer plans");
    for (int q = 0; q < n; ++q)
        if (!xplans[q] || z4c::xplan_plan(xplans[q]) != P)
            return fail(Z4C_EINVAL, "every transfer plan must be one of this plan's");
    P->levels.assign(xplans, xplans + n);
    if (P->device)
        P->clear_graphs();
    ++P->version;
    return Z4C_OK;
}

z4c_status z4c_plan_set_launch(z4c_plan *P, int nx, int ny, int nz, const z4c_launch *L)
{
    if (!P || !L)
        return fail(Z4C_EINVAL, "plan and launch must not be NULL");
    z4c_launch LL = *L;
    if (LL.waves == 0)
        LL.waves = 2;
    if (!stage_shape_supported(P->params.fd_order, LL.tile_x, LL.tile_y, LL.tile_z, LL.waves))
        return fail(Z4C_ENOTSUP, "unsupported tile shape / occupancy for this order");
    if (L->persistent < 0)
        return fail(Z4C_EINVAL, "persistent must be >= 0");
    bool any = false;
    for (auto &c : P->classes)
        if ((nx == 0 && ny == 0 && nz == 0) || (c.nx == nx && c.ny == ny && c.nz == nz)) {
            c.launch = LL;
            any = true;
        }
    if (!any)
        return fail(Z4C_EINVAL, "no blocks of that size");
    return build_groups(P);
}

z4c_status z4c_plan_get_launch(const z4c_plan *P, int nx, int ny, int nz, z4c_launch *L)
{
    if (!P || !L)
        return fail(Z4C_EINVAL, "plan and launch must not be NULL");
    for (const auto &c : P->classes)
        if (c.nx == nx && c.ny == ny && c.nz == nz) {
            *L = c.launch;
            return Z4C_OK;
        }
    return fail(Z4C_EINVAL, "no blocks of that size");
}

long long z4c_plan_tiles(const z4c_plan *P) { return P ? P->total_tiles : -1; }

z4c_status z4c_rhs(z4c_plan *P, const double *u, const double *matter, double *rhs, void *stream)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    if (!u || !rhs)
        return fail(Z4C_EINVAL, "u and rhs must not be NULL");
    if (u == rhs || matter == rhs)
        return fail(Z4C_EINVAL, "rhs must not alias u or matter");
    if (!aligned8(u) || !aligned8(rhs) || !aligned8(matter))
        return fail(Z4C_EALIGN, "arrays must be 8-byte aligned");
    z4c_status st = need_device(P);
    if (st != Z4C_OK)
        return st;
    StageArgs a = base_args(P);
    a.u = u;
    a.matter = matter;
    a.out = rhs;
    return run_groups(P, MODE_RHS, P->params.arith, a, (hipStream_t)stream);
}

z4c_status z4c_rk_stage(z4c_plan *P, const double *u0_in, double *u0_out, double *u1,
                        const double *u2, const double *matter, const z4c_rk_coeffs *c,
                        double dt, void *stream)
{
    z4c_status st = validate_stage(P, u0_in, u0_out, u1, u2, matter, c, dt);
    if (st != Z4C_OK)
        return st;
    st = need_device(P);
    if (st != Z4C_OK)
        return st;
    return enqueue_stage(P, u0_in, u0_out, u1, u2, matter, c, dt, (hipStream_t)stream);
}

z4c_status z4c_rk_stage_monitor(z4c_plan *P, const double *u0_in, double *u0_out, double *u1,
                                const double *u2, const double *matter, const z4c_rk_coeffs *c,
                                double dt, double *cons, double *norms, void *stream)
{
    z4c_status st = validate_stage(P, u0_in, u0_out, u1, u2, matter, c, dt);
    if (st != Z4C_OK)
        return st;
    if (!norms)
        return fail(Z4C_EINVAL, "norms must not be NULL");
    for (const double *x : {u0_in, (const double *)u0_out, (const double *)u1, u2, matter})
        if (x && (x == cons || x == norms))
            return fail(Z4C_EINVAL, "cons and norms must not alias a state or matter array");
    if (cons && cons == norms)
        return fail(Z4C_EINVAL, "cons must not alias norms");
    if (!aligned8(cons) || !aligned8(norms))
        return fail(Z4C_EALIGN, "arrays must be 8-byte aligned");
    if (P->params.arith != Z4C_ARITH_FP64)
        return fail(Z4C_ENOTSUP, "the constraint monitor runs with FP64 arithmetic only");
    if (P->params.advection != Z4C_ADVECT_CENTRED)
        return fail(Z4C_ENOTSUP, "the constraint monitor has centred advection only");
    st = need_device(P);
    if (st != Z4C_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    st = enqueue_stage(P, u0_in, u0_out, u1, u2, matter, c, dt, s, -1, nullptr, true, cons);
    if (st != Z4C_OK)
        return st;
    const hipError_t e = launch_norm_reduce(P->blocks_d, P->nblocks, P->tile_start_d,
                                            P->tile_count_d, P->partial_d, norms, s);
    if (e != hipSuccess)
        return hip_fail(e, "norm reduction launch");
    return Z4C_OK;
}

z4c_status z4c_constraints(z4c_plan *P, const double *u, const double *matter, double *cons,
                           double *norms, void *stream)
{
    z4c_status st = validate_constraints(P, u, matter, cons, norms);
    if (st != Z4C_OK)
        return st;
    return enqueue_constraints(P, u, matter, cons, norms, P->partial_d, (hipStream_t)stream);
}

z4c_status z4c_constraints_noalloc(z4c_plan *P, const double *u, const double *matter,
                                   double *cons, double *norms, void *stream)
{
    z4c_status st = validate_constraints(P, u, matter, cons, norms);
    if (st != Z4C_OK)
        return st;
    if (P->total_tiles > NOALLOC_MAX_TILES) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "z4c_constraints_noalloc: the plan has %lld tiles; the static scratch "
                      "holds the partial sums of at most %d",
                      P->total_tiles, NOALLOC_MAX_TILES);
        return fail(Z4C_ENOTSUP, buf);
    }
    double *partial = nullptr;
    st = noalloc_scratch(&partial);
    if (st != Z4C_OK)
        return st;
    return enqueue_constraints(P, u, matter, cons, norms, partial, (hipStream_t)stream);
}

z4c_status z4c_ghost_fill(z4c_plan *P, int policy, double *u, const double *frozen, void *stream)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    z4c_status st = validate_ghost(P, policy, u, frozen);
    if (st != Z4C_OK)
        return st;
    st = need_device(P);
    if (st != Z4C_OK)
        return st;
    return enqueue_ghost(P, policy, u, frozen, (hipStream_t)stream);
}

z4c_status z4c_sommerfeld_rhs(z4c_plan *P, const double *u, double *rhs, void *stream)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    if (!P->radiative)
        return fail(Z4C_EINVAL, "z4c_plan_set_sommerfeld has not been called");
    if (!u || !rhs)
        return fail(Z4C_EINVAL, "u and rhs must not be NULL");
    if (u == rhs)
        return fail(Z4C_EINVAL, "rhs must not alias u");
    if (!aligned8(u) || !aligned8(rhs))
        return fail(Z4C_EALIGN, "arrays must be 8-byte aligned");
    z4c_status st = need_device(P);
    if (st != Z4C_OK)
        return st;
    return enqueue_radiative(P, u, nullptr, nullptr, nullptr, nullptr, 0.0, rhs,
                             P->halo == Z4C_GHOST_NEIGHBOUR, (hipStream_t)stream);
}

z4c_status z4c_sommerfeld_stage(z4c_plan *P, const double *u0_in, double *u0_out, double *u1,
                                const double *u2, const z4c_rk_coeffs *c, double dt,
                                void *stream)
{
    z4c_status st = validate_stage(P, u0_in, u0_out, u1, u2, nullptr, c, dt);
    if (st != Z4C_OK)
        return st;
    if (!P->radiative)
        return fail(Z4C_EINVAL, "z4c_plan_set_sommerfeld has not been called");
    st = need_device(P);
    if (st != Z4C_OK)
        return st;
    return enqueue_radiative(P, u0_in, u0_out, u1, u2, c, dt, nullptr,
                             P->halo == Z4C_GHOST_NEIGHBOUR, (hipStream_t)stream);
}

z4c_status z4c_step(z4c_plan *P, const z4c_step_desc *d, int *result, void *stream)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    z4c_status st = validate_step(P, d);
    if (st != Z4C_OK)
        return st;
    int in[8], out[8], res;
    st = step_schedule(d, in, out, &res);
    if (st != Z4C_OK)
        return st;
    for (int k = 0; k < d->nstages; ++k) {
        st = validate_stage(P, d->regs[in[k]], d->regs[out[k]], d->regs[3], d->regs[0], d->matter,
                            &d->table[k], d->dt);
        if (st != Z4C_OK)
            return st;
    }
    st = need_device(P);
    if (st != Z4C_OK)
        return st;
    return enqueue_step(P, d, result, (hipStream_t)stream);
}

z4c_status z4c_step_graph(z4c_plan *P, const z4c_step_desc *d, int *result, void *stream)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    z4c_status st = validate_step(P, d);
    if (st != Z4C_OK)
        return st;
    {
        int in0[8], out0[8], r0;
        st = step_schedule(d, in0, out0, &r0);
        if (st != Z4C_OK)
            return st;
        for (int k = 0; k < d->nstages; ++k) {
            st = validate_stage(P, d->regs[in0[k]], d->regs[out0[k]], d->regs[3], d->regs[0],
                                d->matter, &d->table[k], d->dt);
            if (st != Z4C_OK)
                return st;
        }
    }
    st = need_device(P);
    if (st != Z4C_OK)
        return st;
    StepKey key;
    std::memset(&key, 0, sizeof key);
    for (int r = 0; r < 4; ++r)
        key.regs[r] = d->regs[r];
    key.matter = d->matter;
    key.frozen = d->frozen;
    key.dt = d->dt;
    key.nstages = d->nstages;
    key.ghost_policy = d->ghost_policy;
    key.flags = d->flags;
    key.cons = d->cons;
    key.norms = d->norms;
    for (int s = 0; s < d->nstages; ++s)
        key.table[s] = d->table[s];
    key.version = P->version;
    for (const auto &g : P->graphs)
        if (g.key == key) {
            HIP_TRY(hipGraphLaunch(g.exec, (hipStream_t)stream), "hipGraphLaunch");
            if (result)
                *result = g.result;
            return Z4C_OK;
        }
    int in[8], out[8], res;
    st = step_schedule(d, in, out, &res);
    if (st != Z4C_OK)
        return st;
    for (int k = 0; k < d->nstages; ++k) {
        st = validate_stage(P, d->regs[in[k]], d->regs[out[k]], d->regs[3], d->regs[0], d->matter,
                            &d->table[k], d->dt);
        if (st != Z4C_OK)
            return st;
    }
    hipStream_t cs = P->capture_stream;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    st = enqueue_step(P, d, nullptr, cs);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    if (st != Z4C_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return st;
    }
    if (ee != hipSuccess)
        return hip_fail(ee, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess)
        return hip_fail(ei, "hipGraphInstantiate");
    if (P->graphs.size() >= 4) {
        (void)hipGraphExecDestroy(P->graphs.front().exec);
        P->graphs.erase(P->graphs.begin());
    }
    P->graphs.push_back(GraphEntry{key, exec, res});
    HIP_TRY(hipGraphLaunch(exec, (hipStream_t)stream), "hipGraphLaunch");
    if (result)
        *result = res;
    return Z4C_OK;
}

z4c_status z4c_plan_autotune(z4c_plan *P, const double *u0, double *u0_out, double *u1,
                             const double *matter, int reps, void *stream)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    if (!u0 || !u0_out || !u1 || u0 == u0_out || u1 == u0 || u1 == u0_out)
        return fail(Z4C_EINVAL, "autotune needs three distinct state buffers");
    if (reps < 1)
        return fail(Z4C_EINVAL, "reps must be >= 1");
    if (P->params.arith == Z4C_ARITH_FP32_NAIVE)
        return fail(Z4C_ENOTSUP, "the naive FP32 form is a right-hand side only (no autotuning)");
    z4c_status st = need_device(P);
    if (st != Z4C_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    const z4c_rk_coeffs c{0.0, 1.0 / 3.0, 0.0, 0.0, 1.0, 0.5, 1, 1};
    // Candidates: every supported tile shape and occupancy, as a grid launch
    // and as persistent launches of one or two workgroups per CU; earlier
    // candidates win near-ties (a later one must be 1.5 % faster).
    static const int shapes[][4] = {{8, 8, 4, 1}, {8, 4, 8, 1}, {8, 8, 8, 2}, {8, 8, 4, 2}};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    const std::vector<SizeClass> saved = P->classes;
    std::vector<z4c_launch> best(P->classes.size());
    std::vector<float> best_time(P->classes.size(), 0.f);
    TuneCache cache = tune_cache_load();
    std::vector<std::string> keys(saved.size());
    for (size_t ci = 0; ci < saved.size(); ++ci) {
        keys[ci] = tune_key(P, saved[ci]);
        auto hit = cache.entries.find(keys[ci]);
        if (hit != cache.entries.end()
            && stage_shape_supported(P->params.fd_order, hit->second.launch.tile_x,
                                     hit->second.launch.tile_y, hit->second.launch.tile_z,
                                     hit->second.launch.waves)) {
            best[ci] = hit->second.launch;
            best_time[ci] = -1.f;   // from the cache
            continue;
        }
        float best_ms = 1e30f;
        for (const auto &sh : shapes) {
            if (!stage_shape_supported(P->params.fd_order, sh[0], sh[1], sh[2], sh[3]))
                continue;
            for (int pers : {0, 1, 2}) {
                z4c_launch L{sh[0], sh[1], sh[2], pers * P->num_cus, sh[3]};
                // a plan view holding only this size class
                P->classes.assign(1, saved[ci]);
                P->classes[0].launch = L;
                st = build_groups(P);
                if (st != Z4C_OK)
                    break;
                st = enqueue_stage(P, u0, u0_out, u1, u0, matter, &c, 1e-3, s);   // warm-up
                if (st != Z4C_OK)
                    break;
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < reps && st == Z4C_OK; ++r)
                    st = enqueue_stage(P, u0, u0_out, u1, u0, matter, &c, 1e-3, s);
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (st == Z4C_OK && ms < 0.985f * best_ms) {
                    best_ms = ms;
                    best[ci] = L;
                    best_time[ci] = ms / reps;
                }
            }
            if (st != Z4C_OK)
                break;
        }
        if (st != Z4C_OK)
            break;
    }
    // Merge pass.  Classes that share a tile shape and occupancy run as one
    // dispatch when they also share the launch form, which a class timed
    // alone cannot see (one tail instead of several, one work queue for
    // all).  For each such set of two or more classes, time the set with
    // the per-class choices and with each uniform launch form, and keep the
    // fastest (a change must be 1.5 % faster).  Runs only when some class was
    // timed now, so that a plan whose classes all come from the cache keeps
    // exactly the cached launches.
    bool fresh_any = false;
    for (size_t ci = 0; ci < saved.size(); ++ci)
        fresh_any = fresh_any || best_time[ci] >= 0.f;
    if (st == Z4C_OK && fresh_any) {
        std::map<std::vector<int>, std::vector<size_t>> sets;
        for (size_t ci = 0; ci < saved.size(); ++ci)
            sets[{best[ci].tile_x, best[ci].tile_y, best[ci].tile_z, best[ci].waves}].push_back(ci);
        auto time_set = [&](const std::vector<size_t> &members,
                            const std::vector<z4c_launch> &launch, float *ms) -> z4c_status {
            P->classes.clear();
            for (size_t m = 0; m < members.size(); ++m) {
                P->classes.push_back(saved[members[m]]);
                P->classes.back().launch = launch[m];
            }
            z4c_status r = build_groups(P);
            if (r == Z4C_OK)
                r = enqueue_stage(P, u0, u0_out, u1, u0, matter, &c, 1e-3, s);   // warm-up
            if (r != Z4C_OK)
                return r;
            (void)hipEventRecord(e0, s);
            for (int k = 0; k < reps && r == Z4C_OK; ++k)
                r = enqueue_stage(P, u0, u0_out, u1, u0, matter, &c, 1e-3, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            *ms = 0.f;
            (void)hipEventElapsedTime(ms, e0, e1);
            return r;
        };
        for (const auto &kv : sets) {
            const std::vector<size_t> &members = kv.second;
            if (members.size() < 2)
                continue;
            std::vector<z4c_launch> cur(members.size());
            for (size_t m = 0; m < members.size(); ++m)
                cur[m] = best[members[m]];
            float best_ms = 0.f;
            st = time_set(members, cur, &best_ms);
            std::vector<z4c_launch> pick = cur;
            for (int pers : {0, 1, 2}) {
                if (st != Z4C_OK)
                    break;
                std::vector<z4c_launch> uni(members.size(), cur[0]);
                for (auto &L : uni)
                    L.persistent = pers * P->num_cus;
                float ms = 0.f;
                st = time_set(members, uni, &ms);
                if (st == Z4C_OK && ms < 0.985f * best_ms) {
                    best_ms = ms;
                    pick = uni;
                }
            }
            if (st != Z4C_OK)
                break;
            for (size_t m = 0; m < members.size(); ++m) {
                const size_t ci = members[m];
                if (pick[m].persistent != best[ci].persistent)
                    best_time[ci] = best_ms / reps;   // now a member of a merged dispatch
                best[ci] = pick[m];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->classes = saved;
    if (st == Z4C_OK) {
        bool fresh = false;
        for (size_t ci = 0; ci < saved.size(); ++ci) {
            P->classes[ci].launch = best[ci];
            if (best_time[ci] >= 0.f) {
                cache.entries[keys[ci]] = TuneEntry{best[ci], best_time[ci]};
                fresh = true;
            }
        }
        if (fresh)
            tune_cache_store(cache);
    }
    const z4c_status st2 = build_groups(P);
    return st != Z4C_OK ? st : st2;
}

z4c_status z4c_set_tune_cache(const char *path)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_path = path ? std::string(path) : std::string();
    return Z4C_OK;
}

z4c_status z4c_check_finite(z4c_plan *P, const double *u, long long *count, void *stream)
{
    if (!P)
        return fail(Z4C_EINVAL, "plan is NULL");
    if (!u || !count)
        return fail(Z4C_EINVAL, "u and count must not be NULL");
    z4c_status st = need_device(P);
    if (st != Z4C_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_zero_u64(P->count_d, s), "zero kernel");
    HIP_TRY(launch_finite_count(P->blocks_d, P->nblocks, P->pt_start_d, P->total_pts, u, P->count_d,
                                s),
            "finite-count kernel");
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, P->count_d, sizeof h, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    *count = (long long)h;
    return Z4C_OK;
}

}  // extern "C"
