// Internal declarations shared by the kernel and host translation units of
// libz4c.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "z4c.h"

namespace z4c {

// State field indices (order fixed by the ABI).
enum Field : int {
    CHI = 0, GXX = 1, GXY, GXZ, GYY, GYZ, GZZ, KHAT = 7,
    AXX = 8, AXY, AXZ, AYY, AYZ, AZZ, THETA = 14,
    GAMX = 15, GAMY, GAMZ, ALPHA = 18, BETAX = 19, BETAY, BETAZ, NFIELD = 22
};
enum MatterField : int { M_RHO = 0, M_SX, M_SY, M_SZ, M_SXX, M_SXY, M_SXZ, M_SYY, M_SYZ, M_SZZ,
                         NMATTER = 10 };
enum ConsField : int { C_H = 0, C_MX, C_MY, C_MZ, C_THETA, C_ZX, C_ZY, C_ZZ, NCONS = 8 };

// What a tile kernel produces.
enum Mode : int { MODE_RHS = 0, MODE_RK = 1, MODE_CONS = 2, MODE_RK_MON = 3 };

// One work item of a tile kernel: block index and interior origin of the tile.
struct Tile {
    int block, i0, j0, k0;
};

struct StageArgs {
    const z4c_block *blocks;
    const double *fac64;     // per block: 12 stencil scale factors (see block_factors)
    const float *fac32;      // the same factors rounded to float
    const Tile *tiles;
    int ntiles;
    int persistent;          // 0: one workgroup per tile; else that many workgroups
    int *queue;              // persistent: 8 tile counters (one per XCD range), zeroed
    long long tile_base;     // global index of tiles[0] (norm partial sums)
    const double *u;         // input state (u0 for a stage)
    const double *matter;    // nullptr = vacuum
    double *out;             // rhs, u0_out, or constraint fields (may be nullptr for CONS)
    double *u1;
    const double *u2;
    double *partial;         // CONS: per-tile sums, [tile][16]
    double *cons;            // RK_MON: constraint fields of the input (may be nullptr)
    // Runge-Kutta stage
    double delta, eps_dt, g1, g2, g3, beta_dt;
    int read_u1, write_u1, use_u2, u2_is_u0;
    // scheme
    double ko_sigma, kappa1, kappa2, eta, chi_floor, alpha_floor;
    int lapse, shift, advect_gauge;
    // Halo reads: how ghost points of the input are obtained.  GHOST_NONE:
    // the stored ghost values; PERIODIC / NEIGHBOUR / FROZEN: read straight
    // from the source a ghost refresh would copy (own interior wrapped, the
    // neighbour's interior, or `frozen`), so no refresh pass is needed.
    int halo;
    const int *nbr;          // nblocks*27 (NEIGHBOUR)
    const double *frozen;    // state layout (FROZEN, and NEIGHBOUR outer faces)
};

struct GhostArgs {
    const z4c_block *blocks;
    int nblocks;
    const long long *ghost_start;   // nblocks + 1 prefix sums of ghost points
    const int *neighbours;          // nblocks*27 or nullptr
    const double *frozen;
    double *u;
    int policy;
};

// Radiative (Sommerfeld) outer boundary: one box of outer ghost points of a
// block (ghost points in a direction whose neighbour entry is -1).
struct OuterRegion {
    int block;
    int lo[3];   // first point, indices counted from the first interior point
    int n[3];    // extent per direction
};

struct RadiativeArgs {
    const z4c_block *blocks;
    const double *origins;        // 3 per block: coordinates of interior point (0, 0, 0)
    const OuterRegion *regions;
    const long long *start;       // nregions + 1 prefix sums of points
    int nregions;
    long long total;
    const double *u;              // input state
    double *rhs;                  // right-hand side mode: d_t u at the outer points
    double *out;                  // stage mode (rhs == nullptr): u0_out
    double *u1;
    const double *u2;
    double delta, eps_dt, g1, g2, g3, beta_dt;
    int read_u1, write_u1, use_u2;
    double chi_floor, alpha_floor;
    // non-null: stencil samples at ghost points that have a neighbour are
    // read from the neighbour (the neighbour rule of the stage's halo
    // reads); null: every sample is the stored value
    const int *nbr;
};

// Stencil scale factors of one block, in order d1[3], d2[3], mix[3] (xy, xz,
// yz), ko[3]:  d1 = 1/(c1 h), d2 = 1/(c2 h^2), mix = d1_a d1_b,
// ko = (-1)^(r+1) sigma / (2^(2r) h), with (c1, c2) = (12, 12) for order 4 and
// (60, 180) for order 6, r = order/2 + 1.
void block_factors(const z4c_block &b, int fd_order, double sigma, double out[12]);

// Launch entry points implemented in z4c_kernels.hip (tile kernels: one
// variant per order, arithmetic, tile shape and occupancy target `waves`
// = waves per SIMD the kernel is compiled for).
hipError_t launch_stage(int mode, int fd_order, int arith, int tx, int ty, int tz, int waves,
                        const StageArgs &a, hipStream_t s);
bool stage_shape_supported(int fd_order, int tx, int ty, int tz, int waves);
hipError_t launch_p6_f64(int mode, int tx, int ty, int tz, int w, const StageArgs &a,
                         hipStream_t s);
hipError_t launch_p6_f32(int mode, int tx, int ty, int tz, int w, const StageArgs &a,
                         hipStream_t s);
hipError_t launch_p4(int mode, int arith, int tx, int ty, int tz, int w, const StageArgs &a,
                     hipStream_t s);
// Right-hand side / stage with lopsided advection (FP64, z4c_variants_lop.hip).
hipError_t launch_lopsided(int mode, int fd_order, int tx, int ty, int tz, int w,
                           const StageArgs &a, hipStream_t s);
// Naive-FP32 right-hand side (z4c_variants_naive.hip).
hipError_t launch_naive(int fd_order, int tx, int ty, int tz, int w, const StageArgs &a,
                        hipStream_t s);
// Stage with the constraint monitor (FP64, z4c_variants_mon.hip).
hipError_t launch_monitor(int fd_order, int tx, int ty, int tz, int w, const StageArgs &a,
                          hipStream_t s);
hipError_t launch_ghost(const GhostArgs &g, long long total_ghost, hipStream_t s);
// Radiative outer boundary (z4c_boundary.hip).
hipError_t launch_radiative(const RadiativeArgs &a, hipStream_t s);
hipError_t launch_norm_reduce(const z4c_block *blocks, int nblocks, const long long *tile_start,
                              const int *tile_count, const double *partial, double *norms,
                              hipStream_t s);
hipError_t launch_finite_count(const z4c_block *blocks, int nblocks, const long long *pt_start,
                               long long total_pts, const double *u,
                               unsigned long long *count, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s);
// Zero the 8 tile counters of a persistent launch (a kernel, so that captured
// graphs replay it).
hipError_t launch_zero_queue(int *q, hipStream_t s);

// Read access to a plan from other translation units: its host block table,
// its device copy (nullptr without a device).
const std::vector<z4c_block> &plan_blocks(const z4c_plan *P);
const z4c_block *plan_blocks_device(const z4c_plan *P);
// The plan a transfer plan was created on.
const z4c_plan *xplan_plan(const z4c_xplan *X);

// Last-error message of the calling thread (z4c_last_error), for the host
// code of every translation unit; both return their status argument.
z4c_status set_error(z4c_status s, const char *msg);
z4c_status set_hip_error(hipError_t e, const char *what);

}  // namespace z4c
