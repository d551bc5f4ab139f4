/*
 * z4c.h -- C ABI of the MI355X (gfx950) Z4c hot-path library (libz4c.so).
 *
 * The library evaluates, for a batch of MeshBlocks (a level set of a
 * block-based oct-tree mesh, Sec. 3.1 of the paper), the right-hand side of
 * the Z4c formulation of the Einstein equations with matter sources (Sec. 2:
 * the spacetime is evolved in Z4c with the perfect-fluid ADM projections
 * rho, S_i, S_ij as sources), discretised with centred finite differences of
 * order 4 or 6 and Kreiss-Oliger dissipation (opening paragraph of Sec. 4: 6th-order FD,
 * kappa1 = 0.02, kappa2 = 0, sigma_KO = 0.5), and advances it by one stage of
 * a low-storage Runge-Kutta method (same paragraph: RK3; RK4 also supported).
 *
 * Conventions
 *   - G = c = 1.  Every floating-point array is double (FP64) in device
 *     memory, structure of arrays, x fastest.
 *   - State: 22 fields in this order: chi, gt_xx, gt_xy, gt_xz, gt_yy,
 *     gt_yz, gt_zz, Khat, At_xx, At_xy, At_xz, At_yy, At_yz, At_zz, Theta,
 *     Gt^x, Gt^y, Gt^z, alpha, beta^x, beta^y, beta^z.
 *   - Matter: 10 fields rho, S_x, S_y, S_z, S_xx, S_xy, S_xz, S_yy, S_yz,
 *     S_zz (ADM projections, covariant).  A NULL matter pointer means vacuum.
 *   - Constraints (output): 8 fields H, M_x, M_y, M_z, Theta, Z^x, Z^y, Z^z.
 *   - Block b stores (nz+2ng)(ny+2ng)(nx+2ng) points per field; point
 *     (i, j, k), i in [-ng, nx+ng), has element index
 *       offset + f*field_stride + (i+ng) + (nx+2ng)*((j+ng) + (ny+2ng)*(k+ng))
 *     for state field f (moffset / coffset for matter / constraints).
 *   - Interior points are i in [0, nx) etc.; only interior points of an
 *     output array are written by the stage, RHS and constraint calls.
 *
 * Ownership and asynchrony
 *   - The caller owns every field array.  A plan owns only its device copy
 *     of the block table, its tile lists, scratch for norm partial sums and
 *     its captured graphs (and the radiative boundary's outer-point list);
 *     all of it is allocated in z4c_plan_create /
 *     z4c_plan_set_* / on the first z4c_step_graph call, never by
 *     z4c_rhs, z4c_rk_stage, z4c_constraints, z4c_ghost_fill or z4c_step.
 *   - Every compute call is asynchronous on the given HIP stream
 *     (hipStream_t passed as void*, NULL = default stream).
 *   - A plan must not be used from two host threads at once.
 *
 * Errors: every call returns a z4c_status; arguments are validated on the
 * host before anything is enqueued, so every error path is testable without
 * a GPU (z4c_plan_create with Z4C_PLAN_NO_DEVICE).  z4c_last_error() gives
 * a message for the last failure of the calling thread.
 */
#ifndef Z4C_H
#define Z4C_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    Z4C_OK = 0,
    Z4C_EINVAL = -1,    /* NULL pointer, bad size, bad parameter, aliasing     */
    Z4C_ENOGHOST = -2,  /* ng < fd_order/2 + 1 for some block                  */
    Z4C_EALIGN = -3,    /* array pointer not 8-byte aligned                    */
    Z4C_EHIP = -4,      /* a HIP runtime call or kernel launch failed          */
    Z4C_ENOTSUP = -5,   /* valid request the library does not implement      */
    Z4C_ENOMEM = -6,    /* device allocation for plan tables failed            */
    Z4C_ENODEV = -7     /* plan created without a device cannot launch         */
} z4c_status;

typedef enum { Z4C_LAPSE_1PLUSLOG = 0, Z4C_LAPSE_HARMONIC = 1, Z4C_LAPSE_FROZEN = 2 } z4c_lapse;
typedef enum { Z4C_SHIFT_GAMMADRIVER = 0, Z4C_SHIFT_FROZEN = 1 } z4c_shift;
typedef enum { Z4C_ARITH_FP64 = 0, Z4C_ARITH_FP32 = 1, Z4C_ARITH_FP32_NAIVE = 2 } z4c_arith;
typedef enum { Z4C_ADVECT_CENTRED = 0, Z4C_ADVECT_LOPSIDED = 1 } z4c_advection;
typedef enum {
    Z4C_GHOST_NONE = 0,       /* leave ghost values as they are               */
    Z4C_GHOST_PERIODIC = 1,   /* each block periodic on itself                */
    Z4C_GHOST_NEIGHBOUR = 2,  /* same-level neighbour copy, table of 27/block */
    Z4C_GHOST_FROZEN = 3      /* every ghost from the `frozen` array          */
} z4c_ghost;

/* Scheme parameters.
 *   fd_order     4 or 6 (centred first/second derivatives; Sec. 4 uses 6)
 *   ko_sigma     Kreiss-Oliger strength sigma (Sec. 4: 0.5); operator of
 *                order 2r = fd_order + 2, Q = (-1)^(r+1) sigma/(2^(2r) h) D^(2r)
 *   kappa1/2     Z4c constraint damping (Sec. 4: 0.02 / 0)
 *   eta          Gamma-driver damping
 *   lapse        1+log (d_t alpha = -2 alpha Khat + advection), harmonic
 *                (-alpha^2 Khat) or frozen (no lapse source term)
 *   shift        Gamma-driver (d_t beta^i = Gt^i - eta beta^i + advection)
 *                or frozen (no Gt^i source)
 *   advect_gauge 1: beta^k d_k advection terms on alpha and beta
 *   chi_floor    chi is replaced by max(chi, chi_floor) in every 1/chi and
 *                clamped to it after each stage
 *   alpha_floor  alpha clamped to it after each stage
 *   arith        FP64: all arithmetic in double.  FP32: stencil differences
 *                u_m - u_0 are formed in double, then the derivatives,
 *                dissipation and the pointwise algebra run in float; storage,
 *                the Runge-Kutta combination and the floors stay double.
 *                FP32_NAIVE: float arithmetic with every sample rounded to
 *                float before the stencil differences (the form that loses
 *                perturbations below float resolution); right-hand side
 *                only, order 6, centred advection, for precision
 *                comparisons (Z4C_ENOTSUP for stages, steps, autotuning and
 *                other orders).
 *   advection    stencil of the advection terms beta^k d_k u (every field):
 *                CENTRED (the fd_order first derivative) or LOPSIDED, the
 *                fd_order-accurate first derivative on the points shifted by
 *                one towards the sign of beta^k (offsets -p/2+1 .. p/2+1
 *                for beta^k > 0, mirrored otherwise; the paper gives no
 *                advection stencil, this is the usual upwind-biased choice
 *                of moving-puncture codes).  LOPSIDED needs FP64 arithmetic
 *                (Z4C_ENOTSUP otherwise).  The field sits in the padding
 *                after `arith`: the struct stays 80 bytes and a zeroed
 *                struct means CENTRED. */
typedef struct {
    int fd_order;
    double ko_sigma, kappa1, kappa2, eta;
    int lapse, shift, advect_gauge;
    double chi_floor, alpha_floor;
    int arith;
    int advection;
} z4c_params;

/* One MeshBlock (72 bytes). dx, dy, dz > 0; nx, ny, nz >= 1. */
typedef struct {
    long long offset;        /* element offset of state field 0, point (-ng,-ng,-ng)   */
    long long moffset;       /* same for matter field 0 (ignored when matter is NULL)  */
    long long coffset;       /* same for constraint field 0                            */
    long long field_stride;  /* elements between consecutive fields of this block      */
    int nx, ny, nz, ng;
    double dx, dy, dz;
} z4c_block;

/* One Runge-Kutta stage in three-register form (u0 = stage state, u1 =
 * accumulator, u2 = state at the start of the step), k = RHS(u0):
 *   u1'  = (read_u1 ? u1 : 0) + delta*u0 + eps*dt*k      (stored if write_u1)
 *   u0'  = g1*u0 + g2*u1' + g3*u2 + beta*dt*k
 * then on u0': gt <- gt * det(gt)^(-1/3), At <- At - gt tr(At)/3,
 * chi <- max(chi, chi_floor), alpha <- max(alpha, alpha_floor). */
typedef struct {
    double delta, eps, g1, g2, g3, beta;
    int read_u1, write_u1;
} z4c_rk_coeffs;

typedef struct z4c_plan z4c_plan;

/* Flags for z4c_plan_create. */
#define Z4C_PLAN_NO_DEVICE 1   /* validate and build host tables only; no HIP call */

/* Create a plan for `nblocks` blocks described by the HOST array `blocks`
 * (copied).  Validates every block (sizes, spacings, ghosts >= fd_order/2+1,
 * offsets >= 0) and the parameters, builds tile lists and uploads them to the
 * current HIP device.  *out receives the plan (NULL on error).  A block of
 * 2^29 or more stored points ((nx+2ng)(ny+2ng)(nz+2ng)) is Z4C_ENOTSUP: the
 * kernels address a block's points as 32-bit byte offsets. */
z4c_status z4c_plan_create(const z4c_params *params, const z4c_block *blocks, int nblocks,
                           int flags, z4c_plan **out);
z4c_status z4c_plan_destroy(z4c_plan *plan);

/* Replace the scheme parameters (same validation as create). */
z4c_status z4c_plan_set_params(z4c_plan *plan, const z4c_params *params);

/* Same-level neighbour table (HOST, nblocks*27 ints, -1 = outer boundary),
 * entry [b*27 + (oz+1)*9 + (oy+1)*3 + (ox+1)] = block adjacent to b in
 * direction (ox, oy, oz).  Neighbours must have equal nx, ny, nz, ng and
 * field_stride.  Halo reads through the neighbour rule address a point of
 * another block by its 32-bit element offset from the state array base, so
 * they need offset + (nx+2ng)(ny+2ng)(nz+2ng) <= 2^32 for every block named
 * as another block's neighbour (34 GB of FP64 before its end); a table that
 * breaks this is accepted (ghost refreshes address in 64 bits) unless the
 * plan reads halos through the neighbour rule (Z4C_ENOTSUP, plan unchanged).
 * A block's own points, its periodic images and `frozen` have no such
 * limit. */
z4c_status z4c_plan_set_neighbours(z4c_plan *plan, const int *neighbours);

/* Launch shape for the blocks of one size class (nx, ny, nz) (0 = all).
 * tile_x/y/z: interior points per workgroup, one thread per point;
 * persistent: 0 = one workgroup per tile, otherwise that many workgroups
 * taking tiles from a work queue (per-XCD ranges of consecutive tiles, then
 * the other ranges' leftovers); waves: occupancy the kernel variant is
 * compiled for, in waves per SIMD (0 = 2; its register budget is 512/waves
 * per lane).  Supported: 8x8x8 and 8x8x4 with waves 2, and for order 6 also
 * 8x8x4 and 8x4x8 with waves 1. */
typedef struct {
    int tile_x, tile_y, tile_z;
    int persistent;
    int waves;
} z4c_launch;
z4c_status z4c_plan_set_launch(z4c_plan *plan, int nx, int ny, int nz, const z4c_launch *launch);
z4c_status z4c_plan_get_launch(const z4c_plan *plan, int nx, int ny, int nz, z4c_launch *launch);

/* How z4c_rhs, z4c_rk_stage and z4c_constraints obtain the ghost points of
 * their input: Z4C_GHOST_NONE (default) reads the stored ghost values;
 * PERIODIC, NEIGHBOUR (table from z4c_plan_set_neighbours; -1 entries read
 * `frozen`) and FROZEN read, for every ghost point, the value a
 * z4c_ghost_fill with that policy would store there — straight from the
 * source, so no refresh pass is needed and the stored ghosts are ignored.
 * NEIGHBOUR needs the offset limit stated at z4c_plan_set_neighbours
 * (Z4C_ENOTSUP otherwise).  `frozen` (device, state layout) must stay valid
 * while calls that use it are pending. */
z4c_status z4c_plan_set_halo(z4c_plan *plan, int policy, const double *frozen);

/* d_t u at every interior point (dissipation included) -> rhs (state layout).
 * u, rhs: device; rhs must not alias u. */
z4c_status z4c_rhs(z4c_plan *plan, const double *u, const double *matter, double *rhs,
                   void *stream);

/* Fused RHS + Runge-Kutta stage + algebraic enforcement, interior points.
 * u0_in and u0_out must differ (neighbouring tiles still read u0_in); u1
 * may be NULL only if !read_u1 && !write_u1 && g2 == 0; u2 may be NULL only
 * if g3 == 0; u2 may equal u0_in.  `c` is a host pointer. */
z4c_status z4c_rk_stage(z4c_plan *plan, const double *u0_in, double *u0_out, double *u1,
                        const double *u2, const double *matter, const z4c_rk_coeffs *c,
                        double dt, void *stream);

/* Constraints (Sec. 4.1 monitoring): H = R + 2/3 K^2 - At.At - 16 pi rho,
 * M_i (conformal form), Theta, Z^i = (Gt^i - Gt_d^i)/2 at interior points into
 * `cons` (constraint layout, may be NULL) and per-block norms into `norms`
 * (device, nblocks*16 doubles: for field q, [b*16+2q] = sum |c| dV and
 * [b*16+2q+1] = sum c^2 dV, dV = dx dy dz), summed in a fixed order.
 * Halo reads follow z4c_plan_set_halo. */
z4c_status z4c_constraints(z4c_plan *plan, const double *u, const double *matter,
                           double *cons, double *norms, void *stream);

/* z4c_constraints for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results (bitwise), with the per-tile partial sums in
 * a static device array of the library (8 MiB per device, held until the
 * process ends) instead of the plan's buffer; the call allocates nothing.
 * The plan itself (created beforehand) still owns its tables.  Plans of more
 * than 65,536 tiles (z4c_plan_tiles) are refused with Z4C_ENOTSUP.  Every
 * call on one device shares that array: calls that overlap on one device
 * (other streams, other threads) race and must be ordered by the caller. */
z4c_status z4c_constraints_noalloc(z4c_plan *plan, const double *u, const double *matter,
                                   double *cons, double *norms, void *stream);

/* z4c_rk_stage with the constraint monitor fused into the stage kernel (Sec.
 * 4.1 monitoring): the stage as z4c_rk_stage, and the constraints of its
 * input u0_in (the quantities and layouts of z4c_constraints) formed from
 * the derivatives the stage takes anyway, so that monitoring adds no pass
 * over the state.  `cons` (device, constraint layout) may be NULL; `norms`
 * (device, nblocks*16 doubles, as z4c_constraints) must not.  Neither may
 * alias a state or matter array.  FP64-arithmetic plans only (Z4C_ENOTSUP
 * otherwise), centred advection only (the monitor kernel has no lopsided
 * form: Z4C_ENOTSUP).  Values equal those of z4c_constraints up to
 * rounding. */
z4c_status z4c_rk_stage_monitor(z4c_plan *plan, const double *u0_in, double *u0_out, double *u1,
                                const double *u2, const double *matter, const z4c_rk_coeffs *c,
                                double dt, double *cons, double *norms, void *stream);

/* Refresh the ghost points of `u` (device): periodic, neighbour (table set
 * with z4c_plan_set_neighbours; -1 entries take `frozen`, or keep their
 * stored value when `frozen` is NULL), or frozen (`frozen` device array in
 * the state layout). */
z4c_status z4c_ghost_fill(z4c_plan *plan, int policy, double *u, const double *frozen,
                          void *stream);

/* One full Runge-Kutta step of nstages fused stages.  With a ghost policy
 * other than NONE every stage reads the ghost points of its input through
 * that policy (as z4c_plan_set_halo describes), so no refresh pass runs
 * between stages; the ghosts of the final state are then refreshed once
 * (unless Z4C_STEP_NO_FINAL_FILL).  Z4C_STEP_STORED_GHOSTS instead refreshes
 * the stored ghosts of every stage output with z4c_ghost_fill and lets the
 * stages read them; both give bitwise the same interior.  The step takes
 * that form by itself under the neighbour policy when the neighbour table
 * breaks the offset limit of z4c_plan_set_neighbours, and then first
 * refreshes the ghosts of regs[0] (which halo reads would not read), so
 * that the result is the same.  Buffers regs[0..3]:
 * regs[0] holds y_n on entry; regs[1], regs[2] are stage ping-pong buffers;
 * regs[3] is the accumulator.  Stage s reads regs[in_s] (in_0 = 0) and
 * writes regs[out_s]: the one of {1, 2} it does not read, except that the
 * last stage writes regs[0] when its g3 == 0 (it does not read y_n).  The
 * final state's index is returned in *result (0 for classic RK4, so the
 * step can be repeated with the same registers). */
#define Z4C_STEP_STORED_GHOSTS 1   /* refresh stored ghosts after every stage    */
#define Z4C_STEP_NO_FINAL_FILL 2   /* do not refresh the final state's ghosts     */
#define Z4C_STEP_MONITOR 4         /* stage 0 with the fused constraint monitor:
                                      the constraints of y_n (regs[0] on entry) into
                                      cons (may be NULL) and norms, as
                                      z4c_rk_stage_monitor; no extra pass */
#define Z4C_STEP_LEVEL_EXCHANGE 8  /* multi-level set: after every stage the stored
                                      ghosts of its output are refreshed by the
                                      same-level policy, then exchanged across the
                                      level jumps set with
                                      z4c_plan_set_level_exchange (implies stored
                                      ghosts) */
#define Z4C_STEP_SOMMERFELD 16     /* the outer ghost points advance by the radiative
                                      law beside every stage (z4c_sommerfeld_stage
                                      into the stage's output and accumulator), so
                                      every stage reads evolved outer ghosts; needs
                                      z4c_plan_set_sommerfeld, the neighbour policy
                                      and no frozen array (Z4C_EINVAL).  With
                                      Z4C_STEP_LEVEL_EXCHANGE the neighbour table
                                      is the same-level one: its -1 regions facing
                                      another level are advanced too and then
                                      overwritten by the exchange, so only points
                                      no block owns keep the radiative values */
typedef struct {
    double *regs[4];
    const double *matter;
    const z4c_rk_coeffs *table;   /* host, nstages entries */
    int nstages;
    double dt;
    int ghost_policy;
    const double *frozen;
    int flags;                    /* Z4C_STEP_* */
    double *cons;                 /* Z4C_STEP_MONITOR: constraint fields or NULL  */
    double *norms;                /* Z4C_STEP_MONITOR: nblocks*16 doubles         */
} z4c_step_desc;                  /* 104 bytes */
z4c_status z4c_step(z4c_plan *plan, const z4c_step_desc *desc, int *result, void *stream);

/* Same as z4c_step, but the whole step (stages + ghost fills) is captured
 * into a HIP graph on first use (per distinct descriptor, a few cached) and
 * replayed afterwards: one host call per step. */
z4c_status z4c_step_graph(z4c_plan *plan, const z4c_step_desc *desc, int *result,
                          void *stream);

/* Time each supported launch shape per size class on the caller's buffers
 * (u0 read, u0_out/u1 overwritten at interior points, one RK4-like stage)
 * and keep the fastest; `reps` timed launches per candidate.  Candidates:
 * every supported tile shape and occupancy, each as a grid launch and as
 * persistent launches of one and two workgroups per CU.  Then classes that
 * chose the same tile shape and occupancy are timed together, as they
 * launch (one dispatch when their launch forms agree), under their own
 * choices and under each common launch form, and the fastest is kept.
 * With a tuning cache set (z4c_set_tune_cache), size classes found there
 * under the same key (device architecture, order, arithmetic, advection,
 * halo rule, block interior size, ghosts) take the stored launch without
 * timing (and without the joint pass when every class is found), and newly
 * timed ones are added to it.  Results are readable with
 * z4c_plan_get_launch.  Synchronises the stream. */
z4c_status z4c_plan_autotune(z4c_plan *plan, const double *u0, double *u0_out, double *u1,
                             const double *matter, int reps, void *stream);

/* Path of the autotuning cache file used by z4c_plan_autotune (process-wide;
 * NULL or "" = no cache).  One text line per entry; written atomically
 * (temporary file + rename) after a tuning run that timed new classes. */
z4c_status z4c_set_tune_cache(const char *path);

/* Scan the interior of u for non-finite values; *flag = count found (host
 * int, the call synchronises the stream). */
z4c_status z4c_check_finite(z4c_plan *plan, const double *u, long long *count, void *stream);

/* Transfers between refinement levels of a vertex-centred mesh with
 * refinement ratio 2 (Sec. 3.2: the Z4c variables are vertex-centred so that
 * restriction and prolongation between levels stay simple with high-order
 * operators).  Fine vertex i of the fine block lies at coarse position
 * c0 + i/2 of the coarse block (per direction; fine vertex 0 on coarse
 * vertex c0), and the fine spacing is half the coarse one.
 *   prolongation (destination: fine points in [lo, hi), ghosts allowed): an
 *     even index copies the coincident coarse vertex, an odd one takes the
 *     Lagrange polynomial through the `order` nearest coarse vertices at the
 *     midpoint; in 3-D the tensor product of the three directions;
 *   restriction (destination: coarse points in [lo, hi)): injection, coarse
 *     vertex j takes fine vertex 2 (j - c0).
 * All 22 state fields; each call works in place on one state array. */
typedef struct {
    int coarse, fine;   /* block indices of the plan (different blocks)         */
    int c0[3];          /* coarse vertex under fine vertex 0                    */
    int lo[3], hi[3];   /* destination box, half-open, destination block indices */
} z4c_transfer;

typedef struct z4c_xplan z4c_xplan;

/* A set of transfers on the blocks of `plan` (HOST arrays, copied):
 * `nprolong` prolongations and `nrestrict` restrictions, interpolation order
 * 2, 4 or 6.  Validation: block indices, a spacing ratio of 2 (to 1e-12),
 * destination boxes inside the destination's stored points, every source
 * point of every destination point inside the source's stored points (else
 * Z4C_ENOGHOST), and no block written by one transfer and read by another
 * of the same kind (the calls run all transfers of a kind at once).  The
 * xplan keeps a pointer to `plan`, which must outlive it. */
z4c_status z4c_xplan_create(const z4c_plan *plan, const z4c_transfer *prolong, int nprolong,
                            const z4c_transfer *restrict_, int nrestrict, int order, int flags,
                            z4c_xplan **out);
z4c_status z4c_xplan_destroy(z4c_xplan *xplan);

/* Where a block sits in an AMR level set: its refinement level and the
 * position of its interior vertex 0 on the integer lattice of the finest
 * level present (lattice spacing = the spacing of level Lmax; a block of
 * level L has its vertices 2^(Lmax - L) lattice units apart).  A block
 * owns the lattice points of its span [o, o + n step) per direction: its
 * interior vertices and, on a coarse level, the points between its last
 * vertex and the next block; the spans of a level set tile it. */
typedef struct {
    int level;
    int o[3];
} z4c_loc;

/* The transfers of a ghost exchange across the level jump between level
 * `coarse_level` and coarse_level + 1 (Sec. 3.2, vertex-centred refinement
 * by 2), from the blocks of `plan` and their places `locs` (HOST, nblocks
 * entries):
 *   prolongation: every ghost point of a fine block in the span of a coarse
 *     block, one transfer per (fine block, ghost region of the 26, coarse
 *     block) with a non-empty intersection;
 *   restriction: every ghost point of a coarse block in the span of a fine
 *     block (an interior vertex of it), likewise per (coarse block, ghost
 *     region, fine block).
 * Ghost points owned by blocks of the same level are the neighbour ghost
 * fill's; points no block owns are left alone.  Use: restrict, refresh the
 * coarse level's same-level ghosts, prolongate (coarse level pairs first).
 * The arrays are filled up to max_prolong / max_restrict entries; *nprolong
 * and *nrestrict receive the counts needed (call with max = 0 to size
 * them; Z4C_EINVAL when an array is too small).  Errors: a fine block whose
 * vertex 0 is not a coarse lattice vertex, levels outside 0..30, or block
 * spacings that do not halve per level (Z4C_EINVAL). */
z4c_status z4c_level_transfers(const z4c_plan *plan, const z4c_loc *locs, int coarse_level,
                               z4c_transfer *prolong, int max_prolong, int *nprolong,
                               z4c_transfer *restrict_, int max_restrict, int *nrestrict);

/* Apply every prolongation (or every restriction) of `xplan` to the state
 * array `u` (device, the plan's layout), asynchronously on the stream. */
z4c_status z4c_prolongate(const z4c_xplan *xplan, double *u, void *hip_stream);
z4c_status z4c_restrict(const z4c_xplan *xplan, double *u, void *hip_stream);

/* Transfer plans of the level jumps of a multi-level set (Sec. 3.1: all
 * levels advance with one global time step, no subcycling; Sec. 3.2:
 * vertex-centred restriction and prolongation), one per pair of adjacent
 * levels (from z4c_level_transfers), coarsest pair first; n = 0 removes
 * them.  Each must have been created on this plan and outlive its use.
 * With Z4C_STEP_LEVEL_EXCHANGE a step refreshes, after every stage, the
 * stored ghosts of the stage output: the step's ghost policy (same-level
 * copies, frozen outer faces), then every restriction (coarse ghosts inside
 * finer blocks, injected from their vertices) finest pair first, then every
 * prolongation (fine ghosts inside coarser blocks, interpolated from coarse
 * points whose ghosts are then current) coarsest pair first. */
z4c_status z4c_plan_set_level_exchange(z4c_plan *plan, const z4c_xplan *const *xplans, int n);


/* Radiative (Sommerfeld) outer boundary.  The paper states no outer
 * boundary condition for Z4c (its static-star test moves the outer boundary
 * further out instead); this is the usual radiative law of moving-puncture
 * codes, a reading.  Outer points: the ghost points of a block in every
 * direction whose entry of the neighbour table is -1.  At an outer point
 * with coordinates x and r = |x| each of the 22 fields u evolves by
 *   d_t u = -(x^a / r) D_a u - (u - u_inf) / r,
 * u_inf its flat-space value (1 for chi, gt_xx, gt_yy, gt_zz and alpha, 0
 * otherwise), D_a the second-order difference along a: centred where the
 * point's index along a lies in [0, n_a), one-sided towards the interior
 * (three points) otherwise; no dissipation, FP64 whatever the plan's
 * arithmetic.  Stencil samples at ghost points that have a neighbour are
 * read from the neighbour when the plan reads halos through the neighbour
 * rule (z4c_plan_set_halo), as stored otherwise (a step reads them the way
 * its stages do).
 * z4c_plan_set_sommerfeld: `origins` (HOST, nblocks*3 doubles, copied) are
 * the coordinates of each block's interior point (0, 0, 0); point (i, j, k)
 * sits at origin + (i dx, j dy, k dz).  Needs z4c_plan_set_neighbours
 * first (a later table rebuilds the outer point list); Z4C_EINVAL when an
 * outer point may lie within half a grid spacing of x = 0 (in a multi-level
 * set this covers every ghost region without a same-level neighbour,
 * including those another level owns).  NULL removes the boundary.  The
 * plan keeps the point list in device memory. */
z4c_status z4c_plan_set_sommerfeld(z4c_plan *plan, const double *origins);

/* d_t u by the radiative law at every outer point of `rhs` (device, state
 * layout; nothing else is written); rhs must not alias u. */
z4c_status z4c_sommerfeld_rhs(z4c_plan *plan, const double *u, double *rhs, void *stream);

/* One Runge-Kutta stage of the outer points: the combination of
 * z4c_rk_stage with k the radiative right-hand side, then the same
 * enforcement; arguments and aliasing rules as z4c_rk_stage (no matter).
 * Writes only outer points of u0_out and u1, and reads only u0_in, u1, u2,
 * so it runs before or after the z4c_rk_stage of the same stage. */
z4c_status z4c_sommerfeld_stage(z4c_plan *plan, const double *u0_in, double *u0_out, double *u1,
                                const double *u2, const z4c_rk_coeffs *c, double dt,
                                void *stream);

const char *z4c_strerror(z4c_status status);
const char *z4c_last_error(void);

/* Number of tiles the plan launches per stage (all size classes). */
long long z4c_plan_tiles(const z4c_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* Z4C_H */
