/*
 * z4c_matter.h -- matter coupling of the Z4c right-hand side (libz4c.so).
 *
 * The Z4c variables live on a vertex-centred (VC) grid and the fluid on a
 * cell-centred (CC) grid; the two are coupled by Lagrange interpolation whose
 * order may differ between variables (Sec. 3.2 of the paper, intergrid
 * communication): the metric goes VC -> CC for the fluid, the ADM
 * projections of the stress-energy tensor go CC -> VC as the matter input of
 * the Z4c right-hand side (z4c.h: rho, S_i, S_ij).  The projections are those
 * of the perfect fluid (Sec. 2.1, equations for rho_ADM, S_i ADM, S_ij ADM)
 * and, with a magnetic field, of ideal GRMHD with the comoving field b^mu
 * (Sec. 2.2, the GRMHD ADM sources and the relations b^0, b^i, b^2).
 *
 * Grid of one MeshBlock: nc cells per direction and nc + 1 vertices; vertex
 * i sits at x0 + i dx (i = 0 .. nc), the centre of cell i at x0 + (i + 1/2) dx
 * (i = 0 .. nc - 1).  A VC array stores vertices [-ngv, nc + 1 + ngv) per
 * direction, a CC array cells [-ngc, nc + ngc); x fastest, then y, then z, one
 * field after the other (structure of arrays), element index
 *   VC: off + f*vc_stride + (i+ngv) + (ncx+1+2ngv)*((j+ngv) + (ncy+1+2ngv)*(k+ngv))
 *   CC: off + f*cc_stride + (i+ngc) + (ncx+2ngc)*((j+ngc) + (ncy+2ngc)*(k+ngc)).
 * With a Z4c plan (z4c.h) over the same blocks: nx = ncx + 1, ng = ngv,
 * offset = vs_offset, moffset = vm_offset, field_stride = vc_stride.
 *
 * Arrays (all double, device memory, owned by the caller):
 *   VC state   the 22-field Z4c state; fields 0..6 (chi, gt_ij) are read
 *   VC matter  10 fields rho, S_x, S_y, S_z, S_xx, S_xy, S_xz, S_yy, S_yz, S_zz
 *   CC geom    7 fields chi, gt_xx, gt_xy, gt_xz, gt_yy, gt_yz, gt_zz
 *   CC prim    8 fields rho, ut^x, ut^y, ut^z, p, B^x, B^y, B^z: rest-mass
 *              density, the projected 4-velocity ut^i = W v^i, pressure and
 *              the Eulerian magnetic field (the sqrt(4 pi) absorbed, Sec. 2.2);
 *              the B fields are not read for pure hydrodynamics
 *   CC adm     10 fields, the layout of VC matter
 *   CC cons    8 fields D, S_x, S_y, S_z, tau, B^x, B^y, B^z: the conservative
 *              variables of Sec. 2.2, densitised by sqrt(gamma) (B^k too)
 *   CC status  one int per stored cell (primitive recovery)
 *
 * Interpolation: along each direction the Lagrange polynomial through the
 * `order` nearest input points (order 2, 4 or 6) evaluated midway between the
 * two central ones; in 3-D the tensor product of the three.  A cell centre
 * uses vertices i - order/2 + 1 .. i + order/2, a vertex uses cells
 * i - order/2 .. i + order/2 - 1.
 *
 * Ownership, asynchrony and errors are those of z4c.h: an mplan owns only its
 * device tables (allocated in z4c_mplan_create); compute calls allocate
 * nothing, validate on the host, then enqueue on the given HIP stream.
 */
#ifndef Z4C_MATTER_H
#define Z4C_MATTER_H

#include "z4c.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One MeshBlock of the matter coupling (96 bytes). */
typedef struct {
    long long vs_offset;   /* VC state array: element offset of field 0, vertex (-ngv,-ngv,-ngv) */
    long long vm_offset;   /* VC matter array: the same                                      */
    long long vc_stride;   /* elements between consecutive fields of either VC array          */
    long long cg_offset;   /* CC geometry array: element offset of field 0, cell (-ngc,...)   */
    long long cp_offset;   /* CC primitive array                                              */
    long long ca_offset;   /* CC ADM-source array                                             */
    long long cq_offset;   /* CC conservative array                                           */
    long long cf_offset;   /* CC status array (one int per stored cell, no fields)            */
    long long cc_stride;   /* elements between consecutive fields of any CC array             */
    int ncx, ncy, ncz;     /* cells per direction, >= 1                                       */
    int ngv, ngc;          /* ghost layers stored in the VC / CC arrays, >= 0                 */
    int pad;
} z4c_mblock;

/* Fluid description.
 *   mhd        0: perfect fluid (Sec. 2.1), 1: ideal GRMHD (Sec. 2.2)
 *   gamma_ad   ideal-gas adiabatic index Gamma > 1: p = (Gamma - 1) rho eps,
 *              so rho h = rho + Gamma/(Gamma - 1) p
 *   chi_floor  gamma_ij = gt_ij / max(chi, chi_floor), as in the Z4c kernels */
typedef struct {
    int mhd;
    double gamma_ad;
    double chi_floor;
} z4c_fluid;

typedef struct z4c_mplan z4c_mplan;

/* Create a matter-coupling plan for `nblocks` blocks (HOST array, copied);
 * validates sizes (ncx, ncy, ncz >= 1, ngv, ngc >= 0, offsets and strides
 * >= 0) and uploads the tables to the current HIP device (no device with
 * Z4C_PLAN_NO_DEVICE).  Z4C_EINVAL on a bad block, Z4C_ENOMEM / Z4C_EHIP on
 * a failed upload. */
z4c_status z4c_mplan_create(const z4c_mblock *blocks, int nblocks, int flags, z4c_mplan **out);
z4c_status z4c_mplan_destroy(z4c_mplan *plan);

/* Metric to the fluid grid (Sec. 3.2): chi and gt_ij (state fields 0..6)
 * interpolated from the VC state `u` to cells [-ext, nc + ext) of `geom`
 * (CC geometry).  order in {2, 4, 6}; 0 <= ext <= ngc and
 * ngv >= order/2 - 1 + ext for every block (else Z4C_ENOGHOST).
 * `u` and `geom` must not alias. */
z4c_status z4c_metric_to_cc(const z4c_mplan *plan, int order, int ext, const double *u,
                            double *geom, void *hip_stream);

/* ADM projections of the stress-energy tensor (Sec. 2.1 / 2.2) at cells
 * [-ext, nc + ext): from `geom` (CC geometry) and `prim` (CC primitives) to
 * `adm` (CC, 10 fields).  With W = sqrt(1 + gamma_ij ut^i ut^j),
 * v_i = gamma_ij ut^j / W, alpha b^0 = W B^i v_i,
 * b_i = gamma_ij B^j / W + alpha b^0 v_i,
 * b^2 = ((alpha b^0)^2 + gamma_ij B^i B^j) / W^2 (all zero for mhd = 0):
 *   rho_ADM = (rho h + b^2) W^2 - (p + b^2/2) - (alpha b^0)^2
 *   S_i     = (rho h + b^2) W^2 v_i - alpha b^0 b_i
 *   S_ij    = (rho h + b^2) W^2 v_i v_j + (p + b^2/2) gamma_ij - b_i b_j.
 * The lapse cancels from every term, so it is not an input.
 * 0 <= ext <= ngc; `adm` must alias neither input. */
z4c_status z4c_adm_sources(const z4c_mplan *plan, const z4c_fluid *fluid, int ext,
                           const double *geom, const double *prim, double *adm,
                           void *hip_stream);

/* Sources to the Z4c grid (Sec. 3.2): the 10 fields of `adm` (CC)
 * interpolated to vertices [0, nc] of `matter` (VC matter, the matter input
 * of z4c_rhs / z4c_rk_stage).  order in {2, 4, 6}; ngc >= order/2 for every
 * block (else Z4C_ENOGHOST).  Ghost vertices of `matter` are not written. */
z4c_status z4c_sources_to_vc(const z4c_mplan *plan, int order, const double *adm, double *matter,
                             void *hip_stream);

/* Primitive recovery (Sec. 3.5, conservative-to-primitive inversion, and
 * Appendix A).  Ideal gas p = (Gamma - 1) rho eps.  Per cell, with
 * gamma_ij = gt_ij / max(chi, chi_floor) from the CC geometry:
 *   - the conservatives are undensitised; if D / sqrt(gamma) < f_thr rho_atm
 *     the cell becomes atmosphere (status 1);
 *   - otherwise the inversion is the root in mu = 1 / (h W) of the master
 *     function of Kastaun, Kalinani & Ciolfi (the algorithm the paper's
 *     primitive solver is based on): bracketed in [0, mu+] (mu+ from their
 *     auxiliary function), Illinois iterations to a relative width `tol` or
 *     `max_iter` iterations; no sign change or no convergence: atmosphere
 *     (status 3);
 *   - a solution with |ut| = sqrt(W^2 - 1) above ut_max (the velocity
 *     ceiling), or with rho < f_thr rho_atm, becomes atmosphere (status 2 /
 *     status 1);
 *   - atmosphere: rho = rho_atm, ut^i = 0, p = p_atm, B unchanged, and the
 *     conservatives of that state written back (Sec. 3.5: atmosphere
 *     treatment).  Status 0: recovered.
 * `prim` receives rho, ut^i, p and (mhd) the undensitised B^i. */
typedef struct {
    int mhd;               /* 0: no magnetic field (B fields neither read nor written) */
    double gamma_ad;       /* > 1                                                      */
    double chi_floor;      /* > 0                                                      */
    double rho_atm, p_atm; /* atmosphere density (> 0) and pressure (>= 0)             */
    double f_thr;          /* atmosphere threshold factor (>= 0; the paper uses 1)     */
    double ut_max;         /* velocity ceiling on |ut| (> 0; the paper uses 20)        */
    double tol;            /* relative width of the final bracket of mu (> 0)          */
    int max_iter;          /* >= 1                                                     */
} z4c_c2p_params;

/* Conservatives of the primitives (Sec. 2.2) at cells [-ext, nc + ext):
 * from `geom` and `prim` (rho, ut^i, p, B^i) to `cons` (densitised).
 * Uses mhd, gamma_ad, chi_floor of `c`. */
z4c_status z4c_p2c(const z4c_mplan *plan, const z4c_c2p_params *c, int ext, const double *geom,
                   const double *prim, double *cons, void *hip_stream);

/* Primitive recovery at cells [-ext, nc + ext): `cons` (read; rewritten at
 * atmosphere cells) to `prim`; `status` (may be NULL) receives the status
 * of every cell in the range. */
z4c_status z4c_c2p(const z4c_mplan *plan, const z4c_c2p_params *c, int ext, const double *geom,
                   double *cons, double *prim, int *status, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* Z4C_MATTER_H */
