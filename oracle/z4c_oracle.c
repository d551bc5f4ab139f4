/*
 * z4c_oracle.c -- plain, slow, FP64 CPU oracle for the Z4c hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU path and is never called by it.
 *
 * What it computes (one MeshBlock at a time, every interior point):
 *   - the Z4c right-hand side of the 22 evolved fields (the paper evolves
 *     the Einstein equations in the Z4c formulation with constraint damping
 *     kappa1, kappa2 and the moving-puncture gauge, Sec. 2 and the opening
 *     paragraph of Sec. 4; the
 *     equations themselves are those of the standard Z4c system the paper
 *     cites, written out below term by term),
 *   - centred finite differences of order 4 or 6 (Sec. 4: 6th order),
 *     mixed second derivatives as a first derivative of a first derivative,
 *   - Kreiss-Oliger dissipation of order 2r = p + 2 on every field
 *     (Sec. 4: sigma_KO = 0.5),
 *   - ADM matter source terms rho, S_i, S_ij (Sec. 2.1, the perfect-fluid
 *     projections), taken here as given input arrays,
 *   - one low-storage Runge-Kutta stage (Sec. 4: RK3; RK4 also used) with
 *     algebraic enforcement det(gt) = 1, tr(At) = 0 and chi/alpha floors,
 *   - the constraints H, M_i, Theta, Z^i and their L1/L2 norms
 *     (Sec. 4.1, constraint monitoring of the static star),
 *   - ghost refresh by periodic wrap, same-level neighbour copy or frozen
 *     values.
 *
 * Every stencil is applied in centre-subtracted form: differences u_m - u_0
 * (or u_m - u_-m) are formed first, then weighted with integer weights, then
 * divided once by the grid-spacing factor.  Constant data therefore gives
 * exactly zero derivatives.
 *
 * Compiled with -ffp-contract=off: no fused multiply-add, every product and
 * sum rounds as written.  The working type `real` is double; the same source
 * built with -DORACLE_EXTENDED works in x87 extended precision (64-bit
 * significand) and serves only to measure the FP64 oracle's own rounding
 * error.  Built with -DORACLE_FP32 the working type is float while every
 * stencil difference is still formed in double (the FP32-arithmetic form of
 * the right-hand side); adding -DORACLE_NAIVE rounds the samples to float
 * before the differences.  These two builds measure what FP32 arithmetic
 * itself costs in accuracy; only their right-hand side is used.  Arrays
 * crossing the interface are always double.
 */
#include <tgmath.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#if defined(ORACLE_EXTENDED)
typedef long double real;
#elif defined(ORACLE_FP32)
typedef float real;
#else
typedef double real;
#endif

/* Field indices, state (22). */
enum { CHI = 0, GXX, GXY, GXZ, GYY, GYZ, GZZ, KHAT, AXX, AXY, AXZ, AYY, AYZ, AZZ,
       THETA, GAMX, GAMY, GAMZ, ALPHA, BETAX, BETAY, BETAZ, NFIELD };
/* Matter (10). */
enum { M_RHO = 0, M_SX, M_SY, M_SZ, M_SXX, M_SXY, M_SXZ, M_SYY, M_SYZ, M_SZZ, NMATTER };
/* Constraint outputs (8). */
enum { C_H = 0, C_MX, C_MY, C_MZ, C_THETA, C_ZX, C_ZY, C_ZZ, NCONS };

typedef struct {
    long long offset, moffset, coffset, field_stride;
    int nx, ny, nz, ng;
    double dx, dy, dz;
} orc_block;

typedef struct {
    int fd_order;
    double ko_sigma, kappa1, kappa2, eta;
    int lapse;          /* 0: 1+log, 1: harmonic, 2: frozen */
    int shift;          /* 0: Gamma-driver, 1: frozen        */
    int advect_gauge;   /* 1: beta^k d_k on alpha and beta   */
    double chi_floor, alpha_floor;
    int advection;      /* 0: centred, 1: lopsided advection stencils */
} orc_params;

typedef struct {
    double delta, eps, g1, g2, g3, beta;
    int read_u1, write_u1;
} orc_rk;

static const real PI = 3.141592653589793238462643383279502884L;

/* Index pairs of a symmetric 3x3 tensor stored as 6 components. */
static const int SYM_I[6] = {0, 0, 0, 1, 1, 2};
static const int SYM_J[6] = {0, 1, 2, 1, 2, 2};

/* ---------------------------------------------------------------------------
 * 1-D stencils on a strided pointer u (u[0] = centre, u[m*s] = m-th neighbour)
 * ------------------------------------------------------------------------ */

/* Input samples are double; every difference below is formed in `real`. */
#define U(off) ((real)u[(off)])
/* Difference of two samples.  In the FP32-arithmetic reference (ORACLE_FP32)
 * it is formed in double and rounded to float afterwards (the mixed form);
 * with ORACLE_NAIVE as well, from samples already rounded to float. */
#if defined(ORACLE_FP32) && !defined(ORACLE_NAIVE)
#define DIFF(a, b) ((real)(u[(a)] - u[(b)]))
#else
#define DIFF(a, b) (U(a) - U(b))
#endif

/* First derivative, centred, order p: antisymmetric pairs u_m - u_-m. */
static real d1(const double *u, long s, real h, int p)
{
    if (p == 4)
        return (8 * DIFF(s, -s) - DIFF(2 * s, -2 * s)) / (12 * h);
    return (45 * DIFF(s, -s) - 9 * DIFF(2 * s, -2 * s) + DIFF(3 * s, -3 * s)) / (60 * h);
}

/* Lopsided first derivative, order p (the advection stencil of moving-
 * puncture codes; the paper names no advection stencil): the first
 * derivative on the p + 1 points shifted by one towards the sign of beta,
 * offsets -p/2+1 .. p/2+1 for beta > 0 and the mirror image otherwise.  Its
 * weights are, by definition, the unique ones exact on every polynomial of
 * degree <= p: sum_j w_j j^m = [m == 1] (m = 0..p, j over the offsets),
 * solved once per order by Gaussian elimination with partial pivoting.
 * LOPW[q][j] holds the weights of order 4 (q = 0) and 6 (q = 1) for offset
 * -p/2+1 + j. */
static long double LOPW[2][7];

static void lop_solve(int p, long double *w)
{
    const int n = p + 1, lo = -p / 2 + 1;
    long double A[7][8];
    for (int m = 0; m < n; ++m) {
        for (int j = 0; j < n; ++j) {
            long double x = 1.0L;
            for (int e = 0; e < m; ++e)
                x *= (long double)(lo + j);
            A[m][j] = x;
        }
        A[m][n] = (m == 1) ? 1.0L : 0.0L;
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsl(A[r][c]) > fabsl(A[piv][c]))
                piv = r;
        for (int e = 0; e <= n; ++e) {
            const long double t = A[c][e];
            A[c][e] = A[piv][e];
            A[piv][e] = t;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c)
                continue;
            const long double f = A[r][c] / A[c][c];
            for (int e = c; e <= n; ++e)
                A[r][e] -= f * A[c][e];
        }
    }
    for (int j = 0; j < n; ++j)
        w[j] = A[j][n] / A[j][j];
}

static void lop_init(void)
{
    lop_solve(4, LOPW[0]);
    lop_solve(6, LOPW[1]);
}

/* Weights of order p for the offsets -p/2+1 .. p/2+1 (host array of p+1). */
int orc_lopsided_weights(int p, double *w)
{
    if (p != 4 && p != 6)
        return -1;
    long double v[7];
    lop_solve(p, v);
    for (int j = 0; j <= p; ++j)
        w[j] = (double)v[j];
    return 0;
}

static real d1lop(const double *u, long s, real h, int p, int pos)
{
    const long double *w = LOPW[p == 6];
    const int lo = -p / 2 + 1;
    real acc = 0.0;
    for (int j = 0; j <= p; ++j) {
        const long o = pos ? (long)(lo + j) : -(long)(lo + j);
        acc += (real)w[j] * DIFF(o * s, 0);   /* the weights sum to zero */
    }
    return (pos ? acc : -acc) / h;
}

/* Second derivative, centred, order p: weights sum to zero, so it is written
 * in differences from the centre value. */
static real d2(const double *u, long s, real h, int p)
{
    if (p == 4)
        return (16 * (DIFF(s, 0) + DIFF(-s, 0)) - (DIFF(2 * s, 0) + DIFF(-2 * s, 0))) / (12 * h * h);
    return (270 * (DIFF(s, 0) + DIFF(-s, 0)) - 27 * (DIFF(2 * s, 0) + DIFF(-2 * s, 0))
            + 2 * (DIFF(3 * s, 0) + DIFF(-3 * s, 0)))
           / (180 * h * h);
}

/* Mixed second derivative d_a d_b u = D1_a ( D1_b u ): the first-derivative
 * stencil along a applied to first derivatives along b. */
static real d1d1(const double *u, long sa, long sb, real ha, real hb, int p)
{
    real gp[4] = {0}, gm[4] = {0};
    const int q = p / 2;
    for (int m = 1; m <= q; ++m) {
        gp[m] = d1(u + m * sa, sb, hb, p);
        gm[m] = d1(u - m * sa, sb, hb, p);
    }
    if (p == 4)
        return (8 * (gp[1] - gm[1]) - (gp[2] - gm[2])) / (12 * ha);
    return (45 * (gp[1] - gm[1]) - 9 * (gp[2] - gm[2]) + (gp[3] - gm[3])) / (60 * ha);
}

static real binomial(int n, int k)
{
    real r = 1.0;
    for (int i = 1; i <= k; ++i)
        r = r * (real)(n - k + i) / (real)i;
    return r;
}

/* Kreiss-Oliger dissipation along one direction, r = p/2 + 1:
 *   Q u = (-1)^(r+1) sigma / (2^(2r) h) * Delta^(2r) u,
 * Delta^(2r) u_0 = sum_{m != 0} c_m (u_m - u_0),  c_m = (-1)^(m+r) C(2r, r+m).
 * On the highest grid mode (-1)^i it returns exactly -sigma/h * u. */
static real ko1(const double *u, long s, real h, int p, real sigma)
{
    const int r = p / 2 + 1;
    real acc = 0;
    for (int m = 1; m <= r; ++m) {
        const real cm = (((m + r) & 1) ? -1 : 1) * binomial(2 * r, r + m);
        acc += cm * (DIFF(m * s, 0) + DIFF(-m * s, 0));
    }
    const real sign = ((r + 1) & 1) ? -1.0 : 1.0;
    return sign * sigma / (ldexp(1.0, 2 * r) * h) * acc;
}

/* ---------------------------------------------------------------------------
 * Small tensor helpers (plain 3x3)
 * ------------------------------------------------------------------------ */
static real det3(const real g[3][3])
{
    return g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1])
         - g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0])
         + g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
}

/* Inverse through the adjugate divided by the actual determinant. */
static void inv3(const real g[3][3], real gi[3][3])
{
    const real d = det3(g);
    gi[0][0] = (g[1][1] * g[2][2] - g[1][2] * g[2][1]) / d;
    gi[0][1] = (g[0][2] * g[2][1] - g[0][1] * g[2][2]) / d;
    gi[0][2] = (g[0][1] * g[1][2] - g[0][2] * g[1][1]) / d;
    gi[1][0] = (g[1][2] * g[2][0] - g[1][0] * g[2][2]) / d;
    gi[1][1] = (g[0][0] * g[2][2] - g[0][2] * g[2][0]) / d;
    gi[1][2] = (g[0][2] * g[1][0] - g[0][0] * g[1][2]) / d;
    gi[2][0] = (g[1][0] * g[2][1] - g[1][1] * g[2][0]) / d;
    gi[2][1] = (g[0][1] * g[2][0] - g[0][0] * g[2][1]) / d;
    gi[2][2] = (g[0][0] * g[1][1] - g[0][1] * g[1][0]) / d;
}

static void unpack_sym(const real *v6, real t[3][3])
{
    for (int a = 0; a < 6; ++a) {
        t[SYM_I[a]][SYM_J[a]] = v6[a];
        t[SYM_J[a]][SYM_I[a]] = v6[a];
    }
}

/* ---------------------------------------------------------------------------
 * Per-point derivative gathering
 * ------------------------------------------------------------------------ */
typedef struct {
    real u[NFIELD];          /* centre values                         */
    real du[NFIELD][3];      /* d_k u_f                               */
    real ddu[NFIELD][3][3];  /* d_k d_l u_f (only for fields needing it) */
    real ko[NFIELD];         /* sum over directions of the KO operator */
    real dl[NFIELD][3];      /* lopsided d_k u_f (advection = 1 only)  */
    real m[NMATTER];         /* matter at the point (0 if absent)     */
} point_data;

static int needs_second(int f)
{
    return f == CHI || (f >= GXX && f <= GZZ) || f == ALPHA || (f >= BETAX && f <= BETAZ);
}

static void gather(const orc_params *P, const orc_block *B, const double *u,
                   const double *matter, int i, int j, int k, int want_ko, point_data *pd)
{
    const long sx = 1, sy = B->nx + 2 * B->ng, sz = (long)sy * (B->ny + 2 * B->ng);
    const long s[3] = {sx, sy, sz};
    const real h[3] = {B->dx, B->dy, B->dz};
    const int p = P->fd_order;
    const long pt = (long)(i + B->ng) * sx + (long)(j + B->ng) * sy + (long)(k + B->ng) * sz;
    memset(pd, 0, sizeof(*pd));
    for (int f = 0; f < NFIELD; ++f) {
        const double *c = u + B->offset + (long long)f * B->field_stride + pt;
        pd->u[f] = c[0];
        for (int a = 0; a < 3; ++a)
            pd->du[f][a] = d1(c, s[a], h[a], p);
        if (needs_second(f)) {
            for (int a = 0; a < 3; ++a) {
                pd->ddu[f][a][a] = d2(c, s[a], h[a], p);
                for (int b = a + 1; b < 3; ++b) {
                    /* d_a d_b = D1_a ( D1_b u ) */
                    const real v = d1d1(c, s[a], s[b], h[a], h[b], p);
                    pd->ddu[f][a][b] = v;
                    pd->ddu[f][b][a] = v;
                }
            }
        }
        if (want_ko) {
            real q = 0.0;
            for (int a = 0; a < 3; ++a)
                q += ko1(c, s[a], h[a], p, P->ko_sigma);
            pd->ko[f] = q;
        }
    }
    if (P->advection == 1) {
        for (int f = 0; f < NFIELD; ++f) {
            const double *c = u + B->offset + (long long)f * B->field_stride + pt;
            for (int a = 0; a < 3; ++a)
                pd->dl[f][a] = d1lop(c, s[a], h[a], p, pd->u[BETAX + a] > 0.0);
        }
    }
    if (matter) {
        for (int f = 0; f < NMATTER; ++f)
            pd->m[f] = matter[B->moffset + (long long)f * B->field_stride + pt];
    }
}

/* ---------------------------------------------------------------------------
 * Z4c pointwise algebra
 * ------------------------------------------------------------------------ */
typedef struct {
    real g[3][3], gi[3][3], A[3][3];
    real Gl[3][3][3];   /* Gt_{k ij}  = 1/2 (d_i gt_jk + d_j gt_ik - d_k gt_ij) */
    real Gu[3][3][3];   /* Gt^k_{ij}  = gt^{kl} Gt_{l ij}                       */
    real Gd[3];         /* Gt_d^i     = gt^{jk} Gt^i_{jk}                       */
    real R[3][3];       /* R_ij = Rt_ij + R^chi_ij                             */
    real Rs;            /* R = chi gt^{ij} R_ij                                */
    real DDa[3][3];     /* D_i D_j alpha (physical covariant derivative)       */
    real D2a;           /* chi gt^{ij} D_i D_j alpha                            */
    real Aup[3][3];     /* At^{ij}                                             */
    real Amix[3][3];    /* At^i_j = gt^{ik} At_kj                               */
    real AA;            /* At_ij At^ij                                         */
    real K;             /* Khat + 2 Theta                                      */
    real chis;          /* max(chi, chi_floor), used in every 1/chi             */
    real dchi[3], dalpha[3];
} geometry;

static void compute_geometry(const orc_params *P, const point_data *pd, geometry *G)
{
    real dg[3][3][3];       /* dg[k][i][j]    = d_k gt_ij        */
    real ddg[3][3][3][3];   /* ddg[k][l][i][j]= d_k d_l gt_ij    */
    real dGam[3][3];        /* dGam[j][k]     = d_j Gt^k (evolved) */
    unpack_sym(&pd->u[GXX], G->g);
    unpack_sym(&pd->u[AXX], G->A);
    inv3(G->g, G->gi);
    for (int a = 0; a < 6; ++a) {
        const int i = SYM_I[a], j = SYM_J[a];
        for (int k = 0; k < 3; ++k) {
            dg[k][i][j] = dg[k][j][i] = pd->du[GXX + a][k];
            for (int l = 0; l < 3; ++l)
                ddg[k][l][i][j] = ddg[k][l][j][i] = pd->ddu[GXX + a][k][l];
        }
    }
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
            dGam[j][k] = pd->du[GAMX + k][j];

    const real chi = pd->u[CHI];
    G->chis = chi > P->chi_floor ? chi : P->chi_floor;
    for (int a = 0; a < 3; ++a) {
        G->dchi[a] = pd->du[CHI][a];
        G->dalpha[a] = pd->du[ALPHA][a];
    }

    /* Christoffel symbols of the conformal metric. */
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                G->Gl[k][i][j] = 0.5 * (dg[i][j][k] + dg[j][i][k] - dg[k][i][j]);
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                real s = 0.0;
                for (int l = 0; l < 3; ++l)
                    s += G->gi[k][l] * G->Gl[l][i][j];
                G->Gu[k][i][j] = s;
            }
    for (int i = 0; i < 3; ++i) {
        real s = 0.0;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                s += G->gi[j][k] * G->Gu[i][j][k];
        G->Gd[i] = s;
    }

    /* Conformal Ricci tensor Rt_ij. */
    real Rt[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            real t1 = 0.0;
            for (int l = 0; l < 3; ++l)
                for (int m = 0; m < 3; ++m)
                    t1 += G->gi[l][m] * ddg[l][m][i][j];
            real t2 = 0.0;
            for (int k = 0; k < 3; ++k)
                t2 += G->g[k][i] * dGam[j][k] + G->g[k][j] * dGam[i][k];
            real t3 = 0.0;
            for (int k = 0; k < 3; ++k)
                t3 += G->Gd[k] * (G->Gl[i][j][k] + G->Gl[j][i][k]);
            real t4 = 0.0;
            for (int l = 0; l < 3; ++l)
                for (int m = 0; m < 3; ++m) {
                    real s = 0.0;
                    for (int k = 0; k < 3; ++k)
                        s += G->Gu[k][l][i] * G->Gl[j][k][m] + G->Gu[k][l][j] * G->Gl[i][k][m]
                           + G->Gu[k][i][m] * G->Gl[k][l][j];
                    t4 += G->gi[l][m] * s;
                }
            Rt[i][j] = -0.5 * t1 + 0.5 * t2 + 0.5 * t3 + t4;
        }

    /* Conformal-factor part R^chi_ij. */
    real DDchi[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            real s = 0.0;
            for (int k = 0; k < 3; ++k)
                s += G->Gu[k][i][j] * G->dchi[k];
            DDchi[i][j] = pd->ddu[CHI][i][j] - s;
        }
    real trDDchi = 0.0, dchi2 = 0.0;
    for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) {
            trDDchi += G->gi[l][m] * DDchi[l][m];
            dchi2 += G->gi[l][m] * G->dchi[l] * G->dchi[m];
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const real Rchi = (DDchi[i][j] + G->g[i][j] * trDDchi) / (2.0 * G->chis)
                              - (G->dchi[i] * G->dchi[j] + 3.0 * G->g[i][j] * dchi2)
                                / (4.0 * G->chis * G->chis);
            G->R[i][j] = Rt[i][j] + Rchi;
        }
    real trR = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            trR += G->gi[i][j] * G->R[i][j];
    G->Rs = chi * trR;

    /* D_i D_j alpha of the physical metric gamma_ij = gt_ij / chi. */
    real dchi_dalpha = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            dchi_dalpha += G->gi[k][l] * G->dchi[k] * G->dalpha[l];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            real s = 0.0;
            for (int k = 0; k < 3; ++k)
                s += G->Gu[k][i][j] * G->dalpha[k];
            G->DDa[i][j] = pd->ddu[ALPHA][i][j] - s
                         + (G->dchi[i] * G->dalpha[j] + G->dchi[j] * G->dalpha[i]
                            - G->g[i][j] * dchi_dalpha) / (2.0 * G->chis);
        }
    real trDDa = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            trDDa += G->gi[i][j] * G->DDa[i][j];
    G->D2a = chi * trDDa;

    /* Raised / mixed At and its square. */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            real s = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l)
                    s += G->gi[i][k] * G->gi[j][l] * G->A[k][l];
            G->Aup[i][j] = s;
            real t = 0.0;
            for (int l = 0; l < 3; ++l)
                t += G->gi[i][l] * G->A[l][j];
            G->Amix[i][j] = t;
        }
    real AA = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            AA += G->A[i][j] * G->Aup[i][j];
    G->AA = AA;
    G->K = pd->u[KHAT] + 2.0 * pd->u[THETA];
}

/* The 22 right-hand sides at one point (KO included). */
static void point_rhs(const orc_params *P, const point_data *pd, real rhs[NFIELD])
{
    geometry G;
    compute_geometry(P, pd, &G);
    const real chi = pd->u[CHI], alpha = pd->u[ALPHA], Theta = pd->u[THETA];
    const real Khat = pd->u[KHAT];
    const real beta[3] = {pd->u[BETAX], pd->u[BETAY], pd->u[BETAZ]};
    const real Gam[3] = {pd->u[GAMX], pd->u[GAMY], pd->u[GAMZ]};
    const real K = G.K;
    real dbeta[3][3];        /* dbeta[j][i] = d_j beta^i       */
    real ddbeta[3][3][3];    /* ddbeta[j][k][i] = d_j d_k beta^i */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            dbeta[j][i] = pd->du[BETAX + i][j];
            for (int k = 0; k < 3; ++k)
                ddbeta[j][k][i] = pd->ddu[BETAX + i][j][k];
        }
    real divb = 0.0;
    for (int k = 0; k < 3; ++k)
        divb += dbeta[k][k];

    /* matter */
    const real rho = pd->m[M_RHO];
    const real Si[3] = {pd->m[M_SX], pd->m[M_SY], pd->m[M_SZ]};
    real Sij[3][3];
    unpack_sym(&pd->m[M_SXX], Sij);
    real trS = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            trS += G.gi[i][j] * Sij[i][j];
    const real S = chi * trS;

    real adv[NFIELD];
    for (int f = 0; f < NFIELD; ++f) {
        real s = 0.0;
        for (int k = 0; k < 3; ++k)
            s += beta[k] * (P->advection == 1 ? pd->dl[f][k] : pd->du[f][k]);
        adv[f] = s;
    }

    /* chi */
    rhs[CHI] = adv[CHI] + (2.0 / 3.0) * chi * (alpha * K - divb);

    /* conformal metric */
    for (int a = 0; a < 6; ++a) {
        const int i = SYM_I[a], j = SYM_J[a];
        real lie = 0.0;
        for (int k = 0; k < 3; ++k)
            lie += G.g[i][k] * dbeta[j][k] + G.g[j][k] * dbeta[i][k];
        rhs[GXX + a] = adv[GXX + a] - 2.0 * alpha * G.A[i][j] + lie
                     - (2.0 / 3.0) * G.g[i][j] * divb;
    }

    /* Khat */
    rhs[KHAT] = adv[KHAT] - G.D2a + alpha * (G.AA + K * K / 3.0) + 4.0 * PI * alpha * (S + rho)
              + alpha * P->kappa1 * (1.0 - P->kappa2) * Theta;

    /* traceless conformal extrinsic curvature */
    real X[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            X[i][j] = -G.DDa[i][j] + alpha * (G.R[i][j] - 8.0 * PI * Sij[i][j]);
    real trX = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            trX += G.gi[i][j] * X[i][j];
    for (int a = 0; a < 6; ++a) {
        const int i = SYM_I[a], j = SYM_J[a];
        const real Xtf = X[i][j] - G.g[i][j] * trX / 3.0;
        real AAm = 0.0;
        for (int k = 0; k < 3; ++k)
            AAm += G.A[i][k] * G.Amix[k][j];
        real lie = 0.0;
        for (int k = 0; k < 3; ++k)
            lie += G.A[i][k] * dbeta[j][k] + G.A[j][k] * dbeta[i][k];
        rhs[AXX + a] = adv[AXX + a] + chi * Xtf + alpha * (K * G.A[i][j] - 2.0 * AAm) + lie
                     - (2.0 / 3.0) * G.A[i][j] * divb;
    }

    /* Theta */
    rhs[THETA] = adv[THETA] + 0.5 * alpha * (G.Rs - G.AA + (2.0 / 3.0) * K * K)
               - alpha * (8.0 * PI * rho + P->kappa1 * (2.0 + P->kappa2) * Theta);

    /* Gamma-tilde */
    for (int i = 0; i < 3; ++i) {
        real s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, s5 = 0.0, s6 = 0.0, s7 = 0.0, s8 = 0.0;
        for (int k = 0; k < 3; ++k)
            s1 += G.Gd[k] * dbeta[k][i];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                s2 += G.gi[j][k] * ddbeta[j][k][i];
        for (int j = 0; j < 3; ++j) {
            real dd = 0.0;
            for (int k = 0; k < 3; ++k)
                dd += ddbeta[j][k][k];
            s3 += G.gi[i][j] * dd;
        }
        for (int j = 0; j < 3; ++j)
            s4 += G.Aup[i][j] * G.dalpha[j];
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                s5 += G.Gu[i][j][k] * G.Aup[j][k];
        for (int j = 0; j < 3; ++j)
            s6 += G.Aup[i][j] * G.dchi[j];
        for (int j = 0; j < 3; ++j)
            s7 += G.gi[i][j] * (2.0 * pd->du[KHAT][j] + pd->du[THETA][j]);
        for (int j = 0; j < 3; ++j)
            s8 += G.gi[i][j] * Si[j];
        rhs[GAMX + i] = adv[GAMX + i] - s1 + (2.0 / 3.0) * G.Gd[i] * divb + s2 + s3 / 3.0
                      - 2.0 * s4
                      + 2.0 * alpha * (s5 - 3.0 / (2.0 * G.chis) * s6 - s7 / 3.0 - 8.0 * PI * s8)
                      - 2.0 * alpha * P->kappa1 * (Gam[i] - G.Gd[i]);
    }

    /* lapse */
    real muL_a2;  /* mu_L * alpha^2 */
    if (P->lapse == 0)
        muL_a2 = 2.0 * alpha;
    else if (P->lapse == 1)
        muL_a2 = alpha * alpha;
    else
        muL_a2 = 0.0;
    rhs[ALPHA] = (P->advect_gauge ? adv[ALPHA] : 0.0) - muL_a2 * Khat;

    /* shift */
    const real muS_a2 = P->shift == 0 ? 1.0 : 0.0;
    for (int i = 0; i < 3; ++i)
        rhs[BETAX + i] = (P->advect_gauge ? adv[BETAX + i] : 0.0) + muS_a2 * Gam[i]
                       - P->eta * beta[i];

    for (int f = 0; f < NFIELD; ++f)
        rhs[f] += pd->ko[f];
}

static void point_constraints(const orc_params *P, const point_data *pd, real c[NCONS])
{
    geometry G;
    compute_geometry(P, pd, &G);
    const real rho = pd->m[M_RHO];
    const real Si[3] = {pd->m[M_SX], pd->m[M_SY], pd->m[M_SZ]};
    real dA[3][3][3];   /* dA[k][i][j] = d_k At_ij */
    for (int a = 0; a < 6; ++a)
        for (int k = 0; k < 3; ++k)
            dA[k][SYM_I[a]][SYM_J[a]] = dA[k][SYM_J[a]][SYM_I[a]] = pd->du[AXX + a][k];
    c[C_H] = G.Rs + (2.0 / 3.0) * G.K * G.K - G.AA - 16.0 * PI * rho;
    for (int i = 0; i < 3; ++i) {
        real div = 0.0;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) {
                real s = dA[k][i][j];
                for (int l = 0; l < 3; ++l)
                    s -= G.Gu[l][j][k] * G.A[l][i] + G.Gu[l][j][i] * G.A[k][l];
                div += G.gi[j][k] * s;
            }
        real t = 0.0;
        for (int j = 0; j < 3; ++j)
            t += G.Amix[j][i] * G.dchi[j];
        const real dK = pd->du[KHAT][i] + 2.0 * pd->du[THETA][i];
        c[C_MX + i] = div - 3.0 / (2.0 * G.chis) * t - (2.0 / 3.0) * dK - 8.0 * PI * Si[i];
    }
    c[C_THETA] = pd->u[THETA];
    for (int i = 0; i < 3; ++i)
        c[C_ZX + i] = 0.5 * (pd->u[GAMX + i] - G.Gd[i]);
}

/* ---------------------------------------------------------------------------
 * Algebraic enforcement after a stage: det(gt) = 1, tr(At) = 0, floors.
 * ------------------------------------------------------------------------ */
static void enforce(const orc_params *P, real v[NFIELD])
{
    real g[3][3], gi[3][3], A[3][3];
    unpack_sym(&v[GXX], g);
    const real f = 1.0 / cbrt(det3(g));
    for (int a = 0; a < 6; ++a)
        v[GXX + a] *= f;
    unpack_sym(&v[GXX], g);
    inv3(g, gi);
    unpack_sym(&v[AXX], A);
    real tr = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            tr += gi[i][j] * A[i][j];
    for (int a = 0; a < 6; ++a)
        v[AXX + a] -= g[SYM_I[a]][SYM_J[a]] * tr / 3.0;
    if (!(v[CHI] > P->chi_floor))
        v[CHI] = P->chi_floor;
    if (!(v[ALPHA] > P->alpha_floor))
        v[ALPHA] = P->alpha_floor;
}

/* ---------------------------------------------------------------------------
 * Work lists: (block, z-plane) pairs for OpenMP
 * ------------------------------------------------------------------------ */
typedef struct { int b, k; } work_item;

static work_item *make_work(const orc_block *blocks, int nb, long *count)
{
    long n = 0;
    for (int b = 0; b < nb; ++b)
        n += blocks[b].nz;
    work_item *w = (work_item *)malloc(sizeof(work_item) * (size_t)(n > 0 ? n : 1));
    long c = 0;
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < blocks[b].nz; ++k) {
            w[c].b = b;
            w[c].k = k;
            ++c;
        }
    *count = n;
    return w;
}

/* nthreads > 0: that many threads; 0: the OpenMP default of the process
 * (as it was before the first call here). */
static void set_threads(int nthreads)
{
#ifdef _OPENMP
    static int default_threads = 0;
    if (default_threads == 0)
        default_threads = omp_get_max_threads();
    omp_set_num_threads(nthreads > 0 ? nthreads : default_threads);
#else
    (void)nthreads;
#endif
}

static long point_index(const orc_block *B, int i, int j, int k)
{
    const long sy = B->nx + 2 * B->ng, sz = sy * (B->ny + 2 * B->ng);
    return (long)(i + B->ng) + (long)(j + B->ng) * sy + (long)(k + B->ng) * sz;
}

/* ---------------------------------------------------------------------------
 * Exported entry points (host pointers; interior points only are written)
 * ------------------------------------------------------------------------ */

int orc_rhs(const orc_params *P, const orc_block *blocks, int nb, const double *u,
            const double *matter, double *rhs, int nthreads)
{
    long nw;
    work_item *w = make_work(blocks, nb, &nw);
    set_threads(nthreads);
    lop_init();
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < nw; ++t) {
        const orc_block *B = &blocks[w[t].b];
        const int k = w[t].k;
        point_data pd;
        real r[NFIELD];
        for (int j = 0; j < B->ny; ++j)
            for (int i = 0; i < B->nx; ++i) {
                gather(P, B, u, matter, i, j, k, 1, &pd);
                point_rhs(P, &pd, r);
                const long pt = point_index(B, i, j, k);
                for (int f = 0; f < NFIELD; ++f)
                    rhs[B->offset + (long long)f * B->field_stride + pt] = (double)r[f];
            }
    }
    free(w);
    return 0;
}

/* One stage: k = RHS(u0);  u1 <- [u1] + delta u0 + eps dt k;
 * u0_out <- g1 u0 + g2 u1 + g3 u2 + beta dt k;  enforce on u0_out. */
int orc_rk_stage(const orc_params *P, const orc_block *blocks, int nb, const double *u0,
                 double *u0_out, double *u1, const double *u2, const double *matter,
                 const orc_rk *c, double dt, int nthreads)
{
    long nw;
    work_item *w = make_work(blocks, nb, &nw);
    set_threads(nthreads);
    lop_init();
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < nw; ++t) {
        const orc_block *B = &blocks[w[t].b];
        const int k = w[t].k;
        point_data pd;
        real r[NFIELD], v[NFIELD];
        for (int j = 0; j < B->ny; ++j)
            for (int i = 0; i < B->nx; ++i) {
                gather(P, B, u0, matter, i, j, k, 1, &pd);
                point_rhs(P, &pd, r);
                const long pt = point_index(B, i, j, k);
                for (int f = 0; f < NFIELD; ++f) {
                    const long long e = B->offset + (long long)f * B->field_stride + pt;
                    const real a1 = c->read_u1 ? (real)u1[e] : 0;
                    const real epsdt = (real)c->eps * (real)dt, betadt = (real)c->beta * (real)dt;
                    const real n1 = a1 + (real)c->delta * pd.u[f] + epsdt * r[f];
                    v[f] = (real)c->g1 * pd.u[f] + (real)c->g2 * n1
                         + (c->g3 != 0.0 ? (real)c->g3 * (real)u2[e] : 0) + betadt * r[f];
                    if (c->write_u1)
                        u1[e] = (double)n1;
                }
                enforce(P, v);
                for (int f = 0; f < NFIELD; ++f)
                    u0_out[B->offset + (long long)f * B->field_stride + pt] = (double)v[f];
            }
    }
    free(w);
    return 0;
}

/* Constraints at every interior point (cons may be NULL) and per-block norms:
 * norms[b*16 + 2*c + 0] = sum |c| dV,  norms[b*16 + 2*c + 1] = sum c^2 dV. */
int orc_constraints(const orc_params *P, const orc_block *blocks, int nb, const double *u,
                    const double *matter, double *cons, double *norms, int nthreads)
{
    set_threads(nthreads);
    for (int b = 0; b < nb; ++b) {
        const orc_block *B = &blocks[b];
        const double dV = B->dx * B->dy * B->dz;
        real l1[NCONS] = {0}, l2[NCONS] = {0};
        for (int k = 0; k < B->nz; ++k) {
            real pl1[NCONS] = {0}, pl2[NCONS] = {0};
#pragma omp parallel for reduction(+ : pl1[:NCONS], pl2[:NCONS]) schedule(static)
            for (int j = 0; j < B->ny; ++j) {
                point_data pd;
                real cv[NCONS];
                for (int i = 0; i < B->nx; ++i) {
                    gather(P, B, u, matter, i, j, k, 0, &pd);
                    point_constraints(P, &pd, cv);
                    const long pt = point_index(B, i, j, k);
                    for (int q = 0; q < NCONS; ++q) {
                        if (cons)
                            cons[B->coffset + (long long)q * B->field_stride + pt] = (double)cv[q];
                        pl1[q] += fabs(cv[q]);
                        pl2[q] += cv[q] * cv[q];
                    }
                }
            }
            for (int q = 0; q < NCONS; ++q) {
                l1[q] += pl1[q];
                l2[q] += pl2[q];
            }
        }
        if (norms)
            for (int q = 0; q < NCONS; ++q) {
                norms[b * 16 + 2 * q] = (double)(l1[q] * dV);
                norms[b * 16 + 2 * q + 1] = (double)(l2[q] * dV);
            }
    }
    return 0;
}

/* Ghost refresh.  policy 1: each block periodic on itself; 2: neighbour copy
 * from nbr[b*27 + dir] (dir = (oz+1)*9 + (oy+1)*3 + (ox+1); -1 means outer
 * boundary, filled from `frozen`); 3: all ghosts from `frozen`.
 * Neighbours must have the same nx, ny, nz, ng. */
int orc_ghost_fill(int policy, const orc_block *blocks, int nb, const int *nbr, double *u,
                   const double *frozen)
{
    for (int b = 0; b < nb; ++b) {
        const orc_block *B = &blocks[b];
        const int ng = B->ng;
        for (int f = 0; f < NFIELD; ++f)
            for (int k = -ng; k < B->nz + ng; ++k)
                for (int j = -ng; j < B->ny + ng; ++j)
                    for (int i = -ng; i < B->nx + ng; ++i) {
                        const int ox = i < 0 ? -1 : (i >= B->nx ? 1 : 0);
                        const int oy = j < 0 ? -1 : (j >= B->ny ? 1 : 0);
                        const int oz = k < 0 ? -1 : (k >= B->nz ? 1 : 0);
                        if (!ox && !oy && !oz)
                            continue;
                        const long long dst = B->offset + (long long)f * B->field_stride
                                            + point_index(B, i, j, k);
                        int src_b = -1;
                        if (policy == 1)
                            src_b = b;
                        else if (policy == 2)
                            src_b = nbr[b * 27 + (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)];
                        if (src_b < 0) {
                            if (frozen)
                                u[dst] = frozen[dst];
                            continue;
                        }
                        const orc_block *S = &blocks[src_b];
                        const int si = i - ox * B->nx, sj = j - oy * B->ny, sk = k - oz * B->nz;
                        u[dst] = u[S->offset + (long long)f * S->field_stride
                                   + point_index(S, si, sj, sk)];
                    }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Radiative (Sommerfeld) outer boundary.  The paper states no outer boundary
 * condition for Z4c; this is the usual radiative law of moving-puncture
 * codes, taken as a reading:
 *   outer points: the ghost points of block b in a direction (ox, oy, oz)
 *     whose neighbour entry nbr[b*27 + dir] is -1;
 *   at an outer point with coordinates x (x0 of the block, the coordinates
 *     of its interior point (0,0,0), plus index times spacing) and r = |x|,
 *     every field u evolves by
 *       d_t u = -(x^a / r) D_a u - (u - u_inf) / r,
 *     u_inf its flat-space value (1 for chi, gt_xx, gt_yy, gt_zz, alpha; 0
 *     otherwise), D_a the second-order difference along a: centred where
 *     the point's index along a lies in [0, n_a), one-sided towards the
 *     interior otherwise;
 *   the outer points then take the same Runge-Kutta stage and enforcement
 *     as the interior points (orc_rk_stage); no dissipation.
 * ------------------------------------------------------------------------ */
static real flat_value(int f)
{
    return (f == CHI || f == GXX || f == GYY || f == GZZ || f == ALPHA) ? 1.0 : 0.0;
}

/* Second-order difference along one direction at index i of n interior
 * points (stride s between neighbours, spacing h), in differences from the
 * centre. */
static real d1_radiative(const double *u, long s, int i, int n, real h)
{
    if (i < 0)
        return (4 * DIFF(s, 0) - DIFF(2 * s, 0)) / (2 * h);
    if (i >= n)
        return (-4 * DIFF(-s, 0) + DIFF(-2 * s, 0)) / (2 * h);
    return DIFF(s, -s) / (2 * h);
}

/* rhs != NULL: d_t u at every outer point of rhs (nothing else written).
 * rhs == NULL: one stage at the outer points, u1 <- [u1] + delta u0 +
 * eps dt k (if write_u1), u0_out <- g1 u0 + g2 u1' + g3 u2 + beta dt k,
 * then enforcement, as orc_rk_stage does for the interior.  x0: 3 per
 * block. */
int orc_sommerfeld(const orc_params *P, const orc_block *blocks, int nb, const int *nbr,
                   const double *x0, const double *u0, double *rhs, double *u0_out, double *u1,
                   const double *u2, const orc_rk *c, double dt)
{
    for (int b = 0; b < nb; ++b) {
        const orc_block *B = &blocks[b];
        const int ng = B->ng;
        const int n[3] = {B->nx, B->ny, B->nz};
        const real h[3] = {B->dx, B->dy, B->dz};
        const long sy = B->nx + 2 * ng, sz = sy * (B->ny + 2 * ng);
        const long st[3] = {1, sy, sz};
        for (int k = -ng; k < B->nz + ng; ++k)
            for (int j = -ng; j < B->ny + ng; ++j)
                for (int i = -ng; i < B->nx + ng; ++i) {
                    const int ox = i < 0 ? -1 : (i >= B->nx ? 1 : 0);
                    const int oy = j < 0 ? -1 : (j >= B->ny ? 1 : 0);
                    const int oz = k < 0 ? -1 : (k >= B->nz ? 1 : 0);
                    if (!ox && !oy && !oz)
                        continue;
                    if (nbr[b * 27 + (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)] >= 0)
                        continue;
                    const int idx[3] = {i, j, k};
                    real X[3];
                    for (int a = 0; a < 3; ++a)
                        X[a] = (real)x0[3 * b + a] + idx[a] * h[a];
                    const real r = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
                    const long pt = point_index(B, i, j, k);
                    real kf[NFIELD], v[NFIELD];
                    for (int f = 0; f < NFIELD; ++f) {
                        const double *cf = u0 + B->offset + (long long)f * B->field_stride + pt;
                        real adv = 0;
                        for (int a = 0; a < 3; ++a)
                            adv += X[a] * d1_radiative(cf, st[a], idx[a], n[a], h[a]);
                        kf[f] = -adv / r - ((real)cf[0] - flat_value(f)) / r;
                    }
                    if (rhs) {
                        for (int f = 0; f < NFIELD; ++f)
                            rhs[B->offset + (long long)f * B->field_stride + pt] = (double)kf[f];
                        continue;
                    }
                    for (int f = 0; f < NFIELD; ++f) {
                        const long long e = B->offset + (long long)f * B->field_stride + pt;
                        const real a1 = c->read_u1 ? (real)u1[e] : 0;
                        const real epsdt = (real)c->eps * (real)dt, betadt = (real)c->beta * (real)dt;
                        const real n1 = a1 + (real)c->delta * (real)u0[e] + epsdt * kf[f];
                        v[f] = (real)c->g1 * (real)u0[e] + (real)c->g2 * n1
                             + (c->g3 != 0.0 ? (real)c->g3 * (real)u2[e] : 0) + betadt * kf[f];
                        if (c->write_u1)
                            u1[e] = (double)n1;
                    }
                    enforce(P, v);
                    for (int f = 0; f < NFIELD; ++f)
                        u0_out[B->offset + (long long)f * B->field_stride + pt] = (double)v[f];
                }
    }
    return 0;
}

/* Derivative probe for the operator pins: one field array of block shape in,
 * 12 interior-sized arrays out, in order
 * D1x D1y D1z  D2xx D2xy D2xz D2yy D2yz D2zz  KOx KOy KOz   (x fastest). */
int orc_derivs(const orc_params *P, const orc_block *B, const double *u, double *out)
{
    const long sx = 1, sy = B->nx + 2 * B->ng, sz = sy * (B->ny + 2 * B->ng);
    const long s[3] = {sx, sy, sz};
    const double h[3] = {B->dx, B->dy, B->dz};
    const int p = P->fd_order;
    const long n = (long)B->nx * B->ny * B->nz;
    for (int k = 0; k < B->nz; ++k)
        for (int j = 0; j < B->ny; ++j)
            for (int i = 0; i < B->nx; ++i) {
                const double *c = u + point_index(B, i, j, k);
                const long o = (long)i + (long)B->nx * (j + (long)B->ny * k);
                for (int a = 0; a < 3; ++a)
                    out[a * n + o] = (double)d1(c, s[a], h[a], p);
                int q = 3;
                for (int a = 0; a < 3; ++a)
                    for (int b = a; b < 3; ++b) {
                        out[q * n + o] = (double)((a == b) ? d2(c, s[a], h[a], p)
                                                           : d1d1(c, s[a], s[b], h[a], h[b], p));
                        ++q;
                    }
                for (int a = 0; a < 3; ++a)
                    out[(9 + a) * n + o] = (double)ko1(c, s[a], h[a], p, P->ko_sigma);
            }
    return 0;
}

/* Number of OpenMP threads the oracle would use. */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

