"""Pins of the FP64 CPU oracle against what mathematics and general
relativity fix (no GPU).  Each test names the property it relies on; none
re-types the oracle's formulas.

* stencil weights: exactness on polynomials (unique for these stencil
  widths) and the leading truncation term one degree higher;
* Kreiss-Oliger operator: annihilates polynomials of degree < 2r and acts as
  -sigma/h on the highest grid mode in every direction;
* flat space: every right-hand side and constraint is exactly 0;
* Kerr-Schild Schwarzschild (vacuum, shifted, static), generic smooth data
  with matter that satisfies the ADM constraints, the x and diagonal gauge
  waves: right-hand side -> exact time derivative from textbook ADM
  evolution at order p; H and M_i -> 0 at order p;
* the linearised system about flat space (1+log lapse, Gamma-driver shift,
  constraint damping, dissipation) and its RK4 / SSPRK3 amplification;
* long-run robust stability on noise;
* a full evolution of the gauge wave converging at min(p, 4);
* algebraic enforcement and floors; ghost refresh index maps.
"""
import math

import numpy as np
import pytest

import exact as E
import linear_mode as LM
import oracle as O
from paper_2311_04989_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _build_oracle():
    O.build(force=False)


# --- stencils ---------------------------------------------------------------------

def _poly_block(n=9, ng=4):
    return W.Block(n, n, n, ng, 1.0, 1.0, 1.0, -3.0, 2.0, 5.0)


def _monomial(blk, a, b, c):
    X, Y, Z = blk.coords()
    return X ** a * Y ** b * Z ** c, (X, Y, Z)


@pytest.mark.parametrize("p", [4, 6])
def test_first_and_second_derivatives_exact_on_polynomials(p):
    """D1 is exact for degree <= p, D2 for degree <= p+1, D1_a D1_b for
    x^a y^b with a, b <= p: with integer points and h = 1 every value is
    computed exactly, so the comparison is bitwise."""
    blk = _poly_block()
    g = blk.ng
    sl = (slice(g, -g),) * 3
    for deg in range(0, p + 2):
        for (a, b, c) in [(deg, 0, 0), (0, deg, 0), (0, 0, deg)]:
            u, (X, Y, Z) = _monomial(blk, a, b, c)
            out = O.derivs(blk, u, p)
            exact_d = [a * X ** max(a - 1, 0) * Y ** b * Z ** c,
                       b * X ** a * Y ** max(b - 1, 0) * Z ** c,
                       c * X ** a * Y ** b * Z ** max(c - 1, 0)]
            exact_dd = [a * (a - 1) * X ** max(a - 2, 0) * Y ** b * Z ** c,
                        b * (b - 1) * X ** a * Y ** max(b - 2, 0) * Z ** c,
                        c * (c - 1) * X ** a * Y ** b * Z ** max(c - 2, 0)]
            if deg <= p:
                for q in range(3):
                    np.testing.assert_array_equal(out[q], exact_d[q][sl])
            # pure second derivatives: D2xx (3), D2yy (6), D2zz (8)
            for q, e in zip((3, 6, 8), exact_dd):
                np.testing.assert_array_equal(out[q], e[sl])
    # mixed derivatives on x^a y^b (a, b <= p) and permutations
    for a in range(0, p + 1):
        for b in range(0, p + 1):
            for (pa, pb, q) in [((a, b, 0), None, 4), ((a, 0, b), None, 5), ((0, a, b), None, 7)]:
                u, (X, Y, Z) = _monomial(blk, *pa)
                out = O.derivs(blk, u, p)
                i, j, k = pa
                if q == 4:
                    e = i * j * X ** max(i - 1, 0) * Y ** max(j - 1, 0) * Z ** k
                elif q == 5:
                    e = i * k * X ** max(i - 1, 0) * Y ** j * Z ** max(k - 1, 0)
                else:
                    e = j * k * X ** i * Y ** max(j - 1, 0) * Z ** max(k - 1, 0)
                np.testing.assert_array_equal(out[q], e[sl])


@pytest.mark.parametrize("p", [4, 6])
def test_leading_truncation_terms(p):
    """One degree past exactness the error equals the Taylor remainder of
    the central stencils: D1 x^(p+1) - (p+1) x^p = c1 h^p (p+1)!,
    c1 = -1/30 (p=4), +1/140 (p=6);  D2 x^(p+2) - exact = c2 h^p (p+2)!,
    c2 = -1/90 (p=4), +1/560 (p=6)."""
    blk = _poly_block()
    g = blk.ng
    sl = (slice(g, -g),) * 3
    X, Y, Z = blk.coords()
    c1 = {4: -1.0 / 30.0, 6: 1.0 / 140.0}[p]
    c2 = {4: -1.0 / 90.0, 6: 1.0 / 560.0}[p]
    out = O.derivs(blk, X ** (p + 1), p)
    err = out[0] - ((p + 1) * X ** p)[sl]
    np.testing.assert_allclose(err, c1 * math.factorial(p + 1), rtol=1e-12)
    out = O.derivs(blk, Y ** (p + 2), p)
    err = out[6] - ((p + 2) * (p + 1) * Y ** p)[sl]
    np.testing.assert_allclose(err, c2 * math.factorial(p + 2), rtol=1e-12)


@pytest.mark.parametrize("p", [4, 6])
def test_ko_annihilates_low_degree_and_damps_highest_mode(p):
    r = p // 2 + 1
    blk = _poly_block()
    for deg in range(0, 2 * r):
        for pa in [(deg, 0, 0), (0, deg, 0), (0, 0, deg)]:
            u, _ = _monomial(blk, *pa)
            out = O.derivs(blk, u, p, ko_sigma=0.5)
            for q in (9, 10, 11):
                assert np.all(out[q] == 0.0), (deg, pa, q)
    # degree 2r is not annihilated: Delta^(2r) x^(2r) = (2r)!
    u, _ = _monomial(blk, 2 * r, 0, 0)
    out = O.derivs(blk, u, p, ko_sigma=0.5)
    expect = (-1.0) ** (r + 1) * 0.5 / 2.0 ** (2 * r) * math.factorial(2 * r)
    np.testing.assert_array_equal(out[9], np.full_like(out[9], expect))
    # highest grid mode: each direction gives -sigma/h * u exactly
    for h in (1.0, 0.5, 0.25):
        blk2 = W.Block(6, 7, 8, r, h, h, h)
        I = np.indices(blk2.shape)
        u = (-1.0) ** (I[0] + I[1] + I[2])
        out = O.derivs(blk2, u, p, ko_sigma=0.5)
        g = blk2.ng
        uc = u[g:-g, g:-g, g:-g]
        for q in (9, 10, 11):
            np.testing.assert_array_equal(out[q], -0.5 / h * uc)


def test_ko_fourier_symbol():
    """On cos(k x) the operator returns -(sigma/h) sin(kh/2)^(2r) cos(k x)."""
    for p in (4, 6):
        r = p // 2 + 1
        h = 0.1
        blk = W.Block(20, 4, 4, r, h, h, h)
        X, _, _ = blk.coords()
        for k in (1.0, 7.0, 20.0):
            out = O.derivs(blk, np.cos(k * X), p, ko_sigma=0.3)
            g = blk.ng
            pred = -(0.3 / h) * math.sin(0.5 * k * h) ** (2 * r) * np.cos(k * X)[g:-g, g:-g, g:-g]
            np.testing.assert_allclose(out[9], pred, atol=1e-12)


# --- whole right-hand side ------------------------------------------------------------

@pytest.mark.parametrize("p", [4, 6])
def test_flat_space_gives_exact_zero(p):
    blocks = [W.Block(5, 7, 3, p // 2 + 1, 0.1, 0.2, 0.3), W.Block(9, 4, 6, 4, 0.05, 0.05, 0.5)]
    bt = W.Batch(blocks, with_matter=True)
    W.fill_fields(bt, W.flat)
    bt.params = W.Params(fd_order=p, ko_sigma=0.5)
    r = O.rhs(bt)
    assert np.all(r == 0.0)
    cons, norms = O.constraints(bt)
    assert np.all(cons == 0.0) and np.all(norms == 0.0)


def _load_exact(blk, vals, matter=None):
    bt = W.Batch([blk], with_matter=matter is not None)
    for f, nm in enumerate(W.FIELDS):
        bt.view(bt.u, 0, f)[...] = vals[nm]
    if matter is not None:
        for f in range(W.NM):
            bt.view(bt.matter, 0, f, W.NM)[...] = matter[f]
    return bt


FROZEN = dict(lapse=W.LAPSE_FROZEN, shift=W.SHIFT_FROZEN, eta=0.0, advect_gauge=0)


def _adm_convergence(which, p, ns, L, x0, sigma):
    rhs_err, cons_err = [], []
    for n in ns:
        h = L / n
        blk = W.Block(n, n, n, p // 2 + 1, h, h, h, *x0)
        X, Y, Z = blk.coords()
        if which == "kerr_schild":
            vals, dts, matter = E.kerr_schild(X, Y, Z)
        else:
            vals, dts, matter = E.generic_with_matter(X, Y, Z)
        bt = _load_exact(blk, vals, matter)
        bt.params = W.Params(fd_order=p, ko_sigma=sigma, kappa1=0.02, kappa2=0.1, **FROZEN)
        r = O.rhs(bt)
        g = blk.ng
        sl = (slice(g, -g),) * 3
        rhs_err.append(np.array([np.abs(bt.interior(r, 0, f) - dts[nm][sl]).max()
                                 for f, nm in enumerate(W.FIELDS[:18])]))
        cons, _ = O.constraints(bt)
        cons_err.append(np.array([np.abs(bt.interior(cons, 0, c, W.NC)).max() for c in range(4)]))
    return np.array(rhs_err), np.array(cons_err)


@pytest.mark.parametrize("p", [4, 6])
def test_kerr_schild_static_convergence(p):
    """Static Schwarzschild in Kerr-Schild form (M = 1) on [2, 3]^3 with the
    gauge frozen: every non-gauge right-hand side tends to 0 (the exact d_t)
    and H, M_i tend to 0, all at order p."""
    re, ce = _adm_convergence("kerr_schild", p, (12, 24), 1.0, (2.0, 2.0, 2.0), 0.0)
    order = np.log2(re[0].max() / re[1].max())
    assert abs(order - p) < 0.35, (order, re)
    corder = np.log2(ce[0] / ce[1])
    assert np.all(np.abs(corder - p) < 0.35), (corder, ce)


@pytest.mark.parametrize("p", [4, 6])
def test_generic_data_with_matter_matches_adm_evolution(p):
    """Generic shifted data with a non-trivial lapse, rho and S_i defined by
    the ADM constraints, arbitrary S_ij: every non-gauge right-hand side
    (with dissipation on) converges at order p to d_t of the Z4c variables
    implied by the ADM evolution equations with matter, and H, M_i -> 0."""
    re, ce = _adm_convergence("generic", p, (12, 24), 0.5, (0.3, -0.2, 0.1), 0.5)
    orders = np.log2(re[0] / re[1])
    assert np.all(orders > p - 1.0), (orders, re)
    assert abs(np.log2(re[0].max() / re[1].max()) - p) < 0.35
    corder = np.log2(ce[0] / ce[1])
    assert np.all(np.abs(corder - p) < 0.35), (corder, ce)


@pytest.mark.parametrize("p", [4, 6])
@pytest.mark.parametrize("direction", ["x", "xy"])
def test_gauge_wave_rhs_convergence(p, direction):
    """Gauge wave (A = 0.1, harmonic slicing, zero shift) is an exact
    solution: the right-hand side of all 22 fields converges to the exact
    time derivative at order p.  The diagonal wave exercises the mixed
    second derivatives."""
    errs = []
    for n in (16, 32):
        blk = W.Block(n, n, 4, p // 2 + 1, 1.0 / n, 1.0 / n, 1.0 / n)
        X, Y, Z = blk.coords()
        vals, dts = E.gauge_wave(X, Y, Z, 0.1, direction)
        bt = _load_exact(blk, vals)
        bt.params = W.Params(fd_order=p, ko_sigma=0.0, lapse=W.LAPSE_HARMONIC,
                             shift=W.SHIFT_FROZEN, eta=0.0, advect_gauge=0)
        r = O.rhs(bt)
        g = blk.ng
        sl = (slice(g, -g),) * 3
        errs.append(max(np.abs(bt.interior(r, 0, f) - dts[nm][sl]).max()
                        for f, nm in enumerate(W.FIELDS)))
    order = math.log2(errs[0] / errs[1])
    assert order > p - 0.45, (order, errs)


def test_config1_gauge_wave_data_matches_exact_solution():
    """The workload generator's gauge wave equals the exact solution built
    from ADM quantities (up to the seeded 1e-10 noise and periodic ghosts)."""
    bt = W.config1()
    blk = bt.blocks[0]
    X, Y, Z = blk.coords()
    vals, _ = E.gauge_wave(X, Y, Z, 0.01, "x")
    g = blk.ng
    for f, nm in enumerate(W.FIELDS):
        d = bt.interior(bt.u, 0, f) - vals[nm][g:-g, g:-g, g:-g]
        assert np.abs(d).max() <= 1.0e-10 + 1e-15, nm


# --- linearised system --------------------------------------------------------------

def _mode_batch(blk, c, coord, k, eps, prm):
    bt = W.Batch([blk])
    W.fill_fields(bt, W.flat)
    vals = LM.field_values(c, coord, k)
    for f in range(W.NF):
        bt.view(bt.u, 0, f)[...] += eps * vals[f]
    bt.params = prm
    bt.ghost = W.GHOST_PERIODIC
    return bt


@pytest.mark.parametrize("p", [4, 6])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_linear_mode_closed_form(p, d):
    """Small plane waves about flat space along each axis: the odd-in-eps part
    of the right-hand side, and of one RK4 and one SSPRK3 step with periodic
    ghosts, equals the closed-form linear semi-discrete evolution (1+log,
    Gamma-driver, kappa1/kappa2 damping, KO) to O(eps^2)."""
    rng = np.random.default_rng(100 + 10 * p + d)
    n, m = 16, 2
    h = 1.0 / n
    k = 2.0 * math.pi * m / (n * h)
    dims = [4, 4, 4]
    dims[d] = n
    blk = W.Block(dims[0], dims[1], dims[2], p // 2 + 1, h, h, h)
    coord = blk.coords()[d]
    c = LM.random_amplitudes(rng)
    prm = W.Params(fd_order=p, ko_sigma=0.3, kappa1=0.07, kappa2=0.3, eta=1.7)
    eps = 1e-5
    bp = _mode_batch(blk, c, coord, k, eps, prm)
    bm = _mode_batch(blk, c, coord, k, -eps, prm)
    M = LM.matrix(k, h, p, prm.ko_sigma, d, prm.kappa1, prm.kappa2, prm.eta)
    g = blk.ng
    sl = (slice(g, -g),) * 3

    def check(lin, amp):
        pred = LM.field_values(amp, coord, k)
        scale = max(np.abs(pv).max() for pv in pred)
        err = max(np.abs(bp.interior(lin, 0, f) - pred[f][sl]).max() for f in range(W.NF))
        assert err <= 1e-7 * scale, err / scale

    check((O.rhs(bp) - O.rhs(bm)) / (2 * eps), M @ c)
    O.ghost_fill(bp, bp.u)
    O.ghost_fill(bm, bm.u)
    dt = 0.25 * h
    for tab, name in ((O.RK4, "rk4"), (O.SSPRK3, "ssprk3")):
        up = O.rk_step(bp, bp.u, table=tab, dt=dt)
        um = O.rk_step(bm, bm.u, table=tab, dt=dt)
        check((up - um) / (2 * eps), LM.rk_polynomial(dt * M, name) @ c)


def test_rk_amplification_polynomials_on_pure_damping():
    """With the lapse frozen and gauge advection off, alpha obeys
    d_t alpha = Q alpha exactly (Q = KO, linear).  On the highest grid mode
    Q = -3 sigma/h, so one RK4 step multiplies the perturbation by
    1+z+z^2/2+z^3/6+z^4/24 and one SSPRK3 step by 1+z+z^2/2+z^3/6,
    z = -3 sigma dt / h."""
    h, sigma, p = 0.5, 0.4, 4
    blk = W.Block(6, 6, 6, 3, h, h, h)
    I = np.indices(blk.shape)
    mode = (-1.0) ** (I[0] + I[1] + I[2])
    bt = W.Batch([blk])
    W.fill_fields(bt, W.flat)
    f = W.F["alpha"]
    eps = 1e-3
    bt.view(bt.u, 0, f)[...] += eps * mode
    bt.params = W.Params(fd_order=p, ko_sigma=sigma, lapse=W.LAPSE_FROZEN,
                         shift=W.SHIFT_FROZEN, eta=0.0, advect_gauge=0)
    bt.ghost = W.GHOST_PERIODIC
    dt = 0.3
    z = -3.0 * sigma / h * dt
    g = blk.ng
    for tab, amp in ((O.RK4, 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24),
                     (O.SSPRK3, 1 + z + z ** 2 / 2 + z ** 3 / 6)):
        out = O.rk_step(bt, bt.u.copy(), table=tab, dt=dt)
        got = bt.interior(out, 0, f) - 1.0
        np.testing.assert_allclose(got, amp * eps * mode[g:-g, g:-g, g:-g], rtol=1e-12)


# --- stability, evolution convergence --------------------------------------------------

def test_robust_stability_on_noise():
    """Flat space + U(-1e-10, 1e-10) noise on all fields, periodic 8^3 block,
    p = 4, sigma = 0.02, 1+log / Gamma-driver (eta = 2), 1000 RK4 steps with
    dt = dx/4: the Hamiltonian-constraint L2 norm never exceeds 10x its
    initial value and shows no exponential growth."""
    n = 8
    h = 1.0 / n
    blk = W.Block(n, n, n, 3, h, h, h)
    bt = W.Batch([blk])
    W.fill_fields(bt, W.flat)
    W.add_noise(bt, np.random.default_rng(W.SEED_BASE + 99), 1e-10)
    bt.params = W.Params(fd_order=4, ko_sigma=0.02, eta=2.0)
    bt.ghost = W.GHOST_PERIODIC
    O.ghost_fill(bt, bt.u)
    u = bt.u
    H = []
    for s in range(1001):
        if s % 25 == 0:
            _, nr = O.constraints(bt, u=u, want_fields=False)
            H.append(math.sqrt(nr[0, 0, 1]))
        if s < 1000:
            u = O.rk_step(bt, u, dt=0.25 * h)
    H = np.array(H)
    assert np.all(np.isfinite(H))
    assert H.max() <= 10.0 * H[0]
    slope = np.polyfit(np.arange(len(H)) * 25.0, np.log(H), 1)[0]
    assert slope <= 0.01


@pytest.mark.parametrize("p", [4, 6])
def test_gauge_wave_evolution_convergence(p):
    """Full evolution of the 1-D gauge wave (A = 0.1, harmonic slicing) to
    t = 0.25 with RK4, dt = dx/4, periodic ghosts: the error against the
    exact solution converges at min(p, 4) = 4."""
    errs = []
    T = 0.25
    for n in (16, 32):
        h = 1.0 / n
        blk = W.Block(n, 4, 4, p // 2 + 1, h, h, h)
        X, Y, Z = blk.coords()
        vals, _ = E.gauge_wave(X, Y, Z, 0.1, "x")
        bt = _load_exact(blk, vals)
        bt.params = W.Params(fd_order=p, ko_sigma=0.0, lapse=W.LAPSE_HARMONIC,
                             shift=W.SHIFT_FROZEN, eta=0.0, advect_gauge=0)
        bt.ghost = W.GHOST_PERIODIC
        dt = 0.25 * h
        u = bt.u
        for _ in range(int(round(T / dt))):
            u = O.rk_step(bt, u, dt=dt)
        ex, _ = E.gauge_wave(X - T, Y, Z, 0.1, "x")
        g = blk.ng
        sl = (slice(g, -g),) * 3
        errs.append(max(np.abs(bt.interior(u, 0, f) - ex[nm][sl]).max()
                        for f, nm in enumerate(W.FIELDS)))
    order = math.log2(errs[0] / errs[1])
    assert order > 3.6, (order, errs)


def test_convergence_factor_definition():
    """The paper's self-convergence factor Q_n = (dx_c^n - dx_m^n) /
    (dx_c^n - dx_f^n) is the expected ratio (u_c - u_m)/(u_c - u_f) of
    differences between coarse, medium and fine solutions converging at
    order n; check it on the gauge-wave right-hand side of the oracle."""
    p = 4
    hs, vals = [], []
    for n in (16, 24, 32):
        h = 1.0 / n
        blk = W.Block(n, 4, 4, 3, h, h, h)
        X, Y, Z = blk.coords()
        v, _ = E.gauge_wave(X, Y, Z, 0.1, "x")
        bt = _load_exact(blk, v)
        bt.params = W.Params(fd_order=p, ko_sigma=0.0, lapse=W.LAPSE_HARMONIC,
                             shift=W.SHIFT_FROZEN, eta=0.0, advect_gauge=0)
        r = O.rhs(bt)
        # sample the K-hat right-hand side at x = 1/8 (a point common to all grids)
        i = int(round(0.125 / h))
        hs.append(h)
        vals.append(bt.interior(r, 0, W.F["Khat"])[1, 1, i])
    Q = (hs[0] ** p - hs[1] ** p) / (hs[0] ** p - hs[2] ** p)
    measured = (vals[0] - vals[1]) / (vals[0] - vals[2])
    assert abs(measured - Q) < 0.02 * Q


# --- enforcement, floors, ghosts ------------------------------------------------------

def test_stage_enforces_unit_determinant_and_traceless_At():
    bt = W.random_batch(5, nblocks=1, nmax=6, fd_order=4, amp=0.05)
    bt.params.ko_sigma = 0.1
    u0 = bt.u
    out = u0.copy()
    u1 = np.zeros_like(u0)
    O.rk_stage(bt, u0, out, u1, u0, O.RK4[0], 0.05)
    blk = bt.blocks[0]
    g = [bt.interior(out, 0, W.F[n]) for n in ("gxx", "gxy", "gxz", "gyy", "gyz", "gzz")]
    det = (g[0] * (g[3] * g[5] - g[4] ** 2) - g[1] * (g[1] * g[5] - g[4] * g[2])
           + g[2] * (g[1] * g[4] - g[3] * g[2]))
    np.testing.assert_allclose(det, 1.0, atol=2e-15)
    Gm = np.stack([np.stack([g[0], g[1], g[2]]), np.stack([g[1], g[3], g[4]]),
                   np.stack([g[2], g[4], g[5]])])
    Gi = np.linalg.inv(np.moveaxis(Gm, (0, 1), (-2, -1)))
    A = [bt.interior(out, 0, W.F[n]) for n in ("Axx", "Axy", "Axz", "Ayy", "Ayz", "Azz")]
    Am = np.moveaxis(np.stack([np.stack([A[0], A[1], A[2]]), np.stack([A[1], A[3], A[4]]),
                               np.stack([A[2], A[4], A[5]])]), (0, 1), (-2, -1))
    tr = np.einsum("...ij,...ij->...", Gi, Am)
    assert np.abs(tr).max() < 1e-16 + 1e-15 * np.abs(Am).max()
    assert blk.nx >= 1


def test_floors_clamp_chi_and_alpha():
    bt = W.random_batch(6, nblocks=1, nmax=5, fd_order=4, amp=0.01)
    u0 = bt.u.copy()
    for b in range(1):
        bt.view(u0, b, W.F["chi"])[...] = 1e-9
        bt.view(u0, b, W.F["alpha"])[...] = -3.0
    out = u0.copy()
    u1 = np.zeros_like(u0)
    c = dict(delta=0.0, eps=0.0, g1=1.0, g2=0.0, g3=0.0, beta=0.0, read_u1=0, write_u1=0)
    O.rk_stage(bt, u0, out, u1, u0, c, 0.1)
    assert np.all(bt.interior(out, 0, W.F["chi"]) == bt.params.chi_floor)
    assert np.all(bt.interior(out, 0, W.F["alpha"]) == bt.params.alpha_floor)


def test_ghost_fill_periodic_and_neighbour_index_maps():
    """Periodic refresh equals numpy's modular indexing of the interior; a
    2x1x1 neighbour tiling equals the periodic fill of the joined array
    along x (with frozen values on the open faces)."""
    rng = np.random.default_rng(3)
    blk = W.Block(5, 6, 7, 3, 1.0, 1.0, 1.0)
    bt = W.Batch([blk])
    bt.u[:] = rng.normal(size=bt.u.shape)
    O.ghost_fill(bt, bt.u, W.GHOST_PERIODIC)
    g = blk.ng
    for f in (0, 13, 21):
        v = bt.view(bt.u, 0, f)
        inner = v[g:-g, g:-g, g:-g]
        iz = (np.arange(blk.shape[0]) - g) % blk.nz
        iy = (np.arange(blk.shape[1]) - g) % blk.ny
        ix = (np.arange(blk.shape[2]) - g) % blk.nx
        np.testing.assert_array_equal(v, inner[np.ix_(iz, iy, ix)])
    # two blocks side by side along x, each periodic in y, z through the table
    b0 = W.Block(4, 5, 6, 3, 1.0, 1.0, 1.0)
    bt2 = W.Batch([b0, b0])
    bt2.u[:] = rng.normal(size=bt2.u.shape)
    nbr = np.full((2, 27), -1, dtype=np.int32)
    for b in range(2):
        for oz in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for ox in (-1, 0, 1):
                    cx = b + ox
                    nbr[b, W.dir_index(ox, oy, oz)] = cx % 2   # periodic in x too
    bt2.neighbours = nbr
    O.ghost_fill(bt2, bt2.u, W.GHOST_NEIGHBOUR)
    for f in (2, 17):
        joined = np.concatenate([bt2.interior(bt2.u, 0, f), bt2.interior(bt2.u, 1, f)], axis=2)
        iz = (np.arange(b0.shape[0]) - g) % b0.nz
        iy = (np.arange(b0.shape[1]) - g) % b0.ny
        for b in range(2):
            ix = (np.arange(b0.shape[2]) - g + b * b0.nx) % (2 * b0.nx)
            np.testing.assert_array_equal(bt2.view(bt2.u, b, f), joined[np.ix_(iz, iy, ix)])
    # open faces: -1 entries take frozen values
    bt2.frozen = rng.normal(size=bt2.u.shape)
    nbr2 = nbr.copy()
    nbr2[0, :9] = -1   # oz = -1 side of block 0
    bt2.neighbours = nbr2
    O.ghost_fill(bt2, bt2.u, W.GHOST_NEIGHBOUR)
    v = bt2.view(bt2.u, 0, 5)
    fz = bt2.view(bt2.frozen, 0, 5)
    np.testing.assert_array_equal(v[:g], fz[:g])
