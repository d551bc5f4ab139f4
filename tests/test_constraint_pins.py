"""Pins of the oracle's constraint outputs that the other pins leave open
(CPU only): the Z^i vector and the per-block L1 / L2^2 norms.

Z^i = (Gt^i - Gt_d^i)/2 (constraint monitoring of the static star, Sec. 4.1;
Gt_d^i = gt^{jk} Gt^i_jk from the metric derivatives).  Every other pin runs
on data with Gt^i = Gt_d^i, where Z vanishes whatever its form; here Gt^i is a
constant and the conformal metric a quadratic polynomial, which the order-4
stencils differentiate exactly, so Gt_d follows from the analytic metric
derivatives (numpy, not the oracle's stencils).  A dropped 1/2 or a flipped
sign fails.

Norms: L1 = sum |c| dV and L2^2 = sum c^2 dV over interior points, dV =
dx dy dz.  On a block with three different spacings, flat conformal data and
Theta a separable polynomial, the constraints are known in closed form
(K = Khat + 2 Theta with Khat = 0, At = 0, flat metric):
    H = 2/3 K^2 = 8/3 Theta^2,   M_i = -2/3 d_i K = -4/3 d_i Theta,
    Theta,   Z^i = 0,
and each norm is a product of one-dimensional sums over the x, y and z
coordinates, evaluated here from those sums alone.  A volume element dx^3,
a missing dV or a sum over ghost points fails."""
import numpy as np
import pytest

import oracle as O
from paper_2311_04989_amd import workloads as W

F = W.F
CI = {n: i for i, n in enumerate(W.CONSTRAINTS)}

# gt_ij = delta_ij + eps (a_ij x y + b_ij z^2 + c_ij x), symmetric a, b, c
EPS = 0.05
RNG = np.random.default_rng(23)
A, B, C = [(lambda m: (m + m.T) / 2)(RNG.normal(size=(3, 3))) for _ in range(3)]


def metric(x, y, z):
    return np.eye(3) + EPS * (A * x * y + B * z * z + C * x)


def dmetric(x, y, z):
    """d_k gt_ij as [k][i][j]."""
    return EPS * np.array([A * y + C, A * x, 2.0 * B * z])


def gamma_d(x, y, z):
    g = metric(x, y, z)
    gi = np.linalg.inv(g)
    dg = dmetric(x, y, z)
    Gl = 0.5 * (np.einsum("ijk->kij", dg) + np.einsum("jik->kij", dg) - dg)   # Gt_{k ij}
    Gu = np.einsum("il,ljk->ijk", gi, Gl)
    return np.einsum("jk,ijk->i", gi, Gu)


def test_z_vector_is_half_the_gamma_mismatch():
    n, ng, h = 7, 3, 0.09
    bt = W.Batch([W.Block(n, n + 1, n - 1, ng, h, 0.8 * h, 1.1 * h, x0=0.1, y0=-0.2, z0=0.3)],
                 with_matter=False)
    X, Y, Zc = bt.blocks[0].coords()
    for nm, (i, j) in zip(["gxx", "gxy", "gxz", "gyy", "gyz", "gzz"], W.SYM):
        bt.view(bt.u, 0, F[nm])[...] = (i == j) + EPS * (A[i, j] * X * Y + B[i, j] * Zc * Zc
                                                         + C[i, j] * X)
    bt.view(bt.u, 0, F["chi"])[...] = 1.0
    bt.view(bt.u, 0, F["alpha"])[...] = 1.0
    gam = (0.13, -0.21, 0.05)
    for k, nm in enumerate(("Gx", "Gy", "Gz")):
        bt.view(bt.u, 0, F[nm])[...] = gam[k]
    bt.view(bt.u, 0, F["Theta"])[...] = 0.004 * X - 0.002
    bt.params = W.Params(fd_order=4, ko_sigma=0.0)
    cons, _ = O.constraints(bt)
    g = ng
    xs, ys, zs = X[g:-g, g:-g, g:-g], Y[g:-g, g:-g, g:-g], Zc[g:-g, g:-g, g:-g]
    for i, nm in enumerate(("Zx", "Zy", "Zz")):
        got = bt.interior(cons, 0, CI[nm], W.NC)
        want = np.empty_like(got)
        for idx in np.ndindex(got.shape):
            want[idx] = 0.5 * (gam[i] - gamma_d(xs[idx], ys[idx], zs[idx])[i])
        scale = np.abs(want).max()
        assert scale > 1e-3
        assert np.abs(got - want).max() <= 1e-13 * scale, (nm, np.abs(got - want).max(), scale)
    # the Theta constraint is the Theta field itself
    assert np.array_equal(bt.interior(cons, 0, CI["Theta"], W.NC),
                          bt.interior(bt.u, 0, F["Theta"]))


def _flat_theta_block(theta_fn, p):
    """One block with spacings 0.3, 0.17, 0.11, flat conformal data, Khat = 0
    and Theta = theta_fn(X, Y, Z) at every stored point."""
    blk = W.Block(5, 7, 6, p // 2 + 1, 0.3, 0.17, 0.11, x0=-0.4, y0=0.25, z0=0.6)
    bt = W.Batch([blk], with_matter=False)
    W.fill_fields(bt, W.flat)
    X, Y, Zc = blk.coords()
    bt.view(bt.u, 0, F["Theta"])[...] = theta_fn(X, Y, Zc)
    bt.params = W.Params(fd_order=p)
    return bt, blk


@pytest.mark.parametrize("p", [4, 6])
def test_norms_of_a_constant_theta(p):
    c = -0.37
    bt, blk = _flat_theta_block(lambda X, Y, Z: np.full_like(X, c), p)
    _, norms = O.constraints(bt, want_fields=False)
    npts = blk.nx * blk.ny * blk.nz
    dV = blk.dx * blk.dy * blk.dz
    want = {"Theta": (abs(c) * npts * dV, c * c * npts * dV),
            "H": (8.0 / 3.0 * c * c * npts * dV, (8.0 / 3.0 * c * c) ** 2 * npts * dV)}
    for nm, (l1, l2) in want.items():
        np.testing.assert_allclose(norms[0, CI[nm]], (l1, l2), rtol=1e-14, err_msg=nm)
    for nm in ("Mx", "My", "Mz", "Zx", "Zy", "Zz"):
        assert np.all(norms[0, CI[nm]] == 0.0), nm


@pytest.mark.parametrize("p", [4, 6])
def test_norms_of_a_separable_polynomial_theta(p):
    a, b, cc = 0.8, 1.3, -0.6
    fx = lambda x: 1.0 + a * x           # noqa: E731  positive on the block
    fy = lambda y: 2.0 + b * y * y       # noqa: E731
    fz = lambda z: 3.0 + cc * z          # noqa: E731
    bt, blk = _flat_theta_block(lambda X, Y, Z: fx(X) * fy(Y) * fz(Z), p)
    cons, norms = O.constraints(bt)
    x = blk.x0 + np.arange(blk.nx) * blk.dx   # interior coordinates only
    y = blk.y0 + np.arange(blk.ny) * blk.dy
    z = blk.z0 + np.arange(blk.nz) * blk.dz
    assert fx(x).min() > 0 and fz(z).min() > 0
    dV = blk.dx * blk.dy * blk.dz
    S = lambda v, k=1: float(np.sum(np.abs(v) ** k))   # noqa: E731
    # Theta = fx fy fz;  H = 8/3 Theta^2;  M_x = -4/3 a fy fz, M_y = -4/3 fx (2 b y) fz,
    # M_z = -4/3 fx fy cc  (the stencils are exact on these polynomials)
    want = {
        "Theta": (S(fx(x)) * S(fy(y)) * S(fz(z)), S(fx(x), 2) * S(fy(y), 2) * S(fz(z), 2)),
        "H": (8 / 3 * S(fx(x), 2) * S(fy(y), 2) * S(fz(z), 2),
              (8 / 3) ** 2 * S(fx(x), 4) * S(fy(y), 4) * S(fz(z), 4)),
        "Mx": (4 / 3 * abs(a) * blk.nx * S(fy(y)) * S(fz(z)),
               (4 / 3 * a) ** 2 * blk.nx * S(fy(y), 2) * S(fz(z), 2)),
        "My": (4 / 3 * S(fx(x)) * S(2 * b * y) * S(fz(z)),
               (4 / 3) ** 2 * S(fx(x), 2) * S(2 * b * y, 2) * S(fz(z), 2)),
        "Mz": (4 / 3 * abs(cc) * S(fx(x)) * S(fy(y)) * blk.nz,
               (4 / 3 * cc) ** 2 * S(fx(x), 2) * S(fy(y), 2) * blk.nz),
    }
    for nm, (l1, l2) in want.items():
        np.testing.assert_allclose(norms[0, CI[nm]], (l1 * dV, l2 * dV), rtol=1e-12,
                                   err_msg=nm)
    for nm in ("Zx", "Zy", "Zz"):
        assert np.all(norms[0, CI[nm]] == 0.0), nm
    # the pointwise fields behind the norms
    X, Y, Zc = blk.coords()
    g = blk.ng
    th = (fx(X) * fy(Y) * fz(Zc))[g:-g, g:-g, g:-g]
    np.testing.assert_allclose(bt.interior(cons, 0, CI["H"], W.NC), 8 / 3 * th ** 2, rtol=1e-13)
    np.testing.assert_allclose(bt.interior(cons, 0, CI["My"], W.NC),
                               -4 / 3 * (fx(X) * 2 * b * Y * fz(Zc))[g:-g, g:-g, g:-g],
                               rtol=1e-12, atol=1e-14)


def test_norms_sum_each_block_separately():
    """Two blocks with different spacings: each block's norms use its own dV
    and its own points only."""
    b0 = W.Block(4, 5, 6, 4, 0.2, 0.3, 0.5)
    b1 = W.Block(6, 3, 5, 4, 0.05, 0.07, 0.02)
    bt = W.Batch([b0, b1], with_matter=False)
    W.fill_fields(bt, W.flat)
    bt.view(bt.u, 0, F["Theta"])[...] = 0.5
    bt.view(bt.u, 1, F["Theta"])[...] = -2.0
    bt.params = W.Params(fd_order=6)
    _, norms = O.constraints(bt, want_fields=False)
    for b, c in ((0, 0.5), (1, -2.0)):
        blk = bt.blocks[b]
        nv = blk.nx * blk.ny * blk.nz * blk.dx * blk.dy * blk.dz
        np.testing.assert_allclose(norms[b, CI["Theta"]], (abs(c) * nv, c * c * nv), rtol=1e-14)
