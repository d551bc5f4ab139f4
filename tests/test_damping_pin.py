"""Pin of the Gamma-tilde damping term of the oracle (CPU only).

The paper gives kappa1 but not the form of the term; the reading taken is
-2 alpha kappa1 (Gt^i - Gt_d^i), with Gt_d^i = gt^{jk} Gt^i_jk from the
metric derivatives.  On data where Gt^i differs from Gt_d^i, with Theta = 0
(so no other kappa1 term acts) and a non-constant lapse alpha != 1, the
kappa1-dependent part of the right-hand side of Gt^i must be exactly that
term.  Gt_d is computed here from the analytic derivatives of a quadratic
conformal metric (which the order-4 stencils differentiate exactly), not
from the oracle's stencils; a dropped alpha, a wrong sign or a wrong
contraction fails."""
import numpy as np
import pytest

import oracle as O
from paper_2311_04989_amd import workloads as W

# gt_ij = delta_ij + eps * (a_ij x y + b_ij z^2 + c_ij x), symmetric a, b, c
EPS = 0.05
RNG = np.random.default_rng(17)
A, B, C = (lambda m: (m + m.T) / 2)(RNG.normal(size=(3, 3))), \
    (lambda m: (m + m.T) / 2)(RNG.normal(size=(3, 3))), \
    (lambda m: (m + m.T) / 2)(RNG.normal(size=(3, 3)))


def metric(x, y, z):
    return np.eye(3) + EPS * (A * x * y + B * z * z + C * x)


def dmetric(x, y, z):
    """d_k gt_ij as [k][i][j]."""
    return EPS * np.array([A * y + C, A * x, 2.0 * B * z])


def gamma_d(x, y, z):
    g = metric(x, y, z)
    gi = np.linalg.inv(g)
    dg = dmetric(x, y, z)
    # Gt_{k ij} = 1/2 (d_i g_jk + d_j g_ik - d_k g_ij)
    Gl = 0.5 * (np.einsum("ijk->kij", dg) + np.einsum("jik->kij", dg) - dg)
    Gu = np.einsum("il,ljk->ijk", gi, Gl)
    return np.einsum("jk,ijk->i", gi, Gu)


@pytest.mark.parametrize("kappa1", [0.3, 0.02])
def test_gamma_damping_term(kappa1):
    n, ng, h = 8, 3, 0.07
    bt = W.Batch([W.Block(n, n, n, ng, h, h, h, x0=0.2, y0=-0.3, z0=0.15)], with_matter=False)
    X, Y, Zc = bt.blocks[0].coords()
    F = W.F
    names = ["gxx", "gxy", "gxz", "gyy", "gyz", "gzz"]
    pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for nm, (i, j) in zip(names, pairs):
        bt.view(bt.u, 0, F[nm])[...] = (i == j) + EPS * (A[i, j] * X * Y + B[i, j] * Zc * Zc
                                                         + C[i, j] * X)
    bt.view(bt.u, 0, F["chi"])[...] = 1.0
    bt.view(bt.u, 0, F["alpha"])[...] = 0.6 + 0.1 * X
    gam = (0.11, -0.23, 0.07)
    for k, nm in enumerate(("Gx", "Gy", "Gz")):
        bt.view(bt.u, 0, F[nm])[...] = gam[k]
    common = dict(fd_order=4, ko_sigma=0.0, lapse=W.LAPSE_FROZEN, shift=W.SHIFT_FROZEN,
                  eta=0.0, advect_gauge=0, kappa2=0.3)
    bt.params = W.Params(kappa1=kappa1, **common)
    r1 = O.rhs(bt)
    bt.params = W.Params(kappa1=0.0, **common)
    r0 = O.rhs(bt)
    for i, nm in enumerate(("Gx", "Gy", "Gz")):
        got = bt.interior(r1, 0, F[nm]) - bt.interior(r0, 0, F[nm])
        g = ng
        xs, ys, zs = X[g:-g, g:-g, g:-g], Y[g:-g, g:-g, g:-g], Zc[g:-g, g:-g, g:-g]
        want = np.empty_like(got)
        for idx in np.ndindex(got.shape):
            x, y, z = xs[idx], ys[idx], zs[idx]
            want[idx] = -2.0 * (0.6 + 0.1 * x) * kappa1 * (gam[i] - gamma_d(x, y, z)[i])
        scale = np.abs(want).max()
        assert scale > 1e-4
        assert np.abs(got - want).max() <= 1e-12 * scale, (nm, np.abs(got - want).max(), scale)
