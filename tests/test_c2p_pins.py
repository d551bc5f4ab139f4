"""Pins of the primitive <-> conservative oracle (oracle/c2p.py), CPU only.

* p2c against the ADM projections pinned in test_matter_pins.py (the energy
  and momentum densities seen by the Eulerian observer are the same physical
  quantities: (tau + D) / sqrt(gamma) = rho_ADM, S_j / sqrt(gamma) = S_j ADM)
  and its static and hydrodynamic limits.
* c2p as the inverse of p2c: primitives recovered to 1e-10 (the relative
  error the paper states for its primitive solver's self-consistency tests,
  Appendix A) on states up to W = 10 and magnetisation b^2 / rho = 10; the
  conservatives reproduced to 1e-12 on harder states (W up to 30, cold gas)
  whose primitives are ill-conditioned.
"""
import math

import numpy as np
import pytest

from oracle import c2p as OC
from oracle import matter as OM


def _metric(rng):
    while True:
        a = rng.normal(size=(3, 3))
        gam = np.eye(3) + 0.15 * (a + a.T)
        if np.all(np.linalg.eigvalsh(gam) > 0.3):
            return gam * rng.uniform(0.8, 3.0)


def _state(rng, wmax=10.0, cold=1e-3, mag=10.0):
    gam = _metric(rng)
    rho = 10 ** rng.uniform(-8, -2)
    p = rho * 10 ** rng.uniform(math.log10(cold), 1)
    d = rng.normal(size=3)
    d /= math.sqrt(d @ gam @ d)
    W = 10 ** rng.uniform(0, math.log10(wmax))
    ut = d * math.sqrt(W * W - 1.0)
    B = rng.normal(size=3)
    B *= math.sqrt(rho * 10 ** rng.uniform(-4, math.log10(mag)) / (B @ gam @ B))
    return gam, rho, ut, p, B


def test_p2c_energy_and_momentum_are_the_adm_projections():
    rng = np.random.default_rng(8)
    for _ in range(100):
        gam, rho, ut, p, B = _state(rng)
        alpha, beta = rng.uniform(0.4, 1.2), rng.uniform(-0.3, 0.3, size=3)
        D, S, tau, Bc = OC.p2c(rho, ut, p, B, gam, 5.0 / 3.0, alpha, beta)
        r, Sa, _ = OM.adm_point(rho, ut, p, B, gam, 5.0 / 3.0, alpha, beta)
        sg = math.sqrt(np.linalg.det(gam))
        assert (tau + D) / sg == pytest.approx(r, rel=1e-12)
        np.testing.assert_allclose(np.asarray(S) / sg, Sa, rtol=0, atol=1e-12 * r)
        np.testing.assert_allclose(Bc, sg * B, rtol=1e-15)


def test_p2c_limits():
    gam = np.array([[1.2, 0.1, 0.0], [0.1, 0.9, 0.05], [0.0, 0.05, 1.1]])
    sg = math.sqrt(np.linalg.det(gam))
    rho, p, G = 2e-3, 3e-4, 2.0
    eps = p / ((G - 1.0) * rho)
    D, S, tau, _ = OC.p2c(rho, np.zeros(3), p, np.zeros(3), gam, G)
    assert D == pytest.approx(sg * rho, rel=1e-15)
    assert np.all(np.asarray(S) == 0.0)
    assert tau == pytest.approx(sg * rho * eps, rel=1e-14)
    ut = np.array([0.3, -0.2, 0.5])
    W = math.sqrt(1.0 + ut @ gam @ ut)
    h = 1.0 + eps + p / rho
    D, S, tau, _ = OC.p2c(rho, ut, p, np.zeros(3), gam, G)
    assert D == pytest.approx(sg * rho * W, rel=1e-15)
    np.testing.assert_allclose(S, sg * rho * h * W * (gam @ ut), rtol=1e-14)
    assert tau == pytest.approx(sg * (rho * h * W * W - rho * W - p), rel=1e-13)


@pytest.mark.parametrize("mag", [0.0, 10.0])
def test_c2p_inverts_p2c(mag):
    rng = np.random.default_rng(21 if mag else 22)
    for _ in range(150):
        gam, rho, ut, p, B = _state(rng, mag=mag if mag > 0.0 else 1.0)
        if mag == 0.0:
            B = np.zeros(3)
        q = OC.p2c(rho, ut, p, B, gam, 5.0 / 3.0)
        r2, u2, p2 = OC.c2p(*q, gam, 5.0 / 3.0)
        assert abs(r2 - rho) <= 1e-10 * rho
        assert abs(p2 - p) <= 1e-10 * p
        assert np.abs(u2 - ut).max() <= 1e-10 * max(np.abs(ut).max(), 1.0)


def test_c2p_reproduces_conservatives_of_hard_states():
    rng = np.random.default_rng(23)
    for _ in range(100):
        gam, rho, ut, p, B = _state(rng, wmax=30.0, cold=1e-5, mag=100.0)
        q = OC.p2c(rho, ut, p, B, gam, 4.0 / 3.0)
        r2, u2, p2 = OC.c2p(*q, gam, 4.0 / 3.0)
        q2 = OC.p2c(r2, u2, p2, B, gam, 4.0 / 3.0)
        scale = q[0] + q[2]
        assert abs(q2[0] - q[0]) <= 1e-12 * scale
        assert abs(q2[2] - q[2]) <= 1e-12 * scale
        np.testing.assert_allclose(q2[1], q[1], rtol=0, atol=1e-12 * scale)
