"""FP64 CPU oracle of the primitive <-> conservative maps of ideal GRMHD
(numpy / pure Python, one point at a time).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU
baseline leg, never by the product path; shares no code with the GPU library.

* p2c: the conservative variables of Sec. 2.2 (q = sqrt(gamma) (rho W,
  (rho h + b^2) W ut_j - alpha b^0 b_j, (rho h + b^2) W^2 - rho W - (p +
  b^2/2) - (alpha b^0)^2, B^k)), written out in the paper's notation with the
  comoving field b^0, b_i, b^2 of Sec. 2.2; ideal gas p = (Gamma - 1) rho eps.
* c2p: the inverse of p2c by its definition: with z = rho h W^2, the
  conservatives satisfy (derived from the formulas above)
      S_j   = (z + B^2) v_j - (B.v) B_j,       B.v = (S.B) / z,
      S^2   = (z + B^2)^2 v^2 - (2 z + B^2) (B.v)^2,
      tau + D = z + B^2 - p - B^2 / (2 W^2) - (B.v)^2 / 2,
  so v^2(z) and W(z) are explicit, rho = D / W, p = (Gamma - 1)/Gamma (z /
  W^2 - rho), and the energy equation is one equation in z, solved here by
  plain bisection to the last bit after a scan for the sign change above the
  smallest z with v < 1.  This is
  a different route from the GPU kernel's (a root of the master function in
  mu = 1 / (h W) of Kastaun, Kalinani & Ciolfi, which the paper's primitive
  solver follows); both must agree with p2c's inverse.
"""
from __future__ import annotations

import math

import numpy as np


def p2c(rho, ut, p, B, gam, gamma_ad, alpha=1.0, beta=(0.0, 0.0, 0.0)):
    """Conservatives (D, S_j[3], tau, Bcons^k[3]) of one point (Sec. 2.2).
    ut: ut^i; B: Eulerian B^i; gam: gamma_ij (3x3)."""
    gam = np.asarray(gam, dtype=float)
    ut = np.asarray(ut, dtype=float)
    B = np.asarray(B, dtype=float)
    beta = np.asarray(beta, dtype=float)
    sg = math.sqrt(np.linalg.det(gam))
    W = math.sqrt(1.0 + ut @ gam @ ut)
    v_up = ut / W
    v_lo = gam @ v_up
    ut_lo = gam @ ut
    eps = p / ((gamma_ad - 1.0) * rho)
    h = 1.0 + eps + p / rho
    b0 = W * (B @ v_lo) / alpha
    b_up = (B + alpha * b0 * W * (v_up - beta / alpha)) / W
    b_lo = gam @ b_up + (gam @ beta) * b0
    b2 = ((alpha * b0) ** 2 + B @ gam @ B) / W ** 2
    D = sg * rho * W
    S = sg * ((rho * h + b2) * W * ut_lo - alpha * b0 * b_lo)
    tau = sg * ((rho * h + b2) * W ** 2 - rho * W - (p + 0.5 * b2) - (alpha * b0) ** 2)
    return D, S, tau, sg * B


def _state(z, D, S2, SB, B2, E, gamma_ad):
    """v^2, W, rho, p and the energy residual at z = rho h W^2."""
    v2 = (S2 + (2.0 * z + B2) * SB * SB / (z * z)) / ((z + B2) ** 2)
    if not v2 < 1.0:
        return None
    W = 1.0 / math.sqrt(1.0 - v2)
    rho = D / W
    p = (gamma_ad - 1.0) / gamma_ad * (z / (W * W) - rho)
    res = z + B2 - p - B2 / (2.0 * W * W) - SB * SB / (2.0 * z * z) - E
    return v2, W, rho, p, res


def c2p(D, S, tau, Bc, gam, gamma_ad):
    """Primitives (rho, ut^i[3], p) whose p2c is (D, S_j, tau, Bc^k), by the
    definition; raises if no physical solution is found."""
    gam = np.asarray(gam, dtype=float)
    sg = math.sqrt(np.linalg.det(gam))
    gi = np.linalg.inv(gam)
    D, tau = D / sg, tau / sg
    S = np.asarray(S, dtype=float) / sg
    B = np.asarray(Bc, dtype=float) / sg
    S2 = S @ gi @ S
    B2 = B @ gam @ B
    SB = S @ B
    E = tau + D
    # physical states have z >= D (h >= 1, W >= 1) and v^2(z) < 1, i.e.
    # g(z) = (z + B^2)^2 - S^2 - (2 z + B^2)(S.B)^2 / z^2 > 0; g increases
    # with z, so the admissible z form an interval (z0, inf): find z0 by
    # bisection, then scan upward from it on a geometric grid of offsets for
    # the sign change of the energy residual
    def g(z):
        return (z + B2) ** 2 - S2 - (2.0 * z + B2) * SB * SB / (z * z)

    z0 = D
    if not g(D) > 0.0:
        a, b = D, 2.0 * D
        while not g(b) > 0.0:
            a, b = b, 2.0 * b
        for _ in range(200):
            m = 0.5 * (a + b)
            if m <= a or m >= b:
                break
            if g(m) > 0.0:
                b = m
            else:
                a = m
        z0 = b
    prev = None
    lo = hi = None
    for off in np.logspace(-15.0, 9.0, 6000):
        z = z0 * (1.0 + off)
        st = _state(z, D, S2, SB, B2, E, gamma_ad)
        if st is None:
            prev = None
            continue
        if prev is not None and (prev[1] <= 0.0) != (st[4] <= 0.0):
            lo, hi = prev[0], z
            break
        prev = (z, st[4])
    if lo is None:
        raise ValueError("no sign change of the energy residual")
    flo = _state(lo, D, S2, SB, B2, E, gamma_ad)[4]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        fm = _state(mid, D, S2, SB, B2, E, gamma_ad)[4]
        if (fm <= 0.0) == (flo <= 0.0):
            lo, flo = mid, fm
        else:
            hi = mid
    z = 0.5 * (lo + hi)
    v2, W, rho, p, _ = _state(z, D, S2, SB, B2, E, gamma_ad)
    Bv = SB / z
    v_lo = (S + Bv * gam @ B) / (z + B2)
    ut = W * (gi @ v_lo)
    return rho, ut, p
