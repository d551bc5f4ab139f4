"""Closed-form semi-discrete evolution of a small plane-wave perturbation of
flat space (test infrastructure).

Background: chi = alpha = 1, gt = delta, everything else 0.  A perturbation
depending on x_d only, v_f = Re(c_f exp(i k x_d)), evolves under the
linearisation of the Z4c system (1+log lapse, Gamma-driver shift with
coefficient 1 and damping eta, constraint damping kappa1, kappa2) about
flat space.  With n = e_d and the discrete operators replaced by their
Fourier symbols

    D1  ->  i k1,   k1 = (1/h) sum_m w_m 2 sin(m k h)     (central, order p)
    D2  ->  -k2sq,  k2sq = -(1/h^2) sum_m v_m 2 (cos(m k h) - 1)
    KO  ->  -(sigma/h) sin(k h / 2)^(2r),   r = p/2 + 1   (only along d)

the linear system (c = chi - 1, h_ij = gt_ij - delta_ij, a = alpha - 1) is

  c'     = 2/3 (Khat + 2 Theta) - 2/3 D beta^d
  h_ij'  = -2 At_ij + n_j D beta^i + n_i D beta^j - 2/3 delta_ij D beta^d
  Khat'  = -D2 a + kappa1 (1 - kappa2) Theta
  At_ij' = [X]^TF,  X_ij = -n_i n_j D2 a + R_ij,
           R_ij  = -1/2 D2 h_ij + 1/2 (n_j D Gt^i + n_i D Gt^j)
                   + 1/2 (n_i n_j + delta_ij) D2 c
  Theta' = 1/2 tr R - kappa1 (2 + kappa2) Theta
  Gt^i'  = D2 beta^i + 1/3 n^i D2 beta^d - 2/3 n^i D (2 Khat + Theta)
           - 2 kappa1 (Gt^i - Gd^i),   Gd^i = n_k D h_ik - 1/2 n_i D tr h
  a'     = -2 Khat
  beta^i'= Gt^i - eta beta^i
plus the KO symbol on every field.  The linearisation drops every product of
perturbations (advection, Christoffel products, At^2, K^2, ...).
"""
from __future__ import annotations

import math

import numpy as np

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
CHI, GXX, KHAT, AXX, THETA, GAM, ALPHA, BETA = 0, 1, 7, 8, 14, 15, 18, 19

_W1 = {4: [(1, 8.0 / 12.0), (2, -1.0 / 12.0)],
       6: [(1, 45.0 / 60.0), (2, -9.0 / 60.0), (3, 1.0 / 60.0)]}
_W2 = {4: [(1, 16.0 / 12.0), (2, -1.0 / 12.0)],
       6: [(1, 270.0 / 180.0), (2, -27.0 / 180.0), (3, 2.0 / 180.0)]}


def symbols(k, h, p, sigma):
    k1 = sum(w * 2.0 * math.sin(m * k * h) for m, w in _W1[p]) / h
    k2sq = -sum(w * 2.0 * (math.cos(m * k * h) - 1.0) for m, w in _W2[p]) / (h * h)
    r = p // 2 + 1
    ko = -(sigma / h) * math.sin(0.5 * k * h) ** (2 * r)
    return k1, k2sq, ko


def sidx(i, j):
    return SYM.index((min(i, j), max(i, j)))


def matrix(k, h, p, sigma, d, kappa1, kappa2, eta):
    """22x22 complex matrix M with d/dt c = M c for the modal amplitudes."""
    k1, k2sq, ko = symbols(k, h, p, sigma)
    D = 1j * k1
    D2 = -k2sq
    n = [1.0 if a == d else 0.0 for a in range(3)]
    M = np.zeros((22, 22), dtype=complex)
    # chi
    M[CHI, KHAT] += 2.0 / 3.0
    M[CHI, THETA] += 4.0 / 3.0
    M[CHI, BETA + d] += -2.0 / 3.0 * D
    # gt_ij
    for a, (i, j) in enumerate(SYM):
        M[GXX + a, AXX + a] += -2.0
        M[GXX + a, BETA + i] += n[j] * D
        M[GXX + a, BETA + j] += n[i] * D
        if i == j:
            M[GXX + a, BETA + d] += -2.0 / 3.0 * D
    # Khat
    M[KHAT, ALPHA] += -D2
    M[KHAT, THETA] += kappa1 * (1.0 - kappa2)
    # R_ij as rows over the 22 amplitudes
    R = np.zeros((3, 3, 22), dtype=complex)
    for i in range(3):
        for j in range(3):
            R[i, j, GXX + sidx(i, j)] += -0.5 * D2
            R[i, j, GAM + i] += 0.5 * n[j] * D
            R[i, j, GAM + j] += 0.5 * n[i] * D
            R[i, j, CHI] += 0.5 * (n[i] * n[j] + (1.0 if i == j else 0.0)) * D2
    Xm = R.copy()
    for i in range(3):
        for j in range(3):
            Xm[i, j, ALPHA] += -n[i] * n[j] * D2
    trX = sum(Xm[i, i] for i in range(3))
    for a, (i, j) in enumerate(SYM):
        M[AXX + a] += Xm[i, j] - (trX / 3.0 if i == j else 0.0)
    # Theta
    trR = sum(R[i, i] for i in range(3))
    M[THETA] += 0.5 * trR
    M[THETA, THETA] += -kappa1 * (2.0 + kappa2)
    # Gamma-tilde
    for i in range(3):
        M[GAM + i, BETA + i] += D2
        M[GAM + i, BETA + d] += n[i] * D2 / 3.0
        M[GAM + i, KHAT] += -2.0 / 3.0 * n[i] * D * 2.0
        M[GAM + i, THETA] += -2.0 / 3.0 * n[i] * D
        M[GAM + i, GAM + i] += -2.0 * kappa1
        # + 2 kappa1 Gd^i
        for kk in range(3):
            M[GAM + i, GXX + sidx(i, kk)] += 2.0 * kappa1 * n[kk] * D
        for jj in range(3):
            M[GAM + i, GXX + sidx(jj, jj)] += -2.0 * kappa1 * 0.5 * n[i] * D
    # gauge
    M[ALPHA, KHAT] += -2.0
    for i in range(3):
        M[BETA + i, GAM + i] += 1.0
        M[BETA + i, BETA + i] += -eta
    M += ko * np.eye(22)
    return M


def rk_polynomial(Z, table="rk4"):
    I = np.eye(Z.shape[0], dtype=complex)
    if table == "rk4":
        return I + Z + Z @ Z / 2.0 + Z @ Z @ Z / 6.0 + Z @ Z @ Z @ Z / 24.0
    return I + Z + Z @ Z / 2.0 + Z @ Z @ Z / 6.0


def random_amplitudes(rng):
    """Complex amplitudes with traceless gt and At perturbations (so that the
    algebraic det/trace enforcement acts only at second order)."""
    c = rng.normal(size=22) + 1j * rng.normal(size=22)
    for base in (GXX, AXX):
        tr = c[base + 0] + c[base + 3] + c[base + 5]
        c[base + 0] -= tr / 3.0
        c[base + 3] -= tr / 3.0
        c[base + 5] -= tr / 3.0
    return c


def field_values(c, coord, k):
    """Real perturbation values Re(c_f exp(i k x)) for all 22 fields."""
    e = np.exp(1j * k * coord)
    return [np.real(c[f] * e) for f in range(22)]
