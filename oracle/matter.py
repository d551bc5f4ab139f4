"""FP64 CPU oracle of the matter coupling (numpy): Lagrange interpolation
between the vertex-centred Z4c grid and the cell-centred fluid grid, and the
ADM projections of the perfect-fluid / ideal-GRMHD stress-energy tensor.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU
baseline leg, never by the product path.  It shares no code with the GPU
library.  Every function is the definition written out, slowly:

* interpolation (Sec. 3.2, intergrid communication: Lagrange interpolation
  between the VC and CC representations, order chosen per variable): the
  value at a cell centre / vertex is the full tensor-product sum over the
  order^3 nearest input points with the 1-D Lagrange weights of the midpoint;
  the weights are computed here from the Lagrange basis in exact rationals.
* ADM sources: the projections rho_ADM, S_i ADM, S_ij ADM of the perfect
  fluid (Sec. 2.1) and of ideal GRMHD (Sec. 2.2), in the paper's notation,
  with the comoving field b^0, b^i, b^2 from its relations to the Eulerian
  field B^i; lapse and shift are explicit inputs (they cancel).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from paper_2311_04989_amd.workloads import NM, NGEOM


def midpoint_weights(order: int) -> np.ndarray:
    """Weights l_k(0) of the Lagrange basis on the nodes x_k = k - (order-1)/2
    (k = 0 .. order-1), i.e. at the midpoint of the two central nodes."""
    nodes = [Fraction(2 * k - (order - 1), 2) for k in range(order)]
    w = []
    for k, xk in enumerate(nodes):
        num, den = Fraction(1), Fraction(1)
        for m, xm in enumerate(nodes):
            if m != k:
                num *= (0 - xm)
                den *= (xk - xm)
        w.append(num / den)
    return np.array([float(x) for x in w])


def _tensor_interp(src: np.ndarray, starts, counts, order: int) -> np.ndarray:
    """out[k, j, i] = sum_{a,b,c} w_a w_b w_c src[s_z + k + c, s_y + j + b, s_x + i + a]
    with (s_x, s_y, s_z) = starts and (n_x, n_y, n_z) = counts."""
    w = midpoint_weights(order)
    sx, sy, sz = starts
    nx, ny, nz = counts
    out = np.zeros((nz, ny, nx))
    for c in range(order):
        for b in range(order):
            for a in range(order):
                out += w[a] * w[b] * w[c] * src[sz + c:sz + c + nz, sy + b:sy + b + ny,
                                                sx + a:sx + a + nx]
    return out


def metric_to_cc(mb, order: int, ext: int, u: np.ndarray = None) -> np.ndarray:
    """chi and gt_ij (state fields 0..6) at cells [-ext, nc + ext) of every
    block; a cell centre uses vertices i - order/2 + 1 .. i + order/2.
    Returns a CC geometry array (cells outside the range left at zero)."""
    u = mb.u if u is None else u
    geom = np.zeros_like(mb.geom)
    for b, blk in enumerate(mb.blocks):
        n = (blk.ncx, blk.ncy, blk.ncz)
        start = [-ext - order // 2 + 1 + blk.ngv] * 3     # stored vertex index
        counts = [m + 2 * ext for m in n]
        for f in range(NGEOM):
            val = _tensor_interp(mb.view("u", u, b, f), start, counts, order)
            g0 = blk.ngc - ext
            mb.view("geom", geom, b, f)[g0:g0 + counts[2], g0:g0 + counts[1], g0:g0 + counts[0]] = val
    return geom


def sources_to_vc(mb, order: int, adm: np.ndarray = None) -> np.ndarray:
    """The 10 ADM fields at vertices [0, nc] of every block; a vertex uses
    cells i - order/2 .. i + order/2 - 1.  Returns a VC matter array (ghost
    vertices left at zero)."""
    adm = mb.adm if adm is None else adm
    matter = np.zeros_like(mb.matter)
    for b, blk in enumerate(mb.blocks):
        counts = [blk.ncx + 1, blk.ncy + 1, blk.ncz + 1]
        start = [blk.ngc - order // 2] * 3                 # stored cell index
        for f in range(NM):
            val = _tensor_interp(mb.view("adm", adm, b, f), start, counts, order)
            g = blk.ngv
            mb.view("matter", matter, b, f)[g:g + counts[2], g:g + counts[1], g:g + counts[0]] = val
    return matter


def adm_point(rho, ut, p, Bv, gam, gamma_ad, alpha=1.0, beta=(0.0, 0.0, 0.0)):
    """ADM projections at one point, in the paper's notation (Sec. 2.1, 2.2).

    rho, p: rest-mass density and pressure; ut: ut^i (contravariant); Bv:
    Eulerian B^i (None: perfect fluid); gam: 3x3 spatial metric gamma_ij;
    ideal gas p = (Gamma - 1) rho eps.  Returns (rho_ADM, S_i[3], S_ij[3x3])."""
    gam = np.asarray(gam, dtype=float)
    ut = np.asarray(ut, dtype=float)
    beta = np.asarray(beta, dtype=float)
    eps = p / ((gamma_ad - 1.0) * rho) if rho != 0.0 else 0.0
    rhoh = rho * (1.0 + eps) + p if rho != 0.0 else gamma_ad / (gamma_ad - 1.0) * p
    W = np.sqrt(1.0 + ut @ gam @ ut)          # W^2 = 1 + gamma_ij ut^i ut^j
    v_up = ut / W                             # v^i = ut^i / W
    v_lo = gam @ v_up                         # v_i
    if Bv is None:
        b0, b_lo, b2 = 0.0, np.zeros(3), 0.0
    else:
        Bv = np.asarray(Bv, dtype=float)
        b0 = W * (Bv @ v_lo) / alpha                             # b^0
        vt = v_up - beta / alpha                                 # v-tilde^i
        b_up = (Bv + alpha * b0 * W * vt) / W                    # b^i
        b_lo = gam @ b_up + gam @ beta * b0                      # b_i = g_{i mu} b^mu
        b2 = ((alpha * b0) ** 2 + Bv @ gam @ Bv) / W ** 2        # b^2
    e = (rhoh + b2) * W ** 2
    ptot = p + 0.5 * b2
    rho_adm = e - ptot - (alpha * b0) ** 2
    S = e * v_lo - alpha * b0 * b_lo
    Sij = e * np.outer(v_lo, v_lo) + ptot * gam - np.outer(b_lo, b_lo)
    return rho_adm, S, Sij


def adm_sources(mb, mhd: bool, gamma_ad: float, chi_floor: float, ext: int,
                geom: np.ndarray = None, prim: np.ndarray = None) -> np.ndarray:
    """adm_point at every cell [-ext, nc + ext) of every block (pure-Python
    loop over points: for small batches), with gamma_ij = gt_ij / max(chi,
    chi_floor).  Returns a CC ADM array (cells outside the range at zero)."""
    geom = mb.geom if geom is None else geom
    prim = mb.prim if prim is None else prim
    adm = np.zeros_like(mb.adm)
    sym = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for b, blk in enumerate(mb.blocks):
        g = [mb.view("geom", geom, b, f) for f in range(NGEOM)]
        w = [mb.view("prim", prim, b, f) for f in range(8)]
        out = [mb.view("adm", adm, b, f) for f in range(NM)]
        lo = blk.ngc - ext
        for k in range(lo, blk.ngc + blk.ncz + ext):
            for j in range(lo, blk.ngc + blk.ncy + ext):
                for i in range(lo, blk.ngc + blk.ncx + ext):
                    chi = max(g[0][k, j, i], chi_floor)
                    gam = np.zeros((3, 3))
                    for q, (a, c) in enumerate(sym):
                        gam[a, c] = gam[c, a] = g[1 + q][k, j, i] / chi
                    ut = [w[1][k, j, i], w[2][k, j, i], w[3][k, j, i]]
                    Bv = [w[5][k, j, i], w[6][k, j, i], w[7][k, j, i]] if mhd else None
                    r, S, Sij = adm_point(w[0][k, j, i], ut, w[4][k, j, i], Bv, gam, gamma_ad)
                    out[0][k, j, i] = r
                    for a in range(3):
                        out[1 + a][k, j, i] = S[a]
                    for q, (a, c) in enumerate(sym):
                        out[4 + q][k, j, i] = Sij[a, c]
    return adm
