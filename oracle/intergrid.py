"""FP64 CPU oracle of the vertex-centred intergrid operators between
refinement levels (numpy, point by point).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, never by the product path;
shares no code with the GPU library.

Vertex-centred refinement by 2 (Sec. 3.2: the Z4c variables live on a
vertex-centred grid so that restriction and prolongation between refinement
levels stay simple with high-order operators): fine vertex i of a fine
block sits at coarse position c0 + i/2 of its coarse block (fine vertex 0 on
coarse vertex c0).
* prolongation (coarse -> fine): along each direction, an even fine index
  coincides with coarse vertex c0 + i/2 (the value is copied); an odd one
  lies midway between c0 + (i-1)/2 and c0 + (i+1)/2 and takes the Lagrange
  polynomial through the `order` nearest coarse vertices (symmetric);
  in 3-D the tensor product of the three rules (applied one direction after
  the other with numpy.tensordot).
* restriction (fine -> coarse): injection, coarse vertex j takes the fine
  value at i = 2 (j - c0).
"""
from __future__ import annotations

import numpy as np

from oracle.matter import midpoint_weights


def _rule(i: int, c0: int, order: int):
    """(coarse indices, weights) of fine index i along one direction."""
    if i % 2 == 0:
        return [c0 + i // 2], np.array([1.0])
    left = c0 + (i - 1) // 2
    idx = [left - (order // 2 - 1) + k for k in range(order)]
    return idx, midpoint_weights(order)


def _matrix(lo: int, hi: int, c0: int, cng: int, ncs: int, order: int) -> np.ndarray:
    """Interpolation matrix of one direction: row r (fine index lo + r) holds
    the weights of the stored coarse points (index + cng) of its rule."""
    M = np.zeros((hi - lo, ncs))
    for r, i in enumerate(range(lo, hi)):
        idx, w = _rule(i, c0, order)
        for c, wc in zip(idx, w):
            M[r, c + cng] += wc
    return M


def prolong(batch, u, transfers, order):
    """Apply every prolongation transfer (dict with coarse, fine, c0, lo, hi)
    to a copy of the state array u: the tensor product of the three
    direction rules, applied one direction after the other."""
    out = u.copy()
    from paper_2311_04989_amd.workloads import NF
    for t in transfers:
        cb, fb = t["coarse"], t["fine"]
        cblk = batch.blocks[cb]
        cng, fng = cblk.ng, batch.blocks[fb].ng
        shp = cblk.shape                                  # (z, y, x) stored
        Mx = _matrix(t["lo"][0], t["hi"][0], t["c0"][0], cng, shp[2], order)
        My = _matrix(t["lo"][1], t["hi"][1], t["c0"][1], cng, shp[1], order)
        Mz = _matrix(t["lo"][2], t["hi"][2], t["c0"][2], cng, shp[0], order)
        for f in range(NF):
            src = batch.view(u, cb, f)
            v = np.tensordot(src, Mx, axes=([2], [1]))                    # (z, y, X)
            v = np.tensordot(v, My, axes=([1], [1]))                      # (z, X, Y)
            v = np.tensordot(v, Mz, axes=([0], [1]))                      # (X, Y, Z)
            dst = batch.view(out, fb, f)
            dst[t["lo"][2] + fng:t["hi"][2] + fng, t["lo"][1] + fng:t["hi"][1] + fng,
                t["lo"][0] + fng:t["hi"][0] + fng] = np.transpose(v, (2, 1, 0))
    return out


def restrict(batch, u, transfers):
    """Apply every restriction transfer (coarse box lo..hi) to a copy of u."""
    out = u.copy()
    from paper_2311_04989_amd.workloads import NF
    for t in transfers:
        cb, fb = t["coarse"], t["fine"]
        cng, fng = batch.blocks[cb].ng, batch.blocks[fb].ng
        c0 = t["c0"]
        for f in range(NF):
            src = batch.view(u, fb, f)
            dst = batch.view(out, cb, f)
            for k in range(t["lo"][2], t["hi"][2]):
                for j in range(t["lo"][1], t["hi"][1]):
                    for i in range(t["lo"][0], t["hi"][0]):
                        dst[k + cng, j + cng, i + cng] = src[2 * (k - c0[2]) + fng,
                                                             2 * (j - c0[1]) + fng,
                                                             2 * (i - c0[0]) + fng]
    return out
