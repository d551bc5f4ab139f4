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


def level_exchange(batch, locs, u, frozen=None, order=6, acc=np.float64):
    """Refresh every ghost point of every block of a multi-level set from the
    block that owns its position (Sec. 3.1: blocks of an oct-tree level set
    with ghost zones; Sec. 3.2: vertex-centred data moved between levels by
    restriction and prolongation), on a copy of u.

    Positions live on the integer lattice of the finest level: block b of
    level L has its vertex i at o_b + i s_L (s_L = 2^(Lmax - L)) and owns the
    half-open span [o_b, o_b + n s_L) per direction.  A ghost point takes
      * the owner's vertex, when the owner is on the same level (copy);
      * the owner's coincident vertex, when the owner is one level finer
        (injection);
      * the tensor product of the direction rules of `prolong` applied to
        the owner's stored points, when the owner is one level coarser;
      * `frozen` (if given, else its stored value), when no block owns it.
    Copies and injections read interior vertices only and run first;
    interpolations read the coarse block's ghosts as well and run level by
    level, coarsest first, so that every point they read is already current.
    `acc` is the type the interpolation sums are formed in (numpy.longdouble
    for the extended-precision reference); results are stored as double."""
    from paper_2311_04989_amd.workloads import NF
    out = u.copy()
    lmax = max(L for L, _ in locs)
    st = [1 << (lmax - L) for L in range(lmax + 1)]
    blocks = batch.blocks
    spans = [(np.array(o), np.array(o) + np.array([b.nx, b.ny, b.nz]) * st[L])
             for b, (L, o) in zip(blocks, locs)]

    def owner(X):
        """Owner index per point (N, 3) -> (N,), -1 where none."""
        res = np.full(len(X), -1, dtype=np.int64)
        for ob, (lo, hi) in enumerate(spans):
            inside = np.all((X >= lo) & (X < hi), axis=1)
            assert not np.any(res[inside] >= 0), "spans overlap"
            res[inside] = ob
        return res

    def view(arr, b, f):
        return batch.view(arr, b, f)

    w_mid = midpoint_weights(order)
    pending = []     # (level, block, idx (N,3) stored indices, owner, X)
    for b, (blk, (L, o)) in enumerate(zip(blocks, locs)):
        g = blk.ng
        k, j, i = np.meshgrid(np.arange(-g, blk.nz + g), np.arange(-g, blk.ny + g),
                              np.arange(-g, blk.nx + g), indexing="ij")
        ghost = ~((i >= 0) & (i < blk.nx) & (j >= 0) & (j < blk.ny) & (k >= 0) & (k < blk.nz))
        I = np.stack([i[ghost], j[ghost], k[ghost]], axis=1)        # (N, 3) x, y, z
        X = np.array(o) + I * st[L]
        own = owner(X)
        dst = I + g                                                  # stored indices
        for ob in np.unique(own):
            sel = own == ob
            if ob < 0:
                if frozen is not None:
                    for f in range(NF):
                        view(out, b, f)[dst[sel, 2], dst[sel, 1], dst[sel, 0]] = \
                            view(frozen, b, f)[dst[sel, 2], dst[sel, 1], dst[sel, 0]]
                continue
            Lo, oo = locs[ob]
            if Lo == L - 1:
                pending.append((L, b, dst[sel], ob, X[sel]))
                continue
            assert Lo in (L, L + 1), "levels of neighbouring blocks differ by more than one"
            rel = X[sel] - np.array(oo)
            assert np.all(rel % st[Lo] == 0)
            src = rel // st[Lo] + blocks[ob].ng
            for f in range(NF):
                view(out, b, f)[dst[sel, 2], dst[sel, 1], dst[sel, 0]] = \
                    view(u, ob, f)[src[:, 2], src[:, 1], src[:, 0]]
    # interpolation from the coarser owner, coarse levels first
    for L, b, dst, ob, X in sorted(pending, key=lambda p: p[0]):
        Lo, oo = locs[ob]
        cng = blocks[ob].ng
        rel2 = 2 * (X - np.array(oo)) // st[Lo]       # twice the coarse index
        for parity in {tuple(p) for p in (rel2 % 2)}:
            sel = np.all(rel2 % 2 == np.array(parity), axis=1)
            taps = []
            for d in range(3):
                if parity[d] == 0:
                    taps.append(([0], [1.0]))
                else:
                    taps.append((list(range(-(order // 2 - 1), order // 2 + 1)), list(w_mid)))
            base = rel2[sel] // 2 + cng            # left coarse node (stored index)
            for f in range(NF):
                src = view(out, ob, f)
                total = np.zeros(int(sel.sum()), dtype=acc)
                for oz, wz in zip(*taps[2]):
                    for oy, wy in zip(*taps[1]):
                        for ox, wx in zip(*taps[0]):
                            total += acc(wx * wy * wz) * src[base[:, 2] + oz, base[:, 1] + oy,
                                                             base[:, 0] + ox].astype(acc)
                view(out, b, f)[dst[sel, 2], dst[sel, 1], dst[sel, 0]] = total.astype(np.float64)
    return out


def rk_step_levels(batch, locs, u, table, dt, orc, frozen=None, order=6, ext=False):
    """One Runge-Kutta step of every block of a multi-level set with the
    oracle's stage (`orc.rk_stage`), with batch.sommerfeld the radiative
    stage of the outer ghost points (`orc.sommerfeld_stage`, batch.neighbours
    the same-level table), and after every stage the ghost exchange
    `level_exchange` (one global time step for all levels).  Returns the new
    state (a new array)."""
    y = u
    u1 = np.zeros_like(u)
    cur = u
    for c in table:
        nxt = cur.copy()
        orc.rk_stage(batch, cur, nxt, u1, y, c, dt, ext=ext)
        if getattr(batch, "sommerfeld", False):
            # radiative law on the ghost regions without a same-level
            # neighbour; the exchange below overwrites those another level
            # owns, so only points no block owns keep it
            orc.sommerfeld_stage(batch, cur, nxt, u1, y, c, dt, ext=ext)
        nxt = level_exchange(batch, locs, nxt, frozen, order,
                             acc=np.longdouble if ext else np.float64)
        cur = nxt
    return cur
