"""Pins of the intergrid oracle (oracle/intergrid.py), CPU only: vertex-
centred prolongation reproduces tensor-product polynomials of degree
< order along each direction bitwise (integer coarse coordinates, fine ones
half-integers, all values dyadic) and fails one degree higher; restriction
of a prolongation returns the coarse data bitwise (even fine vertices copy
coarse vertices, injection takes them back)."""
import numpy as np
import pytest

from oracle import intergrid as OI
from paper_2311_04989_amd import workloads as W


def _poly(X, Y, Z, a, b, c):
    return (X ** a - 2 * X + 3) * (Y ** b + Y - 1) * (2 * Z ** c - Z + 5)


def _ghost_boxes(blk):
    """The six ghost slabs of a block (destination boxes of a prolongation)."""
    n, g = blk.nx, blk.ng
    full = (-g, n + g)
    boxes = []
    for d in range(3):
        for lo, hi in ((-g, 0), (n, n + g)):
            b_lo, b_hi = [full[0]] * 3, [full[1]] * 3
            b_lo[d], b_hi[d] = lo, hi
            boxes.append((b_lo, b_hi))
    return boxes


@pytest.mark.parametrize("order", [2, 4, 6])
def test_prolongation_exact_on_polynomials(order):
    deg = order - 1
    for d in range(3):
        for extra, exact in ((0, True), (1, False)):
            degs = [0, 0, 0]
            degs[d] = deg + extra
            bt, origins = W.refined_pair(fill=lambda X, Y, Z, f: _poly(X, Y, Z, *degs) + f)
            tr = [dict(coarse=0, fine=1 + m, c0=origins[m], lo=lo, hi=hi)
                  for m in range(len(origins)) for lo, hi in _ghost_boxes(bt.blocks[1 + m])]
            out = OI.prolong(bt, bt.u, tr, order)
            ok = True
            for m in range(len(origins)):
                blk = bt.blocks[1 + m]
                X, Y, Z = blk.coords()
                for f in range(W.NF):
                    ok &= np.array_equal(bt.view(out, 1 + m, f), _poly(X, Y, Z, *degs) + f)
            assert ok == exact, (order, degs)


def test_restriction_inverts_prolongation_on_coincident_points():
    bt, origins = W.refined_pair(seed=3)
    fine_all = [dict(coarse=0, fine=1 + m, c0=origins[m], lo=[-4] * 3, hi=[20] * 3)
                for m in range(len(origins))]
    u1 = OI.prolong(bt, bt.u, fine_all, 6)
    back = [dict(coarse=0, fine=1 + m, c0=origins[m], lo=list(origins[m]),
                 hi=[origins[m][0] + 8, origins[m][1] + 8, origins[m][2] + 8])
            for m in range(len(origins))]
    u2 = OI.restrict(bt, u1, back)
    for f in range(W.NF):          # the coarse block is back bit for bit
        assert np.array_equal(bt.view(u2, 0, f), bt.view(bt.u, 0, f))
    # and restriction really reads the fine block: perturb it, the coarse values follow
    for m in range(len(origins)):
        for f in range(W.NF):
            bt.view(u1, 1 + m, f)[...] += 1.0
    u3 = OI.restrict(bt, u1, back)
    diff = sum(np.count_nonzero(bt.view(u3, 0, f) - bt.view(bt.u, 0, f)) for f in range(W.NF))
    assert diff == W.NF * len(origins) * 8 ** 3
