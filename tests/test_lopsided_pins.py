"""Pins of the lopsided advection stencil of the oracle (CPU only).

The paper names no advection stencil; the lopsided reading taken here is
the first derivative of order p on the p + 1 points shifted by one towards
the sign of beta^k, whose weights are fixed by exactness on polynomials of
degree <= p.  Pinned here without the oracle's own solve:
* its weights equal the exact rational solution of the exactness conditions
  (fractions.Fraction elimination in this file) and fail at degree p + 1;
* the oracle's right-hand side of chi on flat space with a constant shift
  of mixed signs and chi - 1 a polynomial of degree p + 2 (where every
  stencil errs) equals beta^k times the shifted stencil evaluated exactly in
  rational arithmetic, in each direction towards the sign of beta^k;
* with data of degree <= p the lopsided and centred right-hand sides agree
  (both stencils exact), with degree p + 2 they do not.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2311_04989_amd import workloads as W


def exact_weights(p):
    """Solve sum_j w_j j^m = [m == 1], m = 0..p, offsets -p/2+1 .. p/2+1,
    in rational arithmetic."""
    offs = list(range(-p // 2 + 1, p // 2 + 2))
    n = len(offs)
    A = [[Fraction(o) ** m for o in offs] + [Fraction(int(m == 1))] for m in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return offs, [A[j][n] / A[j][j] for j in range(n)]


@pytest.mark.parametrize("p", [4, 6])
def test_weights_are_the_exact_solution(p):
    offs, w = exact_weights(p)
    got = O.lopsided_weights(p)
    for a, b in zip(got, w):
        assert abs(a - float(b)) <= 1e-16 * max(1.0, abs(float(b))), (p, got, w)
    # exact to degree p, not to degree p + 1
    for m in range(p + 1):
        assert sum(wj * Fraction(o) ** m for wj, o in zip(w, offs)) == int(m == 1)
    assert sum(wj * Fraction(o) ** (p + 1) for wj, o in zip(w, offs)) != 0
    # the integer forms (denominators 12 and 60)
    den = 12 if p == 4 else 60
    ints = [int(x * den) for x in w]
    assert ints == ([-3, -10, 18, -6, 1] if p == 4 else [2, -24, -35, 80, -30, 8, -1])


def _flat_block(p, deg, beta, h=(0.1, 0.13, 0.07), n=10, eps=1e-3):
    ng = p // 2 + 1
    bt = W.Batch([W.Block(n, n, n, ng, *h, x0=0.3, y0=-0.2, z0=0.1)], with_matter=False)
    F = W.F
    for f, v in (("chi", 1.0), ("gxx", 1.0), ("gyy", 1.0), ("gzz", 1.0), ("alpha", 1.0)):
        bt.view(bt.u, 0, F[f])[...] = v
    for k, name in enumerate(("bx", "by", "bz")):
        bt.view(bt.u, 0, F[name])[...] = beta[k]
    X, Y, Z = bt.blocks[0].coords()
    poly = lambda x, y, z: (x ** deg - 0.5 * x + 0.2) * (y ** deg + 0.3) * (z ** deg - 0.1)  # noqa: E731
    bt.view(bt.u, 0, F["chi"])[...] = 1.0 + eps * poly(X, Y, Z)
    bt.params = W.Params(fd_order=p, ko_sigma=0.0, lapse=W.LAPSE_FROZEN,
                         shift=W.SHIFT_FROZEN, eta=0.0, advect_gauge=0, advection=1)
    return bt, poly, eps


@pytest.mark.parametrize("p", [4, 6])
@pytest.mark.parametrize("beta", [(0.3, -0.2, 0.5), (-0.4, 0.25, -0.1)])
def test_chi_rhs_is_the_shifted_stencil(p, beta):
    """rhs(chi) = beta^k d_k chi here (K = 0, constant shift, no dissipation);
    each d_k is the rational stencil sum over the stored chi values on the
    points shifted towards the sign of beta^k."""
    bt, _, _ = _flat_block(p, p + 2, beta)
    got = bt.interior(O.rhs(bt), 0, W.F["chi"])
    chi = bt.view(bt.u, 0, W.F["chi"])          # stored (z, y, x), ghosts included
    offs, w = exact_weights(p)
    blk = bt.blocks[0]
    g = blk.ng
    steps = (blk.dx, blk.dy, blk.dz)
    rng = np.random.default_rng(3)
    for _ in range(16):
        i, j, k = (int(v) for v in rng.integers(0, blk.nx, size=3))
        total = Fraction(0)
        for a in range(3):
            s = 1 if beta[a] > 0 else -1
            acc = Fraction(0)
            for wj, oj in zip(w, offs):
                idx = [i + g, j + g, k + g]
                idx[a] += s * oj
                acc += wj * Fraction(float(chi[idx[2], idx[1], idx[0]]))
            total += Fraction(beta[a]) * s * acc / Fraction(steps[a])
        want = float(total)
        assert abs(got[k, j, i] - want) <= 1e-10 * abs(want) + 1e-18, (p, beta, got[k, j, i], want)


@pytest.mark.parametrize("p", [4, 6])
def test_lopsided_equals_centred_on_exact_data_only(p):
    beta = (0.3, -0.2, 0.5)
    for deg, same in ((p, True), (p + 2, False)):
        bt, _, _ = _flat_block(p, deg, beta)
        lop = bt.interior(O.rhs(bt), 0, W.F["chi"])
        bt.params.advection = 0
        cen = bt.interior(O.rhs(bt), 0, W.F["chi"])
        scale = np.abs(cen).max()
        d = np.abs(lop - cen).max()
        if same:
            assert d <= 1e-10 * scale, (p, deg, d, scale)
        else:
            assert d > 1e-6 * scale, (p, deg, d, scale)
