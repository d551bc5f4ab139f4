"""Pins of the oracle's ghost exchange on a multi-level set (CPU only):
every ghost point owned by a block of the same level is a copy, one owned by
a finer block an injection, one owned by a coarser block the tensor-product
Lagrange interpolation of order p -- exact on polynomials of degree < p along
each direction, so a polynomial of total degree p - 1 comes back to rounding
at every owned ghost point of a two- and a three-level set; points no block
owns take `frozen`.  A wrong stencil offset or weight fails."""
import numpy as np
import pytest

from oracle.intergrid import level_exchange
from paper_2311_04989_amd import workloads as W

CASES = [dict(refine=(1, 0, 0)), dict(refine=(0, 0, 0), refine2=0)]


def _coords(bt, locs):
    lmax = max(L for L, _ in locs)
    out = []
    for blk, (L, o) in zip(bt.blocks, locs):
        s = 1 << (lmax - L)
        g = blk.ng
        k, j, i = np.meshgrid(np.arange(-g, blk.nz + g), np.arange(-g, blk.ny + g),
                              np.arange(-g, blk.nx + g), indexing="ij")
        X = np.stack([o[0] + i * s, o[1] + j * s, o[2] + k * s]).astype(float)
        inner = (i >= 0) & (i < blk.nx) & (j >= 0) & (j < blk.ny) & (k >= 0) & (k < blk.nz)
        out.append((X, inner))
    return out


def _poly(X, deg):
    x, y, z = X / 16.0
    return 0.3 + x ** deg - 2 * x ** 2 * y ** (deg - 2) + y * z ** (deg - 1) - z ** deg + x * y * z


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_exchange_exact_on_polynomials(case, order):
    bt, locs = W.refined_level_set(**CASES[case])
    co = _coords(bt, locs)
    # the exact data everywhere in `frozen` (the outer ghosts, which no block
    # owns and coarse stencils near the outer boundary read); in the state
    # only the interiors, the ghosts poisoned with NaN
    frozen = np.zeros_like(bt.u)
    for b, (X, inner) in enumerate(co):
        for f in range(W.NF):
            bt.view(frozen, b, f)[...] = _poly(X, order - 1) * (f + 1)
            v = bt.view(bt.u, b, f)
            v[...] = _poly(X, order - 1) * (f + 1)
            v[~inner] = np.nan
    out = level_exchange(bt, locs, bt.u, frozen, order)
    for b, (X, inner) in enumerate(co):
        for f in (0, 13, 21):
            v = bt.view(out, b, f)
            want = _poly(X, order - 1) * (f + 1)
            assert not np.any(np.isnan(v))
            np.testing.assert_allclose(v, want, rtol=0, atol=1e-13 * np.abs(want).max())
            # interiors untouched
            assert np.array_equal(v[inner], bt.view(bt.u, b, f)[inner])
    # the outer ghosts are frozen values, every other ghost is computed: with
    # frozen set to garbage only the outer ghosts (and stencils touching them)
    # change
    junk = np.full_like(bt.u, 1e6)
    out2 = level_exchange(bt, locs, bt.u, junk, order)
    nowned = sum(int((bt.view(out2, b, 0) != 1e6).sum() - inner.sum())
                 for b, (X, inner) in enumerate(co))
    assert nowned > 10000
    # one degree higher the interpolation is no longer exact
    for b, (X, inner) in enumerate(co):
        bt.view(frozen, b, 0)[...] = _poly(X, order)
        v = bt.view(bt.u, b, 0)
        v[...] = _poly(X, order)
        v[~inner] = np.nan
    out = level_exchange(bt, locs, bt.u, frozen, order)
    err = max(float(np.abs(bt.view(out, b, 0) - _poly(X, order)).max())
              for b, (X, inner) in enumerate(co))
    assert err > 1e-6


def test_same_level_copies_and_injections_are_bitwise():
    bt, locs = W.refined_level_set(refine=(1, 0, 0))
    rng = np.random.default_rng(3)
    bt.u[:] = rng.integers(-1000, 1000, size=bt.u.shape).astype(float)
    out = level_exchange(bt, locs, bt.u, None, 6)
    lmax = max(L for L, _ in locs)
    spans = [(np.array(o), np.array(o) + 8 * (1 << (lmax - L))) for L, o in locs]
    ncopy = ninj = 0
    for b, (blk, (L, o)) in enumerate(zip(bt.blocks, locs)):
        s = 1 << (lmax - L)
        g = blk.ng
        for (i, j, k) in [(-1, 3, 2), (blk.nx + 2, 0, 5), (4, -3, blk.nz), (-2, -2, -2)]:
            X = np.array([o[0] + i * s, o[1] + j * s, o[2] + k * s])
            own = [ob for ob, (lo, hi) in enumerate(spans) if np.all((X >= lo) & (X < hi))]
            if not own or locs[own[0]][0] < L:
                continue
            ob = own[0]
            so = 1 << (lmax - locs[ob][0])
            src = (X - np.array(locs[ob][1])) // so + g
            for f in range(W.NF):
                assert bt.view(out, b, f)[k + g, j + g, i + g] == \
                    bt.view(bt.u, ob, f)[src[2], src[1], src[0]]
            if locs[ob][0] == L:
                ncopy += 1
            else:
                ninj += 1
    assert ncopy > 0 and ninj > 0
