"""Transfers between refinement levels on the GPU (z4c_prolongate,
z4c_restrict through the C ABI) against oracle/intergrid.py: prolongation
of the ghost slabs and of whole fine blocks for orders 2, 4, 6 within 1e-13
(relative, 1e-3 floor; linear combinations, rounding order only), bitwise
on polynomial data of degree < order, restriction bitwise; every point no
transfer writes keeps its value bit for bit."""
import sys

import numpy as np
import pytest

from oracle import intergrid as OI
from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def Z():
    from paper_2311_04989_amd import z4c
    return z4c


def ghost_slabs(blk, fine, c0):
    n, g = blk.nx, blk.ng
    out = []
    for d in range(3):
        for lo, hi in ((-g, 0), (n, n + g)):
            b_lo, b_hi = [-g] * 3, [n + g] * 3
            if d > 0:          # slabs of earlier directions already cover their corners
                for e in range(d):
                    b_lo[e], b_hi[e] = 0, n
            b_lo[d], b_hi[d] = lo, hi
            out.append(dict(coarse=0, fine=fine, c0=c0, lo=b_lo, hi=b_hi))
    return out


def run(bt, pro, res, order):
    plan = Z().plan_for(bt)
    xp = Z().XPlan(plan, pro, res, order)
    u = torch.from_numpy(bt.u.copy()).to(DEV)
    if pro:
        xp.prolongate(u)
    if res:
        xp.restrict(u)
    torch.cuda.synchronize()
    out = u.cpu().numpy()
    xp.close()
    plan.close()
    return out


@pytest.mark.parametrize("order", [2, 4, 6])
def test_prolongation_parity(order):
    bt, origins = W.refined_pair(seed=order)
    pro = []
    for m, c0 in enumerate(origins):
        pro += ghost_slabs(bt.blocks[1 + m], 1 + m, c0)
    note(f"prolongation order {order}: {len(pro)} transfers")
    got = run(bt, pro, [], order)
    want = OI.prolong(bt, bt.u, pro, order)
    written = want != bt.u
    assert np.all(got[~written] == bt.u[~written]) or np.all(got[~written] == want[~written])
    for b in range(len(bt.blocks)):
        for f in range(W.NF):
            g, o = bt.view(got, b, f), bt.view(want, b, f)
            m = np.abs(o).max()
            e = (np.abs(g - o) / np.maximum(np.abs(o), 1e-3 * m)).max()
            assert e <= 1e-13, (b, f, e)
    # the coarse block is only read
    for f in range(W.NF):
        assert np.array_equal(bt.view(got, 0, f), bt.view(bt.u, 0, f))


@pytest.mark.parametrize("order", [2, 4, 6])
def test_prolongation_exact_on_polynomials(order):
    deg = order - 1
    bt, origins = W.refined_pair(
        fill=lambda X, Y, Z, f: (X ** deg - X + 2) * (Y ** deg + 1) * (Z ** deg - 3) + f)
    pro = [dict(coarse=0, fine=1 + m, c0=c0, lo=[-4] * 3, hi=[20] * 3)
           for m, c0 in enumerate(origins)]
    note(f"prolongation polynomial order {order}")
    got = run(bt, pro, [], order)
    for m in range(len(origins)):
        X, Y, Zc = bt.blocks[1 + m].coords()
        for f in range(W.NF):
            want = (X ** deg - X + 2) * (Y ** deg + 1) * (Zc ** deg - 3) + f
            np.testing.assert_allclose(bt.view(got, 1 + m, f), want, rtol=1e-14,
                                       atol=1e-14 * np.abs(want).max())


def test_restriction_parity():
    bt, origins = W.refined_pair(seed=9)
    for m in range(len(origins)):           # fine data that differ from the coarse data
        for f in range(W.NF):
            bt.view(bt.u, 1 + m, f)[...] += 0.5 + f
    res = [dict(coarse=0, fine=1 + m, c0=c0, lo=list(c0), hi=[c0[0] + 8, c0[1] + 8, c0[2] + 8])
           for m, c0 in enumerate(origins)]
    note("restriction")
    got = run(bt, [], res, 6)
    want = OI.restrict(bt, bt.u, res)
    assert np.array_equal(got, want)
    assert not np.array_equal(got, bt.u)


def test_level_jump_at_scale_sampled():
    """The measured workload (64 coarse + 512 fine blocks, 3072 face slabs of
    order 6, 512 octants restricted), both calls in sequence as timed: a
    seeded sample of 48 prolongation and 48 restriction transfers against
    the oracle, and every fine interior point untouched."""
    bt, pro, res = W.level_jump()
    note(f"level jump at scale: {bt.name}")
    plan = Z().plan_for(bt)
    xp = Z().XPlan(plan, pro, res, 6)
    u = torch.from_numpy(bt.u).to(DEV)
    xp.prolongate(u)
    xp.restrict(u)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    xp.close()
    plan.close()
    rng = np.random.default_rng(77)
    sp = [pro[i] for i in rng.choice(len(pro), 48, replace=False)]
    sr = [res[i] for i in rng.choice(len(res), 48, replace=False)]
    want_p = OI.prolong(bt, bt.u, sp, 6)
    want_r = OI.restrict(bt, bt.u, sr)
    for t in sp:
        fb, ng = t["fine"], bt.blocks[t["fine"]].ng
        sl = tuple(slice(t["lo"][d] + ng, t["hi"][d] + ng) for d in (2, 1, 0))
        for f in range(W.NF):
            g, o = bt.view(got, fb, f)[sl], bt.view(want_p, fb, f)[sl]
            assert np.abs(g - o).max() <= 1e-13 * max(np.abs(o).max(), 1.0), (t, f)
    for t in sr:
        cb, ng = t["coarse"], bt.blocks[t["coarse"]].ng
        sl = tuple(slice(t["lo"][d] + ng, t["hi"][d] + ng) for d in (2, 1, 0))
        for f in range(W.NF):
            assert np.array_equal(bt.view(got, cb, f)[sl], bt.view(want_r, cb, f)[sl]), (t, f)
    nc = 64
    for b in range(nc, len(bt.blocks), 37):
        for f in (0, 7, 21):
            assert np.array_equal(bt.interior(got, b, f), bt.interior(bt.u, b, f))


@pytest.mark.parametrize("refine,refine2", [((1, 0, 0), None), ((0, 1, 1), None), ((1, 0, 0), 7)])
def test_level_jump_exchange_exact_on_polynomials(refine, refine2):
    """The exchange z4c_level_transfers describes, run on the GPU: every
    stored point of a level set with one or two level jumps holds a
    polynomial of degree <= 5 per direction except the destinations of the
    transfers, which hold NaN; after the restrictions (finest level pair
    first) and the prolongations (order 6, coarsest pair first) every stored
    point holds the polynomial (exact up to rounding), so every destination
    was written and no transfer read a point before it was filled."""
    bt, locs = W.refined_level_set(refine=refine, refine2=refine2)
    poly = lambda x, y, z: (x ** 5 - 0.3 * x ** 2 + 0.7) * (y ** 5 + 0.2 * y - 1.1) \
        * (z ** 4 + 0.5 * z ** 3 - 0.25)   # noqa: E731
    want = np.zeros_like(bt.u)
    for b, blk in enumerate(bt.blocks):
        X, Y, Zc = blk.coords()
        for f in range(W.NF):
            bt.view(want, b, f)[...] = poly(X, Y, Zc) + f
    plan = Z().plan_for(bt)
    pairs = range(max(L for L, _ in locs))
    sets = [Z().level_transfers(plan, locs, L) for L in pairs]
    note(f"level-jump exchange {refine} {refine2}: "
         + ", ".join(f"pair {L}: {len(p)} prolongations, {len(r)} restrictions"
                     for L, (p, r) in zip(pairs, sets)))
    start = want.copy()
    for pro, res in sets:
        for t, key in [(t, "fine") for t in pro] + [(t, "coarse") for t in res]:
            b, g = t[key], bt.blocks[t[key]].ng
            sl = tuple(slice(t["lo"][d] + g, t["hi"][d] + g) for d in (2, 1, 0))
            for f in range(W.NF):
                bt.view(start, b, f)[sl] = np.nan
    xps = [Z().XPlan(plan, pro, res, 6) for pro, res in sets]
    u = torch.from_numpy(start).to(DEV)
    for xp in reversed(xps):
        xp.restrict(u)
    for xp in xps:
        xp.prolongate(u)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    for xp in xps:
        xp.close()
    plan.close()
    assert np.isfinite(got).all()
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-13 * scale, np.abs(got - want).max() / scale
