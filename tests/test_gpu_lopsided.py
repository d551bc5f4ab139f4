"""Lopsided advection on the GPU (plans with advection = LOPSIDED, through
the C ABI) against the oracle's lopsided reading (tests/test_lopsided_pins.py
pins it): right-hand side and RK4 stage 2 with the parity metric of
tests/parity.py, on random shapes (orders 4 and 6, default launch shapes), in
the one-wave kernel (order 6, 8x8x4 tiles, plain and persistent), and with
ghosts read through the neighbour rule (bitwise equal to stored ghosts).
The shift of every case has both signs in every direction."""
import sys

import numpy as np
import pytest

import oracle as O
from parity import assert_parity, compare, report
from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def Z():
    from paper_2311_04989_amd import z4c
    return z4c


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def with_shift(bt, amp=0.05):
    """A smooth shift of both signs (a function of position, so neighbouring
    blocks agree on their shared points)."""
    for b, blk in enumerate(bt.blocks):
        X, Y, Zc = blk.coords()
        for k, f in enumerate(("bx", "by", "bz")):
            bt.view(bt.u, b, W.F[f])[...] += amp * np.sin(1.3 * X + 0.7 * (k + 1) * Y
                                                          - 0.9 * Zc + k)
    bt.params.advection = 1
    return bt


def check(bt, plan, label):
    u, m = dev(bt.u), dev(bt.matter)
    out = torch.zeros(bt.total_u, dtype=torch.float64, device=DEV)
    plan.rhs(u, m, out)
    g = host(out)
    rows = compare(bt, g, O.rhs(bt), O.rhs(bt, ext=True))
    assert_parity(rows, f"{label} rhs\n" + report(rows))
    out2, u1 = dev(bt.u), dev(bt.u)
    plan.rk_stage(u, out2, u1, u, m, Z().RK4[1], 0.01)
    gout = host(out2)
    o64, o80 = bt.u.copy(), bt.u.copy()
    O.rk_stage(bt, bt.u, o64, bt.u.copy(), bt.u, O.RK4[1], 0.01)
    O.rk_stage(bt, bt.u, o80, bt.u.copy(), bt.u, O.RK4[1], 0.01, ext=True)
    rows = compare(bt, gout, o64, o80, base=bt.u)
    assert_parity(rows, f"{label} stage\n" + report(rows))
    return g


@pytest.mark.parametrize("seed", range(4))
def test_random_shapes_lopsided(seed):
    bt = with_shift(W.random_batch(seed, nblocks=3, nmax=24, amp=0.02))
    note(f"lopsided random shapes seed {seed} p={bt.params.fd_order}: "
         + ", ".join(f"{b.nx}x{b.ny}x{b.nz}" for b in bt.blocks))
    plan = Z().plan_for(bt)
    g = check(bt, plan, f"lopsided random {seed}")
    plan.close()
    # the stencil choice matters for these data
    bt.params.advection = 0
    c = O.rhs(bt)
    assert np.abs(g - c).max() > 1e-9 * np.abs(c).max()


@pytest.mark.parametrize("pers", [0, 3])
def test_one_wave_lopsided(pers):
    bt = with_shift(W.random_batch(11, nblocks=3, nmax=30, fd_order=6, amp=0.02))
    note(f"lopsided one-wave persistent={pers}: "
         + ", ".join(f"{b.nx}x{b.ny}x{b.nz}" for b in bt.blocks))
    plan = Z().plan_for(bt)
    plan.set_launch(0, 0, 0, (8, 8, 4), pers, 1)
    check(bt, plan, f"lopsided one-wave p{pers}")
    plan.close()


def test_lopsided_neighbour_halo():
    bt = with_shift(W.config5(n=12))
    bt.frozen = bt.u.copy()
    O.ghost_fill(bt, bt.u)              # stored ghosts = the neighbour rule
    bt.frozen = bt.u.copy()
    note("lopsided neighbour halo, 8 x 12^3")
    plan = Z().plan_for(bt)
    ref = check(bt, plan, "lopsided 8x12^3")
    stale = bt.u.copy()
    rng = np.random.default_rng(9)
    for b in range(len(bt.blocks)):
        g = bt.blocks[b].ng
        for f in range(W.NF):
            v = bt.view(stale, b, f)
            keep = v[g:-g, g:-g, g:-g].copy()
            v[...] = rng.normal(size=v.shape)
            v[g:-g, g:-g, g:-g] = keep
    fr = dev(bt.frozen)                 # the plan keeps the pointer: keep the array alive
    plan.set_halo(Z().GHOST_NEIGHBOUR, fr)
    out = torch.zeros(bt.total_u, dtype=torch.float64, device=DEV)
    plan.rhs(dev(stale), dev(bt.matter), out)
    got = host(out)
    plan.close()
    for b in range(len(bt.blocks)):
        for f in range(W.NF):
            assert np.array_equal(bt.interior(got, b, f), bt.interior(ref, b, f)), (b, f)


def test_level_set_lopsided_stage_sampled():
    """At full size in the launch configuration the benchmark times: the
    uneven level set (1,024 blocks, ghosts read through the periodic rule,
    autotuned shapes), lopsided advection, RK4 stage 2; 16 sampled blocks
    (4 of each size) against the oracle."""
    bt = W.config4()
    O.ghost_fill(bt, bt.u)                   # stored ghosts = the periodic rule
    bt.params.advection = 1
    note(f"lopsided level set: {bt.name}")
    Zm = Z()
    plan = Zm.plan_for(bt)
    u0 = dev(bt.u)
    plan.set_halo(Zm.GHOST_PERIODIC)
    out, u1 = u0.clone(), torch.zeros_like(u0)
    plan.autotune(u0, out, u1, None, reps=2)
    out, u1 = u0.clone(), torch.zeros_like(u0)
    plan.rk_stage(u0, out, u1, u0, None, Zm.RK4[1], bt.dt)
    got = host(out)
    plan.close()
    sizes = np.array([b.nx for b in bt.blocks])
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(np.nonzero(sizes == s)[0], size=4, replace=False)
                          for s in (8, 16, 24, 32)])
    sub = bt.subset(idx)
    o64, o80 = sub.u.copy(), sub.u.copy()
    O.rk_stage(sub, sub.u, o64, np.zeros_like(sub.u), sub.u, O.RK4[1], bt.dt)
    O.rk_stage(sub, sub.u, o80, np.zeros_like(sub.u), sub.u, O.RK4[1], bt.dt, ext=True)
    gsub = bt.subset(idx)
    for j, i in enumerate(idx):
        for f in range(W.NF):
            gsub.view(gsub.u, j, f)[...] = bt.view(got, i, f)
    rows = compare(sub, gsub.u, o64, o80, base=sub.u)
    assert_parity(rows, "lopsided level set sampled stage\n" + report(rows))
