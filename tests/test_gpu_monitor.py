"""The constraint monitor fused into the stage kernel (z4c_rk_stage_monitor
through the C ABI): one call gives the stage and the constraints of its
input (Sec. 4.1 monitoring).

* configuration 2 (star metric + matter, 64^3, order 6), RK4 stage 2, in
  every launch shape the order-6 kernels have (one wave per SIMD on 8x8x4
  tiles, two waves on 8x8x4 and 8x8x8, persistent or not): the stage
  against the oracle's stage and the constraints against the oracle's
  constraints with the parity metric of tests/parity.py, the per-block
  norms within 1e-10;
* the uneven level set of the benchmark (1,024 blocks, ghosts read through
  the periodic rule, autotuned shapes): constraints and norms against
  z4c_constraints on the same state (same quantities, other rounding
  order), and the stage bit for bit against z4c_rk_stage's where the
  compiler leaves the stage's arithmetic unchanged, else within 1e-13;
* the star level set reduced to 8 x 16^3 with neighbour ghosts and frozen
  outer ghosts read through the rule: stage and constraints against the
  oracle.
"""
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


@pytest.fixture(scope="module")
def config2_oracle():
    bt = W.config2()
    rng = np.random.default_rng(5)
    u1 = bt.u + rng.uniform(-1e-3, 1e-3, size=bt.u.shape)
    y = bt.u + rng.uniform(-1e-3, 1e-3, size=bt.u.shape)
    c = O.RK4[1]
    o64, o64u1 = bt.u.copy(), u1.copy()
    O.rk_stage(bt, bt.u, o64, o64u1, y, c, bt.dt)
    o80, o80u1 = bt.u.copy(), u1.copy()
    O.rk_stage(bt, bt.u, o80, o80u1, y, c, bt.dt, ext=True)
    c64, n64 = O.constraints(bt)
    c80, n80 = O.constraints(bt, ext=True)
    return bt, u1, y, (o64, o80, o64u1, o80u1), (c64, c80, n80)


@pytest.mark.parametrize("shape", [((8, 8, 4), 0, 1), ((8, 8, 4), 0, 2), ((8, 8, 8), 0, 2),
                                   ((8, 8, 4), 64, 1)])
def test_config2_stage_monitor(config2_oracle, shape):
    bt, u1_init, y, (o64, o80, o64u1, o80u1), (c64, c80, n80) = config2_oracle
    tile, pers, waves = shape
    note(f"config2 stage monitor tile {tile} persistent {pers} waves {waves}")
    plan = Z().plan_for(bt)
    b = bt.blocks[0]
    plan.set_launch(b.nx, b.ny, b.nz, tile=tile, persistent=pers, waves=waves)
    u0, out, u1 = dev(bt.u), dev(bt.u), dev(u1_init)
    cons = torch.zeros(bt.total_c, dtype=torch.float64, device=DEV)
    norms = torch.zeros(16 * len(bt.blocks), dtype=torch.float64, device=DEV)
    plan.rk_stage_monitor(u0, out, u1, dev(y), dev(bt.matter), Z().RK4[1], bt.dt, cons, norms)
    gout, gu1, gc = host(out), host(u1), host(cons)
    gn = host(norms).reshape(-1, 8, 2)
    plan.close()
    rows = compare(bt, gout, o64, o80, base=y)
    assert_parity(rows, "monitor stage state - y\n" + report(rows))
    rows = compare(bt, gu1, o64u1, o80u1, base=u1_init)
    assert_parity(rows, "monitor stage accumulator increment\n" + report(rows))
    rows = compare(bt, gc, c64, c80, nfields=W.NC)
    assert_parity(rows, "monitor constraints\n" + report(rows))
    np.testing.assert_allclose(gn, n80, rtol=1e-10, atol=1e-300)


def test_level_set_monitor_matches_constraints():
    bt = W.config4()
    note(f"level set monitor: {bt.name}")
    Zm = Z()
    plan = Zm.plan_for(bt)
    u0 = dev(bt.u)
    plan.ghost_fill(Zm.GHOST_PERIODIC, u0)   # stored ghosts = what the rule reads
    plan.set_halo(Zm.GHOST_PERIODIC)
    regs = [u0.clone(), torch.zeros_like(u0)]
    plan.autotune(u0, regs[0], regs[1], None, reps=2)
    a_out, a_u1 = u0.clone(), torch.zeros_like(u0)
    b_out, b_u1 = u0.clone(), torch.zeros_like(u0)
    nb = len(bt.blocks)
    cons_m = torch.zeros(bt.total_c, dtype=torch.float64, device=DEV)
    norms_m = torch.zeros(16 * nb, dtype=torch.float64, device=DEV)
    cons_c = torch.zeros(bt.total_c, dtype=torch.float64, device=DEV)
    norms_c = torch.zeros(16 * nb, dtype=torch.float64, device=DEV)
    plan.rk_stage(u0, a_out, a_u1, u0, None, Zm.RK4[0], bt.dt)
    plan.rk_stage_monitor(u0, b_out, b_u1, u0, None, Zm.RK4[0], bt.dt, cons_m, norms_m)
    plan.constraints(u0, None, cons_c, norms_c)
    ga, gb = host(a_out), host(b_out)
    gu_a, gu_b = host(a_u1), host(b_u1)
    cm, cc = host(cons_m), host(cons_c)
    nm, nc = host(norms_m).reshape(nb, 8, 2), host(norms_c).reshape(nb, 8, 2)
    plan.close()
    d = np.abs(gb - ga)
    assert d.max() <= 1e-13 * np.abs(ga).max(), d.max()
    d1 = np.abs(gu_b - gu_a)
    assert d1.max() <= 1e-13 * max(np.abs(gu_a).max(), 1e-300), d1.max()
    note(f"  stage: bitwise equal {np.array_equal(ga, gb)}, max diff {d.max():.3g}")
    # constraints: per field, relative to the field's largest magnitude
    for b in range(0, nb, 7):
        for q in range(W.NC):
            x, r = bt.view(cm, b, q, W.NC), bt.view(cc, b, q, W.NC)
            scale = np.abs(r).max()
            assert np.abs(x - r).max() <= 1e-9 * scale + 1e-300, (b, q, np.abs(x - r).max(), scale)
    np.testing.assert_allclose(nm, nc, rtol=1e-9, atol=1e-300)


def test_graph_step_with_monitor():
    """Z4C_STEP_MONITOR in the graph-replayed RK4 step of the level set: each
    of three replays (eager work and synchronisation between them) gives the
    norms of z4c_constraints on the state it started from (within 1e-9), and
    the same state as the step without the monitor (within 1e-13)."""
    bt = W.config4()
    note(f"graph step with monitor: {bt.name}")
    Zm = Z()
    plan = Zm.plan_for(bt)
    u0 = dev(bt.u)
    plan.ghost_fill(Zm.GHOST_PERIODIC, u0)
    nb = len(bt.blocks)
    regs = [u0.clone(), u0.clone(), u0.clone(), torch.zeros_like(u0)]
    ref = [u0.clone(), u0.clone(), u0.clone(), torch.zeros_like(u0)]
    cons = torch.zeros(bt.total_c, dtype=torch.float64, device=DEV)
    norms = torch.zeros(16 * nb, dtype=torch.float64, device=DEV)
    cons_c = torch.zeros(bt.total_c, dtype=torch.float64, device=DEV)
    norms_c = torch.zeros(16 * nb, dtype=torch.float64, device=DEV)
    for rep in range(3):
        plan.set_halo(Zm.GHOST_PERIODIC)
        plan.constraints(regs[0], None, cons_c, norms_c)
        want = host(norms_c).copy()
        r = plan.step(regs, None, Zm.RK4, bt.dt, Zm.GHOST_PERIODIC, graph=True,
                      flags=Zm.STEP_MONITOR, cons=cons, norms=norms)
        r2 = plan.step(ref, None, Zm.RK4, bt.dt, Zm.GHOST_PERIODIC, graph=True)
        assert r == r2 == 0
        got = host(norms)
        np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-300)
        a, b = host(regs[0]), host(ref[0])
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
        note(f"  replay {rep}: norms within 1e-9, state max diff {np.abs(a - b).max():.3g}")
        ref[0].copy_(regs[0])     # both continue from the same state
    plan.close()


def test_level_set_monitor_sampled_against_oracle():
    """At full size in the benchmark's launch configuration (autotuned
    shapes, ghosts through the periodic rule), RK4 stage 2 with the monitor:
    the constraints and per-block norms of 16 sampled blocks (4 of each
    size) against the oracle's."""
    bt = W.config4()
    O.ghost_fill(bt, bt.u)
    note(f"monitor level set vs oracle: {bt.name}")
    Zm = Z()
    plan = Zm.plan_for(bt)
    u0 = dev(bt.u)
    plan.set_halo(Zm.GHOST_PERIODIC)
    out, u1 = u0.clone(), torch.zeros_like(u0)
    plan.autotune(u0, out, u1, None, reps=2)
    nb = len(bt.blocks)
    cons = torch.zeros(bt.total_c, dtype=torch.float64, device=DEV)
    norms = torch.zeros(16 * nb, dtype=torch.float64, device=DEV)
    plan.rk_stage_monitor(u0, out, u1, u0, None, Zm.RK4[1], bt.dt, cons, norms)
    gc, gn = host(cons), host(norms).reshape(nb, 8, 2)
    plan.close()
    sizes = np.array([b.nx for b in bt.blocks])
    rng = np.random.default_rng(6)
    idx = np.concatenate([rng.choice(np.nonzero(sizes == s)[0], size=4, replace=False)
                          for s in (8, 16, 24, 32)])
    sub = bt.subset(idx)
    c64, _ = O.constraints(sub)
    c80, n80 = O.constraints(sub, ext=True)
    gsub = np.zeros_like(c64)
    for j, i in enumerate(idx):
        for q in range(W.NC):
            sub.view(gsub, j, q, W.NC)[...] = bt.view(gc, i, q, W.NC)
    rows = compare(sub, gsub, c64, c80, nfields=W.NC)
    assert_parity(rows, "monitor level set sampled constraints\n" + report(rows))
    np.testing.assert_allclose(gn[idx], n80.reshape(len(idx), 8, 2), rtol=1e-10, atol=1e-300)


def test_eager_step_with_monitor_and_stored_ghosts():
    """Z4C_STEP_MONITOR with Z4C_STEP_STORED_GHOSTS (stage 0 reads stored
    ghosts, refreshed by the step after each stage), eager: the norms equal
    those of z4c_constraints on the state the step started from (within
    1e-9), the state equals the monitor-free step's (within 1e-13), and the
    constraint fields are written."""
    bt = W.config4()
    note(f"eager stored-ghost step with monitor: {bt.name}")
    Zm = Z()
    plan = Zm.plan_for(bt)
    u0 = dev(bt.u)
    plan.ghost_fill(Zm.GHOST_PERIODIC, u0)
    nb = len(bt.blocks)
    cons_c = torch.zeros(bt.total_c, dtype=torch.float64, device=DEV)
    norms_c = torch.zeros(16 * nb, dtype=torch.float64, device=DEV)
    plan.constraints(u0, None, cons_c, norms_c)
    want = host(norms_c).copy()
    regs = [u0.clone(), u0.clone(), u0.clone(), torch.zeros_like(u0)]
    ref = [u0.clone(), u0.clone(), u0.clone(), torch.zeros_like(u0)]
    cons = torch.full((bt.total_c,), float("nan"), dtype=torch.float64, device=DEV)
    norms = torch.zeros(16 * nb, dtype=torch.float64, device=DEV)
    flags = Zm.STEP_MONITOR | Zm.STEP_STORED_GHOSTS
    r = plan.step(regs, None, Zm.RK4, bt.dt, Zm.GHOST_PERIODIC, flags=flags, cons=cons,
                  norms=norms)
    r2 = plan.step(ref, None, Zm.RK4, bt.dt, Zm.GHOST_PERIODIC, flags=Zm.STEP_STORED_GHOSTS)
    np.testing.assert_allclose(host(norms), want, rtol=1e-9, atol=1e-300)
    a, b = host(regs[r]), host(ref[r2])
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    gc, cc = host(cons), host(cons_c)
    for blk in range(0, nb, 97):
        for q in range(W.NC):
            x, y = bt.interior(gc, blk, q, W.NC), bt.interior(cc, blk, q, W.NC)
            assert np.isfinite(x).all()
            assert np.abs(x - y).max() <= 1e-9 * np.abs(y).max() + 1e-300
    plan.close()


def test_monitor_with_neighbour_and_frozen_halo_reads():
    """The star level set reduced to 8 blocks of 16^3 (matter, neighbour
    ghosts between the blocks, frozen outer ghosts) read through the rule by
    the monitor kernel in the one-wave shape: the stage and the constraints
    against the oracle on the same state with refreshed stored ghosts."""
    Zm = Z()
    bt = W.config5(n=16)
    O.ghost_fill(bt, bt.u)
    note("monitor, neighbour + frozen halo reads, 8 x 16^3")
    rng = np.random.default_rng(8)
    u1_init = bt.u + rng.uniform(-1e-4, 1e-4, size=bt.u.shape)
    c = O.RK4[1]
    o64, o64u1 = bt.u.copy(), u1_init.copy()
    O.rk_stage(bt, bt.u, o64, o64u1, bt.u, c, bt.dt)
    o80, o80u1 = bt.u.copy(), u1_init.copy()
    O.rk_stage(bt, bt.u, o80, o80u1, bt.u, c, bt.dt, ext=True)
    c64, _ = O.constraints(bt)
    c80, n80 = O.constraints(bt, ext=True)
    plan = Zm.plan_for(bt)
    plan.set_launch(0, 0, 0, tile=(8, 8, 4), persistent=0, waves=1)
    frozen = dev(bt.frozen)
    plan.set_halo(Zm.GHOST_NEIGHBOUR, frozen)
    u0 = dev(bt.u)
    out, u1 = dev(bt.u), dev(u1_init)
    cons = torch.zeros(bt.total_c, dtype=torch.float64, device=DEV)
    norms = torch.zeros(16 * len(bt.blocks), dtype=torch.float64, device=DEV)
    plan.rk_stage_monitor(u0, out, u1, u0, dev(bt.matter), Zm.RK4[1], bt.dt, cons, norms)
    gout, gu1, gc = host(out), host(u1), host(cons)
    gn = host(norms).reshape(-1, 8, 2)
    plan.close()
    rows = compare(bt, gout, o64, o80, base=bt.u)
    assert_parity(rows, "monitor neighbour-rule stage\n" + report(rows))
    rows = compare(bt, gu1, o64u1, o80u1, base=u1_init)
    assert_parity(rows, "monitor neighbour-rule accumulator\n" + report(rows))
    rows = compare(bt, gc, c64, c80, nfields=W.NC)
    assert_parity(rows, "monitor neighbour-rule constraints\n" + report(rows))
    np.testing.assert_allclose(gn, n80, rtol=1e-10, atol=1e-300)
