"""Parity of the HIP path (through the C ABI) with the oracle, on the GPU.

Inputs are the seeded workload generators; the metric and its tolerance are
described in tests/parity.py.  Full-size configurations run on the GPU in
the launch configuration the benchmark uses and are checked on sampled
blocks (blocks are independent within one stage given their ghosts, and
each block of the uneven level set is periodic on itself).
"""
import sys

import numpy as np
import pytest

import oracle as O
from parity import assert_parity, compare, report
from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def z4c():
    from paper_2311_04989_amd import z4c as Z
    return Z


DEV = "cuda:0"


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def zeros(n):
    return torch.zeros(n, dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_rhs(bt, arith=0, plan=None):
    Z = z4c()
    plan = plan or Z.plan_for(bt, arith)
    u, m, out = dev(bt.u), dev(bt.matter), zeros(bt.total_u)
    plan.rhs(u, m, out)
    return host(out)


def gpu_stage(bt, coeffs, dt, u1_init=None, u2=None, arith=0, plan=None):
    Z = z4c()
    plan = plan or Z.plan_for(bt, arith)
    u0 = dev(bt.u)
    out = dev(bt.u)   # ghosts carried over, interior overwritten
    u1 = dev(u1_init) if u1_init is not None else zeros(bt.total_u)
    u2d = dev(u2) if u2 is not None else u0
    plan.rk_stage(u0, out, u1, u2d, dev(bt.matter), coeffs, dt)
    return host(out), host(u1)


def gpu_step(bt, table, dt, graph=False, arith=0, plan=None, replays=1):
    Z = z4c()
    plan = plan or Z.plan_for(bt, arith)
    regs = [dev(bt.u), dev(bt.u), dev(bt.u), zeros(bt.total_u)]
    frozen = dev(bt.frozen) if bt.frozen is not None else None
    res = plan.step(regs, dev(bt.matter), table, dt, bt.ghost, frozen, graph=graph)
    return host(regs[res])


ORACLE_RK4 = O.RK4


# --- exactness -------------------------------------------------------------------

@pytest.mark.parametrize("p", [4, 6])
def test_flat_space_bitwise_zero(p):
    Z = z4c()
    blocks = [W.Block(1, 1, 1, p // 2 + 1, 0.1, 0.1, 0.1), W.Block(5, 9, 13, 4, 0.3, 0.2, 0.1),
              W.Block(16, 16, 16, p // 2 + 1, 0.05, 0.05, 0.05), W.Block(17, 3, 8, 4, 1.0, 2.0, 3.0)]
    bt = W.Batch(blocks, with_matter=False)
    W.fill_fields(bt, W.flat)
    bt.params = W.Params(fd_order=p, ko_sigma=0.5)
    note(f"flat p={p}")
    for arith in (Z.ARITH_FP64, Z.ARITH_FP32):
        r = gpu_rhs(bt, arith)
        assert np.all(r == 0.0)
        out, _ = gpu_stage(bt, Z.RK4[0], 0.01, arith=arith)
        assert np.array_equal(out, bt.u)


# --- configuration 1: gauge wave 16^3, p = 4 ---------------------------------------

def test_config1_rhs_and_rk4_step():
    Z = z4c()
    bt = W.config1()
    O.ghost_fill(bt, bt.u)
    note("config1 rhs")
    g = gpu_rhs(bt)
    rows = compare(bt, g, O.rhs(bt), O.rhs(bt, ext=True))
    assert_parity(rows, "config1 rhs\n" + report(rows))
    note("config1 rk4 step")
    gs = gpu_step(bt, Z.RK4, bt.dt)
    o64 = O.rk_step(bt, bt.u.copy(), dt=bt.dt)
    o80 = O.rk_step(bt, bt.u.copy(), dt=bt.dt, ext=True)
    rows = compare(bt, gs, o64, o80, base=bt.u)
    assert_parity(rows, "config1 step increments\n" + report(rows))
    note("config1 ssprk3 step")
    gs = gpu_step(bt, Z.SSPRK3, bt.dt)
    o64 = O.rk_step(bt, bt.u.copy(), table=O.SSPRK3, dt=bt.dt)
    o80 = O.rk_step(bt, bt.u.copy(), table=O.SSPRK3, dt=bt.dt, ext=True)
    rows = compare(bt, gs, o64, o80, base=bt.u)
    assert_parity(rows, "config1 ssprk3 increments\n" + report(rows))


# --- configuration 2: star metric + matter 64^3, p = 6 --------------------------------

def test_config2_rhs_stage_constraints():
    Z = z4c()
    bt = W.config2()
    note("config2 rhs")
    g = gpu_rhs(bt)
    rows = compare(bt, g, O.rhs(bt), O.rhs(bt, ext=True))
    assert_parity(rows, "config2 rhs\n" + report(rows))
    # a middle RK4 stage: reads u0, u1 and u2 = y_n, writes u0' and u1
    rng = np.random.default_rng(5)
    u1 = bt.u + rng.uniform(-1e-3, 1e-3, size=bt.u.shape)
    y = bt.u + rng.uniform(-1e-3, 1e-3, size=bt.u.shape)
    c = ORACLE_RK4[1]
    note("config2 stage")
    gout, gu1 = gpu_stage(bt, Z.RK4[1], bt.dt, u1_init=u1, u2=y)
    o64 = bt.u.copy()
    o64u1 = u1.copy()
    O.rk_stage(bt, bt.u, o64, o64u1, y, c, bt.dt)
    o80 = bt.u.copy()
    o80u1 = u1.copy()
    O.rk_stage(bt, bt.u, o80, o80u1, y, c, bt.dt, ext=True)
    rows = compare(bt, gout, o64, o80, base=y)
    assert_parity(rows, "config2 stage state - y\n" + report(rows))
    rows = compare(bt, gu1, o64u1, o80u1, base=u1)
    assert_parity(rows, "config2 stage accumulator increment\n" + report(rows))
    note("config2 constraints")
    plan = Z.plan_for(bt)
    cons, norms = zeros(bt.total_c), zeros(16 * len(bt.blocks))
    plan.constraints(dev(bt.u), dev(bt.matter), cons, norms)
    gc, gn = host(cons), host(norms).reshape(-1, 8, 2)
    c64, n64 = O.constraints(bt)
    c80, n80 = O.constraints(bt, ext=True)
    rows = compare(bt, gc, c64, c80, nfields=W.NC)
    assert_parity(rows, "config2 constraints\n" + report(rows))
    np.testing.assert_allclose(gn, n80, rtol=1e-10, atol=1e-300)


# --- random shapes --------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_random_shapes_rhs_and_stage(seed):
    Z = z4c()
    bt = W.random_batch(seed, nblocks=3, nmax=24)
    note(f"random shapes seed {seed}: " + ", ".join(f"{b.nx}x{b.ny}x{b.nz}/ng{b.ng}"
                                                  for b in bt.blocks)
         + f" p={bt.params.fd_order}")
    g = gpu_rhs(bt)
    rows = compare(bt, g, O.rhs(bt), O.rhs(bt, ext=True))
    assert_parity(rows, f"random {seed} rhs\n" + report(rows))
    gout, _ = gpu_stage(bt, Z.RK4[0], 0.01)
    o64 = bt.u.copy()
    o80 = bt.u.copy()
    O.rk_stage(bt, bt.u, o64, np.zeros_like(bt.u), bt.u, ORACLE_RK4[0], 0.01)
    O.rk_stage(bt, bt.u, o80, np.zeros_like(bt.u), bt.u, ORACLE_RK4[0], 0.01, ext=True)
    rows = compare(bt, gout, o64, o80, base=bt.u)
    assert_parity(rows, f"random {seed} stage\n" + report(rows))


def _launch_plan(bt, arith, tile, pers, waves):
    Z = z4c()
    plan = Z.plan_for(bt, arith)
    plan.set_launch(0, 0, 0, tile, pers, waves)
    return plan


def test_launch_shape_and_persistence_do_not_change_results():
    """Within one kernel family (the same per-point arithmetic) results are
    bitwise independent of tile shape, persistence (work-queue order) and
    tile order: two waves per SIMD (8x8x8 and 8x8x4 tiles), and one wave per
    SIMD (8x8x4 and 8x4x8, mixed derivatives in two passes, compared with the
    oracle in test_one_wave_variant_parity)."""
    Z = z4c()
    bt = W.random_batch(11, nblocks=4, nmax=30, fd_order=6)
    note("launch-shape invariance")
    families = {2: [((8, 8, 8), 0), ((8, 8, 4), 0), ((8, 8, 8), 7), ((8, 8, 4), 3),
                    ((8, 8, 8), 1), ((8, 8, 4), 1000)],
                1: [((8, 8, 4), 0), ((8, 8, 4), 5), ((8, 8, 4), 1), ((8, 8, 4), 1000),
                    ((8, 4, 8), 0), ((8, 4, 8), 3), ((8, 4, 8), 256)]}
    for waves, shapes in families.items():
        for arith in (Z.ARITH_FP64, Z.ARITH_FP32):
            ref = stage_ref = None
            for tile, pers in shapes:
                plan = _launch_plan(bt, arith, tile, pers, waves)
                r = gpu_rhs(bt, plan=plan)
                out, _ = gpu_stage(bt, Z.RK4[1], 0.01, u1_init=bt.u, plan=plan)
                if ref is None:
                    ref, stage_ref = r, out
                    continue
                assert np.array_equal(r, ref), (tile, pers, waves, arith)
                assert np.array_equal(out, stage_ref), (tile, pers, waves, arith)


@pytest.mark.parametrize("seed", [3, 17, 29])
def test_one_wave_variant_parity(seed):
    """The one-wave-per-SIMD kernels (two-pass mixed derivatives) against the
    oracle: right-hand side and a stage increment, FP64; flat space stays
    exactly zero in both arithmetic types."""
    Z = z4c()
    bt = W.random_batch(seed, nblocks=3, nmax=30, fd_order=6)
    note(f"one-wave variant seed {seed}: " + ", ".join(f"{b.nx}x{b.ny}x{b.nz}" for b in bt.blocks))
    g = gpu_rhs(bt, plan=_launch_plan(bt, Z.ARITH_FP64, (8, 8, 4), 0, 1))
    rows = compare(bt, g, O.rhs(bt), O.rhs(bt, ext=True))
    assert_parity(rows, f"one-wave {seed} rhs\n" + report(rows))
    g2 = gpu_rhs(bt, plan=_launch_plan(bt, Z.ARITH_FP64, (8, 4, 8), 7, 1))
    assert np.array_equal(g2, g)
    gout, _ = gpu_stage(bt, Z.RK4[1], 0.01, u1_init=bt.u,
                        plan=_launch_plan(bt, Z.ARITH_FP64, (8, 8, 4), 3, 1))
    o64 = bt.u.copy()
    o80 = bt.u.copy()
    O.rk_stage(bt, bt.u, o64, bt.u.copy(), bt.u, ORACLE_RK4[1], 0.01)
    O.rk_stage(bt, bt.u, o80, bt.u.copy(), bt.u, ORACLE_RK4[1], 0.01, ext=True)
    rows = compare(bt, gout, o64, o80, base=bt.u)
    assert_parity(rows, f"one-wave {seed} stage\n" + report(rows))
    flat = W.Batch([W.Block(9, 17, 6, 4, 0.1, 0.2, 0.3), W.Block(16, 16, 16, 4, 0.05, 0.05, 0.05)],
                   with_matter=False)
    W.fill_fields(flat, W.flat)
    flat.params = W.Params(fd_order=6, ko_sigma=0.5)
    for arith in (Z.ARITH_FP64, Z.ARITH_FP32):
        assert np.all(gpu_rhs(flat, plan=_launch_plan(flat, arith, (8, 8, 4), 0, 1)) == 0.0)


# --- level sets at full size (sampled oracle) -------------------------------------------

def test_config3_level_set_one_stage_sampled():
    Z = z4c()
    bt = W.config3()
    note("config3 full stage")
    plan = Z.plan_for(bt)
    out, _ = gpu_stage(bt, Z.RK4[0], bt.dt, plan=plan)
    plan_p = Z.plan_for(bt)
    plan_p.set_launch(0, 0, 0, (8, 8, 8), 512)
    out_p, _ = gpu_stage(bt, Z.RK4[0], bt.dt, plan=plan_p)
    assert np.array_equal(out, out_p)
    idx = np.random.default_rng(0).choice(len(bt.blocks), size=24, replace=False)
    sub = bt.subset(idx)
    o64 = sub.u.copy()
    o80 = sub.u.copy()
    O.rk_stage(sub, sub.u, o64, np.zeros_like(sub.u), sub.u, ORACLE_RK4[0], bt.dt)
    O.rk_stage(sub, sub.u, o80, np.zeros_like(sub.u), sub.u, ORACLE_RK4[0], bt.dt, ext=True)
    gsub = bt.subset(idx)
    for j, i in enumerate(idx):
        for f in range(W.NF):
            gsub.view(gsub.u, j, f)[...] = bt.view(out, i, f)
    rows = compare(sub, gsub.u, o64, o80, base=sub.u)
    assert_parity(rows, "config3 sampled stage\n" + report(rows))


def test_config4_graph_step_sampled():
    Z = z4c()
    bt = W.config4()
    O.ghost_fill(bt, bt.u)
    note("config4 eager and graph steps")
    plan = Z.plan_for(bt)
    frozen = None
    y = dev(bt.u)
    eager = [dev(bt.u), dev(bt.u), dev(bt.u), zeros(bt.total_u)]
    res = plan.step(eager, None, Z.RK4, bt.dt, Z.GHOST_PERIODIC, frozen)
    ref = host(eager[res])
    graph_regs = [dev(bt.u), dev(bt.u), dev(bt.u), zeros(bt.total_u)]
    for rep in range(3):
        graph_regs[0].copy_(y)
        torch.cuda.synchronize()
        # eager work of the program between replays
        scratch = torch.empty_like(y).copy_(y) * 1.0
        torch.cuda.synchronize()
        r = plan.step(graph_regs, None, Z.RK4, bt.dt, Z.GHOST_PERIODIC, frozen, graph=True)
        got = host(graph_regs[r])
        assert np.array_equal(got, ref), f"graph replay {rep} differs from eager"
        del scratch
    sizes = np.array([b.nx for b in bt.blocks])
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(np.nonzero(sizes == s)[0], size=4, replace=False)
                          for s in (8, 16, 24, 32)])
    sub = bt.subset(idx)
    o64 = O.rk_step(sub, sub.u.copy(), dt=bt.dt)
    o80 = O.rk_step(sub, sub.u.copy(), dt=bt.dt, ext=True)
    gsub = bt.subset(idx)
    for j, i in enumerate(idx):
        for f in range(W.NF):
            gsub.view(gsub.u, j, f)[...] = bt.view(ref, i, f)
    rows = compare(sub, gsub.u, o64, o80, base=sub.u)
    assert_parity(rows, "config4 sampled step increments\n" + report(rows))



def test_level_set_ssprk3_graph_step_sampled():
    """The paper's third-order Runge-Kutta (SSPRK(3,3)) on the benchmark's
    level set, ghosts through the periodic rule, in the launch shapes of the
    committed autotuning cache, graph-replayed: 16 sampled blocks (4 per
    size) against the oracle's step of the same blocks."""
    import os
    Z = z4c()
    bt = W.config4()
    O.ghost_fill(bt, bt.u)
    note("level set SSPRK3 graph step, 16 sampled blocks")
    Z.set_tune_cache(os.path.join(os.path.dirname(Z.__file__), "tune_gfx950.txt"))
    try:
        plan = Z.plan_for(bt)
        regs = [dev(bt.u), dev(bt.u), dev(bt.u), zeros(bt.total_u)]
        plan.set_halo(Z.GHOST_PERIODIC)
        plan.autotune(regs[0], regs[1], regs[3], None, reps=3)
        res = plan.step(regs, None, Z.SSPRK3, bt.dt, Z.GHOST_PERIODIC, None, graph=True)
        got = host(regs[res])
        plan.close()
    finally:
        Z.set_tune_cache(None)
    sizes = np.array([b.nx for b in bt.blocks])
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(np.nonzero(sizes == s)[0], size=4, replace=False)
                          for s in (8, 16, 24, 32)])
    sub = bt.subset(idx)
    o64 = O.rk_step(sub, sub.u.copy(), table=O.SSPRK3, dt=bt.dt)
    o80 = O.rk_step(sub, sub.u.copy(), table=O.SSPRK3, dt=bt.dt, ext=True)
    gsub = bt.subset(idx)
    for j, i in enumerate(idx):
        for f in range(W.NF):
            gsub.view(gsub.u, j, f)[...] = bt.view(got, i, f)
    rows = compare(sub, gsub.u, o64, o80, base=sub.u)
    assert_parity(rows, "level set ssprk3 sampled step increments\n" + report(rows))

def test_config5_reduced_neighbour_step():
    Z = z4c()
    bt = W.config5(n=24)
    O.ghost_fill(bt, bt.u)
    note("config5 reduced (8 x 24^3) rk4 step with neighbour ghosts")
    gs = gpu_step(bt, Z.RK4, bt.dt)
    o64 = O.rk_step(bt, bt.u.copy(), dt=bt.dt)
    o80 = O.rk_step(bt, bt.u.copy(), dt=bt.dt, ext=True)
    rows = compare(bt, gs, o64, o80, base=bt.u)
    assert_parity(rows, "config5 reduced step increments\n" + report(rows))


def test_config5_full_size_rhs_one_block():
    bt = W.config5()
    note("config5 full rhs")
    g = gpu_rhs(bt)
    sub = bt.subset([5])
    gsub = bt.subset([5])
    for f in range(W.NF):
        gsub.view(gsub.u, 0, f)[...] = bt.view(g, 5, f)
    rows = compare(sub, gsub.u, O.rhs(sub), O.rhs(sub, ext=True))
    assert_parity(rows, "config5 rhs block 5\n" + report(rows))


# --- ghosts through the refresh rule --------------------------------------------------

def test_steps_reading_ghosts_through_the_rule_equal_stored_refresh():
    """A step whose stages read ghost points through the refresh rule equals,
    bitwise, a step that refreshes the stored ghosts after every stage."""
    Z = z4c()
    cases = [W.config1(), W.config5(n=16)]
    fb = W.random_batch(8, nblocks=2, nmax=14, ng=4, fd_order=6)
    fb.ghost = W.GHOST_FROZEN
    fb.frozen = fb.u.copy() * (1.0 + 1e-3)
    cases.append(fb)
    for bt in cases:
        note(f"rule-read vs stored ghosts: {bt.name}")
        O.ghost_fill(bt, bt.u)
        plan = Z.plan_for(bt)
        frozen = dev(bt.frozen) if bt.frozen is not None else None
        outs = []
        for flags in (Z.STEP_STORED_GHOSTS, 0, Z.STEP_NO_FINAL_FILL):
            regs = [dev(bt.u), dev(bt.u), dev(bt.u), zeros(bt.total_u)]
            r = plan.step(regs, dev(bt.matter), Z.RK4, bt.dt, bt.ghost, frozen, flags=flags)
            outs.append(host(regs[r]))
        assert np.array_equal(outs[0], outs[1])      # whole array: final ghosts refreshed
        for b in range(len(bt.blocks)):
            for f in range(W.NF):
                assert np.array_equal(bt.interior(outs[0], b, f), bt.interior(outs[2], b, f))


def test_halo_reads_ignore_stale_stored_ghosts():
    Z = z4c()
    bt = W.config5(n=12)
    O.ghost_fill(bt, bt.u)
    ref = gpu_rhs(bt)
    stale = bt.u.copy()
    rng = np.random.default_rng(9)
    for b in range(len(bt.blocks)):
        for f in range(W.NF):
            v = bt.view(stale, b, f)
            g = bt.blocks[b].ng
            keep = v[g:-g, g:-g, g:-g].copy()
            v[...] = rng.normal(size=v.shape)
            v[g:-g, g:-g, g:-g] = keep
    plan = Z.plan_for(bt)
    fr = dev(bt.frozen)
    plan.set_halo(Z.GHOST_NEIGHBOUR, fr)
    u, out = dev(stale), zeros(bt.total_u)
    plan.rhs(u, dev(bt.matter), out)
    got = host(out)
    for b in range(len(bt.blocks)):
        for f in range(W.NF):
            assert np.array_equal(bt.interior(got, b, f), bt.interior(ref, b, f))


# --- ghosts, finiteness ------------------------------------------------------------------

def test_ghost_fill_matches_oracle_bitwise():
    Z = z4c()
    for bt in (W.config1(), W.config5(n=12), W.random_batch(3, nblocks=2, nmax=12, ng=4)):
        rng = np.random.default_rng(2)
        u = rng.normal(size=bt.u.shape)
        bt.frozen = rng.normal(size=bt.u.shape)
        policies = [Z.GHOST_PERIODIC, Z.GHOST_FROZEN]
        if bt.neighbours is not None:
            policies.append(Z.GHOST_NEIGHBOUR)
        for pol in policies:
            note(f"ghost fill {bt.name} policy {pol}")
            plan = Z.plan_for(bt)
            ud = dev(u)
            plan.ghost_fill(pol, ud, dev(bt.frozen))
            ref = u.copy()
            O.ghost_fill(bt, ref, pol)
            assert np.array_equal(host(ud), ref)


def test_check_finite_counts_bad_points():
    Z = z4c()
    bt = W.random_batch(4, nblocks=2, nmax=10)
    u = bt.u.copy()
    bt.interior(u, 1, 7)[0, 0, 0] = np.nan
    bt.interior(u, 0, 3)[-1, -1, -1] = np.inf
    bt.view(u, 0, 2)[0, 0, 0] = np.nan     # a ghost point: not counted
    plan = Z.plan_for(bt)
    assert plan.check_finite(dev(u)) == 2


def test_autotune_cache_round_trip(tmp_path):
    """The autotuner stores the shape it picked per size class in the cache
    file, and a second plan of the same level set takes it from there
    without timing (the same shapes, the file unchanged)."""
    Z = z4c()
    bt = W.random_batch(12, nblocks=3, nmax=20, fd_order=6)
    path = tmp_path / "tune.txt"
    Z.set_tune_cache(path)
    try:
        note("autotune cache")
        u0, out, u1 = dev(bt.u), dev(bt.u), dev(bt.u)
        p1 = Z.plan_for(bt)
        p1.autotune(u0, out, u1, dev(bt.matter), reps=1)
        text = path.read_text()
        assert len(text.strip().splitlines()) == len({(b.nx, b.ny, b.nz) for b in bt.blocks})
        assert "gfx950" in text and ":p6:" in text
        p2 = Z.plan_for(bt)
        p2.autotune(u0, out, u1, dev(bt.matter), reps=1)
        for b in bt.blocks:
            assert p1.get_launch(b.nx, b.ny, b.nz) == p2.get_launch(b.nx, b.ny, b.nz)
        assert path.read_text() == text
        # the tuned plan still matches the oracle
        g = gpu_rhs(bt, plan=p2)
        rows = compare(bt, g, O.rhs(bt), O.rhs(bt, ext=True))
        assert_parity(rows, "autotuned rhs\n" + report(rows))
    finally:
        Z.set_tune_cache(None)
