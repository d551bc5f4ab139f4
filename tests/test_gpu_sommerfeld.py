"""Radiative (Sommerfeld) outer boundary on the GPU against the oracle.

Workload: the star level set reduced to 8 blocks of 24^3 + 4 ghosts tiling
[-16, 16]^3 (star metric, matter blobs, 1e-6 noise), neighbour copies
between the blocks and the outer ghost points (the ghost regions of every
direction without a neighbour) advanced by the radiative law instead of
being frozen.  Checked with the parity metric of tests/parity.py:
* the radiative right-hand side at every outer point (nothing else written);
* one radiative stage (RK4 stage 2: accumulator read and written) at the
  outer points, as increments, other points untouched;
* one RK4 step with Z4C_STEP_SOMMERFELD against the oracle's step that
  advances the outer points in every stage: interior and outer points as
  increments; halo-rule and stored-ghost forms and the graph replay
  bitwise equal;
* the same on a two-level set with the exchange across the level jump;
* one SSPRK(3,3) step;
* the step flag together with the constraint monitor.
"""
import sys

import numpy as np
import pytest

import oracle as O
from parity import assert_parity, compare, outer_masks, report
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _batch():
    """The reduced star level set with its neighbour ghosts refreshed (so
    that the stored-ghost and halo-rule step forms start from the same data)
    and its outer ghosts as generated."""
    bt = W.config5(n=24)
    bt.frozen = None
    bt.sommerfeld = True
    O.ghost_fill(bt, bt.u)
    return bt


def test_radiative_rhs_at_outer_points():
    from paper_2311_04989_amd import z4c as Z
    bt = _batch()
    masks = outer_masks(bt)
    note(f"radiative rhs: 8 x 24^3 star level set, {sum(int(m.sum()) for m in masks)} outer points")
    plan = Z.plan_for(bt)
    u = dev(bt.u)
    rhs = torch.zeros_like(u)
    plan.sommerfeld_rhs(u, rhs)
    g = host(rhs)
    rows = compare(bt, g, O.sommerfeld_rhs(bt), O.sommerfeld_rhs(bt, ext=True), masks=masks)
    assert_parity(rows, "radiative rhs 8x24^3 outer points\n" + report(rows))
    for b in range(len(bt.blocks)):
        for f in range(W.NF):
            assert np.all(bt.view(g, b, f)[~masks[b]] == 0.0), (b, W.FIELDS[f])
    # Under the neighbour rule the samples at ghost points with a neighbour
    # come from the neighbour: stale stored values there change nothing.
    stale = bt.u.copy()
    for b, blk in enumerate(bt.blocks):
        ng = blk.ng
        inner = np.zeros(masks[b].shape, dtype=bool)
        inner[ng:ng + blk.nz, ng:ng + blk.ny, ng:ng + blk.nx] = True
        for f in range(W.NF):
            bt.view(stale, b, f)[~masks[b] & ~inner] = -7.0
    plan.set_halo(Z.GHOST_NEIGHBOUR)
    rhs2 = torch.zeros_like(u)
    plan.sommerfeld_rhs(dev(stale), rhs2)
    assert np.array_equal(host(rhs2), g)
    plan.close()
    # the law runs in FP64 whatever the plan's arithmetic
    p32 = Z.plan_for(bt, Z.ARITH_FP32)
    rhs3 = torch.zeros_like(u)
    p32.sommerfeld_rhs(u, rhs3)
    assert np.array_equal(host(rhs3), g)
    p32.close()


def test_radiative_stage_at_outer_points():
    from paper_2311_04989_amd import z4c as Z
    bt = _batch()
    masks = outer_masks(bt)
    note("radiative stage (RK4 stage 2): 8 x 24^3 star level set")
    rng = np.random.default_rng(17)
    u0 = bt.u.copy()
    u1_in = u0 * (1.0 + rng.uniform(-1e-3, 1e-3, size=u0.shape))
    plan = Z.plan_for(bt)
    gu0, gu1 = dev(u0), dev(u1_in)
    gout = torch.full_like(gu0, -7.0)
    plan.sommerfeld_stage(gu0, gout, gu1, gu0, Z.RK4[1], bt.dt)
    out, u1 = host(gout), host(gu1)
    res = {}
    for ext in (False, True):
        o, a1 = np.full_like(u0, -7.0), u1_in.copy()
        O.sommerfeld_stage(bt, u0, o, a1, u0, O.RK4[1], bt.dt, ext=ext)
        res[ext] = (o, a1)
    rows = compare(bt, out, res[False][0], res[True][0], base=u0, masks=masks)
    assert_parity(rows, "radiative stage u0' outer points\n" + report(rows))
    rows = compare(bt, u1, res[False][1], res[True][1], base=u1_in, masks=masks)
    assert_parity(rows, "radiative stage u1 outer points\n" + report(rows))
    for b in range(len(bt.blocks)):
        for f in range(W.NF):
            assert np.all(bt.view(out, b, f)[~masks[b]] == -7.0)
            assert np.array_equal(bt.view(u1, b, f)[~masks[b]], bt.view(u1_in, b, f)[~masks[b]])
    plan.close()


def test_rk4_step_with_radiative_outer_ghosts():
    from paper_2311_04989_amd import z4c as Z
    bt = _batch()
    masks = outer_masks(bt)
    note("RK4 step with radiative outer ghosts: 8 x 24^3 star level set")
    plan = Z.plan_for(bt)
    m = dev(bt.matter)
    finals = []
    graph_regs = [torch.empty(bt.total_u, dtype=torch.float64, device=DEV) for _ in range(4)]
    for flags, graph in ((0, False), (Z.STEP_STORED_GHOSTS, False), (0, True), (0, True)):
        if graph:   # the same registers twice: the second call replays the graph
            regs = graph_regs
            regs[0].copy_(dev(bt.u))
            for r in regs[1:]:
                r.fill_(-7.0)
        else:
            regs = [dev(bt.u)] + [torch.full((bt.total_u,), -7.0, dtype=torch.float64,
                                             device=DEV) for _ in range(3)]
        note(f"  step flags {flags} graph {graph}")
        res = plan.step(regs, m, Z.RK4, bt.dt, Z.GHOST_NEIGHBOUR, None, graph=graph,
                        flags=flags | Z.STEP_SOMMERFELD)
        finals.append(host(regs[res]))
    for q in range(1, len(finals)):
        assert np.array_equal(finals[q], finals[0]), f"step form {q} differs from the first"
    ref64 = O.rk_step(bt, bt.u.copy())
    ref80 = O.rk_step(bt, bt.u.copy(), ext=True)
    rows = compare(bt, finals[0], ref64, ref80, base=bt.u)
    assert_parity(rows, "RK4 step with radiative boundary, interior\n" + report(rows))
    rows = compare(bt, finals[0], ref64, ref80, base=bt.u, masks=masks)
    assert_parity(rows, "RK4 step with radiative boundary, outer points\n" + report(rows))
    # the outer points moved (the law is not the identity on this data)
    moved = sum(int(np.count_nonzero(bt.view(finals[0], b, W.F["chi"])[masks[b]]
                                      != bt.view(bt.u, b, W.F["chi"])[masks[b]]))
                for b in range(len(bt.blocks)))
    assert moved > 0
    plan.close()


def test_rk4_step_of_a_level_set_with_level_exchange_and_radiative_boundary():
    """A two-level set (19 blocks, one level-0 block refined into 8): one RK4
    step with the exchange across the level jump and the radiative outer
    boundary in every stage, against the oracle step (its stage, the
    radiative stage on the ghost regions without a same-level neighbour,
    then its level exchange, which overwrites those that another level
    owns).  The law's origin is the centre of a level-0 block away from the
    refined region, so that no ghost region without a same-level neighbour
    comes near r = 0; interior and those ghost regions are compared as
    increments; graph replay equals the eager step."""
    from oracle.intergrid import rk_step_levels
    from paper_2311_04989_amd import z4c as Z
    bt, locs = W.refined_level_set(refine=(1, 0, 0))
    rng = np.random.default_rng(71)
    for b, blk in enumerate(bt.blocks):
        X, Y, Zc = blk.coords()
        for f in range(W.NF):
            k = 2 * np.pi * np.array([1.0, 1.5, 2.0]) * (1 + 0.1 * f)
            base = 1.0 if W.FIELDS[f] in ("chi", "gxx", "gyy", "gzz", "alpha") else 0.0
            bt.view(bt.u, b, f)[...] = base + 2e-3 * np.sin(k[0] * X + k[1] * Y + k[2] * Zc + f)
    W.add_noise(bt, rng, 1e-7)
    bt.params = W.Params(fd_order=6, ko_sigma=0.5)
    bt.dt = 0.25 * min(b.dx for b in bt.blocks)
    # the radiative law's origin: the centre of the level-0 block spanning
    # [0, 0.5] x [0.5, 1] x [0.5, 1] (the refined block spans [0.5, 1] x
    # [0, 0.5] x [0, 0.5])
    centre = np.array([0.25, 0.75, 0.75])
    for b in bt.blocks:
        b.x0, b.y0, b.z0 = b.x0 - centre[0], b.y0 - centre[1], b.z0 - centre[2]
    bt.neighbours = W.level_neighbours(bt, locs)
    bt.frozen = None
    bt.sommerfeld = True
    masks = outer_masks(bt)
    note(f"two-level set with radiative boundary: {len(bt.blocks)} blocks, "
         f"{sum(int(m.sum()) for m in masks)} ghost points without a same-level neighbour")
    plan = Z.plan_for(bt)
    nlev = max(L for L, _ in locs) + 1
    xps = []
    for pair in range(nlev - 1):
        pro, res = Z.level_transfers(plan, locs, pair)
        xps.append(Z.XPlan(plan, pro, res, 6))
    plan.set_level_exchange(xps)
    regs = [torch.empty(bt.total_u, dtype=torch.float64, device=DEV) for _ in range(4)]
    finals = []
    for graph in (False, True, True):
        regs[0].copy_(dev(bt.u))
        for r in regs[1:]:
            r.copy_(regs[0])
        res = plan.step(regs, None, Z.RK4, bt.dt, Z.GHOST_NEIGHBOUR, None, graph=graph,
                        flags=Z.STEP_LEVEL_EXCHANGE | Z.STEP_SOMMERFELD)
        finals.append(host(regs[res]))
    assert np.array_equal(finals[1], finals[0]) and np.array_equal(finals[2], finals[0])
    o64 = rk_step_levels(bt, locs, bt.u, O.RK4, bt.dt, O, None, 6)
    o80 = rk_step_levels(bt, locs, bt.u, O.RK4, bt.dt, O, None, 6, ext=True)
    rows = compare(bt, finals[0], o64, o80, base=bt.u)
    assert_parity(rows, "two-level RK4 step with radiative boundary, interior\n" + report(rows))
    rows = compare(bt, finals[0], o64, o80, base=bt.u, masks=masks)
    assert_parity(rows, "two-level RK4 step with radiative boundary, ghost regions without a "
                  "same-level neighbour\n" + report(rows))
    plan.close()
    for x in xps:
        x.close()


def test_ssprk3_step_with_radiative_outer_ghosts():
    """The paper's third-order Runge-Kutta (read as SSPRK(3,3): u0 and the
    step's start state combined, no accumulator) with the radiative outer
    ghosts, against the oracle step."""
    from paper_2311_04989_amd import z4c as Z
    bt = _batch()
    masks = outer_masks(bt)
    note("SSPRK3 step with radiative outer ghosts: 8 x 24^3 star level set")
    plan = Z.plan_for(bt)
    regs = [dev(bt.u)] + [torch.full((bt.total_u,), -7.0, dtype=torch.float64, device=DEV)
                          for _ in range(3)]
    res = plan.step(regs, dev(bt.matter), Z.SSPRK3, bt.dt, Z.GHOST_NEIGHBOUR, None,
                    flags=Z.STEP_SOMMERFELD)
    got = host(regs[res])
    ref64 = O.rk_step(bt, bt.u.copy(), table=O.SSPRK3)
    ref80 = O.rk_step(bt, bt.u.copy(), table=O.SSPRK3, ext=True)
    rows = compare(bt, got, ref64, ref80, base=bt.u)
    assert_parity(rows, "SSPRK3 step with radiative boundary, interior\n" + report(rows))
    rows = compare(bt, got, ref64, ref80, base=bt.u, masks=masks)
    assert_parity(rows, "SSPRK3 step with radiative boundary, outer points\n" + report(rows))
    plan.close()


def test_radiative_step_with_the_constraint_monitor():
    """Z4C_STEP_SOMMERFELD together with Z4C_STEP_MONITOR: the monitor
    (constraints of the state the step starts from) and the new state equal
    bitwise those of the two flags used apart."""
    from paper_2311_04989_amd import z4c as Z
    bt = _batch()
    note("radiative step with the constraint monitor: 8 x 24^3 star level set")
    plan = Z.plan_for(bt)
    m = dev(bt.matter)
    nb = len(bt.blocks)

    def run(flags):
        regs = [dev(bt.u)] + [torch.full((bt.total_u,), -7.0, dtype=torch.float64, device=DEV)
                              for _ in range(3)]
        cons = torch.zeros(bt.total_c, dtype=torch.float64, device=DEV)
        norms = torch.zeros(16 * nb, dtype=torch.float64, device=DEV)
        mon = flags & Z.STEP_MONITOR
        res = plan.step(regs, m, Z.RK4, bt.dt, Z.GHOST_NEIGHBOUR, None, flags=flags,
                        cons=cons if mon else None, norms=norms if mon else None)
        return host(regs[res]), host(cons), host(norms)

    both = run(Z.STEP_SOMMERFELD | Z.STEP_MONITOR)
    som = run(Z.STEP_SOMMERFELD)
    mon = run(Z.STEP_MONITOR)
    assert np.array_equal(both[0], som[0])
    assert np.array_equal(both[1], mon[1]) and np.array_equal(both[2], mon[2])
    assert np.all(both[2][1::2] > 0.0)
    plan.close()
