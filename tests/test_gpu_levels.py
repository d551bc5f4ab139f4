"""One RK4 step of a multi-level MeshBlock set on the GPU with the ghost
exchange across level jumps between stages, against the oracle.

All levels advance with one global time step (no subcycling, Sec. 3.1).
After every stage the GPU step (Z4C_STEP_LEVEL_EXCHANGE) refreshes the stored
ghosts of the stage output: same-level copies and frozen outer faces, then
the restrictions and prolongations of z4c_level_transfers (Sec. 3.2,
vertex-centred).  The oracle step applies its own stage and, between stages,
oracle.intergrid.level_exchange, which fills every ghost point from the block
that owns its position (copy, injection or Lagrange interpolation), computed
from the block positions alone -- not from the library's transfer lists.
Both levels sets are 2:1 balanced (no ghost point lies two levels away).
"""
import sys

import numpy as np
import pytest

import oracle as O
from oracle.intergrid import rk_step_levels, level_exchange
from parity import assert_parity, compare, report
from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [dict(refine=(1, 0, 0)), dict(refine=(0, 0, 0), refine2=0)]


def _level_set(case):
    bt, locs = W.refined_level_set(**CASES[case])
    rng = np.random.default_rng(60 + case)
    for b, blk in enumerate(bt.blocks):
        X, Y, Z = blk.coords()
        for f in range(W.NF):
            base = 1.0 if W.FIELDS[f] in ("chi", "gxx", "gyy", "gzz", "alpha") else 0.0
            k = 2 * np.pi * np.array([1.0, 1.5, 2.0]) * (1 + 0.1 * f)
            bt.view(bt.u, b, f)[...] = base + 2e-3 * np.sin(k[0] * X + k[1] * Y + k[2] * Z + f)
    W.add_noise(bt, rng, 1e-7)
    bt.params = W.Params(fd_order=6, ko_sigma=0.5)
    bt.frozen = bt.u.copy()
    bt.dt = 0.25 * min(b.dx for b in bt.blocks)
    return bt, locs


@pytest.mark.parametrize("case", range(len(CASES)))
def test_rk4_step_with_level_exchange(case):
    from paper_2311_04989_amd import z4c as Z
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    bt, locs = _level_set(case)
    nlev = max(L for L, _ in locs) + 1
    print(f"multi-level step: {bt.name} ({len(bt.blocks)} blocks, {nlev} levels)", flush=True)
    sys.stdout.flush()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")   # noqa: E731
    plan = Z.plan_for(bt)
    plan.set_neighbours(W.level_neighbours(bt, locs))
    xps = []
    for pair in range(nlev - 1):
        pro, res = Z.level_transfers(plan, locs, pair)
        xps.append(Z.XPlan(plan, pro, res, 6))
    plan.set_level_exchange(xps)
    frozen = dev(bt.frozen)
    for graph in (False, True):
        regs = [dev(bt.u), dev(bt.u), dev(bt.u), torch.zeros(bt.total_u, dtype=torch.float64,
                                                              device="cuda:0")]
        r = plan.step(regs, None, Z.RK4, bt.dt, Z.GHOST_NEIGHBOUR, frozen, graph=graph,
                      flags=Z.STEP_LEVEL_EXCHANGE)
        torch.cuda.synchronize()
        got = regs[r].cpu().numpy()
        if not graph:
            eager = got
        else:
            assert np.array_equal(got, eager), "graph replay differs from the eager step"
    o64 = rk_step_levels(bt, locs, bt.u, O.RK4, bt.dt, O, bt.frozen, 6)
    o80 = rk_step_levels(bt, locs, bt.u, O.RK4, bt.dt, O, bt.frozen, 6, ext=True)
    rows = compare(bt, eager, o64, o80, base=bt.u)
    assert_parity(rows, f"multi-level RK4 step {case}\n" + report(rows))
    # the final ghosts are the exchange of the final interiors
    ref = level_exchange(bt, locs, eager, bt.frozen, 6)
    np.testing.assert_allclose(eager, ref, rtol=1e-13, atol=1e-15)
    for x in xps:
        x.close()
    plan.close()
