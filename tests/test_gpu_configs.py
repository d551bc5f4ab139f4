"""GPU parity for parts of the scheme the configuration tests leave idle:
the chi/alpha floors (enforcement after a stage and max(chi, chi_floor) in
every 1/chi), the harmonic and frozen lapse, the frozen shift and no gauge
advection; the right-hand side of every stage inside full Runge-Kutta
steps (held to the right-hand-side gate, not only to the step increments),
on the gauge wave, the uneven level set and the full-size star level set;
and launch-to-launch reproducibility of the stage kernel at full size.
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


def Zm():
    from paper_2311_04989_amd import z4c as Z
    return Z


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _coeffs(c):
    return dict(zip(("delta", "eps", "g1", "g2", "g3", "beta", "read_u1", "write_u1"), c))


# --- floors ----------------------------------------------------------------------

def _floor_batch(seed):
    """Smooth data with chi = 1e-9 and alpha = -3 on random interior points
    (and on some ghost points, which only enter through the stencils)."""
    bt = W.random_batch(seed, nblocks=3, nmax=18, fd_order=6, amp=0.01)
    rng = np.random.default_rng(seed)
    for b in range(len(bt.blocks)):
        for name, val in (("chi", 1e-9), ("alpha", -3.0)):
            v = bt.view(bt.u, b, W.F[name])
            v[rng.random(v.shape) < 0.2] = val
    return bt


@pytest.mark.parametrize("seed", [21, 22])
def test_floors_in_rhs_and_stage(seed):
    Z = Zm()
    bt = _floor_batch(seed)
    p = bt.params
    note(f"floors seed {seed}: chi_floor {p.chi_floor}, alpha_floor {p.alpha_floor}")
    plan = Z.plan_for(bt)
    u = dev(bt.u)
    # right-hand side: 1/chi -> 1/max(chi, chi_floor) everywhere
    rhs = torch.zeros_like(u)
    plan.rhs(u, dev(bt.matter), rhs)
    rows = compare(bt, host(rhs), O.rhs(bt), O.rhs(bt, ext=True))
    assert_parity(rows, f"floors {seed} rhs\n" + report(rows))
    # identity stage (u0' = u0 before enforcement): every chi / alpha below
    # its floor is clamped to the floor exactly, the rest is unchanged
    ident = (0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0, 0)
    out = dev(bt.u)
    plan.rk_stage(u, out, None, None, dev(bt.matter), ident, 0.01)
    g = host(out)
    o64 = bt.u.copy()
    O.rk_stage(bt, bt.u, o64, np.zeros_like(bt.u), bt.u, _coeffs(ident), 0.01)
    nclamped = 0
    for b in range(len(bt.blocks)):
        for name, fl in (("chi", p.chi_floor), ("alpha", p.alpha_floor)):
            f = W.F[name]
            src = bt.interior(bt.u, b, f)
            got = bt.interior(g, b, f)
            low = src < fl
            nclamped += int(low.sum())
            assert np.all(got[low] == fl), (b, name)
            assert np.array_equal(got[~low], src[~low]), (b, name)
            assert np.array_equal(got, bt.interior(o64, b, f)), (b, name)
    assert nclamped > 100
    # a real RK4 stage: parity of the increments, and every point the oracle
    # clamps is clamped on the GPU to the same bits
    rng = np.random.default_rng(seed + 100)
    u1 = bt.u + rng.uniform(-1e-3, 1e-3, size=bt.u.shape)
    c = Z.RK4[1]
    out = dev(bt.u)
    u1d = dev(u1)
    plan.rk_stage(u, out, u1d, u, dev(bt.matter), c, 0.01)
    g = host(out)
    o64, o80 = bt.u.copy(), bt.u.copy()
    O.rk_stage(bt, bt.u, o64, u1.copy(), bt.u, _coeffs(c), 0.01)
    O.rk_stage(bt, bt.u, o80, u1.copy(), bt.u, _coeffs(c), 0.01, ext=True)
    rows = compare(bt, g, o64, o80, base=bt.u)
    assert_parity(rows, f"floors {seed} stage increments\n" + report(rows))
    for b in range(len(bt.blocks)):
        for name, fl in (("chi", p.chi_floor), ("alpha", p.alpha_floor)):
            f = W.F[name]
            clamped = bt.interior(o80, b, f) == fl
            assert np.all(bt.interior(g, b, f)[clamped] == fl), (b, name)
    plan.close()


# --- gauge options ------------------------------------------------------------------

GAUGES = [
    dict(lapse=W.LAPSE_HARMONIC, shift=W.SHIFT_GAMMADRIVER, advect_gauge=1),
    dict(lapse=W.LAPSE_FROZEN, shift=W.SHIFT_FROZEN, advect_gauge=0),
    dict(lapse=W.LAPSE_1PLUSLOG, shift=W.SHIFT_FROZEN, advect_gauge=1),
    dict(lapse=W.LAPSE_HARMONIC, shift=W.SHIFT_GAMMADRIVER, advect_gauge=0, eta=0.0),
]


@pytest.mark.parametrize("k", range(len(GAUGES)))
@pytest.mark.parametrize("p", [4, 6])
def test_gauge_options_rhs_and_stage(k, p):
    Z = Zm()
    bt = W.random_batch(40 + k, nblocks=2, nmax=20, fd_order=p, amp=0.02)
    for key, v in GAUGES[k].items():
        setattr(bt.params, key, v)
    note(f"gauge option {GAUGES[k]} p={p}")
    plan = Z.plan_for(bt)
    u = dev(bt.u)
    rhs = torch.zeros_like(u)
    plan.rhs(u, dev(bt.matter), rhs)
    g = host(rhs)
    rows = compare(bt, g, O.rhs(bt), O.rhs(bt, ext=True))
    assert_parity(rows, f"gauge {k} p{p} rhs\n" + report(rows))
    out = dev(bt.u)
    plan.rk_stage(u, out, torch.zeros_like(u), u, dev(bt.matter), Z.RK4[0], 0.01)
    o64, o80 = bt.u.copy(), bt.u.copy()
    O.rk_stage(bt, bt.u, o64, np.zeros_like(bt.u), bt.u, O.RK4[0], 0.01)
    O.rk_stage(bt, bt.u, o80, np.zeros_like(bt.u), bt.u, O.RK4[0], 0.01, ext=True)
    rows = compare(bt, host(out), o64, o80, base=bt.u)
    assert_parity(rows, f"gauge {k} p{p} stage\n" + report(rows))
    plan.close()


# --- every stage of a step held to the right-hand-side gate -------------------------------

def _stagewise(bt, plan, idx=None):
    """Run one RK4 step stage by stage on the GPU (ghosts through the refresh
    rule) and, before every stage, compare the GPU's right-hand side of that
    stage's input with the oracle's right-hand side of the same input (all
    blocks, or the sampled blocks `idx`)."""
    Z = Zm()
    frozen = dev(bt.frozen) if bt.frozen is not None else None
    plan.set_halo(bt.ghost, frozen)
    y = dev(bt.u)
    regs = [y, dev(bt.u), dev(bt.u), torch.zeros_like(y)]
    sched_in, sched_out = [0, 1, 2, 1], [1, 2, 1, 0]
    worst = 0.0
    for s in range(4):
        cur = regs[sched_in[s]]
        plan.ghost_fill(bt.ghost, cur, frozen)      # the stored ghosts the oracle reads
        rhs = torch.zeros_like(y)
        plan.rhs(cur, dev(bt.matter), rhs)
        ucur, g = host(cur), host(rhs)
        sub = bt if idx is None else bt.subset(idx)
        gsub = bt if idx is None else bt.subset(idx)
        if idx is not None:
            for j, i in enumerate(idx):
                for f in range(W.NF):
                    sub.view(sub.u, j, f)[...] = bt.view(ucur, i, f)
                    gsub.view(gsub.u, j, f)[...] = bt.view(g, i, f)
            uu, gg = sub.u, gsub.u
        else:
            uu, gg = ucur, g
        rows = compare(sub, gg, O.rhs(sub, u=uu), O.rhs(sub, u=uu, ext=True))
        assert_parity(rows, f"{bt.name} stage {s} rhs inside the step\n" + report(rows))
        worst = max(worst, max((eg / tol) for _, eg, _, tol, m in rows if m != 0.0))
        plan.rk_stage(cur, regs[sched_out[s]], regs[3], regs[0], dev(bt.matter), Z.RK4[s],
                      bt.dt)
    return host(regs[0]), worst


def test_config1_every_stage_rhs_at_the_rhs_gate():
    Z = Zm()
    bt = W.config1()
    O.ghost_fill(bt, bt.u)
    note("config1 stagewise")
    plan = Z.plan_for(bt)
    stepped, worst = _stagewise(bt, plan)
    # the stagewise step equals the fused step bitwise
    regs = [dev(bt.u), dev(bt.u), dev(bt.u), torch.zeros(bt.total_u, dtype=torch.float64,
                                                          device=DEV)]
    r = plan.step(regs, None, Z.RK4, bt.dt, Z.GHOST_PERIODIC, flags=Z.STEP_NO_FINAL_FILL)
    fused = host(regs[r])
    for f in range(W.NF):
        assert np.array_equal(bt.interior(stepped, 0, f), bt.interior(fused, 0, f))
    note(f"config1 stagewise worst e/tol {worst:.3f}")
    plan.close()


def test_config4_every_stage_rhs_at_the_rhs_gate_sampled():
    Z = Zm()
    bt = W.config4()
    O.ghost_fill(bt, bt.u)
    note("config4 stagewise (16 sampled blocks)")
    plan = Z.plan_for(bt)
    sizes = np.array([b.nx for b in bt.blocks])
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(np.nonzero(sizes == s)[0], size=4, replace=False)
                          for s in (8, 16, 24, 32)])
    _, worst = _stagewise(bt, plan, idx)
    note(f"config4 stagewise worst e/tol {worst:.3f}")
    plan.close()


def test_config5_full_size_every_stage_rhs_at_the_rhs_gate_sampled():
    """The full star level set (8 blocks of 128^3 with matter, neighbour
    ghosts between the blocks, frozen outer ghosts): one RK4 step stage by
    stage, each stage's right-hand side of block 6 (three neighbour faces,
    three frozen faces) against the oracle at the right-hand-side gate."""
    Z = Zm()
    bt = W.config5()
    note("config5 full size stagewise (block 6)")
    plan = Z.plan_for(bt)
    _, worst = _stagewise(bt, plan, [6])
    note(f"config5 stagewise worst e/tol {worst:.3f}")
    plan.close()


# --- reproducibility -------------------------------------------------------------------

@pytest.mark.parametrize("launch", [((8, 8, 4), 1), ((8, 8, 8), 2)])
def test_stage_kernel_bitwise_reproducible_over_20_launches(launch):
    """The adopted stage kernel, in one launch shape at the benchmark's full
    size, gives the same bits on 20 launches (u1 re-seeded each time)."""
    Z = Zm()
    bt = W.config4()
    note(f"reproducibility {launch}")
    plan = Z.plan_for(bt)
    plan.set_halo(Z.GHOST_PERIODIC)
    plan.set_launch(0, 0, 0, launch[0], 0, launch[1])
    u0 = dev(bt.u)
    u1_init = u0 * (1.0 + 1e-7)
    out = torch.empty_like(u0)
    u1 = torch.empty_like(u0)
    ref = ref1 = None
    for rep in range(20):
        out.fill_(0.0)
        u1.copy_(u1_init)
        plan.rk_stage(u0, out, u1, u0, None, Z.RK4[1], bt.dt)
        torch.cuda.synchronize()
        if ref is None:
            ref, ref1 = out.clone(), u1.clone()
        else:
            assert torch.equal(out, ref), f"launch {rep} differs"
            assert torch.equal(u1, ref1), f"launch {rep} accumulator differs"
    plan.close()
