"""FP32-arithmetic right-hand side against the oracle, on the GPU.

The FP32 form keeps storage, the stencil differences u_m - u_0 and the
Runge-Kutta combination in double and runs the derivatives, dissipation and
the pointwise algebra in float.  Its error is measured against the
extended-precision oracle with the metric of tests/parity.py (per field,
relative to max(|o|, 1e-3 max|o_f|)), and the gate is fixed by the
arithmetic, not by the GPU result:

    tol_f = max(8 e32_f, 8 * 2^-24),

where e32_f is the same error of the FP32 reference build of the oracle
(float working type, differences formed in double): the GPU's FP32 path must
be within 8x of what a plain FP32 evaluation of the same formulas loses
(the FP64 gate uses the same factor against the FP64 oracle).

The naive form (every sample rounded to float before the differences) is
built as well.  On data whose perturbations sit near float resolution (the
star metric with U(-1e-6, 1e-6) noise of the precision study) its error
exceeds that gate by orders of magnitude on the fields whose right-hand side
is carried by the perturbation (the diagonal conformal metric, whose
right-hand side there is dissipation of the noise), which is why the
differences stay in double.  The naive kernel itself is checked against the
naive reference build with the same rule.
"""
import sys

import numpy as np
import pytest

import oracle as O
from parity import assert_parity, compare, report
from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
FLOOR = 8 * U32


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_rhs(bt, arith, launch=None):
    from paper_2311_04989_amd import z4c as Z
    plan = Z.plan_for(bt, arith)
    if launch is not None:
        plan.set_launch(0, 0, 0, launch[0], 0, launch[1])
    out = torch.zeros(bt.total_u, dtype=torch.float64, device="cuda:0")
    plan.rhs(dev(bt.u), dev(bt.matter), out)
    torch.cuda.synchronize()
    r = out.cpu().numpy()
    plan.close()
    return r


def _cases():
    c1 = W.config1()
    O.ghost_fill(c1, c1.u)
    c5 = W.config5(n=16)
    O.ghost_fill(c5, c5.u)
    return [("config1", c1, None), ("config2", W.config2(), None),
            ("random0", W.random_batch(0, nblocks=3, nmax=24), None),
            ("random1", W.random_batch(1, nblocks=3, nmax=24, fd_order=6), ((8, 8, 4), 1)),
            ("random2", W.random_batch(2, nblocks=3, nmax=24), ((8, 8, 8), 2)),
            ("config5 8x16^3", c5, None)]


@pytest.mark.parametrize("case", range(6))
def test_fp32_rhs_within_fp32_reference_error(case):
    from paper_2311_04989_amd import z4c as Z
    name, bt, launch = _cases()[case]
    note(f"fp32 rhs {name} launch {launch}")
    g = gpu_rhs(bt, Z.ARITH_FP32, launch)
    rows = compare(bt, g, O.rhs(bt, ext="f32"), O.rhs(bt, ext=True), gate=FLOOR)
    assert_parity(rows, f"fp32 {name} rhs (gate 8x the FP32 reference)\n" + report(rows))


def test_naive_fp32_breaks_the_fp32_gate_on_near_resolution_noise():
    from paper_2311_04989_amd import z4c as Z
    bt = W.config5(n=16)
    O.ghost_fill(bt, bt.u)
    note("naive fp32 rhs config5 8x16^3")
    o80 = O.rhs(bt, ext=True)
    mixed_rows = compare(bt, gpu_rhs(bt, Z.ARITH_FP32), O.rhs(bt, ext="f32"), o80, gate=FLOOR)
    naive = gpu_rhs(bt, Z.ARITH_FP32_NAIVE)
    # the naive kernel is what it claims to be: within 8x the naive reference
    naive_rows = compare(bt, naive, O.rhs(bt, ext="f32naive"), o80, gate=FLOOR)
    assert_parity(naive_rows, "naive fp32 against the naive reference\n" + report(naive_rows))
    # ... and it breaks the gate of the mixed form
    tol = {n: t for n, eg, ec, t, m in mixed_rows}
    err = {n: eg for n, eg, ec, t, m in naive_rows}
    broken = [n for n in tol if err[n] > tol[n]]
    msg = "\n".join(f"  {n:6s} naive {err[n]:.2e} vs gate {tol[n]:.2e}" for n in tol)
    for n in ("gxx", "gyy", "gzz"):
        assert err[n] > 1e3 * tol[n], f"{n}: naive form within 1000x of the gate\n{msg}"
    assert len(broken) >= 15, f"naive form breaks the gate on only {broken}\n{msg}"
    note(msg)


def test_naive_form_is_refused_for_stages():
    from paper_2311_04989_amd import z4c as Z
    bt = W.random_batch(4, nblocks=1, nmax=10, fd_order=6)
    plan = Z.plan_for(bt, Z.ARITH_FP32_NAIVE)
    u = dev(bt.u)
    out = torch.zeros_like(u)
    with pytest.raises(Z.Z4cError) as e:
        plan.rk_stage(u, out, torch.zeros_like(u), u, None, Z.RK4[0], 0.01)
    assert e.value.status == Z.ENOTSUP


def test_fp32_rhs_on_the_level_set_sampled():
    """The benchmark's FP32 configuration: the uneven level set (1,024 blocks,
    ghosts through the periodic rule) in the launch shapes of the committed
    autotuning cache; 16 sampled blocks (4 per size) against the FP32
    reference gate."""
    import os
    from paper_2311_04989_amd import z4c as Z
    bt = W.config4()
    O.ghost_fill(bt, bt.u)
    note("fp32 rhs level set, 16 sampled blocks")
    cache = os.path.join(os.path.dirname(Z.__file__), "tune_gfx950.txt")
    Z.set_tune_cache(cache)
    try:
        plan = Z.plan_for(bt, Z.ARITH_FP32)
        u = dev(bt.u)
        scratch = [torch.empty_like(u), torch.empty_like(u)]
        plan.set_halo(Z.GHOST_PERIODIC)
        plan.autotune(u, scratch[0], scratch[1], None, reps=3)
        note(f"launch shapes {dict((n, plan.get_launch(n, n, n)) for n in (8, 16, 24, 32))}")
        out = torch.zeros_like(u)
        plan.rhs(u, None, out)
        torch.cuda.synchronize()
        g = out.cpu().numpy()
        plan.close()
    finally:
        Z.set_tune_cache(None)
    sizes = np.array([b.nx for b in bt.blocks])
    rng = np.random.default_rng(32)
    idx = np.concatenate([rng.choice(np.nonzero(sizes == s)[0], size=4, replace=False)
                          for s in (8, 16, 24, 32)])
    sub = bt.subset(idx)
    gsub = bt.subset(idx)
    for j, i in enumerate(idx):
        for f in range(W.NF):
            gsub.view(gsub.u, j, f)[...] = bt.view(g, i, f)
    rows = compare(sub, gsub.u, O.rhs(sub, ext="f32"), O.rhs(sub, ext=True), gate=FLOOR)
    assert_parity(rows, "fp32 level set sampled rhs (gate 8x the FP32 reference)\n" + report(rows))


@pytest.mark.parametrize("launch", [None, ((8, 8, 4), 1)])
def test_fp32_rhs_through_the_neighbour_rule(launch):
    """FP32 arithmetic in the kernels that read their halo through the
    neighbour rule (neighbour copies between the 8 blocks, frozen outer
    faces): the GPU reads the stored state with its ghosts as generated, the
    oracle the same state after a ghost refresh; the FP32 gate applies."""
    from paper_2311_04989_amd import z4c as Z
    bt = W.config5(n=16)
    filled = bt.u.copy()
    O.ghost_fill(bt, filled)
    note(f"fp32 rhs config5 8x16^3 through the neighbour rule, launch {launch}")
    plan = Z.plan_for(bt, Z.ARITH_FP32)
    frozen = dev(bt.frozen)
    plan.set_halo(Z.GHOST_NEIGHBOUR, frozen)
    if launch is not None:
        plan.set_launch(0, 0, 0, launch[0], 0, launch[1])
    out = torch.zeros(bt.total_u, dtype=torch.float64, device="cuda:0")
    plan.rhs(dev(bt.u), dev(bt.matter), out)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    plan.close()
    rows = compare(bt, g, O.rhs(bt, filled, ext="f32"), O.rhs(bt, filled, ext=True), gate=FLOOR)
    assert_parity(rows, f"fp32 config5 neighbour rule rhs {launch}\n" + report(rows))
