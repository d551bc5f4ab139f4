"""The largest block the library takes, on the GPU: 800^3 interior points
with 4 ghosts, 808^3 = 527,514,112 stored points per field (the limit is
2^29 = 536,870,912), 92.8 GB per state array.  The kernels address a
block's points as 32-bit byte offsets from the field base, up to 4.22e9 of
the 4.29e9 a 32-bit offset holds here.

Smooth data is generated on the GPU field by field; the right-hand side and
the constraints of the whole block run on the GPU; at sampled points (the
eight corners of the interior and random ones) the oracle evaluates the
same quantities on the point's stencil neighbourhood (a 1^3-interior block
with the same 4 ghost layers cut out of the big array, which is all a
point's right-hand side reads), and the parity metric of tests/parity.py
applies per field over the samples.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from parity import assert_parity, compare, report
from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, NG = 800, 4
S = N + 2 * NG
NPTS = S ** 3
H = 0.01


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def fill(u):
    """Field f: base_f + a_f sin(kx x + p) sin(ky y + q) sin(kz z + r) over
    the stored points (x = (i - ng) h), built in place field by field."""
    rng = np.random.default_rng(7)
    x = (torch.arange(S, dtype=torch.float64, device="cuda:0") - NG) * H
    for f in range(W.NF):
        kx, ky, kz = rng.uniform(0.5, 3.0, size=3)
        p, q, r = rng.uniform(0, 2 * math.pi, size=3)
        base = 1.0 if W.FIELDS[f] in ("chi", "gxx", "gyy", "gzz", "alpha") else 0.0
        amp = 0.02 if base else 0.05
        v = u[f * NPTS:(f + 1) * NPTS].view(S, S, S)
        sz = torch.sin(kz * x + r)
        sy = torch.sin(ky * x + q)
        sx = torch.sin(kx * x + p)
        v.copy_(sz[:, None, None] * sy[None, :, None])
        v.mul_(sx[None, None, :])
        v.mul_(amp)
        v.add_(base)


def samples():
    corners = [(a, b, c) for a in (0, N - 1) for b in (0, N - 1) for c in (0, N - 1)]
    rng = np.random.default_rng(11)
    rand = [tuple(int(v) for v in rng.integers(0, N, size=3)) for _ in range(8)]
    return corners + rand


def windows(arr, nfields, pts):
    """Batch of 1^3-interior blocks (4 ghosts), one per sample, holding the
    9^3 stencil neighbourhood of each sample point of `arr`."""
    blocks = [W.Block(1, 1, 1, NG, H, H, H) for _ in pts]
    bt = W.Batch(blocks)
    bt.params = W.Params(fd_order=6, ko_sigma=0.5)
    view = arr.view(nfields, S, S, S)
    for b, (i, j, k) in enumerate(pts):
        w = view[:, k:k + 2 * NG + 1, j:j + 2 * NG + 1, i:i + 2 * NG + 1].cpu().numpy()
        for f in range(nfields):
            bt.view(bt.u, b, f)[...] = w[f]
    return bt


def test_largest_block_rhs_and_constraints_sampled():
    from paper_2311_04989_amd import z4c as Z
    note(f"largest block {N}^3 + {NG} ghosts: {NPTS} stored points per field")
    table = np.zeros(1, dtype=W.BLOCK_DTYPE)
    table[0] = (0, 0, 0, NPTS, N, N, N, NG, H, H, H)
    plan = Z.Plan(Z.make_params(W.Params(fd_order=6, ko_sigma=0.5)), Z.make_blocks(table), 0)
    u = torch.empty(W.NF * NPTS, dtype=torch.float64, device="cuda:0")
    fill(u)
    pts = samples()
    bt = windows(u, W.NF, pts)

    rhs = torch.zeros_like(u)
    plan.rhs(u, None, rhs)
    torch.cuda.synchronize()
    rv = rhs.view(W.NF, S, S, S)
    g = np.zeros(bt.total_u)
    for b, (i, j, k) in enumerate(pts):
        vals = rv[:, k + NG, j + NG, i + NG].cpu().numpy()
        for f in range(W.NF):
            bt.view(g, b, f)[NG, NG, NG] = vals[f]
    del rhs, rv
    torch.cuda.empty_cache()
    rows = compare(bt, g, O.rhs(bt), O.rhs(bt, ext=True))
    assert_parity(rows, f"largest block {N}^3 rhs at {len(pts)} points\n" + report(rows))

    cons = torch.zeros(W.NC * NPTS, dtype=torch.float64, device="cuda:0")
    norms = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    plan.constraints(u, None, cons, norms)
    torch.cuda.synchronize()
    cv = cons.view(W.NC, S, S, S)
    gc = np.zeros(bt.total_c)
    for b, (i, j, k) in enumerate(pts):
        vals = cv[:, k + NG, j + NG, i + NG].cpu().numpy()
        for q in range(W.NC):
            bt.view(gc, b, q, W.NC)[NG, NG, NG] = vals[q]
    c64, _ = O.constraints(bt)
    c80, _ = O.constraints(bt, ext=True)
    rows = compare(bt, gc, c64, c80, nfields=W.NC)
    assert_parity(rows, f"largest block {N}^3 constraints at {len(pts)} points\n" + report(rows))
    assert np.isfinite(norms.cpu().numpy()).all()
    plan.close()
    del u, cons
