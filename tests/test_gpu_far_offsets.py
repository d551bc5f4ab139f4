"""Blocks far into the state array (element offsets beyond 2^32), on the GPU.

The stage and constraint kernels address a block's own points, its periodic
images and the same point of `frozen` relative to the block's base (any
offset), and a point of another block under the neighbour rule by a 32-bit
element offset from the array base (the plan refuses that rule unless every
block named as a neighbour ends within 2^32 elements; a step then refreshes
stored ghosts instead).  Every case runs the same two blocks twice — packed
at the start of the arrays, and with block 1 moved beyond or up to the
2^32-element mark — and requires bitwise equal results.  The arrays of the
moved layout hold about 2^32 doubles (34 GB) each; at most five are live.
"""
import math
import sys

import numpy as np
import pytest

from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N = 12                     # interior points per direction, 4 ghosts
NPTS = (N + 8) ** 3        # stored points per field


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(autouse=True)
def _release():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def Zm():
    from paper_2311_04989_amd import z4c as Z
    return Z


def pair(seed):
    """Two 12^3 blocks (+4 ghosts) of smooth data, x-neighbours of each other
    (periodic pair along x; every other face reads `frozen`)."""
    rng = np.random.default_rng(seed)
    blocks = [W.Block(N, N, N, 4, 0.1, 0.1, 0.1, 0.0, 0.0, 0.0),
              W.Block(N, N, N, 4, 0.1, 0.1, 0.1, 1.2, 0.0, 0.0)]
    bt = W.Batch(blocks)
    for b, blk in enumerate(bt.blocks):
        X, Y, Zc = blk.coords()
        for f in range(W.NF):
            kx, ky, kz = rng.uniform(0.5, 2.0, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            base = 1.0 if W.FIELDS[f] in ("chi", "gxx", "gyy", "gzz", "alpha") else 0.0
            bt.view(bt.u, b, f)[...] = base + 0.01 * np.sin(kx * X + ky * Y + kz * Zc + ph)
    bt.params = W.Params(fd_order=6, ko_sigma=0.3, kappa1=0.02, kappa2=0.1)
    nbr = np.full((2, 27), -1, dtype=np.int32)
    for b in range(2):
        nbr[b, 13] = b
        nbr[b, 12] = nbr[b, 14] = 1 - b          # -x and +x
    bt.neighbours = nbr
    bt.frozen = bt.u * (1.0 + 1e-3)
    return bt


class Layout:
    """Block table and array length with block 1 at element offset `off1`."""

    def __init__(self, bt, off1=None):
        self.bt = bt
        self.table = bt.block_table()
        if off1 is not None:
            assert off1 >= int(self.table[0]["offset"]) + W.NF * int(bt.field_stride[0])
            self.table[1]["offset"] = off1
        self.length = max(int(r["offset"]) + W.NF * int(r["field_stride"]) for r in self.table)

    def plan(self):
        Z = Zm()
        p = Z.Plan(Z.make_params(self.bt.params), Z.make_blocks(self.table), 0)
        p.set_neighbours(self.bt.neighbours)
        return p

    def device(self, host=None):
        """A device array of the layout; the block regions hold `host` (packed
        layout) or zeros, the rest is never read or written."""
        d = torch.empty(self.length, dtype=torch.float64, device=DEV)
        for b in range(2):
            o, n = int(self.table[b]["offset"]), W.NF * int(self.bt.field_stride[b])
            c = int(self.bt.offsets[b])
            src = torch.zeros(n, dtype=torch.float64) if host is None else \
                torch.from_numpy(np.ascontiguousarray(host[c:c + n]))
            d[o:o + n].copy_(src.to(DEV))
        return d

    def host(self, d):
        """The block regions of a device array, back in the packed layout."""
        torch.cuda.synchronize()
        out = np.zeros(self.bt.total_u)
        for b in range(2):
            o, n = int(self.table[b]["offset"]), W.NF * int(self.bt.field_stride[b])
            c = int(self.bt.offsets[b])
            out[c:c + n] = d[o:o + n].cpu().numpy()
        return out


def same_interior(bt, a, b, what):
    for blk in range(2):
        for f in range(W.NF):
            assert np.array_equal(bt.interior(a, blk, f), bt.interior(b, blk, f)), \
                f"{what}: block {blk} field {W.FIELDS[f]} differs"


def rhs_and_stage(L, halo):
    Z = Zm()
    plan = L.plan()
    frozen = L.device(L.bt.frozen) if halo in (Z.GHOST_NEIGHBOUR, Z.GHOST_FROZEN) else None
    plan.set_halo(halo, frozen)
    u = L.device(L.bt.u)
    rhs = L.device()
    plan.rhs(u, None, rhs)
    r = L.host(rhs)
    del rhs
    out = L.device()
    u1 = L.device(L.bt.u * 0.5)
    plan.rk_stage(u, out, u1, u, None, Z.RK4[1], L.bt.dt)
    o, o1 = L.host(out), L.host(u1)
    plan.close()
    return r, o, o1


def test_periodic_rule_beyond_2_32_elements():
    Z = Zm()
    bt = pair(1)
    far = (1 << 32) + 64
    note(f"periodic halo reads, block 1 at element offset {far}")
    packed = rhs_and_stage(Layout(bt), Z.GHOST_PERIODIC)
    moved = rhs_and_stage(Layout(bt, far), Z.GHOST_PERIODIC)
    for a, b, what in zip(packed, moved, ("rhs", "u0'", "u1")):
        same_interior(bt, a, b, what)
    assert np.abs(packed[0]).max() > 0


def constraints(L, halo):
    Z = Zm()
    plan = L.plan()
    frozen = L.device(L.bt.frozen) if halo == Z.GHOST_NEIGHBOUR else None
    plan.set_halo(halo, frozen)
    u = L.device(L.bt.u)
    cons = torch.zeros(L.bt.total_c, dtype=torch.float64, device=DEV)
    norms = torch.zeros(2 * 16, dtype=torch.float64, device=DEV)
    plan.constraints(u, None, cons, norms)
    torch.cuda.synchronize()
    res = cons.cpu().numpy(), norms.cpu().numpy()
    plan.close()
    return res


def test_constraints_beyond_2_32_elements():
    Z = Zm()
    bt = pair(2)
    far = (1 << 32) + 64
    note(f"constraints with periodic halo reads, block 1 at element offset {far}")
    c0, n0 = constraints(Layout(bt), Z.GHOST_PERIODIC)
    c1, n1 = constraints(Layout(bt, far), Z.GHOST_PERIODIC)
    assert np.array_equal(c0, c1)
    assert np.array_equal(n0, n1)
    assert np.abs(n0).max() > 0


def test_neighbour_rule_up_to_the_limit():
    """Block 1 ends exactly at element 2^32 (its later fields lie beyond it):
    the neighbour rule reads it through 32-bit offsets from the array base."""
    Z = Zm()
    bt = pair(3)
    edge = (1 << 32) - NPTS
    note(f"neighbour halo reads, block 1 at element offset {edge}")
    packed = rhs_and_stage(Layout(bt), Z.GHOST_NEIGHBOUR)
    moved = rhs_and_stage(Layout(bt, edge), Z.GHOST_NEIGHBOUR)
    for a, b, what in zip(packed, moved, ("rhs", "u0'", "u1")):
        same_interior(bt, a, b, what)
    c0, n0 = constraints(Layout(bt), Z.GHOST_NEIGHBOUR)
    c1, n1 = constraints(Layout(bt, edge), Z.GHOST_NEIGHBOUR)
    assert np.array_equal(c0, c1) and np.array_equal(n0, n1)


def test_step_beyond_the_neighbour_limit_refreshes_stored_ghosts():
    """Block 1 one element past the limit: the plan refuses neighbour-rule
    halo reads, and a step under the neighbour policy refreshes stored ghosts
    instead, with bitwise the same result as the packed layout's halo-read
    step (interior and refreshed ghosts)."""
    Z = Zm()
    bt = pair(4)
    res = []
    for off1 in (None, (1 << 32) - NPTS + 2):
        L = Layout(bt, off1)
        note(f"RK4 step, neighbour policy, block 1 at {off1}")
        plan = L.plan()
        frozen = L.device(bt.frozen)
        if off1 is not None:
            with pytest.raises(Z.Z4cError) as e:
                plan.set_halo(Z.GHOST_NEIGHBOUR, frozen)
            assert e.value.status == Z.ENOTSUP
        regs = [L.device(bt.u), L.device(bt.u), L.device(bt.u), L.device()]
        r = plan.step(regs, None, Z.RK4, bt.dt, Z.GHOST_NEIGHBOUR, frozen)
        res.append(L.host(regs[r]))
        plan.close()
        del regs, frozen
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    for blk in range(2):
        for f in range(W.NF):
            assert np.array_equal(bt.view(res[0], blk, f), bt.view(res[1], blk, f)), \
                f"block {blk} field {W.FIELDS[f]} differs"
    assert not np.array_equal(res[0], bt.u)
