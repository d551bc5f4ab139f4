"""z4c_constraints_noalloc captured in a HIP graph (through torch's graph
capture on its capture stream) and replayed: the call allocates nothing and
issues only kernel launches, which is what lets a caller capture it.  The
graph is replayed three times with eager work between the replays (the
state is rescaled), and every replay's constraint fields and norms equal
bitwise those of an eager z4c_constraints call on the same state."""
import sys

import numpy as np
import pytest

from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_constraints_noalloc_replayed_from_a_captured_graph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_04989_amd import z4c as Z
    bt = W.random_batch(6, nblocks=3, nmax=16, fd_order=6)
    print("noalloc constraints in a captured graph: random 3 blocks", flush=True)
    sys.stdout.flush()
    plan = Z.plan_for(bt)
    dev = "cuda:0"
    u = torch.from_numpy(bt.u).to(dev)
    m = torch.from_numpy(bt.matter).to(dev)
    cons = torch.zeros(bt.total_c, dtype=torch.float64, device=dev)
    norms = torch.zeros(16 * len(bt.blocks), dtype=torch.float64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):          # warm-up off the default stream
        plan.constraints_noalloc(u, m, cons, norms, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.constraints_noalloc(u, m, cons, norms, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        u.mul_(1.0 + 1e-3 * (rep + 1))       # eager work between the replays
        cons.fill_(-7.0)
        norms.fill_(-7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got_c, got_n = cons.cpu().numpy(), norms.cpu().numpy()
        ref_c = torch.full_like(cons, -7.0)
        ref_n = torch.full_like(norms, -7.0)
        plan.constraints(u, m, ref_c, ref_n)
        torch.cuda.synchronize()
        assert np.array_equal(got_c, ref_c.cpu().numpy()), f"replay {rep}: fields differ"
        assert np.array_equal(got_n, ref_n.cpu().numpy()), f"replay {rep}: norms differ"
        assert np.all(got_n[1::2] > 0.0)
    del g
    plan.close()
