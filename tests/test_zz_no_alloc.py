"""z4c_constraints_noalloc (partial sums in the library's static device
scratch, nothing allocated) against z4c_constraints, on the GPU: two calls in
a row through the C ABI, the second on a smaller level set, each equal
bitwise to the allocating entry point (same kernels, same summation order),
and both within the oracle's parity metric on one sampled block."""
import sys

import numpy as np
import pytest

import oracle as O
from parity import assert_parity, compare, report
from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_constraints_noalloc_matches_constraints_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_04989_amd import z4c as Z
    O.build(force=False)
    for label, bt in (("config2 64^3 + matter", W.config2()),
                      ("random 2 blocks", W.random_batch(7, nblocks=2, nmax=12, fd_order=6))):
        print(f"noalloc constraints: {label}", flush=True)
        sys.stdout.flush()
        plan = Z.plan_for(bt)
        u = torch.from_numpy(bt.u).to("cuda:0")
        m = None if bt.matter is None else torch.from_numpy(bt.matter).to("cuda:0")
        results = []
        for fn in (plan.constraints, plan.constraints_noalloc):
            cons = torch.full((bt.total_c,), -7.0, dtype=torch.float64, device="cuda:0")
            norms = torch.full((16 * len(bt.blocks),), -7.0, dtype=torch.float64,
                               device="cuda:0")
            fn(u, m, cons, norms)
            torch.cuda.synchronize()
            results.append((cons.cpu().numpy(), norms.cpu().numpy()))
        (c_ref, n_ref), (c_na, n_na) = results
        assert np.array_equal(c_na, c_ref), label
        assert np.array_equal(n_na, n_ref), label
        c64, n64 = O.constraints(bt)
        c80, n80 = O.constraints(bt, ext=True)
        rows = compare(bt, c_na, c64, c80, nfields=W.NC)
        assert_parity(rows, f"noalloc constraints {label}\n" + report(rows))
        np.testing.assert_allclose(n_na.reshape(-1, 8, 2), n80, rtol=1e-10, atol=1e-300)
        plan.close()
