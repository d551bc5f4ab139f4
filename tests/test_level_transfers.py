"""Bookkeeping of a ghost exchange across a level jump (z4c_level_transfers,
host only): on a level set with one refined block among coarse neighbours,
the transfers cover exactly the ghost points a brute-force ownership scan
assigns -- every ghost point of a fine block in a coarse block's span is
prolongated from that block (with the right c0), every ghost point of a
coarse block in a fine block's span is restricted from that block, nothing
else -- and the sets pass the transfer-plan
validation (stencils inside the sources' stored points, no overlaps)."""
import numpy as np
import pytest

from paper_2311_04989_amd import workloads as W
from paper_2311_04989_amd import z4c as Z


def _plan(bt):
    return Z.Plan(Z.make_params(bt.params), Z.make_blocks(bt.block_table()), Z.PLAN_NO_DEVICE)


def step(locs, lev):
    return 1 << (max(L for L, _ in locs) - lev)


def owner(bt, locs, X):
    """Block whose span [o, o + n step) holds lattice point X (the spans
    tile the level set), or None outside it."""
    found = [b for b, (blk, (lev, o)) in enumerate(zip(bt.blocks, locs))
             if all(o[d] <= X[d] < o[d] + n * step(locs, lev)
                    for d, n in enumerate((blk.nx, blk.ny, blk.nz)))]
    assert len(found) <= 1, (X, found)
    return (found[0], None) if found else (None, None)


def ghost_points(blk):
    g = blk.ng
    for k in range(-g, blk.nz + g):
        for j in range(-g, blk.ny + g):
            for i in range(-g, blk.nx + g):
                if 0 <= i < blk.nx and 0 <= j < blk.ny and 0 <= k < blk.nz:
                    continue
                yield (i, j, k)


def covered(transfers, dest_key):
    out = {}
    for t in transfers:
        b = t[dest_key]
        for k in range(t["lo"][2], t["hi"][2]):
            for j in range(t["lo"][1], t["hi"][1]):
                for i in range(t["lo"][0], t["hi"][0]):
                    key = (b, i, j, k)
                    assert key not in out, ("point written twice", key)
                    out[key] = t
    return out


@pytest.mark.parametrize("refine,refine2,pair", [((1, 0, 0), None, 0), ((0, 1, 1), None, 0),
                                                 ((1, 0, 0), 7, 0), ((1, 0, 0), 7, 1)])
def test_transfers_match_ownership(refine, refine2, pair):
    bt, locs = W.refined_level_set(refine=refine, refine2=refine2)
    plan = _plan(bt)
    pro, res = Z.level_transfers(plan, locs, pair)
    P, R = covered(pro, "fine"), covered(res, "coarse")
    want_p, want_r = set(), set()
    for b, (blk, (lev, o)) in enumerate(zip(bt.blocks, locs)):
        if lev not in (pair, pair + 1):
            continue
        s = step(locs, lev)
        for (i, j, k) in ghost_points(blk):
            X = (o[0] + i * s, o[1] + j * s, o[2] + k * s)
            ob, _ = owner(bt, locs, X)
            if ob is None:
                continue
            lo_ = locs[ob][0]
            if lev == pair + 1 and lo_ == pair:     # fine ghost in a coarse span
                want_p.add((b, i, j, k))
                t = P[(b, i, j, k)]
                assert t["coarse"] == ob
                oc = locs[ob][1]
                sc = step(locs, pair)
                assert [(o[d] - oc[d]) // sc for d in range(3)] == t["c0"]
            elif lev == pair and lo_ == pair + 1:   # coarse ghost in a fine span
                want_r.add((b, i, j, k))
                assert R[(b, i, j, k)]["fine"] == ob
    assert want_p == set(P) and want_r == set(R)
    assert len(want_p) > 0 and len(want_r) > 0
    # the transfer plan accepts both sets (stencils inside the stored points)
    xp = Z.XPlan(plan, pro, res, 6, Z.PLAN_NO_DEVICE)
    xp.close()
    plan.close()


def test_level_transfers_errors():
    bt, locs = W.refined_level_set()
    plan = _plan(bt)
    with pytest.raises(Z.Z4cError) as e:
        Z.level_transfers(plan, locs, 1)                       # no level 2
    assert e.value.status == Z.EINVAL
    bad = list(locs)
    bad[-1] = (1, (bad[-1][1][0] + 1, bad[-1][1][1], bad[-1][1][2]))   # off the coarse lattice
    with pytest.raises(Z.Z4cError) as e:
        Z.level_transfers(plan, bad, 0)
    assert e.value.status == Z.EINVAL
    plan.close()
