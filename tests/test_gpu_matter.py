"""Parity of the matter-coupling kernels (through the C ABI) with the oracle
in oracle/matter.py, on the GPU.

Metric per field over the points a call writes: e = |g - o| / max(|o|,
1e-3 max|o|) <= 1e-12 (the interpolations are linear combinations with
positive and negative weights of sum 1, the projections a few dozen
operations: both differ from the oracle only in rounding order).  Points a
call must not write keep a sentinel value bit for bit.
"""
import sys

import numpy as np
import pytest

from oracle import matter as OM
from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SENTINEL = -7.25e33
GATE = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def Z():
    from paper_2311_04989_amd import z4c
    return z4c


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def check(mb, kind, got, want, nfields, region):
    """region(b) -> tuple of slices of the written points of block b."""
    for b in range(len(mb.blocks)):
        sl = region(b)
        for f in range(nfields):
            g = mb.view(kind, got, b, f)
            o = mb.view(kind, want, b, f)
            gi, oi = g[sl], o[sl]
            m = np.abs(oi).max()
            den = np.maximum(np.abs(oi), 1e-3 * m) if m > 0 else 1.0
            e = (np.abs(gi - oi) / den).max()
            assert e <= GATE, f"{kind} block {b} field {f}: e = {e:.3e}"
            mask = np.ones(g.shape, dtype=bool)
            mask[sl] = False
            assert np.all(g[mask] == SENTINEL), f"{kind} block {b} field {f}: wrote outside range"


def cc_region(mb, ext):
    def r(b):
        blk = mb.blocks[b]
        lo = blk.ngc - ext
        return (slice(lo, lo + blk.ncz + 2 * ext), slice(lo, lo + blk.ncy + 2 * ext),
                slice(lo, lo + blk.ncx + 2 * ext))
    return r


def vc_region(mb):
    def r(b):
        blk = mb.blocks[b]
        g = blk.ngv
        return (slice(g, g + blk.ncz + 1), slice(g, g + blk.ncy + 1), slice(g, g + blk.ncx + 1))
    return r


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("order", [2, 4, 6])
def test_interpolation_parity(seed, order):
    mb = W.random_matter_batch(seed, nblocks=3, nmax=21 if seed < 3 else 40)
    plan = Z().mplan_for(mb)
    # fill the CC sources with smooth seeded data
    rng = np.random.default_rng(seed)
    mb.adm[:] = rng.uniform(-1.0, 1.0, size=mb.adm.size) + 2.0
    # every block: ngv = 4 ghost vertices, ngc = 3 ghost cells
    for ext in (0, min(3, 4 - (order // 2 - 1))):
        note(f"matter interp seed {seed} order {order} ext {ext}")
        geom = dev(np.full(mb.geom.size, SENTINEL))
        plan.metric_to_cc(order, ext, dev(mb.u), geom)
        check(mb, "geom", host(geom), OM.metric_to_cc(mb, order, ext), W.NGEOM, cc_region(mb, ext))
    note(f"matter sources_to_vc seed {seed} order {order}")
    matter = dev(np.full(mb.matter.size, SENTINEL))
    plan.sources_to_vc(order, dev(mb.adm), matter)
    check(mb, "matter", host(matter), OM.sources_to_vc(mb, order), W.NM, vc_region(mb))
    plan.close()


@pytest.mark.parametrize("mhd", [0, 1])
@pytest.mark.parametrize("ext", [0, 3])
def test_adm_sources_parity(mhd, ext):
    mb = W.random_matter_batch(10 + ext, nblocks=2, nmax=12)
    plan = Z().mplan_for(mb)
    mb.geom[:] = OM.metric_to_cc(mb, 4, 3)
    note(f"matter adm mhd {mhd} ext {ext}")
    adm = dev(np.full(mb.adm.size, SENTINEL))
    plan.adm_sources(mhd, 2.0, 1e-6, ext, dev(mb.geom), dev(mb.prim), adm)
    want = OM.adm_sources(mb, bool(mhd), 2.0, 1e-6, ext)
    check(mb, "adm", host(adm), want, W.NM, cc_region(mb, ext))
    plan.close()


def test_chain_matches_oracle_chain():
    """Metric VC -> CC (order 4 over the three ghost cells), GRMHD sources on
    those cells, sources CC -> VC (order 6): every kernel's output against the
    oracle applied to the same inputs, and the whole chain against the
    oracle chain."""
    mb = W.random_matter_batch(21, nblocks=3, nmax=18)
    plan = Z().mplan_for(mb)
    note("matter chain")
    geom = dev(np.zeros(mb.geom.size))
    adm = dev(np.zeros(mb.adm.size))
    matter = dev(np.full(mb.matter.size, SENTINEL))
    plan.metric_to_cc(4, 3, dev(mb.u), geom)
    plan.adm_sources(1, 2.0, 1e-6, 3, geom, dev(mb.prim), adm)
    plan.sources_to_vc(6, adm, matter)
    og = OM.metric_to_cc(mb, 4, 3)
    oa = OM.adm_sources(mb, True, 2.0, 1e-6, 3, geom=og)
    om = OM.sources_to_vc(mb, 6, adm=oa)
    check(mb, "matter", host(matter), om, W.NM, vc_region(mb))
    plan.close()


def test_level_set_full_size_sampled():
    """The benchmark's level set (8 blocks of 128^3 cells) in the benchmark's
    launch configuration, checked on sampled vertices: the oracle evaluates
    the chain only at the cells and vertices those samples need."""
    mb = W.matter_level_set()
    plan = Z().mplan_for(mb)
    note("matter level set full size")
    geom = dev(np.zeros(mb.geom.size))
    adm = dev(np.zeros(mb.adm.size))
    matter = dev(np.zeros(mb.matter.size))
    plan.metric_to_cc(4, 3, dev(mb.u), geom)
    plan.adm_sources(1, 2.0, 1e-6, 3, geom, dev(mb.prim), adm)
    plan.sources_to_vc(6, adm, matter)
    g_geom, g_adm, g_matter = host(geom), host(adm), host(matter)
    rng = np.random.default_rng(4)
    w4, w6 = OM.midpoint_weights(4), OM.midpoint_weights(6)
    w4c = np.einsum("z,y,x->zyx", w4, w4, w4)
    sym = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    samples = []
    for _ in range(24):
        b = int(rng.integers(len(mb.blocks)))
        blk = mb.blocks[b]
        v = rng.integers(0, blk.ncx + 1, size=3)          # vertex (i, j, k)
        gv_ = blk.ngv
        acc = np.zeros(W.NM)
        # the 6^3 cells of the vertex's stencil: geometry of each from the
        # 4^3 vertices around it, its sources, then the weighted sum
        for c_ in range(6):
            for b_ in range(6):
                for a_ in range(6):
                    ci, cj, ck = v[0] - 3 + a_, v[1] - 3 + b_, v[2] - 3 + c_
                    gv = np.array([
                        (w4c * mb.view("u", mb.u, b, f)[ck - 1 + gv_:ck + 3 + gv_,
                                                         cj - 1 + gv_:cj + 3 + gv_,
                                                         ci - 1 + gv_:ci + 3 + gv_]).sum()
                        for f in range(W.NGEOM)])
                    chi = max(gv[0], 1e-6)
                    gam = np.zeros((3, 3))
                    for q, (i, j) in enumerate(sym):
                        gam[i, j] = gam[j, i] = gv[1 + q] / chi
                    P = [mb.view("prim", mb.prim, b, f)[ck + blk.ngc, cj + blk.ngc, ci + blk.ngc]
                         for f in range(8)]
                    r, S, Sij = OM.adm_point(P[0], P[1:4], P[4], P[5:8], gam, 2.0)
                    vals = [r, *S] + [Sij[i, j] for i, j in sym]
                    acc += w6[a_] * w6[b_] * w6[c_] * np.array(vals)
        got = np.array([mb.view("matter", g_matter, b, f)[v[2] + gv_, v[1] + gv_, v[0] + gv_]
                        for f in range(W.NM)])
        samples.append((b, v.tolist(), got, acc))
    scale = np.max([np.abs(o) for _, _, _, o in samples], axis=0)
    for b, v, got, acc in samples:
        e = np.abs(got - acc) / np.maximum(np.abs(acc), 1e-3 * scale)
        assert e.max() <= GATE, (b, v, e.max())
    assert np.isfinite(g_geom).all() and np.isfinite(g_adm).all()
    plan.close()
