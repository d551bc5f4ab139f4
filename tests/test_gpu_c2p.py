"""Primitive <-> conservative maps on the GPU (through the C ABI) against the
oracle in oracle/c2p.py.

* z4c_p2c: every cell against the oracle's p2c, 1e-13 relative to the sum
  of the magnitudes of the cell's conservatives (a few dozen operations,
  rounding order only).
* z4c_c2p on conservatives made by the oracle's p2c: recovered primitives
  within 1e-10 of the generating ones at every cell (the relative error the
  paper states for its primitive solver), and of the oracle's c2p on sampled
  cells; atmosphere cells (below the density threshold) and cells above the
  velocity ceiling get the atmosphere state, its conservatives and their
  status; cells outside the requested range are not touched.
* The 8 x 128^3-cell level set: z4c_p2c then z4c_c2p at full size; the
  generator's vacuum cells (rho below the threshold) become atmosphere, every
  other cell is recovered within 1e-10 (in cold, strongly magnetised cells
  the pressure to the rounding of the energy budget and the velocity to
  rounding amplified by B^2 / rho); p2c checked on sampled cells.
"""
import math
import sys

import numpy as np
import pytest

from oracle import c2p as OC
from paper_2311_04989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SENTINEL = -7.25e33
SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


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


def cell_metric(mb, b, k, j, i, geom=None):
    geom = mb.geom if geom is None else geom
    chi = max(mb.view("geom", geom, b, 0)[k, j, i], 1e-6)
    gam = np.zeros((3, 3))
    for q, (a, c) in enumerate(SYM):
        gam[a, c] = gam[c, a] = mb.view("geom", geom, b, 1 + q)[k, j, i] / chi
    return gam


def cell_prim(mb, arr, b, k, j, i):
    v = [mb.view("prim", arr, b, f)[k, j, i] for f in range(8)]
    return v[0], np.array(v[1:4]), v[4], np.array(v[5:8])


def cells(mb, b, ext):
    blk = mb.blocks[b]
    lo = blk.ngc - ext
    for k in range(lo, blk.ngc + blk.ncz + ext):
        for j in range(lo, blk.ngc + blk.ncy + ext):
            for i in range(lo, blk.ngc + blk.ncx + ext):
                yield k, j, i


def oracle_cons(mb, G, ext):
    cons = np.zeros_like(mb.cons)
    for b in range(len(mb.blocks)):
        for k, j, i in cells(mb, b, ext):
            rho, ut, p, Bv = cell_prim(mb, mb.prim, b, k, j, i)
            D, S, tau, Bc = OC.p2c(rho, ut, p, Bv, cell_metric(mb, b, k, j, i), G)
            vals = [D, *S, tau, *Bc]
            for f in range(8):
                mb.view("cons", cons, b, f)[k, j, i] = vals[f]
    return cons


@pytest.mark.parametrize("mhd", [0, 1])
def test_p2c_parity(mhd):
    mb = W.random_matter_batch(40 + mhd, nblocks=2, nmax=10)
    W.c2p_states(mb, np.random.default_rng(mhd))
    if not mhd:
        for b in range(len(mb.blocks)):
            for f in (5, 6, 7):
                mb.view("prim", mb.prim, b, f)[...] = 0.0
    c = Z().c2p_params(mhd=mhd, gamma_ad=5.0 / 3.0)
    plan = Z().mplan_for(mb)
    note(f"p2c parity mhd {mhd}")
    cons = dev(np.full(mb.cons.size, SENTINEL))
    plan.p2c(c, 2, dev(mb.geom), dev(mb.prim), cons)
    got = host(cons)
    want = oracle_cons(mb, 5.0 / 3.0, 2)
    nq = 8 if mhd else 5
    for b in range(len(mb.blocks)):
        scale = sum(np.abs(mb.view("cons", want, b, f)) for f in range(nq))
        for f in range(nq):
            g, o = mb.view("cons", got, b, f), mb.view("cons", want, b, f)
            for k, j, i in cells(mb, b, 2):
                assert abs(g[k, j, i] - o[k, j, i]) <= 1e-13 * scale[k, j, i], (b, f, k, j, i)
    plan.close()


@pytest.mark.parametrize("mhd", [0, 1])
def test_c2p_recovers_primitives(mhd):
    G = 5.0 / 3.0 if mhd else 2.0
    mb = W.random_matter_batch(50 + mhd, nblocks=3, nmax=9)
    W.c2p_states(mb, np.random.default_rng(10 + mhd))
    if not mhd:
        for b in range(len(mb.blocks)):
            for f in (5, 6, 7):
                mb.view("prim", mb.prim, b, f)[...] = 0.0
    cons0 = oracle_cons(mb, G, 3)
    c = Z().c2p_params(mhd=mhd, gamma_ad=G, rho_atm=1e-12)
    plan = Z().mplan_for(mb)
    note(f"c2p mhd {mhd}")
    cons = dev(cons0)
    prim = dev(np.full(mb.prim.size, SENTINEL))
    status = dev(np.full(mb.status.size, -1, dtype=np.int32))
    plan.c2p(c, 3, dev(mb.geom), cons, prim, status)
    gp, gs, gc = host(prim), host(status), host(cons)
    assert np.all(gc == cons0), "conservatives of recovered cells must not change"
    rng = np.random.default_rng(3)
    for b in range(len(mb.blocks)):
        st = mb.view("status", gs, b, 0)
        assert np.all(st == 0), np.unique(st)
        for k, j, i in cells(mb, b, 3):
            rho, ut, p, _ = cell_prim(mb, mb.prim, b, k, j, i)
            r2, u2, p2, _ = cell_prim(mb, gp, b, k, j, i)
            assert abs(r2 - rho) <= 1e-10 * rho and abs(p2 - p) <= 1e-10 * p, (b, k, j, i)
            assert np.abs(u2 - ut).max() <= 1e-10 * max(np.abs(ut).max(), 1.0), (b, k, j, i)
        # the oracle's inversion on sampled cells
        all_cells = list(cells(mb, b, 3))
        for n in rng.choice(len(all_cells), size=40, replace=False):
            k, j, i = all_cells[n]
            q = [mb.view("cons", cons0, b, f)[k, j, i] for f in range(8)]
            r3, u3, p3 = OC.c2p(q[0], q[1:4], q[4], q[5:8], cell_metric(mb, b, k, j, i), G)
            r2, u2, p2, _ = cell_prim(mb, gp, b, k, j, i)
            assert abs(r2 - r3) <= 1e-10 * r3 and abs(p2 - p3) <= 1e-10 * p3
            assert np.abs(u2 - u3).max() <= 1e-10 * max(np.abs(u3).max(), 1.0)
    plan.close()


def test_c2p_atmosphere_ceiling_and_range():
    G = 2.0
    mb = W.random_matter_batch(60, nblocks=2, nmax=8)
    W.c2p_states(mb, np.random.default_rng(60), n_atm=6, n_fast=5, ut_fast=30.0)
    cons0 = oracle_cons(mb, G, 3)
    c = Z().c2p_params(mhd=1, gamma_ad=G, rho_atm=1e-12, ut_max=20.0)
    plan = Z().mplan_for(mb)
    ext = 1
    note("c2p atmosphere")
    cons = dev(cons0)
    prim = dev(np.full(mb.prim.size, SENTINEL))
    status = dev(np.full(mb.status.size, -1, dtype=np.int32))
    plan.c2p(c, ext, dev(mb.geom), cons, prim, status)
    gp, gs, gc = host(prim), host(status), host(cons)
    seen = set()
    for b, blk in enumerate(mb.blocks):
        st = mb.view("status", gs, b, 0)
        inside = np.zeros(st.shape, dtype=bool)
        lo = blk.ngc - ext
        inside[lo:lo + blk.ncz + 2 * ext, lo:lo + blk.ncy + 2 * ext, lo:lo + blk.ncx + 2 * ext] = True
        assert np.all(st[~inside] == -1)
        for f in range(8):
            assert np.all(mb.view("prim", gp, b, f)[~inside] == SENTINEL)
            assert np.all(mb.view("cons", gc, b, f)[~inside] == mb.view("cons", cons0, b, f)[~inside])
        for k, j, i in cells(mb, b, ext):
            rho, ut, p, Bv = cell_prim(mb, mb.prim, b, k, j, i)
            s = st[k, j, i]
            seen.add(int(s))
            W_ = math.sqrt(1.0 + ut @ cell_metric(mb, b, k, j, i) @ ut)
            if rho < 1e-12:
                assert s == 1
            elif math.sqrt(W_ * W_ - 1.0) > 20.0:
                assert s == 2
            else:
                assert s == 0
                continue
            r2, u2, p2, B2 = cell_prim(mb, gp, b, k, j, i)
            assert r2 == c.rho_atm and p2 == c.p_atm and np.all(u2 == 0.0)
            np.testing.assert_allclose(B2, Bv, rtol=1e-14)
            D, S, tau, Bc = OC.p2c(c.rho_atm, np.zeros(3), c.p_atm, Bv,
                                   cell_metric(mb, b, k, j, i), G)
            q = [mb.view("cons", gc, b, f)[k, j, i] for f in range(8)]
            assert q[0] == pytest.approx(D, rel=1e-14) and np.all(np.asarray(q[1:4]) == 0.0)
            assert q[4] == pytest.approx(tau, rel=1e-12)
            np.testing.assert_array_equal(q[5:8], [mb.view("cons", cons0, b, f)[k, j, i]
                                                   for f in (5, 6, 7)])
    assert {0, 1, 2} <= seen
    plan.close()


def test_level_set_round_trip_full_size():
    """p2c then c2p on the 8 x 128^3-cell level set (the benchmark's
    configuration): every cell recovered; p2c sampled against the oracle."""
    G = 2.0
    mb = W.matter_level_set()
    mb.geom[:] = 0.0
    for b, blk in enumerate(mb.blocks):     # cell geometry: chi, gt_ij from the vertex data
        for f in range(W.NGEOM):
            v = mb.view("u", mb.u, b, f)
            g = blk.ngv - blk.ngc
            c8 = [v[g + dz:g + dz + blk.cshape[0], g + dy:g + dy + blk.cshape[1],
                    g + dx:g + dx + blk.cshape[2]] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
            mb.view("geom", mb.geom, b, f)[...] = sum(c8) / 8.0
    c = Z().c2p_params(mhd=1, gamma_ad=G, rho_atm=1e-12)
    plan = Z().mplan_for(mb)
    note("c2p level set full size")
    geom, prim = dev(mb.geom), dev(mb.prim)
    cons = torch.zeros(mb.cons.size, dtype=torch.float64, device=DEV)
    out = torch.zeros(mb.prim.size, dtype=torch.float64, device=DEV)
    status = torch.full((mb.status.size,), -1, dtype=torch.int32, device=DEV)
    plan.p2c(c, 3, geom, prim, cons)
    plan.c2p(c, 3, geom, cons, out, status)
    gp, gs, gc = host(out), host(status), host(cons)
    n_atm = 0
    for b in range(len(mb.blocks)):
        st = mb.view("status", gs, b, 0)
        rho = mb.view("prim", mb.prim, b, 0)
        atm = rho < c.f_thr * c.rho_atm          # the generator's vacuum cells
        n_atm += int(atm.sum())
        assert np.all(st[atm] == 1) and np.all(st[~atm] == 0), np.unique(st, return_counts=True)
        ok = ~atm
        assert np.all(np.abs(mb.view("prim", gp, b, 0) - rho)[ok] <= 1e-10 * rho[ok])
        p = mb.view("prim", mb.prim, b, 4)
        # cold, magnetised cells: p is recovered from the energy budget, whose
        # rounding is ~1e-16 (rho W^2 + B^2); B^2 bounded by 4 |B|^2 here
        Bsq = sum(mb.view("prim", mb.prim, b, f) ** 2 for f in (5, 6, 7))
        tol_p = 1e-10 * p + 1e-13 * (rho + 4.0 * Bsq)
        assert np.all(np.abs(mb.view("prim", gp, b, 4) - p)[ok] <= tol_p[ok])
        # the velocity along B of a strongly magnetised cell follows from
        # S.B = z B.v with z << B^2: rounding amplified by ~B^2 / rho
        tol_u = 1e-10 + 1e-15 * 4.0 * Bsq / np.maximum(rho, 1e-300)
        for f in (1, 2, 3):
            u = mb.view("prim", mb.prim, b, f)
            assert np.all(np.abs(mb.view("prim", gp, b, f) - u)[ok]
                          <= (tol_u * np.maximum(np.abs(u), 1.0))[ok])
    note(f"level set: {n_atm} atmosphere cells of {mb.status.size}")
    rng = np.random.default_rng(9)
    checked = 0
    while checked < 200:
        b = int(rng.integers(len(mb.blocks)))
        k, j, i = rng.integers(0, mb.blocks[b].cshape[0], size=3)
        rho, ut, p, Bv = cell_prim(mb, mb.prim, b, k, j, i)
        if rho < c.f_thr * c.rho_atm:
            continue                     # vacuum cells: no fluid state to compare
        checked += 1
        D, S, tau, Bc = OC.p2c(rho, ut, p, Bv, cell_metric(mb, b, k, j, i), G)
        q = np.array([mb.view("cons", gc, b, f)[k, j, i] for f in range(8)])
        want = np.array([D, *S, tau, *Bc])
        assert np.abs(q - want).max() <= 1e-13 * np.abs(want).sum()
    plan.close()
