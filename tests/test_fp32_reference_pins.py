"""Pins of the oracle's two FP32 reference builds (CPU).

The FP32 gate of the GPU's FP32 path is fixed by the error of the oracle
source built with float as working type and every stencil difference
u_m - u_0 still formed in double (`-DORACLE_FP32`); the naive build
(`-DORACLE_NAIVE` as well) rounds every sample to float first.  Both are
checked here against what the arithmetic fixes, on a perturbation of flat
space whose size sits near float resolution:

  chi = alpha = 1, gt = delta + eps P(x, y, z) on gt_xx only (eps = 1e-6,
  P a periodic sine product), every other field 0 (shift 0, At = 0).

The right-hand side of At_ij is then alpha chi R_ij^TF, a second-derivative
expression of eps P of size eps * |P''|.  In the mixed form the differences
carry eps P exactly (in double), so that right-hand side is right to float
precision relative to its own size; in the naive form each sample of
1 + eps P carries a rounding error of up to 2^-24 (6 % of eps), and the
second differences of that noise over h^2 swamp the signal.  A build that
rounded its samples first, or that still worked in double, fails one of
the three checks.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2311_04989_amd import workloads as W

EPS = 1e-6
N = 16


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


def _batch():
    h = 1.0 / N
    bt = W.Batch([W.Block(N, N, N, 4, h, h, h, 0.0, 0.0, 0.0)])
    X, Y, Z = bt.blocks[0].coords()
    for name in ("chi", "gxx", "gyy", "gzz", "alpha"):
        bt.view(bt.u, 0, W.F[name])[...] = 1.0
    P = np.sin(2 * math.pi * X) * np.cos(2 * math.pi * Y + 0.3) * np.sin(2 * math.pi * Z + 0.7)
    bt.view(bt.u, 0, W.F["gxx"])[...] += EPS * P
    bt.params = W.Params(fd_order=6, ko_sigma=0.0)
    bt.ghost = W.GHOST_PERIODIC
    return bt


def _rel_err(bt, got, ref, names):
    """max |got - ref| / max |ref| over the interior points of the named fields."""
    out = {}
    for n in names:
        g = bt.interior(got, 0, W.F[n])
        r = bt.interior(ref, 0, W.F[n])
        out[n] = float(np.abs(g - r).max() / np.abs(r).max())
    return out


AT = ("Axx", "Axy", "Axz", "Ayy", "Ayz", "Azz")


def test_fp32_builds_against_the_arithmetic():
    bt = _batch()
    ext = O.rhs(bt, ext=True)
    f64 = O.rhs(bt)
    f32 = O.rhs(bt, ext="f32")
    naive = O.rhs(bt, ext="f32naive")
    # the At right-hand side is of size eps |P''| ~ eps (2 pi)^2
    scale = max(np.abs(bt.interior(ext, 0, W.F[n])).max() for n in AT)
    assert 1e-6 < scale < 1e-3
    e64 = _rel_err(bt, f64, ext, AT)
    e32 = _rel_err(bt, f32, ext, AT)
    en = _rel_err(bt, naive, ext, AT)
    msg = "\n".join(f"{n}: f64 {e64[n]:.1e} f32 {e32[n]:.1e} naive {en[n]:.1e}" for n in AT)
    # the FP64 build: double precision
    assert max(e64.values()) < 1e-9, msg
    # the mixed FP32 build is float arithmetic (not double) ...
    assert max(e32.values()) > 1e-9, msg
    # ... on exact differences: float precision relative to the signal
    assert max(e32.values()) < 1e-5, msg
    # the naive build loses the signal in the rounding of its samples
    assert min(en.values()) > 1e-2, msg
