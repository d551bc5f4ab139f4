"""The oracle's operators against the textbook weights in
tests/golden/stencil_weights.json (CPU only): the response of each operator
to a unit impulse, read at the neighbouring points, is its weight vector."""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import matter as OM
from paper_2311_04989_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "stencil_weights.json")))


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


def weights(entry):
    return np.array(entry["num"], dtype=float) / entry["den"]


@pytest.mark.parametrize("p", [4, 6])
def test_fd_and_ko_weights(p):
    r = p // 2 + 1
    n = 2 * r + 3
    h, sigma = 0.5, 0.3
    blk = W.Block(n, n, n, r, h, h, h)
    c = n // 2
    u = np.zeros(blk.shape)
    u[c + r, c + r, c + r] = 1.0                     # impulse at interior point (c, c, c)
    d = O.derivs(blk, u, p, ko_sigma=sigma)
    m = p // 2
    # operator at point x = c - k sees the impulse at offset +k: weight w_k
    w1 = np.array([d[0, c, c, c - k] for k in range(-m, m + 1)]) * h
    w2 = np.array([d[3, c, c, c - k] for k in range(-m, m + 1)]) * h * h
    wk = np.array([d[9, c, c, c - k] for k in range(-r, r + 1)])
    np.testing.assert_allclose(w1, weights(GOLDEN["d1"][str(p)]), rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(w2, weights(GOLDEN["d2"][str(p)]), rtol=1e-15, atol=1e-14)
    ko = (-1) ** (r + 1) * sigma / (2 ** (2 * r) * h) * weights(GOLDEN["ko"][str(p)])
    np.testing.assert_allclose(wk, ko, rtol=1e-14, atol=0)
    # mixed second derivative: the tensor product of the first-derivative weights
    wxy = np.array([[d[4, c, c - j, c - i] for i in range(-m, m + 1)] for j in range(-m, m + 1)])
    np.testing.assert_allclose(wxy * h * h, np.outer(w1, w1) / 1.0, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_midpoint_interpolation_weights(order):
    np.testing.assert_array_equal(OM.midpoint_weights(order),
                                  weights(GOLDEN["midpoint"][str(order)]))
