"""Pins of the oracle's Lagrange interpolation stencil (Eq. propagationInterpolated
with a Lagrange kernel; 4 points by default, 3 points = the paper's "2nd-order"
stencil) against scipy's Lagrange polynomial and polynomial reproduction."""
import math

import numpy as np
import pytest
from scipy.interpolate import lagrange as scipy_lagrange

import oracle


@pytest.mark.parametrize("npts", [3, 4])
def test_base_node_rule(npts):
    for y in [-3.7, -1.0, -0.5, 0.0, 0.2, 0.5, 0.9999, 5.5, 12.25]:
        base, _ = oracle.lagrange(npts, y)
        if npts == 4:
            assert base == math.floor(y) - 1
        else:
            assert base == math.floor(y + 0.5) - 1


@pytest.mark.parametrize("npts", [3, 4])
def test_weights_match_scipy_lagrange(npts):
    rng = np.random.default_rng(npts)
    for _ in range(50):
        y = rng.uniform(-10, 10)
        base, wts = oracle.lagrange(npts, y)
        nodes = base + np.arange(npts, dtype=float)
        for j in range(npts):
            e = np.zeros(npts)
            e[j] = 1.0
            ref = scipy_lagrange(nodes - base, e)(y - base)
            assert abs(wts[j] - ref) < 1e-12


@pytest.mark.parametrize("npts", [3, 4])
def test_polynomial_reproduction(npts):
    rng = np.random.default_rng(10 + npts)
    for _ in range(50):
        y = rng.uniform(-10, 10)
        base, wts = oracle.lagrange(npts, y)
        nodes = base + np.arange(npts, dtype=float)
        assert abs(wts.sum() - 1.0) < 1e-14
        for deg in range(npts):
            assert abs((wts * nodes ** deg).sum() - y ** deg) < 1e-10 * max(1.0, abs(y) ** deg)
        # degree npts is not reproduced in general
    y = 0.37
    base, wts = oracle.lagrange(npts, y)
    nodes = base + np.arange(npts, dtype=float)
    assert abs((wts * nodes ** npts).sum() - y ** npts) > 1e-4


@pytest.mark.parametrize("npts", [3, 4])
def test_on_node_is_copy(npts):
    for y in [-4.0, 0.0, 3.0]:
        base, wts = oracle.lagrange(npts, y)
        e = np.zeros(npts)
        e[int(y) - base] = 1.0
        np.testing.assert_array_equal(wts, e)
