"""Pins of the oracle's lattice (Table I) against the paper's printed values,
a library Gauss-Hermite routine and the exactness of the quadrature."""
import math
import os

import numpy as np

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_lattices.txt")


def _golden():
    out = {}
    with open(GOLD) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            lat, key, val = line.split()
            out[(lat, key)] = float(val)
    return out


def test_d1q4_matches_table1():
    g = _golden()
    c, w = oracle.lattice_1d()
    ci, co = g[("D1Q4", "c_inner")], g[("D1Q4", "c_outer")]
    wi, wo = g[("D1Q4", "w_inner")], g[("D1Q4", "w_outer")]
    np.testing.assert_allclose(c, [-co, -ci, ci, co], rtol=0, atol=4e-16)
    np.testing.assert_allclose(w, [wo, wi, wi, wo], rtol=0, atol=4e-16)


def test_d1q4_is_four_point_gauss_hermite():
    # numpy's probabilists' Gauss-Hermite rule, weights normalised to sum 1
    x, wt = np.polynomial.hermite_e.hermegauss(4)
    c, w = oracle.lattice_1d()
    np.testing.assert_allclose(c, np.sort(x), rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, wt[np.argsort(x)] / math.sqrt(2 * math.pi), rtol=0, atol=1e-14)


def test_quadrature_moments_exact_to_order_seven():
    c, w = oracle.lattice_1d()
    gauss = [1, 0, 1, 0, 3, 0, 15, 0]          # moments of the unit normal, order 0..7
    for n, m in enumerate(gauss):
        assert abs((w * c ** n).sum() - m) < 1e-13 * max(1, m)
    # order 8 is where a 4-point rule stops being exact: 81 instead of 105
    assert abs((w * c ** 8).sum() - 81.0) < 1e-12


def test_d2q16_tensor_product_moments():
    cx, cy, w = oracle.lattice_2d()
    assert cx.shape == (16,)
    gauss = [1, 0, 1, 0, 3, 0, 15, 0]
    for p in range(8):
        for q in range(8):
            got = (w * cx ** p * cy ** q).sum()
            assert abs(got - gauss[p] * gauss[q]) < 1e-12 * max(1, gauss[p] * gauss[q])
    # ordering i = 4a + b: c_i = (c_a, c_b)
    c, _ = oracle.lattice_1d()
    for i in range(16):
        assert cx[i] == c[i // 4] and cy[i] == c[i % 4]
