"""Pins of the oracle's frame transformation (Sec. "Frame transformation").

The transform maps populations living in frame lam_src onto the lattice of
frame lam_dst.  The paper fixes what it must do: keep every moment up to order
three (Eq. genericMomentUptoO3), with a result that is a reduced (N = 3) Grad
expansion (Eq. gradGeneralTransform), i.e. w_i times a polynomial of degree
<= 3 in c_i.  The brute-force check below finds that unique vector by solving
the 10 x 10 moment-matching system with numpy, from monomials rather than the
Hermite formulas the oracle uses.
"""
import itertools

import numpy as np
import pytest

import oracle

EXPS = [(p, q) for n in range(4) for p in range(n, -1, -1) for q in [n - p]]  # 10 (p, q)


def lab_moments(pop, lam):
    cx, cy, _ = oracle.lattice_2d()
    s = np.sqrt(lam[2])
    Vx, Vy = s * cx + lam[0], s * cy + lam[1]
    return np.array([(pop * Vx ** p * Vy ** q).sum() for p, q in EXPS])


def brute_transform(pop, lam_src, lam_dst):
    cx, cy, w = oracle.lattice_2d()
    M = lab_moments(pop, lam_src)
    basis = np.stack([w * cx ** p * cy ** q for p, q in EXPS], axis=1)      # 16 x 10
    A = np.stack([lab_moments(basis[:, j], lam_dst) for j in range(10)], axis=1)
    coef = np.linalg.solve(A, M)
    return basis @ coef


def random_lam(rng):
    return np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.05, 3.0)])


@pytest.mark.parametrize("seed", range(20))
def test_transform_equals_moment_matching_solution(seed):
    rng = np.random.default_rng(seed)
    pop = rng.uniform(0.0, 1.0, 16)
    ls, ld = random_lam(rng), random_lam(rng)
    got = oracle.transform(pop, ls, ld)
    ref = brute_transform(pop, ls, ld)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", range(20))
def test_transform_preserves_moments_to_order_three(seed):
    rng = np.random.default_rng(100 + seed)
    pop = rng.uniform(0.0, 1.0, 16)
    ls, ld = random_lam(rng), random_lam(rng)
    out = oracle.transform(pop, ls, ld)
    m_in, m_out = lab_moments(pop, ls), lab_moments(out, ld)
    assert np.max(np.abs(m_in - m_out)) <= 1e-12 * np.max(np.abs(m_in))


def test_same_frame_is_projection_and_idempotent():
    rng = np.random.default_rng(7)
    pop = rng.uniform(0.0, 1.0, 16)
    lam = random_lam(rng)
    once = oracle.transform(pop, lam, lam)
    twice = oracle.transform(once, lam, lam)
    np.testing.assert_allclose(twice, once, rtol=0, atol=1e-14)
    # a generic 16-vector has components beyond order three: projection is not identity
    assert np.max(np.abs(once - pop)) > 1e-3


def test_round_trip_and_composition():
    rng = np.random.default_rng(11)
    pop = rng.uniform(0.0, 1.0, 16)
    l0, l1, l2 = random_lam(rng), random_lam(rng), random_lam(rng)
    direct = oracle.transform(pop, l0, l2)
    via = oracle.transform(oracle.transform(pop, l0, l1), l1, l2)
    np.testing.assert_allclose(via, direct, rtol=0, atol=1e-11 * np.abs(direct).max())
    back = oracle.transform(oracle.transform(pop, l0, l1), l1, l0)
    np.testing.assert_allclose(back, oracle.transform(pop, l0, l0), rtol=0,
                               atol=1e-11 * np.abs(back).max())


def test_galilean_covariance():
    rng = np.random.default_rng(3)
    pop = rng.uniform(0.0, 1.0, 16)
    ls, ld = random_lam(rng), random_lam(rng)
    U = np.array([1.7, -0.6, 0.0])
    a = oracle.transform(pop, ls, ld)
    b = oracle.transform(pop, ls + U, ld + U)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())


def test_equilibrium_is_invariant_under_frame_change():
    # Maxwellian moments up to order 3 are reproduced exactly in any frame, so
    # the equilibrium of (rho, u, T) expressed in another frame and brought back
    # is the equilibrium itself.
    for rho, ux, uy, T in itertools.product([0.7], [0.3, -1.1], [0.2], [0.5, 1.5]):
        feq, geq = oracle.equilibrium(rho, ux, uy, T, 1.4)
        lam = np.array([ux, uy, T])
        other = np.array([ux + 0.4, uy - 0.3, 0.8 * T])
        for pop in (feq, geq):
            there = oracle.transform(pop, lam, other)
            back = oracle.transform(there, other, lam)
            np.testing.assert_allclose(back, pop, rtol=0, atol=1e-13 * np.abs(pop).max())
