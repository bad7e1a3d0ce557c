"""Pins of the oracle's D2Q25 lattice, its order-4 frame transformation and
the non-translational energy split (Eq. nt_energy_g), against what the paper
fixes independently of the oracle's code: Table I's printed D1Q5 rule, a
library Gauss-Hermite routine, the exactness of the quadrature, the moment
matching that defines the transformation (solved here with numpy from
monomials), the printed a0..a3 formulas (which the general Hermite projection
must reproduce at order three), Maxwellian energy moments, conservation, and
the Navier-Stokes-Fourier limit (shear viscosity, sound speed, thermal
diffusivity)."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from paper_2405_11489_amd import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_lattices.txt")
NT = oracle.NONTRANS
EXPS4 = [(p, n - p) for n in range(5) for p in range(n, -1, -1)]  # 15 (p, q), order <= 4


def _golden():
    out = {}
    with open(GOLD) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            lat, key, val = line.split()
            out[(lat, key)] = float(val)
    return out


# ------------------------------------------------------------------ lattice
def test_d1q5_matches_table1():
    g = _golden()
    c, w = oracle.lattice_1d(5)
    ci, co = g[("D1Q5", "c_inner")], g[("D1Q5", "c_outer")]
    w0, wi, wo = g[("D1Q5", "w_zero")], g[("D1Q5", "w_inner")], g[("D1Q5", "w_outer")]
    np.testing.assert_allclose(c, [-co, -ci, 0.0, ci, co], rtol=0, atol=4e-16)
    np.testing.assert_allclose(w, [wo, wi, w0, wi, wo], rtol=0, atol=4e-16)


def test_d1q5_is_five_point_gauss_hermite():
    x, wt = np.polynomial.hermite_e.hermegauss(5)
    c, w = oracle.lattice_1d(5)
    np.testing.assert_allclose(c, np.sort(x), rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, wt[np.argsort(x)] / math.sqrt(2 * math.pi), rtol=0, atol=1e-14)


def test_d1q5_moments_exact_to_order_nine():
    c, w = oracle.lattice_1d(5)
    for n in range(10):
        exact = 0.0 if n % 2 else float(np.prod(np.arange(n - 1, 0, -2)) if n else 1.0)
        assert (w * c ** n).sum() == pytest.approx(exact, abs=1e-12)
    assert abs((w * c ** 10).sum() - 945.0) > 1.0


def test_d2q25_is_the_tensor_product():
    c, w1 = oracle.lattice_1d(5)
    cx, cy, w = oracle.lattice_2d(5)
    for a in range(5):
        for b in range(5):
            i = 5 * a + b
            assert (cx[i], cy[i]) == (c[a], c[b])
            assert w[i] == pytest.approx(w1[a] * w1[b], rel=1e-15)


# --------------------------------------------------------- transformation
def lab_moments(pop, lam, exps):
    q1 = 4 if len(pop) == 16 else 5
    cx, cy, _ = oracle.lattice_2d(q1)
    s = np.sqrt(lam[2])
    Vx, Vy = s * cx + lam[0], s * cy + lam[1]
    return np.array([(pop * Vx ** p * Vy ** q).sum() for p, q in exps])


def brute_transform(pop, lam_src, lam_dst):
    """The unique w_i x (polynomial of degree <= 4 in c_i) with the source's
    moments up to order four, from a numpy solve on monomials."""
    cx, cy, w = oracle.lattice_2d(5)
    M = lab_moments(pop, lam_src, EXPS4)
    basis = np.stack([w * cx ** p * cy ** q for p, q in EXPS4], axis=1)      # 25 x 15
    A = np.stack([lab_moments(basis[:, j], lam_dst, EXPS4) for j in range(15)], axis=1)
    return basis @ np.linalg.solve(A, M)


def random_lam(rng):
    return np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.05, 3.0)])


@pytest.mark.parametrize("seed", range(12))
def test_hermite_projection_of_order_three_is_the_printed_transform(seed):
    """On D2Q16 the general order-N projection at N = 3 equals the transform
    written with the printed a0..a3 formulas."""
    rng = np.random.default_rng(300 + seed)
    pop = rng.uniform(0.0, 1.0, 16)
    ls, ld = random_lam(rng), random_lam(rng)
    ref = oracle.transform(pop, ls, ld)
    got = oracle.transform_hermite(pop, ls, ld, 3)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", range(12))
def test_d2q25_transform_equals_moment_matching_solution(seed):
    rng = np.random.default_rng(400 + seed)
    pop = rng.uniform(0.0, 1.0, 25)
    ls, ld = random_lam(rng), random_lam(rng)
    got = oracle.transform(pop, ls, ld)
    ref = brute_transform(pop, ls, ld)
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", range(12))
def test_d2q25_transform_preserves_moments_to_order_four(seed):
    rng = np.random.default_rng(500 + seed)
    pop = rng.uniform(0.0, 1.0, 25)
    ls, ld = random_lam(rng), random_lam(rng)
    out = oracle.transform(pop, ls, ld)
    m_in, m_out = lab_moments(pop, ls, EXPS4), lab_moments(out, ld, EXPS4)
    assert np.max(np.abs(m_in - m_out)) <= 1e-11 * np.max(np.abs(m_in))


def test_fourth_moments_survive_a_frame_change_on_d2q25_only():
    """The reason the non-translational split needs the fifth-order lattice:
    its energy needs f's fourth moments, which the N = 3 transformation of
    D2Q16 does not carry across frames."""
    rng = np.random.default_rng(7)
    ls, ld = np.array([0.3, -0.2, 1.0]), np.array([1.1, 0.4, 1.7])
    e4 = [(p, 4 - p) for p in range(5)]
    for q, ok in ((25, True), (16, False)):
        cx, cy, w = oracle.lattice_2d(5 if q == 25 else 4)
        pop = w * (1.0 + 0.2 * rng.uniform(-1, 1, q))
        out = oracle.transform(pop, ls, ld)
        err = np.max(np.abs(lab_moments(out, ld, e4) - lab_moments(pop, ls, e4)))
        assert (err < 1e-12) == ok, (q, err)


def test_d2q25_same_frame_is_projection_and_idempotent():
    rng = np.random.default_rng(11)
    lam = np.array([0.5, -0.7, 1.3])
    pop = rng.uniform(0.0, 1.0, 25)
    once = oracle.transform(pop, lam, lam)
    twice = oracle.transform(once, lam, lam)
    np.testing.assert_allclose(twice, once, rtol=1e-12, atol=1e-14)
    # a Grad expansion of order <= 4 is reproduced exactly
    cx, cy, w = oracle.lattice_2d(5)
    grad = w * (1.0 + 0.1 * cx - 0.2 * cy * cx + 0.05 * (cx ** 4 - 6 * cx ** 2 + 3))
    np.testing.assert_allclose(oracle.transform(grad, lam, lam), grad, rtol=1e-12, atol=1e-15)


def test_d2q25_round_trip_is_the_projection():
    rng = np.random.default_rng(12)
    l1, l2 = np.array([0.2, 0.1, 0.9]), np.array([-1.3, 0.8, 2.2])
    pop = rng.uniform(0.0, 1.0, 25)
    back = oracle.transform(oracle.transform(pop, l1, l2), l2, l1)
    np.testing.assert_allclose(back, oracle.transform(pop, l1, l1), rtol=1e-11, atol=1e-13)


# ------------------------------------------------- non-translational split
@pytest.mark.parametrize("q", [16, 25])
@pytest.mark.parametrize("rho,ux,uy,T,gamma", [(1.0, 0.0, 0.0, 1.0, 1.4),
                                               (0.7, 1.3, -0.4, 0.3, 1.8),
                                               (2.0, -2.5, 0.9, 2.0, 1.4)])
def test_nontrans_equilibrium_energy_moments(q, rho, ux, uy, T, gamma):
    """g^eq = (U'/rho) f^eq carries U' = rho (c_v - 1) T; with f's kinetic
    energy the total is E = rho c_v T + rho |u|^2 / 2, and the energy flux
    sum (g + f |C|^2 / 2) C is the Maxwellian's (E + p) u."""
    cv = 1.0 / (gamma - 1.0)
    f, g = oracle.equilibrium(rho, ux, uy, T, gamma, split=NT, lattice=q)
    cx, cy, w = oracle.lattice_2d(4 if q == 16 else 5)
    s = math.sqrt(T)
    Cx, Cy = s * cx + ux, s * cy + uy
    e = g + 0.5 * (Cx ** 2 + Cy ** 2) * f
    E = rho * cv * T + 0.5 * rho * (ux * ux + uy * uy)
    assert g.sum() == pytest.approx(rho * (cv - 1.0) * T, rel=1e-13)
    assert e.sum() == pytest.approx(E, rel=1e-13)
    p = rho * T
    assert (e * Cx).sum() == pytest.approx((E + p) * ux, rel=1e-12, abs=1e-12)
    assert (e * Cy).sum() == pytest.approx((E + p) * uy, rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(f, rho * w, rtol=1e-14)


@pytest.mark.parametrize("q", [16, 25])
@pytest.mark.parametrize("seed", range(3))
def test_nontrans_collision_conserves_rho_j_E(q, seed):
    rng = np.random.default_rng(600 + seed)
    cx, cy, w = oracle.lattice_2d(4 if q == 16 else 5)
    lam0 = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.5, 2)])
    f0 = w * rng.uniform(0.8, 1.2, q)
    g0 = w * rng.uniform(0.8, 1.2, q)
    s0 = math.sqrt(lam0[2])
    rho = f0.sum()
    u = np.array([(f0 * (s0 * cx + lam0[0])).sum(), (f0 * (s0 * cy + lam0[1])).sum()]) / rho
    # populations re-projected onto the frame of their own moments
    E0 = (g0 + 0.5 * ((s0 * cx + lam0[0]) ** 2 + (s0 * cy + lam0[1]) ** 2) * f0).sum()
    gamma = 1.4
    cv = 1.0 / (gamma - 1.0)
    T = (E0 - 0.5 * rho * (u @ u)) / (rho * cv)
    lam = np.array([u[0], u[1], T])
    f, g = oracle.transform(f0, lam0, lam), oracle.transform(g0, lam0, lam)
    fo, go = oracle.collide(f, g, lam, 0.7, 1.0, gamma, split=NT)
    s = math.sqrt(T)
    Cx, Cy = s * cx + u[0], s * cy + u[1]

    def cons(ff, gg):
        return np.array([ff.sum(), (ff * Cx).sum(), (ff * Cy).sum(),
                         (gg + 0.5 * (Cx ** 2 + Cy ** 2) * ff).sum()])
    np.testing.assert_allclose(cons(fo, go), cons(f, g), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(cons(f, g)[3], E0, rtol=1e-12)


def test_nontrans_requires_unit_prandtl():
    with pytest.raises(ValueError):
        oracle.params(8, 1, tau=0.7, prandtl=0.71, split=NT)


# ------------------------------------------------------------------ steps
@pytest.mark.parametrize("split", [oracle.TOTAL, NT])
def test_d2q25_uniform_flow_is_a_fixed_point(split):
    w = workloads.fourier_modes(n=6, ny=5, mach=1.5, amplitude=0.0, seed=0, tau=0.6,
                                prandtl=1.0)
    P = oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=1.0, split=split,
                      lattice=25)
    s = oracle.init(P, w.rho.ravel(), w.ux.ravel(), w.uy.ravel(), w.T.ravel())
    s1, st = oracle.step(P, s, 3)
    assert st.nonphysical == 0
    np.testing.assert_allclose(s1.f, s.f, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(s1.g, s.g, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(s1.lam, s.lam, rtol=1e-12, atol=1e-14)


def run_mode(w, every, split, lattice=25):
    P = oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl, bc_x=w.bc_x,
                      bc_y=w.bc_y, split=split, lattice=lattice)
    s = oracle.init(P, w.rho.ravel(), w.ux.ravel(), w.uy.ravel(), w.T.ravel())
    kind = w.modes[0][0]
    k, T0, U = w.meta["k"], w.meta["T0"], w.meta["U"]
    cs = math.sqrt(w.gamma * T0)
    ph = np.exp(1j * k * np.arange(w.nx))
    ts, amps = [], []
    for n in range(0, w.steps + 1, every):
        m = oracle.moments(P, s)
        r, vx, vy, p = m["rho"][0], m["ux"][0] - U, m["uy"][0], m["p"][0]
        if kind == "shear":
            obs = vy
        elif kind == "acoustic":
            obs = (p - T0) / cs + vx
        else:
            obs = (r - 1.0) - (p - T0) / cs ** 2
        ts.append(n)
        amps.append((obs * np.conj(ph)).sum() / w.nx)
        if n < w.steps:
            s, st = oracle.step(P, s, every)
            assert st.nonphysical == 0
    ts = np.array(ts, float)
    amps = np.array(amps)
    decay = -np.polyfit(ts, np.log(np.abs(amps)), 1)[0]
    freq = -np.polyfit(ts, np.unwrap(np.angle(amps)), 1)[0]
    return decay, freq


@pytest.mark.parametrize("split,U", [(NT, 0.0), (NT, 2.3664), (oracle.TOTAL, 0.0)])
def test_d2q25_shear_wave_decays_at_nu_k2(split, U):
    w = workloads.shear_wave(L=64, tau=0.8, U=U, steps=120)
    decay, freq = run_mode(w, 10, split)
    k = w.meta["k"]
    assert decay == pytest.approx(cf.shear_viscosity(w.tau, 1.0) * k * k, rel=0.01)
    assert freq == pytest.approx(k * U, abs=1e-6)


@pytest.mark.parametrize("split,gamma,T0", [(NT, 1.4, 1.0), (NT, 1.8, 0.25),
                                            (oracle.TOTAL, 1.4, 1.0)])
def test_d2q25_sound_speed(split, gamma, T0):
    w = workloads.acoustic_wave(L=32, tau=0.6, gamma=gamma, T0=T0, steps=48)
    _, freq = run_mode(w, 2, split)
    assert freq / w.meta["k"] == pytest.approx(cf.sound_speed(gamma, T0), rel=0.005)


@pytest.mark.parametrize("U", [0.0, 2.3664])
def test_d2q25_nontrans_acoustic_attenuation_and_thermal_diffusivity(U):
    w = workloads.acoustic_wave(L=32, tau=0.8, U=U, steps=60)
    decay, freq = run_mode(w, 2, NT)
    s_ac, s_ent = cf.longitudinal_modes(w.meta["k"], w.tau, 1.0, w.gamma, 1.0)
    assert decay == pytest.approx(-s_ac.real, rel=0.03)
    assert freq == pytest.approx(s_ac.imag + w.meta["k"] * U, rel=0.005)
    w = workloads.entropy_wave(L=32, tau=0.8, U=U, steps=80)
    decay, _ = run_mode(w, 4, NT)
    assert decay == pytest.approx(-s_ent.real, rel=0.03)
