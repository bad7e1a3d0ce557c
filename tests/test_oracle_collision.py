"""Pins of the oracle's local equilibria and collision.

Equilibria (Sec. "Discrete velocity solver ...: PonD" and Sec. II): f_i^eq =
rho w_i in the node's own frame must carry the Maxwell-Boltzmann moments up to
order three, and the total-energy-split g^eq must carry E, (E + p) u and the
second moment used in the Chapman-Enskog analysis (appendix, energy flux).
Collision: BGK conserves rho, j and E; with Pr != 1 the quasi-equilibrium
reading relaxes the stress at omega, the Fourier part of the energy flux at
omega_1 and its viscous-heating part u . P^neq at omega.
"""
import numpy as np
import pytest

import oracle

GAMMA = 1.4


def frame_vel(lam):
    cx, cy, w = oracle.lattice_2d()
    s = np.sqrt(lam[2])
    return s * cx + lam[0], s * cy + lam[1], w


@pytest.mark.parametrize("rho,ux,uy,T", [(1.0, 0.0, 0.0, 1.0), (0.4, 2.3, -1.1, 0.3),
                                         (3.0, -0.2, 0.9, 2.5)])
def test_equilibrium_moments(rho, ux, uy, T):
    f, g = oracle.equilibrium(rho, ux, uy, T, GAMMA)
    Cx, Cy, w = frame_vel([ux, uy, T])
    C = np.stack([Cx, Cy])
    u = np.array([ux, uy])
    I = np.eye(2)
    tol = 1e-12 * max(1.0, rho * (T + u @ u) ** 1.5)
    # f: Maxwellian moments up to order three
    assert abs(f.sum() - rho) < tol
    np.testing.assert_allclose(C @ f, rho * u, atol=tol)
    np.testing.assert_allclose(np.einsum("ai,bi,i->ab", C, C, f),
                               rho * (T * I + np.outer(u, u)), atol=tol)
    m3 = np.einsum("ai,bi,ci,i->abc", C, C, C, f)
    exp3 = rho * (np.einsum("a,b,c->abc", u, u, u)
                  + T * (np.einsum("a,bc->abc", u, I) + np.einsum("b,ac->abc", u, I)
                         + np.einsum("c,ab->abc", u, I)))
    np.testing.assert_allclose(m3, exp3, atol=tol)
    # g: total energy, its flux (E + p) u and second moment (p/rho)(E + p) I + (2p + E) uu
    cv = 1.0 / (GAMMA - 1.0)
    p = rho * T
    E = rho * cv * T + 0.5 * rho * (u @ u)
    assert abs(g.sum() - E) < tol * 10
    np.testing.assert_allclose(C @ g, (E + p) * u, atol=tol * 10)
    np.testing.assert_allclose(np.einsum("ai,bi,i->ab", C, C, g),
                               p / rho * (E + p) * I + (2 * p + E) * np.outer(u, u), atol=tol * 10)


def nonequilibrium_state(seed):
    """Random populations in the Grad span, expressed in the frame of their own
    conserved moments (so that the collision sees its actual input)."""
    rng = np.random.default_rng(seed)
    rho, ux, uy, T = 1.3, 0.7, -0.4, 0.6
    f, g = oracle.equilibrium(rho, ux, uy, T, GAMMA)
    f = f * (1 + 0.05 * rng.standard_normal(16))
    g = g * (1 + 0.05 * rng.standard_normal(16))
    lam0 = np.array([ux, uy, T])
    Cx, Cy, _ = frame_vel(lam0)
    r = f.sum()
    jx, jy = Cx @ f, Cy @ f
    E = g.sum()
    cv = 1.0 / (GAMMA - 1.0)
    lam = np.array([jx / r, jy / r, (E - (jx * jx + jy * jy) / (2 * r)) / (r * cv)])
    return oracle.transform(f, lam0, lam), oracle.transform(g, lam0, lam), lam


@pytest.mark.parametrize("prandtl", [1.0, 0.71, 2.0])
@pytest.mark.parametrize("seed", range(4))
def test_collision_conserves_rho_j_E(prandtl, seed):
    f, g, lam = nonequilibrium_state(seed)
    fo, go = oracle.collide(f, g, lam, 0.6, prandtl, GAMMA)
    Cx, Cy, _ = frame_vel(lam)
    for a, b in ((f.sum(), fo.sum()), (Cx @ f, Cx @ fo), (Cy @ f, Cy @ fo), (g.sum(), go.sum())):
        assert abs(a - b) <= 1e-14 * max(1.0, abs(a))


def test_unit_prandtl_is_plain_bgk():
    f, g, lam = nonequilibrium_state(9)
    tau = 0.57
    fo, go = oracle.collide(f, g, lam, tau, 1.0, GAMMA)
    feq, geq = oracle.equilibrium(f.sum(), lam[0], lam[1], lam[2], GAMMA)
    om = 1.0 / tau
    np.testing.assert_allclose(fo, f + om * (feq - f), rtol=0, atol=1e-15)
    np.testing.assert_allclose(go, g + om * (geq - g), rtol=0, atol=1e-15)


@pytest.mark.parametrize("prandtl", [0.71, 1.0, 3.0])
def test_relaxation_rates_of_stress_and_heat_flux(prandtl):
    f, g, lam = nonequilibrium_state(5)
    tau = 0.8
    om = 1.0 / tau
    om1 = 1.0 / (0.5 + (tau - 0.5) / prandtl)
    fo, go = oracle.collide(f, g, lam, tau, prandtl, GAMMA)
    feq, geq = oracle.equilibrium(f.sum(), lam[0], lam[1], lam[2], GAMMA)
    Cx, Cy, _ = frame_vel(lam)
    C = np.stack([Cx, Cy])
    P_in = np.einsum("ai,bi,i->ab", C, C, f - feq)
    P_out = np.einsum("ai,bi,i->ab", C, C, fo - feq)
    np.testing.assert_allclose(P_out, (1 - om) * P_in, atol=1e-13)
    u = lam[:2]
    dq = u @ P_in                                  # viscous-heating part of the flux
    q_in, q_out = C @ (g - geq), C @ (go - geq)
    np.testing.assert_allclose(q_out, (1 - om1) * (q_in - dq) + (1 - om) * dq, atol=1e-13)
