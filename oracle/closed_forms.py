"""Closed forms of the hydrodynamic limit (test infrastructure, oracle package).

Lattice units, r = 1, D = 2.  Each function cites the passage it restates.
"""
from __future__ import annotations

import numpy as np

D = 2


def c_v(gamma: float) -> float:
    """Specific heat at constant volume from gamma = (c_v + r)/c_v (Eq. spec_heat)."""
    return 1.0 / (gamma - 1.0)


def shear_viscosity(tau: float, T: float) -> float:
    """Kinematic viscosity of the discrete BGK step, nu = (tau - 1/2) T.

    Sec. "Measuring dissipation rates" gives nu = tau r T for the continuous
    relaxation time; the time-discrete collision shifts tau by dt/2.
    """
    return (tau - 0.5) * T


def bulk_viscosity_ratio(gamma: float) -> float:
    """eta / (rho nu) = 2/D - r/c_v (Eq. bulk_visc)."""
    return 2.0 / D - 1.0 / c_v(gamma)


def thermal_diffusivity(tau: float, T: float, prandtl: float) -> float:
    """alpha = lambda / ((c_v + r) rho) = nu / Pr.

    Eq. therm_cond with Pr = 1 gives alpha = nu; for Pr != 1 the Fourier flux
    relaxes with tau_1 = 1/2 + (tau - 1/2)/Pr.
    """
    return shear_viscosity(tau, T) / prandtl


def sound_speed(gamma: float, T: float) -> float:
    """c_s = sqrt(gamma r T) (Sec. "Speed of sound")."""
    return float(np.sqrt(gamma * T))


def longitudinal_viscosity(tau: float, T: float, gamma: float) -> float:
    """nu_L = 2(1 - 1/D) nu + eta/rho, from the stress T_NS of Sec. II."""
    nu = shear_viscosity(tau, T)
    return 2.0 * (1.0 - 1.0 / D) * nu + bulk_viscosity_ratio(gamma) * nu


def acoustic_attenuation(k: float, tau: float, T: float, gamma: float, prandtl: float) -> float:
    """Leading-order amplitude decay rate of a sound wave,
    Gamma = k^2/2 [nu_L + (gamma - 1) alpha]."""
    return 0.5 * k * k * (longitudinal_viscosity(tau, T, gamma)
                          + (gamma - 1.0) * thermal_diffusivity(tau, T, prandtl))


def longitudinal_modes(k: float, tau: float, T: float, gamma: float, prandtl: float,
                       rho: float = 1.0):
    """Complex rates s (perturbations ~ exp(s t + i k x), rest frame) of the
    linearised Navier-Stokes-Fourier system of Sec. II for a longitudinal wave:
    continuity, momentum with nu_L, and internal energy
    rho c_v dT/dt + p div u = lambda lap T with lambda = rho c_p alpha.
    Returns (acoustic s with Im > 0, entropy s) as Python complex numbers."""
    cv = c_v(gamma)
    nuL = longitudinal_viscosity(tau, T, gamma)
    alpha = thermal_diffusivity(tau, T, prandtl)
    lam = rho * (cv + 1.0) * alpha
    p = rho * T
    ik = 1j * k
    B = np.array([
        [0.0, -ik * rho, 0.0],
        [-ik * T / rho, -nuL * k * k, -ik],
        [0.0, -ik * p / (rho * cv), -lam * k * k / (rho * cv)],
    ], dtype=complex)
    ev = np.linalg.eigvals(B)
    ac = ev[np.argmax(ev.imag)]
    ent = ev[np.argmin(np.abs(ev.imag))]
    return complex(ac), complex(ent)


def couette_temperature(ny, y, T0, T1, Ec, prandtl):
    """Thermal Couette flow between a wall at rest (T0, at y = -1/2) and a wall
    moving along x (T1, at y = ny - 1/2), constant properties (the solution
    quoted in Sec. "Measuring viscous heating"):
    (T - T0)/(T1 - T0) = eta + Pr Ec / 2 eta (1 - eta), eta = (y + 1/2) / ny."""
    eta = (np.asarray(y, dtype=float) + 0.5) / ny
    return T0 + (T1 - T0) * (eta + 0.5 * prandtl * Ec * eta * (1.0 - eta))
