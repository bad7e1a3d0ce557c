"""Seeded synthetic workloads: initial macroscopic fields only.

This module holds no arithmetic of the method: it draws initial density,
velocity and temperature fields (lattice units, r = 1) and the scalar model
parameters for the flows the paper probes, so that the GPU path and the CPU
oracle can be started from the very same inputs.  Arrays have shape (ny, nx),
x fastest, float64.

Workloads
---------
* ``sod_tube`` -- quasi-1-D shock tube (left rho = 1, p = 1; right
  rho = 0.125, p = 0.1; u = 0), lattice temperature T = 0.04 p / rho
  (a unit domain resolved by nx nodes with dt/dx = 0.2 in physical units).
* ``shear_wave``, ``acoustic_wave``, ``entropy_wave``, ``pressure_front`` --
  single linear modes and the small pressure step of Sec. "Probing
  hydrodynamic limits".
* ``fourier_modes`` -- sum of 8 random-phase shear / acoustic / entropy Fourier
  modes (amplitude 1e-3) on a uniform background advected at a given Mach.
* ``riemann_quadrants`` -- 2-D four-quadrant Riemann problem with seeded states.
* ``batch_instances`` / ``serving_requests`` -- mixes of the above with
  log-uniform sizes, for the batched and served paths.
* ``thermal_couette`` -- channel between a wall at rest (T0) and a wall moving
  along x (T1) at the speed of a given Eckert number (Sec. "Measuring viscous
  heating").
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC, CLAMP, WALL = 0, 1, 2


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    bc_x: int
    bc_y: int
    gamma: float
    prandtl: float
    tau: float
    steps: int
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    modes: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)
    wall_ux: tuple = (0.0, 0.0)   # bc_y == WALL: (bottom, top) wall x-velocity
    wall_T: tuple = (1.0, 1.0)    # bc_y == WALL: (bottom, top) wall temperature

    @property
    def nodes(self) -> int:
        return self.nx * self.ny


def _grid(nx, ny):
    X, Y = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64))
    return X, Y


def tau_for(nu: float, T_ref: float) -> float:
    """Relaxation time giving kinematic viscosity nu at lattice temperature T_ref."""
    return 0.5 + nu / T_ref


def sod_tube(nx=400, ny=1, nu=2e-3, T_scale=0.04, gamma=1.4, prandtl=0.71, steps=None,
             frame_mach=0.0, bc_y=PERIODIC) -> Workload:
    """Sod shock tube; interface between nodes nx/2 - 1 and nx/2.

    ``steps`` defaults to nx (physical t = 0.2 at dt/dx = 0.2).  ``frame_mach``
    adds a uniform velocity (in units of the left sound speed) along x to both
    states.  tau gives ``nu`` at the left-state temperature."""
    X, _ = _grid(nx, ny)
    left = X < nx // 2
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    T = T_scale * p / rho
    U = frame_mach * math.sqrt(gamma * T_scale)
    ux = np.full_like(rho, U)
    return Workload("sod_tube", nx, ny, CLAMP, bc_y, gamma, prandtl, tau_for(nu, T_scale),
                    nx if steps is None else steps, rho, ux, np.zeros_like(rho), T,
                    meta={"T_scale": T_scale, "nu": nu, "frame_velocity": U,
                          "left": (1.0, 0.0, 1.0), "right": (0.125, 0.0, 0.1)})


def _single_mode(kind, L, ny, tau, gamma, prandtl, T0, U, A, steps):
    X, _ = _grid(L, ny)
    k = 2 * math.pi / L
    s = np.sin(k * X)
    cs = math.sqrt(gamma * T0)
    rho = np.ones_like(X)
    ux = np.full_like(X, U)
    uy = np.zeros_like(X)
    T = np.full_like(X, T0)
    if kind == "shear":
        uy = A * s
    elif kind == "acoustic":             # forward-running sound wave
        rho = 1.0 + A * s
        ux = U + cs * A * s
        T = T0 * (1.0 + (gamma - 1.0) * A * s)
    elif kind == "entropy":              # isobaric density/temperature wave
        rho = 1.0 + A * s
        T = T0 / rho
    else:
        raise ValueError(kind)
    return Workload(f"{kind}_wave", L, ny, PERIODIC, PERIODIC, gamma, prandtl, tau, steps,
                    rho, ux, uy, T, modes=[(kind, 1, 0, 0.0)],
                    meta={"k": k, "T0": T0, "U": U, "A": A})


def shear_wave(L=64, ny=1, tau=0.8, gamma=1.4, prandtl=1.0, T0=1.0, U=0.0, A=1e-4, steps=200):
    return _single_mode("shear", L, ny, tau, gamma, prandtl, T0, U, A, steps)


def acoustic_wave(L=32, ny=1, tau=0.8, gamma=1.4, prandtl=1.0, T0=1.0, U=0.0, A=1e-4, steps=60):
    return _single_mode("acoustic", L, ny, tau, gamma, prandtl, T0, U, A, steps)


def entropy_wave(L=32, ny=1, tau=0.8, gamma=1.4, prandtl=1.0, T0=1.0, U=0.0, A=1e-4, steps=80):
    return _single_mode("entropy", L, ny, tau, gamma, prandtl, T0, U, A, steps)


def pressure_front(L=200, tau=0.8, gamma=1.4, prandtl=1.0, T0=1.0, dp=1e-4, steps=60):
    """Quasi-1-D domain split in two halves with a pressure difference dp at
    uniform temperature T0 and zero velocity (left half at the higher pressure)."""
    X, _ = _grid(L, 1)
    left = X < L // 2
    rho = np.where(left, 1.0 + dp / T0, 1.0)
    T = np.full_like(X, T0)
    return Workload("pressure_front", L, 1, CLAMP, PERIODIC, gamma, prandtl, tau, steps,
                    rho, np.zeros_like(X), np.zeros_like(X), T, meta={"dp": dp, "T0": T0})


def _pick_modes(rng, count):
    """count integer wavevectors with 2 <= |m|_inf <= 6 and distinct |m|."""
    seen = set()
    out = []
    while len(out) < count:
        m = rng.integers(-6, 7, size=2)
        if max(abs(int(m[0])), abs(int(m[1]))) < 2:
            continue
        n2 = int(m[0] ** 2 + m[1] ** 2)
        if n2 in seen:
            continue
        seen.add(n2)
        out.append((int(m[0]), int(m[1])))
    return out


def fourier_modes(n=512, ny=None, mach=2.0, angle_deg=30.0, amplitude=1e-3, seed=0, tau=0.55,
                  gamma=1.4, prandtl=0.71, T0=1.0, steps=2000, kinds=None) -> Workload:
    """Uniform background (rho = 1, T = T0) advected at ``mach`` in direction
    ``angle_deg``, plus 8 random-phase Fourier modes of amplitude ``amplitude``:
    3 shear, 3 forward acoustic, 2 isobaric entropy modes, integer wave vectors
    with 2 <= |m|_inf <= 6 and distinct |m|."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    kinds = kinds or ["shear"] * 3 + ["acoustic"] * 3 + ["entropy"] * 2
    ms = _pick_modes(rng, len(kinds))
    phases = rng.uniform(0.0, 2 * math.pi, size=len(kinds))
    X, Y = _grid(n, ny)
    cs = math.sqrt(gamma * T0)
    th = math.radians(angle_deg)
    U = (mach * cs * math.cos(th), mach * cs * math.sin(th))
    drho = np.zeros_like(X)
    dux = np.zeros_like(X)
    duy = np.zeros_like(X)
    dT = np.zeros_like(X)
    modes = []
    for kind, (mx, my), ph in zip(kinds, ms, phases):
        kx, ky = 2 * math.pi * mx / n, 2 * math.pi * my / ny
        kn = math.hypot(kx, ky)
        ex, ey = kx / kn, ky / kn
        s = amplitude * np.sin(kx * X + ky * Y + ph)
        if kind == "shear":
            dux += -ey * cs * s
            duy += ex * cs * s
        elif kind == "acoustic":
            drho += s
            dux += cs * s * ex
            duy += cs * s * ey
            dT += (gamma - 1.0) * T0 * s
        else:
            drho += s
            dT += -T0 * s
        modes.append((kind, mx, my, float(ph)))
    rho = 1.0 + drho
    return Workload("fourier_modes", n, ny, PERIODIC, PERIODIC, gamma, prandtl, tau, steps,
                    rho, U[0] + dux, U[1] + duy, T0 + dT, modes=modes,
                    meta={"mach": mach, "U": U, "T0": T0, "amplitude": amplitude, "seed": seed})


def _quadrant_states(rng, gamma, T_scale, rho_range=(0.5, 2.0), p_range=(0.3, 1.5),
                     mach_range=(0.0, 1.5)):
    states = []
    for _ in range(4):
        r = rng.uniform(*rho_range)
        p = rng.uniform(*p_range)
        ma = rng.uniform(*mach_range)
        d = rng.uniform(0.0, 2 * math.pi)
        T = T_scale * p / r
        c = math.sqrt(gamma * T)
        states.append((r, ma * c * math.cos(d), ma * c * math.sin(d), T))
    return states


def quadrant_jumps(states):
    """(max temperature ratio, max velocity jump in thermal speeds of the colder
    side) over the four pairs of neighbouring quadrants (periodic grid)."""
    pairs = [(0, 1), (2, 3), (0, 2), (1, 3)]
    tr = max(max(states[a][3], states[b][3]) / min(states[a][3], states[b][3]) for a, b in pairs)
    dv = max(math.hypot(states[a][1] - states[b][1], states[a][2] - states[b][2]) /
             math.sqrt(min(states[a][3], states[b][3])) for a, b in pairs)
    return tr, dv


def riemann_quadrants(n=2048, seed=0, gamma=1.4, prandtl=0.71, nu=2e-3, T_scale=0.04,
                      steps=1000, max_temperature_ratio=2.5, max_velocity_jump=2.0,
                      rho_range=(0.5, 2.0), p_range=(0.3, 1.5), mach_range=(0.0, 1.5)) -> Workload:
    """Four-quadrant 2-D Riemann problem on an n x n periodic grid; each quadrant
    draws rho ~ U[0.5, 2], p ~ U[0.3, 1.5], Mach ~ U[0, 1.5] and a direction
    ~ U[0, 2 pi); lattice T = T_scale p / rho; tau gives nu at T_scale.

    Draws whose neighbouring quadrants differ by more than
    ``max_temperature_ratio`` in temperature or by more than
    ``max_velocity_jump`` thermal speeds (of the colder side) in velocity are
    rejected and the next draw of the same generator is taken: the step cannot
    start from stronger jumps (its frame transformation between such
    neighbours leaves the Grad expansion's range)."""
    rng = np.random.default_rng(seed)
    draws = 0
    while True:
        states = _quadrant_states(rng, gamma, T_scale, rho_range, p_range, mach_range)
        draws += 1
        tr, dv = quadrant_jumps(states)
        if tr <= max_temperature_ratio and dv <= max_velocity_jump:
            break
    X, Y = _grid(n, n)
    q = (X >= n // 2).astype(int) + 2 * (Y >= n // 2).astype(int)
    rho = np.empty_like(X)
    ux = np.empty_like(X)
    uy = np.empty_like(X)
    T = np.empty_like(X)
    for i, (r, vx, vy, t) in enumerate(states):
        sel = q == i
        rho[sel], ux[sel], uy[sel], T[sel] = r, vx, vy, t
    return Workload("riemann_quadrants", n, n, PERIODIC, PERIODIC, gamma, prandtl,
                    tau_for(nu, T_scale), steps, rho, ux, uy, T,
                    meta={"states": states, "seed": seed, "draws": draws, "nu": nu,
                          "T_scale": T_scale, "temperature_ratio": tr, "velocity_jump": dv})


def _log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_instances(seed=0, count=256, tube_range=(256, 8192), flow_range=(64, 1024),
                    steps_range=(200, 2000), mach_range=(0.5, 3.0), flow_tau=0.6):
    """Mixed batch: half quasi-1-D shock tubes (nx x 1, clamp / periodic) with a
    uniform frame shift, half 2-D periodic perturbed flows (N x N) on an
    advected background.  Sizes log-uniform, Mach and step counts uniform.

    The flows use tau = ``flow_tau``: at T = 1 the step is linearly unstable at
    tau = 0.55 from Mach ~2.75 on (within 350-1450 steps), stable at 0.6 up to
    Mach 3 over 2000 steps."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        mach = float(rng.uniform(*mach_range))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        if i % 2 == 0:
            nx = _log_uniform_int(rng, *tube_range)
            w = sod_tube(nx=nx, frame_mach=mach, steps=steps)
        else:
            N = _log_uniform_int(rng, *flow_range)
            w = fourier_modes(n=N, mach=mach, angle_deg=float(rng.uniform(0, 360)),
                              seed=int(rng.integers(1 << 30)), steps=steps, tau=flow_tau)
        w.meta["instance"] = i
        out.append(w)
    return out


def serving_requests(seed=0, count=256, size_range=(64, 2048), steps_range=(100, 5000),
                     rate_per_s=1.0, flow_tau=0.6):
    """Poisson request stream: list of (arrival_time_s, Workload).  Kinds are
    uniform over {planar shock tube, shear wave, 2-D Riemann}; size N x N with N
    log-uniform; steps log-uniform.  The Riemann requests draw Mach <= 0.8 and
    p >= 0.5 with neighbour velocity jumps <= 0.75 thermal speed and
    temperature ratios <= 2; the shear flows use tau = ``flow_tau``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        N = _log_uniform_int(rng, *size_range)
        steps = _log_uniform_int(rng, *steps_range)
        kind = int(rng.integers(3))
        if kind == 0:
            w = sod_tube(nx=N, ny=N, steps=steps)
        elif kind == 1:
            w = fourier_modes(n=N, mach=float(rng.uniform(0.5, 3.0)), seed=int(rng.integers(1 << 30)),
                              steps=steps, kinds=["shear"] * 8, tau=flow_tau)
        else:
            # long runs need gentle interfaces: quadrant draws with neighbour velocity
            # jumps near or above 1 thermal speed go non-physical within 250-1750 steps
            w = riemann_quadrants(n=N, seed=int(rng.integers(1 << 30)), nu=2e-3, steps=steps,
                                  p_range=(0.5, 1.5), mach_range=(0.0, 0.8),
                                  max_velocity_jump=0.75, max_temperature_ratio=2.0)
        w.meta["request"] = i
        out.append((t, w))
    return out


def thermal_couette(ny=32, nx=1, Ec=8.0, T0=1.0, T1=1.005, tau=0.8, gamma=1.4, prandtl=1.0,
                    steps=None):
    """Thermal Couette flow: walls at y = -1/2 (at rest, T0) and y = ny - 1/2
    (moving along x at u0, T1), periodic in x; u0 from the Eckert number
    Ec = u0^2 / ((c_v + r) (T1 - T0)).  Starts from the linear velocity and
    temperature profiles at uniform pressure 1; ``steps`` defaults to
    1.2 ny^2 / alpha (alpha = (tau - 1/2) T / Pr), long enough for the
    slowest thermal mode to decay by ~e^-12."""
    cv = 1.0 / (gamma - 1.0)
    dT = T1 - T0
    u0 = math.sqrt(Ec * (cv + 1.0) * dT)
    _, Y = _grid(nx, ny)
    eta = (Y + 0.5) / ny
    T = T0 + dT * eta
    rho = 1.0 / T
    ux = u0 * eta
    uy = np.zeros_like(T)
    alpha = (tau - 0.5) * T0 / prandtl
    if steps is None:
        steps = int(math.ceil(1.2 * ny * ny / alpha))
    return Workload("thermal_couette", nx, ny, PERIODIC, WALL, gamma, prandtl, tau, steps,
                    rho, ux, uy, T, meta={"u0": u0, "Ec": Ec, "T0": T0, "T1": T1},
                    wall_ux=(0.0, u0), wall_T=(T0, T1))

