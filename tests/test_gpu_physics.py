"""GPU runs of the full-size workloads against what the paper fixes (closed
forms of the hydrodynamic limit, the exact Riemann solution), plus the
FP32-vs-FP64 comparison at 2048^2 and the recorded stability finding.

The FP64 kernel itself is tied to the oracle by test_gpu_parity.py; these
tests check the method's physics at sizes the oracle cannot reach.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from oracle import riemann
from paper_2405_11489_amd import workloads
from parity_util import field_errors, field_l1, gpu_run, gpu_solver, oracle_run, plane_errors

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def mode_amplitude(m, kind, mx, my, w):
    """Complex amplitude at wave vector (mx, my) of the mode's characteristic
    observable: shear -> transverse velocity; acoustic (forward) ->
    p'/(rho c) + u'.k_hat; entropy -> rho' - p'/c^2."""
    T0, (Ux, Uy) = w.meta["T0"], w.meta["U"]
    cs = math.sqrt(w.gamma * T0)
    kx, ky = 2 * math.pi * mx / w.nx, 2 * math.pi * my / w.ny
    kn = math.hypot(kx, ky)
    ex, ey = kx / kn, ky / kn
    if kind == "shear":
        obs = -ey * (m["ux"] - Ux) + ex * (m["uy"] - Uy)
    elif kind == "acoustic":
        obs = (m["p"] - T0) / cs + ex * (m["ux"] - Ux) + ey * (m["uy"] - Uy)
    else:
        obs = (m["rho"] - 1.0) - (m["p"] - T0) / cs ** 2
    F = np.fft.fft2(obs) / obs.size
    return F[my % w.ny, mx % w.nx]


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_mach2_modes_decay_and_propagate_as_linear_nsf(prec):
    """The benchmark workload (512^2, Mach 2, 8 modes, 2000 steps): every mode
    decays and oscillates at the rate of the linearised NSF system with
    nu = (tau - 1/2) T, eta/rho = (2 - gamma) nu, alpha = nu / Pr,
    c_s = sqrt(gamma T), Doppler-shifted by k.U."""
    w = workloads.fourier_modes(n=512, mach=2.0, amplitude=1e-3, seed=0, tau=0.55, prandtl=0.71)
    # Doppler-shifted phases advance up to |k||U| ~ 0.25 rad per step: sample
    # every 10 steps so the unwrapped phase is not aliased
    every, steps = 10, w.steps
    ts, amps = [], {i: [] for i in range(len(w.modes))}
    with gpu_solver(w, prec) as sol:
        for n in range(0, steps + 1, every):
            m = sol.moments()
            ts.append(n)
            for i, (kind, mx, my, _) in enumerate(w.modes):
                amps[i].append(mode_amplitude(m, kind, mx, my, w))
            if n < steps:
                sol.step(every)
        st = sol.stats()
    assert st.nonphysical == 0
    ts = np.array(ts, float)
    Ux, Uy = w.meta["U"]
    for i, (kind, mx, my, _) in enumerate(w.modes):
        a = np.array(amps[i])
        decay = -np.polyfit(ts, np.log(np.abs(a)), 1)[0]
        freq = -np.polyfit(ts, np.unwrap(np.angle(a)), 1)[0]
        kx, ky = 2 * math.pi * mx / w.nx, 2 * math.pi * my / w.ny
        k = math.hypot(kx, ky)
        doppler = kx * Ux + ky * Uy
        if kind == "shear":
            exp_decay, exp_freq, tol = cf.shear_viscosity(w.tau, 1.0) * k * k, doppler, 0.02
        elif kind == "acoustic":
            s, _ = cf.longitudinal_modes(k, w.tau, 1.0, w.gamma, w.prandtl)
            exp_decay, exp_freq, tol = -s.real, s.imag + doppler, 0.03
        else:
            _, s = cf.longitudinal_modes(k, w.tau, 1.0, w.gamma, w.prandtl)
            exp_decay, exp_freq, tol = -s.real, doppler, 0.03
        assert decay == pytest.approx(exp_decay, rel=tol), (kind, mx, my)
        assert freq == pytest.approx(exp_freq, rel=5e-3, abs=1e-6), (kind, mx, my)


def test_sod_l1_decreases_with_resolution():
    """Shock tube against the exact Riemann solution at 400, 800, 1600 nodes
    (tau = 0.55, t = 0.2)."""
    errs = []
    for nx in (400, 800, 1600):
        w = workloads.sod_tube(nx=nx, nu=2e-3)
        *_, st, m = gpu_run(w, FP64, w.steps)
        assert st.nonphysical == 0
        x = (np.arange(nx) + 0.5) / nx
        r_ex, _, _ = riemann.sample(w.meta["left"], w.meta["right"], w.gamma, (x - 0.5) / 0.2)
        errs.append(np.abs(m["rho"][0] - r_ex).mean())
    assert errs[0] < 1e-2
    assert errs[0] > errs[1] > errs[2]


def test_quadrants_small_match_oracle():
    """Four-quadrant Riemann problem at oracle size (32^2, 40 steps)."""
    w = workloads.riemann_quadrants(n=32, seed=0, steps=40)
    f, g, fr, _, _, m = gpu_run(w, FP64, w.steps)
    P, s, _ = oracle_run(w, w.steps)
    assert max(plane_errors(f, g, fr, s)) <= 1e-12
    _, _, _, _, _, m32 = gpu_run(w, FP32, w.steps)
    l1 = field_l1(m32, oracle.moments(P, s))
    assert max(l1.values()) <= 1e-4, l1


def test_quadrants_2048_fp32_against_fp64():
    """2048^2 four-quadrant Riemann problem, 1000 steps: FP32 bulk with FP64
    moments against the all-FP64 kernel, L1 <= 1e-4 per field."""
    w = workloads.riemann_quadrants(n=2048, seed=0, steps=1000)
    *_, st64, m64 = gpu_run(w, FP64, w.steps)
    *_, st32, m32 = gpu_run(w, FP32, w.steps)
    assert st64.nonphysical == 0 and st32.nonphysical == 0
    l1 = field_l1(m32, m64)
    assert max(l1.values()) <= 1e-4, l1


def test_low_viscosity_mach2_is_unstable():
    """Recorded finding: at tau = 0.51 on the Mach-2 background the step is
    linearly unstable; FP64 round-off alone grows into a non-physical state
    within 1000 steps (tau = 0.55 decays, see the benchmark workload)."""
    from paper_2405_11489_amd import pond
    w = workloads.fourier_modes(n=512, mach=2.0, amplitude=1e-3, seed=0, tau=0.51)
    bad = False
    with gpu_solver(w, FP64) as sol:
        for _ in range(10):
            sol.step(100)
            try:
                sol.synchronize()
            except pond.PondError:
                bad = True
                break
    assert bad


def _first_nonphysical(w, steps, prec=FP32, chunk=250):
    from paper_2405_11489_amd import pond
    with gpu_solver(w, prec) as sol:
        done = 0
        while done < steps:
            sol.step(min(chunk, steps - done))
            done += min(chunk, steps - done)
            try:
                sol.synchronize()
            except pond.PondError as e:
                assert e.status == pond.ERR_NONPHYSICAL
                return done
    return None


def test_high_mach_stability_needs_tau_above_055():
    """Recorded finding: on the T = 1 background the step at tau = 0.55 turns
    unstable from about Mach 2.75 on; tau = 0.6 runs 2000 steps at Mach 3
    (the advected flows of the batch and serving workloads use tau = 0.6)."""
    unstable = workloads.fourier_modes(n=128, mach=3.0, amplitude=1e-3, seed=0, tau=0.55)
    stable = workloads.fourier_modes(n=128, mach=3.0, amplitude=1e-3, seed=0, tau=0.6)
    assert _first_nonphysical(unstable, 2000) is not None
    assert _first_nonphysical(stable, 2000) is None


def test_riemann_interfaces_with_large_velocity_jumps_fail():
    """Recorded finding: four-quadrant problems drawn from the full ranges
    (Mach <= 1.5) go non-physical within a few hundred steps when neighbouring
    quadrants slide past each other at more than ~1 thermal speed, while the
    gentle draws (Mach <= 0.8, p >= 0.5, jumps <= 1) run 2000 steps."""
    harsh = workloads.riemann_quadrants(n=256, seed=1000, nu=2e-3, steps=2000)
    gentle = workloads.riemann_quadrants(n=256, seed=1000, nu=2e-3, steps=2000,
                                         p_range=(0.5, 1.5), mach_range=(0.0, 0.8),
                                         max_velocity_jump=1.0)
    assert _first_nonphysical(harsh, 2000) is not None
    assert _first_nonphysical(gentle, 2000) is None


@pytest.mark.parametrize("npts", [4, 3])
def test_stencil_accuracy_shear_decay_and_sod(npts):
    """The paper's quadratic stencil (3 points) against the default cubic one
    (4 points): an advected shear wave (L = 64, U = 0.6, T = 1, tau = 0.6,
    800 steps) must decay at nu k^2 with nu = (tau - 1/2) T, and the 400 x 1
    shock tube must match the exact Riemann solution.  The measured errors
    are reported in the design notes (cubic: 0.46 % and 4.0e-3; quadratic:
    L1 1.26e-2); the bars are the cubic stencil's closed-form pins (1 % decay,
    L1 < 1e-2), widened for the quadratic one's extra numerical diffusion."""
    w = workloads.shear_wave(L=64, ny=4, tau=0.6, U=0.6, A=1e-4, steps=800)
    k = 2 * math.pi / w.nx
    amps = []
    with gpu_solver(w, FP64, interp_points=npts) as sol:
        for n in range(0, w.steps + 1, 40):
            m = sol.moments()
            amps.append(np.abs(np.fft.fft(m["uy"][0])[1]) / w.nx)
            if n < w.steps:
                sol.step(40)
    ts = np.arange(0, w.steps + 1, 40)
    decay = -np.polyfit(ts, np.log(amps), 1)[0]
    expected = cf.shear_viscosity(w.tau, 1.0) * k * k
    rel = abs(decay - expected) / expected
    sod = workloads.sod_tube(nx=400, nu=2e-3)
    *_, st, m = gpu_run(sod, FP64, sod.steps, interp_points=npts)
    x = (np.arange(400) + 0.5) / 400
    r_ex, _, _ = riemann.sample(sod.meta["left"], sod.meta["right"], sod.gamma, (x - 0.5) / 0.2)
    l1 = np.abs(m["rho"][0] - r_ex).mean()
    print(f"interp_points {npts}: shear decay error {rel:.4f}, Sod L1(rho) {l1:.5f}")
    assert st.nonphysical == 0
    assert rel < (0.01 if npts == 4 else 0.15), rel
    assert l1 < (1e-2 if npts == 4 else 2e-2), l1
