"""Pins of the oracle's whole step: invariants the method fixes exactly.

* A uniform state is a fixed point of the step, reached in one gather.
* With the frame held at its predictor (one gather) and a uniform frame, the
  gather is a translation-invariant interpolation whose weights sum to one,
  so total mass, momentum and energy are conserved to round-off; the
  collision conserves them node by node.
* Galilean invariance under an integer frame shift U (cells per step): the
  populations live in frames (u + U, T), so their departure points move by
  exactly U cells and a shear wave after n steps is the unshifted one
  translated by n U; for the total-energy g the shift residual is the Grad
  truncation of the added (v.U + U^2/2) f term.
* Self-consistency of the predictor-corrector: every stored frame is the frame
  of the stored populations' own moments.
"""
import numpy as np
import pytest

import oracle
from paper_2405_11489_amd import workloads

GAMMA = 1.4


def make_state(P, rho, ux, uy, T):
    return oracle.init(P, rho.ravel(), ux.ravel(), uy.ravel(), T.ravel())


def conserved_totals(P, s):
    m = oracle.moments(P, s)
    rho = m["rho"]
    cv = 1.0 / (P.gamma - 1.0)
    E = rho * cv * m["T"] + 0.5 * rho * (m["ux"] ** 2 + m["uy"] ** 2)
    return np.array([rho.sum(), (rho * m["ux"]).sum(), (rho * m["uy"]).sum(), E.sum()])


@pytest.mark.parametrize("bc", [0, 1])
def test_uniform_state_is_fixed_point(bc):
    P = oracle.params(7, 5, tau=0.6, gamma=GAMMA, prandtl=0.71, bc_x=bc, bc_y=0)
    sh = (5, 7)
    s0 = make_state(P, np.full(sh, 0.8), np.full(sh, 1.9), np.full(sh, -0.7), np.full(sh, 0.45))
    s1, st = oracle.step(P, s0, 3)
    np.testing.assert_allclose(s1.f, s0.f, rtol=0, atol=1e-14)
    np.testing.assert_allclose(s1.g, s0.g, rtol=0, atol=1e-13)
    np.testing.assert_allclose(s1.lam, s0.lam, rtol=0, atol=1e-13)
    assert (st.iters == 1).all() and st.nonconverged == 0


def test_uniform_frame_single_gather_conserves_exactly():
    nx, ny = 9, 6
    rng = np.random.default_rng(0)
    P = oracle.params(nx, ny, tau=0.7, gamma=GAMMA, prandtl=0.71, pc_max_iter=1)
    rho = 1.0 + 0.2 * rng.uniform(-1, 1, (ny, nx))
    s0 = make_state(P, rho, np.full_like(rho, 0.9), np.full_like(rho, -0.4), np.full_like(rho, 0.8))
    before = conserved_totals(P, s0)
    s1, st = oracle.step(P, s0, 1)
    after = conserved_totals(P, s1)
    np.testing.assert_allclose(after, before, rtol=1e-14, atol=1e-13)
    assert st.nonconverged == nx * ny       # one gather only: flagged, by construction


def test_general_flow_conservation_drift_is_small_and_converges():
    # the pull interpolation is not flux-form: with frames varying in space the
    # global sums drift at truncation level, shrinking as the modes are resolved
    drift = []
    for n in (16, 32):
        w = workloads.fourier_modes(n=n, mach=0.5, amplitude=1e-3, seed=4, tau=0.7)
        P = oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl)
        s0 = make_state(P, w.rho, w.ux, w.uy, w.T)
        before = conserved_totals(P, s0)
        s1, _ = oracle.step(P, s0, 4)
        after = conserved_totals(P, s1)
        drift.append(np.max(np.abs(after - before) / np.abs(before).max()))
    assert drift[0] < 1e-5 and drift[1] < drift[0] / 4


def _shifted_pair(w, U, n):
    P = oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl)
    a = make_state(P, w.rho, w.ux, w.uy, w.T)
    b = make_state(P, w.rho, w.ux + U[0], w.uy + U[1], w.T)
    a, _ = oracle.step(P, a, n)
    b, _ = oracle.step(P, b, n)
    ma, mb = oracle.moments(P, a), oracle.moments(P, b)
    back = {k: np.roll(ma[k], (n * U[1], n * U[0]), axis=(0, 1)) for k in ma}
    return ma, mb, back


@pytest.mark.parametrize("U", [(1, 0), (-2, 0)])
def test_galilean_integer_shift_shear_mode(U):
    """A shear wave seen from a frame moving U cells per step is the same wave
    translated by n U (departure points move by whole cells, the frame
    transformation is covariant)."""
    n = 10
    w = workloads.shear_wave(L=24, tau=0.65, A=1e-3)
    ma, mb, back = _shifted_pair(w, U, n)
    np.testing.assert_allclose(mb["uy"], back["uy"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(mb["ux"] - U[0], back["ux"], rtol=0, atol=1e-12)
    # a wrong-signed departure point would translate the other way
    wrong = np.roll(ma["uy"], (-n * U[1], -n * U[0]), axis=(0, 1))
    assert np.abs(mb["uy"] - wrong).max() > 1e-4


@pytest.mark.parametrize("kind", ["acoustic", "entropy"])
def test_galilean_shift_residual_is_grad_truncation_of_g(kind):
    """g carries total energy, so a frame shift adds (v.U + U^2/2) f to it; with
    the N = 3 Grad projection the fourth-order part of that product is dropped.
    The shift-back residual is therefore not round-off but a truncation error:
    small against the wave and shrinking fast with resolution."""
    res = []
    for L in (16, 32, 64):
        w = getattr(workloads, kind + "_wave")(L=L, tau=0.65, prandtl=0.71, A=1e-3)
        _, mb, back = _shifted_pair(w, (1, 0), 20)
        amp = np.abs(back["rho"] - 1.0).max()
        res.append(max(np.abs(mb["rho"] - back["rho"]).max(), np.abs(mb["T"] - back["T"]).max()) / amp)
    assert res[1] < 5e-3 and res[1] < res[0] / 3 and res[2] < res[1] / 3


def test_stored_frame_is_frame_of_own_moments():
    w = workloads.fourier_modes(n=12, mach=1.5, amplitude=1e-2, seed=2, tau=0.6)
    P = oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl)
    s, st = oracle.step(P, make_state(P, w.rho, w.ux, w.uy, w.T), 2)
    assert st.nonconverged == 0
    m = oracle.moments(P, s)
    np.testing.assert_allclose(m["ux"].ravel(), s.lam[:, 0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(m["uy"].ravel(), s.lam[:, 1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(m["T"].ravel(), s.lam[:, 2], rtol=1e-12, atol=0)
    # populations are centred in their frame: sum_i f_i c_i = 0
    cx, cy, _ = oracle.lattice_2d()
    assert np.abs(s.f @ cx).max() < 1e-13 and np.abs(s.f @ cy).max() < 1e-13
    assert (st.iters >= 2).all()


def test_step_is_deterministic():
    w = workloads.fourier_modes(n=8, mach=2.0, amplitude=1e-2, seed=3, tau=0.55)
    P = oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl)
    s0 = make_state(P, w.rho, w.ux, w.uy, w.T)
    a, _ = oracle.step(P, s0, 2)
    b, _ = oracle.step(P, s0, 2)
    np.testing.assert_array_equal(a.f, b.f)
    np.testing.assert_array_equal(a.g, b.g)
    np.testing.assert_array_equal(a.lam, b.lam)


def test_init_rejects_unphysical_fields():
    P = oracle.params(3, 1, tau=0.6)
    one = np.ones(3)
    with pytest.raises(ValueError):
        oracle.init(P, np.array([1.0, -1.0, 1.0]), 0 * one, 0 * one, one)
    with pytest.raises(ValueError):
        oracle.init(P, one, 0 * one, 0 * one, np.array([1.0, 0.0, 1.0]))
    with pytest.raises(ValueError):
        oracle.init(P, one, np.array([0.0, np.nan, 0.0]), 0 * one, one)
