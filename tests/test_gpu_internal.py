"""GPU parity of the internal-energy split (Eqs. int_energy_g,
int_g_evolution): the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs, with the bars of the total split -- FP64 within 1e-12
per population and frame plane, FP32 within 1e-5 relative on smooth flows --
plus bitwise agreement between the kernel variants and between a batched and
an unbatched instance."""
import numpy as np
import pytest

import oracle
from paper_2405_11489_amd import workloads
from parity_util import (field_errors, field_l1, gpu_run, gpu_solver, oracle_params_for,
                         oracle_run, plane_errors, prev_frame_of, to_oracle_state,
                         velocity_scale)

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
INT = oracle.INTERNAL  # same value as the library's POND_SPLIT_INTERNAL


def modes(n, ny=None, mach=2.0, amp=1e-2, seed=0, tau=0.6, prandtl=0.71, T0=1.0, **kw):
    return workloads.fourier_modes(n=n, ny=ny, mach=mach, amplitude=amp, seed=seed, tau=tau,
                                   prandtl=prandtl, T0=T0, **kw)


def clamp_x(w):
    w.bc_x = workloads.CLAMP
    return w


CASES = {
    "4x4_mach2": lambda: modes(4),
    "7x5_clampx": lambda: clamp_x(modes(7, 5, mach=1.0, seed=3)),
    "16x1_sod": lambda: workloads.sod_tube(nx=16, nu=2e-3, steps=4),
    "1x1": lambda: modes(1, 1, mach=0.7),
    "1x9_column": lambda: modes(1, 9, mach=1.5, seed=5),
    "6x5_hot_fast": lambda: modes(6, 5, mach=1.2, T0=4.0, seed=7),
    "9x7_cold": lambda: modes(9, 7, mach=0.5, T0=0.04, seed=8),
    "8x8_unit_prandtl_gamma18": lambda: workloads.fourier_modes(
        n=8, mach=1.0, amplitude=1e-2, seed=2, tau=0.7, prandtl=1.0, gamma=1.8),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("steps", [1, 5])
def test_fp64_tiny_grids_match_oracle(case, steps):
    w = CASES[case]()
    f, g, fr, _, st, m = gpu_run(w, FP64, steps, split=INT)
    P, s, ost = oracle_run(w, steps, split=INT)
    assert max(plane_errors(f, g, fr, s)) <= 1e-12
    assert st.nonphysical == 0 and ost.nonphysical == 0
    errs = field_errors(m, oracle.moments(P, s))
    assert max(errs.values()) <= 1e-12, errs


@pytest.mark.parametrize("npts", [3, 4])
def test_fp64_interp_points_match_oracle(npts):
    w = modes(10, 6, mach=1.3, seed=11)
    f, g, fr, _, _, _ = gpu_run(w, FP64, 3, interp_points=npts, split=INT)
    _, s, _ = oracle_run(w, 3, interp_points=npts, split=INT)
    assert max(plane_errors(f, g, fr, s)) <= 1e-12


def test_fp64_mach2_modes_32_ragged_tiles():
    """32 x 32 spans four 32 x 8 tiles; 37 x 29 leaves ragged edge tiles."""
    for w in (modes(32, mach=2.0, amp=1e-3, seed=1, tau=0.55),
              clamp_x(modes(37, 29, mach=2.0, amp=1e-2, seed=13, tau=0.6))):
        f, g, fr, _, _, _ = gpu_run(w, FP64, 6, split=INT)
        _, s, _ = oracle_run(w, 6, split=INT)
        assert max(plane_errors(f, g, fr, s)) <= 1e-12


@pytest.mark.parametrize("case", ["4x4_mach2", "7x5_clampx", "6x5_hot_fast", "9x7_cold"])
def test_fp32_tiny_grids_within_1e5(case):
    w = CASES[case]()
    _, _, _, _, _, m = gpu_run(w, FP32, 5, split=INT)
    P, s, _ = oracle_run(w, 5, split=INT)
    errs = field_errors(m, oracle.moments(P, s))
    assert max(errs.values()) <= 1e-5, errs


def test_fp32_mach2_modes_smooth_within_1e5():
    w = modes(32, mach=2.0, amp=1e-3, seed=1, tau=0.55)
    _, _, _, _, _, m = gpu_run(w, FP32, 40, split=INT)
    P, s, _ = oracle_run(w, 40, split=INT)
    errs = field_errors(m, oracle.moments(P, s))
    assert max(errs.values()) <= 1e-5, errs


@pytest.mark.parametrize("prec,bar", [(FP64, 1e-12), (FP32, 1e-5)])
def test_full_size_sampled_nodes(prec, bar):
    """512 x 512 Mach-2 modes, the benchmark's launch configuration: after a
    few GPU steps, the oracle recomputes one step at sampled nodes (edges and
    corners included) from the GPU's own state."""
    w = modes(512, mach=2.0, amp=1e-3, seed=0, tau=0.55)
    rng = np.random.default_rng(2)
    nodes = np.concatenate([rng.integers(0, w.nodes, 96),
                            [0, w.nx - 1, w.nodes - w.nx, w.nodes - 1]])
    with gpu_solver(w, prec, split=INT) as sol:
        sol.step(3)
        f0, g0, fr0, _ = sol.export_state()
        pv0 = sol.export_prev_frame()
        sol.step(1)
        f1, g1, fr1, _ = sol.export_state()
    P = oracle_params_for(w, split=INT)
    fo, go, lo, _, _ = oracle.step_nodes(P, to_oracle_state(f0, g0, fr0, pv0), nodes)
    for a, b in ((f1[:, nodes].T, fo), (g1[:, nodes].T, go)):
        assert np.max(np.abs(a - b) / np.max(np.abs(b), axis=0)) <= bar
    vs = velocity_scale(lo[:, 0], lo[:, 1], lo[:, 2])
    assert np.max(np.abs(fr1[:2, nodes].T - lo[:, :2])) / vs <= bar
    assert np.max(np.abs(fr1[2, nodes] - lo[:, 2]) / lo[:, 2]) <= bar


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_kernels_and_tiles_bitwise_equal(prec):
    """HBM-tap kernel, every tile shape and an LDS capacity that forces the
    HBM fallback give the same bits (ragged 70 x 45 grid, clamp in x)."""
    from paper_2405_11489_amd import pond
    w = clamp_x(modes(70, 45, mach=2.5, amp=2e-2, seed=12))
    ref = gpu_run(w, prec, 4, split=INT, tuning={"kernel": pond.KERNEL_GLOBAL})
    for tile, cap in [(pond.TILE_32x8, 0), (pond.TILE_16x16, 0), (pond.TILE_64x1, 0),
                      (pond.TILE_256x1, 0), (pond.TILE_8x8, 100), (pond.TILE_32x16, 0)]:
        out = gpu_run(w, prec, 4, split=INT,
                      tuning={"kernel": pond.KERNEL_TILED, "tile": tile, "lds_nodes": cap})
        for x, y in zip(out[:3], ref[:3]):
            np.testing.assert_array_equal(x, y, err_msg=f"tile {tile} cap {cap}")


def test_total_split_unchanged_by_the_variant_choice():
    """The same fields under the two splits differ (different g), and the
    internal split's macroscopic fields agree with the oracle's while the
    total split's agree with its own oracle run."""
    w = modes(12, 10, mach=1.5, seed=14)
    for split in (oracle.TOTAL, INT):
        _, _, _, _, _, m = gpu_run(w, FP64, 4, split=split)
        P, s, _ = oracle_run(w, 4, split=split)
        assert max(field_errors(m, oracle.moments(P, s)).values()) <= 1e-12
    a = gpu_run(w, FP64, 4, split=oracle.TOTAL)
    b = gpu_run(w, FP64, 4, split=INT)
    assert np.max(np.abs(a[1] - b[1])) > 1e-3


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_batched_equals_alone_bitwise(prec):
    from paper_2405_11489_amd import pond
    ws = [modes(48, 40, mach=1.5, seed=21), clamp_x(modes(33, 17, mach=2.0, seed=22)),
          workloads.sod_tube(nx=100, nu=2e-3, steps=10)]
    alone, alone_prev = [], []
    for w in ws:
        with gpu_solver(w, prec, split=INT) as s:
            s.step(9)
            alone.append(s.export_state()[:3])
            alone_prev.append(s.export_prev_frame())
    sols = [gpu_solver(w, prec, split=INT) for w in ws]
    try:
        b = pond.pond_batch_create([s.ctx for s in sols])
        try:
            pond.pond_batch_step(b, 9)
            pond.pond_batch_synchronize(b)
        finally:
            pond.pond_batch_destroy(b)
        for s, ref, pv in zip(sols, alone, alone_prev):
            for x, y in zip(s.export_state()[:3], ref):
                np.testing.assert_array_equal(x, y)
            np.testing.assert_array_equal(s.export_prev_frame(), pv)
    finally:
        for s in sols:
            s.close()


def test_batch_rejects_mixed_splits_and_server_another_split():
    from paper_2405_11489_amd import pond
    w = modes(16, 8, mach=1.0, seed=23)
    a, b = gpu_solver(w, FP32), gpu_solver(w, FP32, split=INT)
    try:
        with pytest.raises(pond.PondError) as ei:
            pond.pond_batch_create([a.ctx, b.ctx])
        assert ei.value.status == pond.ERR_INVALID_ARG
    finally:
        a.close()
        b.close()
    srv = pond.pond_server_create(pond.pond_server_config_default())
    try:
        p = pond.pond_params_default(nx=w.nx, ny=w.ny, tau=w.tau, gamma=w.gamma,
                                     prandtl=w.prandtl, split=pond.SPLIT_INTERNAL)
        with pytest.raises(pond.PondError) as ei:  # the server's split is the total one
            pond.pond_server_submit(srv, p, w.rho, w.ux, w.uy, w.T, 4)
        assert ei.value.status == pond.ERR_INVALID_ARG
    finally:
        pond.pond_server_destroy(srv)


def test_sod_tube_matches_oracle():
    """The 400 x 1 shock tube at nu = 2e-3 with the internal split, run to
    t = 0.2 (physical throughout since the source is taken to second order in
    time): FP64 within 1e-12 of the oracle, FP32 fields within 1e-4 (L1)."""
    w = workloads.sod_tube(nx=400, nu=2e-3)
    f, g, fr, _, st, _ = gpu_run(w, FP64, w.steps, split=INT)
    P, s, ost = oracle_run(w, w.steps, split=INT)
    assert st.nonphysical == 0 and ost.nonphysical == 0
    assert max(plane_errors(f, g, fr, s)) <= 1e-12
    _, _, _, _, _, m32 = gpu_run(w, FP32, w.steps, split=INT)
    l1 = field_l1(m32, oracle.moments(P, s))
    assert max(l1.values()) <= 1e-4, l1


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_resume_with_previous_level_is_bitwise(prec):
    """The split's state includes the previous level's frame velocities: a
    state exported with them and imported with them resumes bit for bit; the
    previous level after a step is the frame before it; a fresh import (the
    current frames standing in for the previous level) takes another path."""
    w = modes(40, 24, mach=1.5, amp=1e-2, seed=6)
    with gpu_solver(w, prec, split=INT) as s:
        s.step(5)
        ref = s.export_state()
        ref_prev = s.export_prev_frame()
    with gpu_solver(w, prec, split=INT) as s:
        s.step(2)
        f, g, fr, ur = s.export_state()
        prev = s.export_prev_frame()
        s.step(1)
        np.testing.assert_array_equal(s.export_prev_frame(), fr[:2])
    with gpu_solver(w, prec, split=INT) as s:
        s.import_state(f, g, fr, ur)
        np.testing.assert_array_equal(s.export_prev_frame(), fr[:2])
        s.import_prev_frame(prev)
        s.step(3)
        out = s.export_state()
        np.testing.assert_array_equal(s.export_prev_frame(), ref_prev)
    for x, y in zip(out[:3], ref[:3]):
        np.testing.assert_array_equal(x, y)
    with gpu_solver(w, prec, split=INT) as s:
        s.import_state(f, g, fr, ur)
        s.step(3)
        assert not np.array_equal(s.export_state()[1], ref[1])


def test_previous_level_refused_for_other_splits():
    from paper_2405_11489_amd import pond
    w = modes(8, 6, mach=1.0, seed=4, prandtl=1.0)  # the non-translational split: Pr = 1
    for split in (oracle.TOTAL, oracle.NONTRANS):
        with gpu_solver(w, FP32, split=split) as s:
            for call in (lambda: s.export_prev_frame(),
                         lambda: s.import_prev_frame(np.zeros((2, w.nodes)))):
                with pytest.raises(pond.PondError) as ei:
                    call()
                assert ei.value.status == pond.ERR_UNSUPPORTED


def test_resumed_state_matches_oracle_with_previous_level():
    """The oracle stepping a GPU state that carries the previous level agrees
    with the GPU's own next steps (FP64, 1e-12): the previous level enters
    the source as the oracle reads it."""
    w = clamp_x(modes(24, 20, mach=1.8, amp=2e-2, seed=17))
    with gpu_solver(w, FP64, split=INT) as s:
        s.step(4)
        f, g, fr, _ = s.export_state()
        prev = s.export_prev_frame()
        s.step(3)
        f1, g1, fr1, _ = s.export_state()
    P = oracle_params_for(w, split=INT)
    o, _ = oracle.step(P, to_oracle_state(f, g, fr, prev), 3)
    assert max(plane_errors(f1, g1, fr1, o)) <= 1e-12


def test_mach2_512_stays_physical_for_the_full_run():
    """The 512^2 Mach-2 Fourier-mode workload (tau = 0.55) with this split
    over its full 2000 steps in FP32: no non-physical node, and the
    perturbation decays (its velocity deviation from the background ends
    below where it started)."""
    w = modes(512, mach=2.0, amp=1e-3, seed=0, tau=0.55)
    with gpu_solver(w, FP32, split=INT) as s:
        m0 = s.moments()
        s.step(2000)
        st = s.stats()
        m1 = s.moments()
    assert st.nonphysical == 0 and st.nonconverged == 0

    def dev(m):
        return float(np.max(np.hypot(m["ux"] - m["ux"].mean(), m["uy"] - m["uy"].mean())))

    assert dev(m1) < dev(m0)
