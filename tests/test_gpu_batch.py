"""Batched stepping and the autotuner on the GPU, through the C ABI.

A batch advances every member by the same step as pond_step, with one
pre-pass and one step launch per step for all members (replayed from a
captured HIP graph), so each member's state after k batched steps must equal,
bit for bit, the state of the same instance stepped k times alone.  The mixes
below span 2-D periodic and clamped grids, quasi-1-D tubes, ragged sizes
smaller than one tile, different tile widths and step counts that exercise
both captured graphs (8 steps and 1 step per launch).
"""
import numpy as np
import pytest

import oracle
from paper_2405_11489_amd import workloads
from parity_util import gpu_run, oracle_run, plane_errors

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _mix():
    ws = [
        workloads.fourier_modes(n=48, ny=40, mach=2.0, amplitude=1e-2, seed=1, tau=0.6,
                                prandtl=0.71),
        workloads.sod_tube(nx=300, nu=2e-3, frame_mach=1.0),
        workloads.shear_wave(L=33, ny=20, tau=0.58, U=0.9, A=1e-2),
        workloads.fourier_modes(n=5, ny=3, mach=1.2, amplitude=1e-2, seed=2, tau=0.7,
                                prandtl=1.0),
        workloads.riemann_quadrants(n=40, seed=3),
        workloads.fourier_modes(n=70, ny=17, mach=2.5, amplitude=2e-2, seed=4, tau=0.6,
                                prandtl=0.71),
    ]
    ws[5].bc_x = workloads.CLAMP
    return ws


def _solvers(ws, prec):
    from paper_2405_11489_amd import pond
    return [pond.Solver.from_workload(w, precision=prec) for w in ws]


def _assert_same(a, b, msg):
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y, err_msg=msg)


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_batch_matches_members_alone_bitwise(prec):
    from paper_2405_11489_amd import pond
    ws = _mix()
    steps = 13  # one 8-step graph launch and five 1-step launches
    alone = [gpu_run(w, prec, steps) for w in ws]
    sols = _solvers(ws, prec)
    b = pond.pond_batch_create([s.ctx for s in sols])
    try:
        info = pond.pond_batch_get_info(b)
        assert info.members == len(ws)
        assert info.nodes == sum(w.nodes for w in ws)
        pond.pond_batch_step(b, 5)
        pond.pond_batch_step(b, steps - 5)
        pond.pond_batch_synchronize(b)
        assert pond.pond_batch_get_info(b).steps == steps
        for i, (s, ref) in enumerate(zip(sols, alone)):
            _assert_same(s.export_state(), ref, f"member {i} ({ws[i].name})")
            assert s.stats().steps == steps
    finally:
        pond.pond_batch_destroy(b)
        for s in sols:
            s.close()


def test_batch_tile_widths_bitwise_equal():
    """Every batch tile width computes the same bits (the widths only change
    which lanes share a staged source region)."""
    from paper_2405_11489_amd import pond
    ws = _mix()[:3] + _mix()[5:]
    ref = [gpu_run(w, FP32, 4) for w in ws]
    for width in (16, 32, 64, 128, 256):
        sols = _solvers(ws, FP32)
        for s in sols:
            pond.pond_set_tuning(s.ctx, batch_tile_width=width)
        b = pond.pond_batch_create([s.ctx for s in sols])
        try:
            assert all(pond.pond_batch_member_tile_width(b, i) == width for i in range(len(ws)))
            pond.pond_batch_step(b, 4)
            pond.pond_batch_synchronize(b)
            for i, s in enumerate(sols):
                _assert_same(s.export_state(), ref[i], f"width {width} member {i}")
        finally:
            pond.pond_batch_destroy(b)
            for s in sols:
                s.close()


def test_batch_members_with_different_parity_and_resume_alone():
    """Members enter the batch at different step counts (so different current
    buffers), and step alone again after the batch is destroyed."""
    from paper_2405_11489_amd import pond
    ws = _mix()[:4]
    ref = [gpu_run(w, FP32, 12) for w in ws]
    sols = _solvers(ws, FP32)
    sols[1].step(1)
    sols[3].step(3)
    b = pond.pond_batch_create([s.ctx for s in sols])
    try:
        pond.pond_batch_step(b, 9)
    finally:
        pond.pond_batch_destroy(b)
    try:
        for s, before in zip(sols, [0, 1, 0, 3]):  # every member reaches 12 steps
            if 12 - 9 - before:
                s.step(12 - 9 - before)
        for i, s in enumerate(sols):
            _assert_same(s.export_state(), ref[i], f"member {i}")
    finally:
        for s in sols:
            s.close()


def test_batch_fp64_members_match_oracle():
    from paper_2405_11489_amd import pond
    ws = [workloads.fourier_modes(n=12, ny=10, mach=2.0, amplitude=1e-2, seed=5, tau=0.6,
                                  prandtl=0.71),
          workloads.sod_tube(nx=64, nu=2e-3, frame_mach=2.0)]
    sols = _solvers(ws, FP64)
    b = pond.pond_batch_create([s.ctx for s in sols])
    try:
        pond.pond_batch_step(b, 3)
        pond.pond_batch_synchronize(b)
        for w, s in zip(ws, sols):
            f, g, fr, _ = s.export_state()
            _, o, _ = oracle_run(w, 3)
            assert max(plane_errors(f, g, fr, o)) <= 1e-12, w.name
    finally:
        pond.pond_batch_destroy(b)
        for s in sols:
            s.close()


def test_batch_ownership_rules():
    from paper_2405_11489_amd import pond
    ws = _mix()[:2]
    sols = _solvers(ws, FP32)
    other = _solvers(ws[:1], FP64)[0]
    try:
        ctxs = [s.ctx for s in sols]
        with pytest.raises(pond.PondError) as ei:
            pond.pond_batch_create([ctxs[0], ctxs[0]])
        assert ei.value.status == pond.ERR_INVALID_ARG
        with pytest.raises(pond.PondError) as ei:
            pond.pond_batch_create([ctxs[0], other.ctx])
        assert ei.value.status == pond.ERR_INVALID_ARG
        b = pond.pond_batch_create(ctxs)
        try:
            for call in (lambda: pond.pond_step(ctxs[0], 1),
                         lambda: pond.pond_destroy(ctxs[1]),
                         lambda: pond.pond_set_tuning(ctxs[0], tile=pond.TILE_16x16),
                         lambda: pond.pond_batch_create([ctxs[0]]),
                         lambda: pond.pond_autotune(ctxs[0], 1)):
                with pytest.raises(pond.PondError) as ei:
                    call()
                assert ei.value.status == pond.ERR_STATE
            pond.pond_batch_step(b, 2)
            m = sols[0].moments()  # read-outs stay available, ordered after the steps
            assert np.all(np.isfinite(m["rho"]))
        finally:
            pond.pond_batch_destroy(b)
        sols[0].step(1)
        sols[0].synchronize()
    finally:
        for s in sols + [other]:
            s.close()


def test_nonphysical_member_does_not_disturb_the_others():
    """The shock tube at nu = 1e-4 goes non-physical within 80 steps; batched
    with healthy members, only it is flagged and the others' results are
    unchanged."""
    from paper_2405_11489_amd import pond
    bad = workloads.sod_tube(nx=400, nu=1e-4)
    good = _mix()[:2]
    ref = [gpu_run(w, FP64, 80) for w in good]
    sols = _solvers([good[0], bad, good[1]], FP64)
    b = pond.pond_batch_create([s.ctx for s in sols])
    try:
        pond.pond_batch_step(b, 80)
        with pytest.raises(pond.PondError) as ei:
            pond.pond_batch_synchronize(b)
        assert ei.value.status == pond.ERR_NONPHYSICAL
        with pytest.raises(pond.PondError) as ei:
            pond.pond_batch_step(b, 1)
        assert ei.value.status == pond.ERR_STATE
        _assert_same(sols[0].export_state(), ref[0], "healthy member 0")
        _assert_same(sols[2].export_state(), ref[1], "healthy member 2")
    finally:
        pond.pond_batch_destroy(b)
        for s in sols:
            s.close()


def test_autotune_restores_state_and_caches_the_size_class():
    from paper_2405_11489_amd import pond
    pond.pond_tuning_cache_clear()
    w = workloads.fourier_modes(n=96, ny=80, mach=2.0, amplitude=1e-2, seed=7, tau=0.6,
                                prandtl=0.71)
    ref = gpu_run(w, FP32, 5)
    with pond.Solver.from_workload(w, precision=FP32) as s:
        s.step(2)
        before = s.export_state()
        st0 = s.stats()
        t = pond.pond_autotune(s.ctx, 2)
        assert t.kernel == pond.KERNEL_TILED
        assert t.tile in (pond.TILE_32x8, pond.TILE_16x16, pond.TILE_16x8, pond.TILE_32x16,
                          pond.TILE_8x8)
        assert t.batch_tile_width in (16, 32, 64)
        _assert_same(s.export_state(), before, "state after autotune")
        st1 = s.stats()
        assert (st1.steps, st1.pc_iterations) == (st0.steps, st0.pc_iterations)
        s.step(3)
        _assert_same(s.export_state(), ref, "steps after autotune")
    # a new context of the same size class starts with the tuned configuration
    with pond.Solver.from_workload(w, precision=FP32) as s2:
        t2 = pond.pond_get_tuning(s2.ctx)
        assert (t2.tile, t2.batch_tile_width) == (t.tile, t.batch_tile_width)
    pond.pond_tuning_cache_clear()


def test_quasi_1d_single_row_tiles_bitwise_equal_global():
    """Single-row grids stage one row per tile (every stencil row is that
    row); the result equals the HBM-gather kernel's bit for bit."""
    from paper_2405_11489_amd import pond
    w = workloads.sod_tube(nx=1000, nu=2e-3, frame_mach=2.5)
    ref = gpu_run(w, FP32, 6, tuning={"kernel": pond.KERNEL_GLOBAL})
    for tile in (pond.TILE_64x1, pond.TILE_256x1):
        out = gpu_run(w, FP32, 6, tuning={"kernel": pond.KERNEL_TILED, "tile": tile, "lds_nodes": 0})
        _assert_same(out, ref, f"tile {tile}")
