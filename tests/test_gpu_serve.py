"""Continuous-batching server on the GPU, through the C ABI.

The mix test serves a stream of mixed requests with an HBM budget small
enough that admission binds, a chunk size that forces many batch rebuilds,
and then re-runs requests alone with pond_step: each served result must
equal its solo result bit for bit.  The bookkeeping tests check strict FIFO
admission, the budget, and the failure paths (bad fields, a non-physical
run, refused submissions).
"""
import numpy as np
import pytest

from paper_2405_11489_amd import workloads
from parity_util import gpu_run

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _params(pond, w, prec=FP32):
    return pond.pond_params_default(nx=w.nx, ny=w.ny, tau=w.tau, gamma=w.gamma,
                                    prandtl=w.prandtl, bc_x=w.bc_x, bc_y=w.bc_y, precision=prec)


def _stream(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = i % 4
        n = int(rng.integers(12, 64))
        steps = int(rng.integers(3, 40))
        if kind == 0:
            w = workloads.fourier_modes(n=n, ny=int(rng.integers(8, 48)), mach=float(rng.uniform(0.5, 2.5)),
                                        amplitude=1e-2, seed=int(rng.integers(1 << 20)), tau=0.6)
        elif kind == 1:
            w = workloads.sod_tube(nx=4 * n, frame_mach=float(rng.uniform(0, 2)), nu=2e-3)
        elif kind == 2:
            w = workloads.riemann_quadrants(n=n, seed=int(rng.integers(1 << 20)))
        else:
            w = workloads.shear_wave(L=n, ny=int(rng.integers(1, 20)), tau=0.6,
                                     U=float(rng.uniform(0, 2)), A=1e-2)
        out.append((w, steps))
    return out


def _server(pond, **cfg):
    return pond.pond_server_create(pond.pond_server_config_default(**cfg))


def _unpack_state(x, N):
    return x[:16 * N].reshape(16, N), x[16 * N:32 * N].reshape(16, N), x[32 * N:35 * N].reshape(3, N)


def test_served_results_equal_solo_results_bitwise():
    from paper_2405_11489_amd import pond
    reqs = _stream(0, 24)
    sizes = sorted(pond.pond_state_bytes(_params(pond, w)) for w, _ in reqs)
    budget = sum(sizes[-3:])  # admission binds: at most a few requests run at once
    srv = _server(pond, hbm_budget_bytes=budget, chunk_steps=7)
    try:
        ids = [pond.pond_server_submit(srv, _params(pond, w), w.rho, w.ux, w.uy, w.T, steps,
                                       pond.REQ_KEEP_STATE | pond.REQ_KEEP_MOMENTS)
               for w, steps in reqs]
        pond.pond_server_wait(srv, 0)
        st = pond.pond_server_get_stats(srv)
        assert st.completed == len(reqs) and st.failed == 0
        assert st.admission_waits > 0 and st.batch_builds >= 4
        infos = [pond.pond_server_poll(srv, i) for i in ids]
        assert all(inf.state == pond.REQ_DONE for inf in infos)
        # strict FIFO admission, and the budget holds at every admission
        adm = [inf.t_admit for inf in infos]
        assert adm == sorted(adm)
        for inf in infos:
            live = sum(o.state_bytes for o in infos if o.t_admit <= inf.t_admit < o.t_done)
            assert live <= budget
        for k in range(16):
            w, steps = reqs[k]
            N = w.nodes
            x = np.zeros(35 * N + 2)
            m = np.zeros(5 * N)
            pond.pond_server_result(srv, ids[k], m, x)
            f, g, fr, _, _, mom = gpu_run(w, FP32, steps)
            got = _unpack_state(x, N)
            for a, b in zip(got, (f, g, fr)):
                np.testing.assert_array_equal(a, b, err_msg=f"request {k} ({w.name})")
            np.testing.assert_array_equal(m[:N].reshape(w.ny, w.nx), mom["rho"])
            np.testing.assert_array_equal(m[3 * N:4 * N].reshape(w.ny, w.nx), mom["T"])
            pond.pond_server_release(srv, ids[k])
    finally:
        pond.pond_server_destroy(srv)


@pytest.mark.parametrize("split", [1, 2])
def test_internal_and_nontrans_servers_equal_solo_bitwise(split):
    """A server set to the internal (1) or non-translational (2) split serves
    requests of that split, each equal to its run alone bit for bit; a request
    of another split is refused."""
    from paper_2405_11489_amd import pond
    reqs = [(workloads.fourier_modes(n=24, ny=16, mach=1.5, amplitude=1e-2, seed=31, tau=0.6,
                                     prandtl=1.0), 9),
            (workloads.shear_wave(L=32, ny=4, tau=0.6, U=1.0, A=1e-2), 5),
            (workloads.fourier_modes(n=40, ny=24, mach=0.8, amplitude=1e-2, seed=32, tau=0.7,
                                     prandtl=1.0), 12)]
    srv = _server(pond, split=split, chunk_steps=4)
    try:
        ids = []
        for w, steps in reqs:
            p = _params(pond, w)
            p.split = split
            ids.append(pond.pond_server_submit(srv, p, w.rho, w.ux, w.uy, w.T, steps,
                                               pond.REQ_KEEP_STATE))
        other = _params(pond, reqs[0][0])
        with pytest.raises(pond.PondError) as ei:
            pond.pond_server_submit(srv, other, reqs[0][0].rho, reqs[0][0].ux, reqs[0][0].uy,
                                    reqs[0][0].T, 3)
        assert ei.value.status == pond.ERR_INVALID_ARG
        pond.pond_server_wait(srv, 0)
        for (w, steps), i in zip(reqs, ids):
            N = w.nodes
            x = np.zeros(35 * N + 2)
            pond.pond_server_result(srv, i, None, x)
            f, g, fr, _, _, _ = gpu_run(w, FP32, steps, split=split)
            for a, b in zip(_unpack_state(x, N), (f, g, fr)):
                np.testing.assert_array_equal(a, b, err_msg=w.name)
    finally:
        pond.pond_server_destroy(srv)


def test_server_taking_any_precision_stencil_and_split():
    """A server configured with SERVE_ANY takes requests of every precision,
    stencil and energy split; each round batches requests of one kind, and
    every served state equals the request's run alone bit for bit."""
    from paper_2405_11489_amd import pond
    kinds = [(FP32, 4, 0), (FP64, 4, 1), (FP32, 3, 2), (FP32, 4, 1), (FP64, 3, 0), (FP32, 4, 2),
             (FP32, 4, 0), (FP64, 4, 2)]
    reqs = []
    for k, (prec, npts, split) in enumerate(kinds):
        w = workloads.fourier_modes(n=16 + 4 * k, ny=12 + 2 * k, mach=1.2, amplitude=1e-2,
                                    seed=70 + k, tau=0.6, prandtl=1.0)
        reqs.append((w, 5 + k, prec, npts, split))
    srv = _server(pond, precision=pond.SERVE_ANY, interp_points=pond.SERVE_ANY,
                  split=pond.SERVE_ANY, chunk_steps=3)
    try:
        ids = []
        for w, steps, prec, npts, split in reqs:
            p = _params(pond, w, prec)
            p.interp_points = npts
            p.split = split
            ids.append(pond.pond_server_submit(srv, p, w.rho, w.ux, w.uy, w.T, steps,
                                               pond.REQ_KEEP_STATE))
        pond.pond_server_wait(srv, 0)
        st = pond.pond_server_get_stats(srv)
        assert st.completed == len(reqs) and st.failed == 0
        for (w, steps, prec, npts, split), i in zip(reqs, ids):
            N = w.nodes
            x = np.zeros(35 * N + 2)
            pond.pond_server_result(srv, i, None, x)
            f, g, fr, _, _, _ = gpu_run(w, prec, steps, interp_points=npts, split=split)
            for a_, b_ in zip(_unpack_state(x, N), (f, g, fr)):
                np.testing.assert_array_equal(a_, b_, err_msg=f"{w.name} {prec} {npts} {split}")
    finally:
        pond.pond_server_destroy(srv)


def test_failures_and_refusals():
    from paper_2405_11489_amd import pond
    good = workloads.fourier_modes(n=20, ny=12, mach=1.0, amplitude=1e-2, seed=1, tau=0.6)
    bad_fields = workloads.fourier_modes(n=20, ny=12, mach=1.0, amplitude=1e-2, seed=2, tau=0.6)
    bad_fields.rho[3, 4] = -1.0
    blowup = workloads.sod_tube(nx=400, nu=1e-4)
    srv = _server(pond, hbm_budget_bytes=pond.pond_state_bytes(_params(pond, blowup)) * 3)
    try:
        with pytest.raises(pond.PondError) as ei:  # precision differs from the server's
            pond.pond_server_submit(srv, _params(pond, good, FP64), good.rho, good.ux, good.uy,
                                    good.T, 5)
        assert ei.value.status == pond.ERR_INVALID_ARG
        huge = workloads.fourier_modes(n=400, mach=1.0, amplitude=1e-2, seed=3, tau=0.6)
        with pytest.raises(pond.PondError) as ei:  # larger than the whole budget
            pond.pond_server_submit(srv, _params(pond, huge), huge.rho, huge.ux, huge.uy, huge.T, 5)
        assert ei.value.status == pond.ERR_INVALID_ARG
        ids = [pond.pond_server_submit(srv, _params(pond, w), w.rho, w.ux, w.uy, w.T, n,
                                       pond.REQ_KEEP_MOMENTS)
               for w, n in ((good, 30), (bad_fields, 30), (blowup, 120), (good, 10))]
        pond.pond_server_wait(srv, 0)
        states = [pond.pond_server_poll(srv, i) for i in ids]
        assert [s.state for s in states] == [pond.REQ_DONE, pond.REQ_FAILED, pond.REQ_FAILED,
                                             pond.REQ_DONE]
        assert states[1].error == pond.ERR_INVALID_ARG
        assert states[2].error == pond.ERR_NONPHYSICAL
        with pytest.raises(pond.PondError) as ei:
            pond.pond_server_result(srv, ids[2], np.zeros(5 * blowup.nodes))
        assert ei.value.status == pond.ERR_NONPHYSICAL
        m = np.zeros(5 * good.nodes)
        pond.pond_server_result(srv, ids[0], m)
        ref = gpu_run(good, FP32, 30)[5]
        np.testing.assert_array_equal(m[:good.nodes].reshape(good.ny, good.nx), ref["rho"])
    finally:
        pond.pond_server_destroy(srv)


def test_autotuning_server_and_zero_step_requests():
    from paper_2405_11489_amd import pond
    pond.pond_tuning_cache_clear()
    reqs = _stream(5, 6)
    srv = _server(pond, autotune_steps=1, chunk_steps=0, max_members=2)
    try:
        ids = [pond.pond_server_submit(srv, _params(pond, w), w.rho, w.ux, w.uy, w.T, s,
                                       pond.REQ_KEEP_STATE) for w, s in reqs]
        zid = pond.pond_server_submit(srv, _params(pond, reqs[0][0]), reqs[0][0].rho,
                                      reqs[0][0].ux, reqs[0][0].uy, reqs[0][0].T, 0,
                                      pond.REQ_KEEP_STATE)
        pond.pond_server_wait(srv, 0)
        for (w, steps), i in zip(reqs, ids):
            x = np.zeros(35 * w.nodes + 2)
            pond.pond_server_result(srv, i, None, x)
            f, g, fr, _, _, _ = gpu_run(w, FP32, steps)
            for a, b in zip(_unpack_state(x, w.nodes), (f, g, fr)):
                np.testing.assert_array_equal(a, b)
        assert pond.pond_server_poll(srv, zid).state == pond.REQ_DONE
    finally:
        pond.pond_server_destroy(srv)
        pond.pond_tuning_cache_clear()


def test_fp64_served_requests_match_the_oracle():
    """An FP64 server (continuous batching, a budget that holds about two
    requests at a time, 5-step chunks): every served state equals the CPU
    oracle's on the same inputs within 1e-12 per plane (Eq.
    propagationInterpolated, the step the oracle runs literally)."""
    from paper_2405_11489_amd import pond
    from parity_util import oracle_run, plane_errors
    rng = np.random.default_rng(7)
    reqs = []
    for i in range(6):
        n = int(rng.integers(8, 20))
        steps = int(rng.integers(3, 12))
        if i % 3 == 0:
            w = workloads.fourier_modes(n=n, ny=int(rng.integers(6, 16)), mach=1.5,
                                        amplitude=1e-2, seed=int(rng.integers(1 << 20)), tau=0.6)
        elif i % 3 == 1:
            w = workloads.sod_tube(nx=4 * n, frame_mach=0.7, nu=2e-3)
        else:
            w = workloads.riemann_quadrants(n=n, seed=int(rng.integers(1 << 20)))
        reqs.append((w, steps))
    sizes = sorted(pond.pond_state_bytes(_params(pond, w, FP64)) for w, _ in reqs)
    srv = _server(pond, precision=FP64, hbm_budget_bytes=sizes[-1] + sizes[-2], chunk_steps=5)
    try:
        ids = [pond.pond_server_submit(srv, _params(pond, w, FP64), w.rho, w.ux, w.uy, w.T, steps,
                                       pond.REQ_KEEP_STATE)
               for w, steps in reqs]
        pond.pond_server_wait(srv, 0)
        st = pond.pond_server_get_stats(srv)
        assert st.completed == len(reqs) and st.failed == 0
        for rid, (w, steps) in zip(ids, reqs):
            N = w.nodes
            x = np.zeros(35 * N + 2)
            pond.pond_server_result(srv, rid, None, x)
            f, g, fr = _unpack_state(x, N)
            P, s, ost = oracle_run(w, steps)
            assert ost.nonphysical == 0
            assert max(plane_errors(f, g, fr, s)) <= 1e-12, (w.name, w.nx, w.ny, steps)
    finally:
        pond.pond_server_destroy(srv)
