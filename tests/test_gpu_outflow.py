"""GPU parity of the clamped (zero-gradient) boundary used as an outflow: the
runs the oracle pins in tests/test_oracle_outflow.py -- an acoustic pulse and
the Sod shock leaving through the right edge -- on the HIP path, FP64 within
1e-12 of the oracle, FP32 within 1e-5 (pulse, relative to the field max
norm) and 1e-4 in L1 (shock)."""
import math

import numpy as np
import pytest

import oracle
from paper_2405_11489_amd import workloads
from parity_util import field_errors, field_l1, gpu_run, oracle_run, plane_errors

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
GAMMA = 1.4


def pulse_workload(nx=200, sigma=8.0, A=1e-3, tau=0.6):
    """Right-running isentropic acoustic pulse on gas at rest, clamped in x."""
    x = np.arange(nx, dtype=float)
    cs = math.sqrt(GAMMA)
    rp = A * np.exp(-((x - 100.0) / sigma) ** 2)
    shape = (1, nx)
    return workloads.Workload("acoustic_pulse", nx, 1, workloads.CLAMP, workloads.PERIODIC,
                              GAMMA, 1.0, tau, 120, (1.0 + rp).reshape(shape),
                              (cs * rp).reshape(shape), np.zeros(shape),
                              (1.0 + (GAMMA - 1.0) * rp).reshape(shape))


def test_acoustic_pulse_leaving_matches_oracle():
    w = pulse_workload()
    f, g, fr, _, st, m = gpu_run(w, FP64, w.steps)
    P, s, ost = oracle_run(w, w.steps)
    assert max(plane_errors(f, g, fr, s)) <= 1e-12
    assert st.nonconverged == ost.nonconverged
    _, _, _, _, _, m32 = gpu_run(w, FP32, w.steps)
    errs = field_errors(m32, oracle.moments(P, s))
    assert max(errs.values()) <= 1e-5, errs


def test_sod_shock_leaving_matches_oracle():
    w = workloads.sod_tube(nx=400, nu=2e-3)
    steps = 650  # the shock leaves the tube around step 571
    f, g, fr, _, st, m = gpu_run(w, FP64, steps)
    P, s, ost = oracle_run(w, steps)
    mo = oracle.moments(P, s)
    errs = field_errors(m, mo)
    assert max(errs.values()) <= 1e-12, errs
    assert st.nonconverged == ost.nonconverged and st.nonphysical == 0
    _, _, _, _, _, m32 = gpu_run(w, FP32, steps)
    l1 = field_l1(m32, mo)
    assert max(l1.values()) <= 1e-4, l1
