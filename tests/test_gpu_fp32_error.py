"""Error of the FP32 path over the whole run of the 512 x 512 Mach-2
Fourier-mode workload (2000 steps, tau = 0.55, the benchmark's second
workload).  The FP32 path keeps populations, interpolation and the frame
transformation in float and the conserved moments, temperature recovery and
frame iteration in double.

Stated two ways at step 2000:
  * relative to each field's max norm (velocity components: to the velocity
    scale max(|u|, sqrt T)), against the FP64 GPU path: the 1e-5 bar of smooth
    cases;
  * relative to the amplitude of the perturbation the modes carry (each
    field's deviation from the uniform background, max over the grid).
The FP64 path itself is checked against the CPU oracle at 2048 sampled nodes
of the last step (the oracle steps those nodes from the FP64 state of step
1999): 1e-12.  The test prints the measured figures.
"""
import numpy as np
import pytest

import oracle
from paper_2405_11489_amd import workloads
from parity_util import field_errors, gpu_solver, oracle_params_for, to_oracle_state

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
STEPS = 2000


def test_fp32_error_over_the_full_512_mach2_run():
    w = workloads.fourier_modes(n=512, mach=2.0, angle_deg=30.0, amplitude=1e-3, seed=0,
                                tau=0.55, prandtl=0.71, gamma=1.4, steps=STEPS)
    with gpu_solver(w, FP64) as s:
        s.step(STEPS - 1)
        f, g, fr, _ = s.export_state()
        s.step(1)
        f2, g2, fr2, _ = s.export_state()
        m64 = s.moments()
    with gpu_solver(w, FP32) as s:
        s.step(STEPS)
        st = s.stats()
        m32 = s.moments()
    assert st.nonphysical == 0

    errs = field_errors(m32, m64)
    U = np.array(w.meta["U"])
    background = {"rho": 1.0, "ux": U[0], "uy": U[1], "T": 1.0, "p": 1.0}
    pert = {}
    for k, b in background.items():
        amp = float(np.max(np.abs(m64[k] - b)))
        pert[k] = float(np.max(np.abs(m32[k] - m64[k]))) / amp
    mean_rho = float(np.mean(m32["rho"] - m64["rho"]))
    print(f"\nFP32 - FP64 mean density after {STEPS} steps: {mean_rho:.2e}")
    print(f"FP32 vs FP64 after {STEPS} steps, max-norm relative: "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    print("perturbation-relative: " + ", ".join(f"{k} {v:.2e}" for k, v in pert.items()))
    assert max(errs.values()) <= 1e-5, errs
    assert max(pert.values()) <= 1e-2, pert

    # the FP64 path against the oracle at sampled nodes of the last step
    P = oracle_params_for(w)
    s64 = to_oracle_state(f, g, fr)
    nodes = np.random.default_rng(0).permutation(w.nodes)[:2048]
    fo, go, lo, _, status = oracle.step_nodes(P, s64, nodes)
    assert not status.any()
    for a, b in ((f2[:, nodes].T, fo), (g2[:, nodes].T, go)):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    vs = max(float(np.max(np.abs(lo[:, :2]))), float(np.sqrt(np.max(lo[:, 2]))))
    assert np.max(np.abs(fr2[:2, nodes].T - lo[:, :2])) <= 1e-12 * vs
    assert np.max(np.abs(fr2[2, nodes] - lo[:, 2])) <= 1e-12 * np.max(lo[:, 2])
