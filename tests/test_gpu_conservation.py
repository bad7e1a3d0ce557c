"""A uniform flow of unit density, at rest or advected, through the FP32 path
(Eq. propagationInterpolated on a uniform field), on both lattices and every
energy split.

The step interpolates the stencil nodes' deviations from the tile's reference
moments and adds the reference's own share of the gathered sums once, in FP64
(the Grad reconstruction keeps every moment up to the quadrature's order, so
that share is the reference moments themselves); on a uniform field the
deviations vanish.  What remains is the rounding of the stored populations to
float: the non-equilibrium Grad coefficients of a uniform state are rounding
noise (about 1e-7 of the second moments), which moves the stored populations
by about an ulp, so mass, velocity and temperature drift at that level
(measured over 400 steps: density 1e-8 .. 6e-7, velocity <= 8e-7 of its
scale, temperature <= 2.2e-6).  They must stay within the FP32 bar of smooth
cases (1e-5 of each field's scale; velocity against max(|u|, sqrt T)), and
every node must keep the same values as every other, bit for bit: they see
the same deviations (none) and the same departure fractions.  The test prints
the measured drift.
"""
import numpy as np
import pytest

from paper_2405_11489_amd import workloads
from parity_util import gpu_solver

pytestmark = pytest.mark.gpu

FP32 = 1
STEPS = 400
FLOWS = [(0.0, 1.0), (2.0, 1.0), (1.0, 0.04)]  # (Mach, T)
VARIANTS = [(16, "total"), (16, "internal"), (16, "nontrans"), (25, "total"), (25, "nontrans")]


def _uniform(mach, T, prandtl):
    return workloads.fourier_modes(n=64, ny=32, mach=mach, angle_deg=30.0, amplitude=0.0, seed=0,
                                   tau=0.55, prandtl=prandtl, T0=T, steps=STEPS)


@pytest.mark.parametrize("lattice,split", VARIANTS)
@pytest.mark.parametrize("mach,T", FLOWS)
def test_fp32_uniform_flow_stays_uniform_within_rounding(lattice, split, mach, T):
    from paper_2405_11489_amd import pond
    sp = {"total": pond.SPLIT_TOTAL, "internal": pond.SPLIT_INTERNAL,
          "nontrans": pond.SPLIT_NONTRANS}[split]
    w = _uniform(mach, T, 1.0 if split == "nontrans" else 0.71)
    assert np.all(w.rho == 1.0)
    with gpu_solver(w, FP32, lattice=lattice, split=sp) as s:
        s.step(STEPS)
        m = s.moments()
        st = s.stats()
    assert st.nonphysical == 0
    uscale = max(float(np.max(np.hypot(w.ux, w.uy))), np.sqrt(T))
    drho = float(np.max(np.abs(m["rho"] - 1.0)))
    du = float(max(np.max(np.abs(m["ux"] - w.ux)), np.max(np.abs(m["uy"] - w.uy)))) / uscale
    dT = float(np.max(np.abs(m["T"] - w.T))) / T
    # spread over the grid: the nodes of a uniform flow stay alike
    spread = max(float(np.ptp(m["rho"])), float(np.ptp(m["T"])) / T,
                 float(max(np.ptp(m["ux"]), np.ptp(m["uy"]))) / uscale)
    print(f"D2Q{lattice} {split} Mach {mach} T {T}, {STEPS} steps: |rho - 1| {drho:.1e}, "
          f"u {du:.1e}, T {dT:.1e}, spread {spread:.1e}")
    assert drho <= 1e-5 and du <= 1e-5 and dT <= 1e-5
    assert spread == 0.0
