"""Writes quadrants256_oracle.npz: the FP64 CPU oracle's macroscopic fields
(rho, u_x, u_y, T) after 200 steps of the four-quadrant 2-D Riemann problem on
a 256 x 256 periodic grid -- the same quadrant states as the 2048 x 2048
benchmark workload (workloads.riemann_quadrants, seed 0, nu = 2e-3 at the
lattice temperature scale 0.04, gamma = 1.4, Pr = 0.71), total-energy split,
D2Q16, cubic stencil.

Only the oracle (oracle/) computes anything here; the seeded workload module
supplies the initial fields.  Run from the repository root:

    python tests/golden/make_quadrants256.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2405_11489_amd import workloads  # noqa: E402

N = 256
STEPS = 200
OUT = os.path.join(HERE, "quadrants256_oracle.npz")


def main():
    w = workloads.riemann_quadrants(n=N, seed=0)
    P = oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl, bc_x=w.bc_x,
                      bc_y=w.bc_y)
    s = oracle.init(P, w.rho.ravel(), w.ux.ravel(), w.uy.ravel(), w.T.ravel())
    t0 = time.perf_counter()
    s, st = oracle.step(P, s, STEPS)
    m = oracle.moments(P, s)
    print(f"{STEPS} oracle steps of {N}x{N} in {time.perf_counter() - t0:.0f} s, "
          f"{st.total_iters / (STEPS * N * N):.3f} gathers per node, "
          f"non-converged {st.nonconverged}, non-physical {st.nonphysical}")
    assert st.nonphysical == 0
    np.savez_compressed(OUT, steps=STEPS, n=N, tau=w.tau, prandtl=w.prandtl, gamma=w.gamma,
                        states=np.array(w.meta["states"]),
                        **{k: m[k].reshape(N, N) for k in ("rho", "ux", "uy", "T")})
    print("wrote", OUT)


if __name__ == "__main__":
    main()
