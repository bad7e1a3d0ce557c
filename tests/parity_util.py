"""Helpers of the GPU parity tests: run a workload through the HIP path (via
the C ABI binding) and through the FP64 oracle on identical seeded inputs, and
compare element by element."""
import numpy as np

import oracle


def oracle_params_for(w, **kw):
    if w.bc_y == oracle.WALL:
        kw.setdefault("wall_ux", w.wall_ux)
        kw.setdefault("wall_T", w.wall_T)
    return oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl,
                         bc_x=w.bc_x, bc_y=w.bc_y, **kw)


def oracle_run(w, steps, **kw):
    P = oracle_params_for(w, **kw)
    s = oracle.init(P, w.rho.ravel(), w.ux.ravel(), w.uy.ravel(), w.T.ravel())
    s, st = oracle.step(P, s, steps)
    return P, s, st


def gpu_solver(w, precision, **kw):
    from paper_2405_11489_amd import pond
    return pond.Solver.from_workload(w, precision=precision, **kw)


def gpu_run(w, precision, steps, **kw):
    """Returns (f (16,N), g (16,N), frame (3,N), u_ref, stats, moments).
    ``tuning={...}`` selects the kernel / tile / LDS capacity."""
    with gpu_solver(w, precision, **kw) as s:
        s.step(steps)
        f, g, fr, ur = s.export_state()
        st = s.stats()
        m = s.moments()
    return f, g, fr, ur, st, m


def _rel(a, b, scale=None):
    scale = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / scale)


def velocity_scale(ux, uy, T):
    """Scale of the velocity components: max(|u|_inf, sqrt(max T)).  A velocity
    component that vanishes identically (a 1-D flow) is measured against it."""
    return float(max(np.max(np.abs(ux)), np.max(np.abs(uy)), np.sqrt(np.max(T))))


def plane_errors(f, g, fr, ostate):
    """Max over planes of ||gpu - oracle||_inf / ||oracle||_inf for f planes, g
    planes and the T plane; u_x, u_y planes relative to the velocity scale
    (oracle state in its node-major layout)."""
    ef = max(_rel(f[i], ostate.f[:, i]) for i in range(f.shape[0]))
    eg = max(_rel(g[i], ostate.g[:, i]) for i in range(g.shape[0]))
    vs = velocity_scale(ostate.lam[:, 0], ostate.lam[:, 1], ostate.lam[:, 2])
    el = max(_rel(fr[0], ostate.lam[:, 0], vs), _rel(fr[1], ostate.lam[:, 1], vs),
             _rel(fr[2], ostate.lam[:, 2]))
    return ef, eg, el


def field_errors(m_gpu, m_or):
    """Max-norm error per macroscopic field, relative to the field's max norm
    (velocity components: to the velocity scale)."""
    vs = velocity_scale(m_or["ux"], m_or["uy"], m_or["T"])
    return {k: _rel(m_gpu[k], m_or[k], vs if k in ("ux", "uy") else None)
            for k in ("rho", "ux", "uy", "T", "p")}


def field_l1(m_gpu, m_or):
    """L1 error per macroscopic field: sum|a - b| / sum|b| (velocity
    components: / (N x velocity scale))."""
    vs = velocity_scale(m_or["ux"], m_or["uy"], m_or["T"])
    out = {}
    for k in ("rho", "ux", "uy", "T", "p"):
        d = np.abs(m_gpu[k] - m_or[k]).sum()
        out[k] = float(d / (m_or[k].size * vs) if k in ("ux", "uy") else d / np.abs(m_or[k]).sum())
    return out


def to_oracle_state(f, g, fr, prev=None):
    """GPU export layout (planes) -> oracle node-major state; prev: the
    internal-energy split's previous-level frame velocities (2, N), or None."""
    lam_prev = None
    if prev is not None:
        lam_prev = np.ascontiguousarray(np.vstack([prev, fr[2:3]]).T)
    return oracle.State(np.ascontiguousarray(f.T), np.ascontiguousarray(g.T),
                        np.ascontiguousarray(fr.T), lam_prev)


def prev_frame_of(sol, split):
    """The internal-energy split's previous-level frame velocities of a solver
    (None for the other splits, which keep none)."""
    return sol.export_prev_frame() if split == oracle.INTERNAL else None
