"""FP64 CPU oracle of the PonD f+g step (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (the HIP library and its Python
binding) never imports or calls it, and it shares no code with them.

The arithmetic lives in ``pond_oracle.c`` (plain C99, FP64); this module only
marshals numpy arrays through ctypes.  State layout (oracle only): node
``n = y*nx + x``; ``f[n, i]``, ``g[n, i]`` for velocity ``i = q1*a + b`` with
``c_i = (c_a, c_b)`` (q1 = 4 on D2Q16, 5 on D2Q25); frame
``lam[n] = (u_x, u_y, T)``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import build as _build

NONCONVERGED = 1
NONPHYSICAL = 2

_lib = None


class Params(ctypes.Structure):
    """Mirror of ``oracle_params`` in pond_oracle.c."""
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
        ("interp_points", ctypes.c_int), ("pc_max_iter", ctypes.c_int),
        ("tau", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("gamma", ctypes.c_double), ("pc_tol", ctypes.c_double),
        ("split", ctypes.c_int), ("lattice", ctypes.c_int),
        ("wall_ux", ctypes.c_double * 2), ("wall_T", ctypes.c_double * 2),
    ]


PERIODIC, CLAMP, WALL = 0, 1, 2  # boundary handling (WALL: bc_y only)


# energy splits (Eqs. total_energy_g, int_energy_g, nt_energy_g)
TOTAL, INTERNAL, NONTRANS = 0, 1, 2


def params(nx, ny, *, tau, gamma=1.4, prandtl=1.0, bc_x=0, bc_y=0, interp_points=4,
           pc_tol=1e-13, pc_max_iter=32, split=TOTAL, lattice=16, wall_ux=(0.0, 0.0),
           wall_T=(1.0, 1.0)) -> Params:
    """bc_y = WALL: walls at y = -1/2 (bottom) and ny - 1/2 (top) moving along x
    at wall_ux = (bottom, top) and held at wall_T = (bottom, top)."""
    if lattice not in (16, 25):
        raise ValueError("lattice must be 16 (D2Q16) or 25 (D2Q25)")
    if split == NONTRANS and prandtl != 1.0:
        raise ValueError("the non-translational split is built with Pr = 1 only")
    if bc_x == WALL:
        raise ValueError("walls are built for the y boundaries only")
    return Params(nx, ny, bc_x, bc_y, interp_points, pc_max_iter, tau, prandtl, gamma, pc_tol,
                  split, lattice, (ctypes.c_double * 2)(*wall_ux),
                  (ctypes.c_double * 2)(*wall_T))


def _q1(q):
    if q not in (16, 25):
        raise ValueError("16 or 25 populations expected")
    return 4 if q == 16 else 5


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_abi_version.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        L.oracle_lattice_1d.argtypes = [dp, dp]
        L.oracle_lattice_2d.argtypes = [dp, dp, dp]
        L.oracle_transform.argtypes = [dp, dp, dp, dp]
        L.oracle_lattice_1d_q.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_lattice_1d_q.restype = ctypes.c_int
        L.oracle_lattice_2d_q.argtypes = [ctypes.c_int, dp, dp, dp]
        L.oracle_lattice_2d_q.restype = ctypes.c_int
        L.oracle_transform_hermite.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
        L.oracle_transform_hermite.restype = ctypes.c_int
        L.oracle_transform_q.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        L.oracle_equilibrium_q.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 5 + \
            [dp, dp]
        L.oracle_collide_q.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, dp, dp]
        L.oracle_internal_source_q.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
        L.oracle_init_q.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, dp, dp, dp, dp,
                                    ctypes.c_double, dp, dp, dp]
        L.oracle_init_q.restype = ctypes.c_int
        L.oracle_moments_q.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, dp, dp, dp,
                                       ctypes.c_double, dp, dp, dp, dp, dp]
        L.oracle_equilibrium.argtypes = [ctypes.c_double] * 5 + [dp, dp]
        L.oracle_equilibrium_split.argtypes = [ctypes.c_int] + [ctypes.c_double] * 5 + [dp, dp]
        L.oracle_collide.argtypes = [dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, dp, dp]
        L.oracle_collide_split.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, dp, dp]
        L.oracle_internal_source.argtypes = [dp, dp, dp, dp, dp]
        L.oracle_lagrange.argtypes = [ctypes.c_int, ctypes.c_double, ip, dp]
        L.oracle_lagrange.restype = ctypes.c_int
        L.oracle_step.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp, dp, dp, dp, ip, ip]
        L.oracle_step.restype = ctypes.c_int
        lp = ctypes.POINTER(ctypes.c_long)
        L.oracle_step_nodes.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp, ctypes.c_long, lp,
                                        dp, dp, dp, ip, ip]
        L.oracle_step_nodes.restype = ctypes.c_int
        L.oracle_init_split.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp, dp,
                                        ctypes.c_double, dp, dp, dp]
        L.oracle_init_split.restype = ctypes.c_int
        L.oracle_moments_split.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp,
                                           ctypes.c_double, dp, dp, dp, dp, dp]
        if L.oracle_abi_version() != 5:
            raise RuntimeError("oracle library ABI mismatch; rebuild oracle/")
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's following loops (n >= 1)."""
    lib().oracle_set_num_threads(int(n))


def lattice_1d(q1=4):
    """D1Q4 (q1 = 4) or D1Q5 (q1 = 5) abscissae and weights (Table I),
    ascending abscissae."""
    c = np.zeros(q1)
    w = np.zeros(q1)
    if not lib().oracle_lattice_1d_q(q1, _d(c), _d(w)):
        raise ValueError("q1 must be 4 or 5")
    return c, w


def lattice_2d(q1=4):
    """D2Q16 (q1 = 4) or D2Q25 (q1 = 5) velocities (c_x, c_y) and weights,
    i = q1*a + b."""
    q = q1 * q1
    cx, cy, w = np.zeros(q), np.zeros(q), np.zeros(q)
    if not lib().oracle_lattice_2d_q(q1, _d(cx), _d(cy), _d(w)):
        raise ValueError("q1 must be 4 or 5")
    return cx, cy, w


def transform(pop, lam_src, lam_dst):
    """Frame transformation of 16 (D2Q16: the printed a0..a3) or 25 (D2Q25:
    order-4 Hermite projection) populations from lam_src to lam_dst."""
    pop = _f64(pop).ravel()
    q1 = _q1(len(pop))
    out = np.zeros(len(pop))
    lib().oracle_transform_q(q1, _d(pop), _d(_f64(lam_src, (3,))), _d(_f64(lam_dst, (3,))),
                             _d(out))
    return out


def transform_hermite(pop, lam_src, lam_dst, order):
    """Frame transformation as the Hermite projection of the given order."""
    pop = _f64(pop).ravel()
    q1 = _q1(len(pop))
    out = np.zeros(len(pop))
    if lib().oracle_transform_hermite(q1, order, _d(pop), _d(_f64(lam_src, (3,))),
                                      _d(_f64(lam_dst, (3,))), _d(out)) != 0:
        raise ValueError("order must be <= min(4, q1 - 1)")
    return out


def equilibrium(rho, ux, uy, T, gamma, split=TOTAL, lattice=16):
    q1 = _q1(lattice)
    f = np.zeros(lattice)
    g = np.zeros(lattice)
    lib().oracle_equilibrium_q(q1, split, rho, ux, uy, T, gamma, _d(f), _d(g))
    return f, g


def collide(ft, gt, lam, tau, prandtl, gamma, split=TOTAL):
    ft, gt = _f64(ft).ravel(), _f64(gt).ravel()
    q1 = _q1(len(ft))
    fo, go = np.zeros(len(ft)), np.zeros(len(ft))
    lib().oracle_collide_q(q1, split, _d(ft), _d(gt), _d(_f64(lam, (3,))), tau, prandtl, gamma,
                           _d(fo), _d(go))
    return fo, go


def internal_source(f, lam, a, grad):
    """Source of the internal-energy g-equation over one step, per velocity:
    S_i = -f_i (C_i - u) . (a + C_i . grad u) with grad[alpha][beta] =
    d_alpha u_beta, for populations f in the frame lam."""
    f = _f64(f).ravel()
    S = np.zeros(len(f))
    lib().oracle_internal_source_q(_q1(len(f)), _d(f), _d(_f64(lam, (3,))), _d(_f64(a, (2,))),
                                   _d(_f64(grad, (2, 2))), _d(S))
    return S


def lagrange(npts, y):
    """(first node, weights) of the npts-point Lagrange stencil at coordinate y."""
    base = np.zeros(1, dtype=np.int32)
    w = np.zeros(npts)
    if lib().oracle_lagrange(npts, float(y), _i(base), _d(w)) != 0:
        raise ValueError("interp_points must be 3 or 4")
    return int(base[0]), w


@dataclass
class State:
    """Oracle state: f, g of shape (N, Q), lam of shape (N, 3); lam_prev, the
    frames of the previous time level (the internal-energy split's source
    extrapolates grad u along trajectories from them); None stands for lam
    itself (a state that has not been stepped yet)."""
    f: np.ndarray
    g: np.ndarray
    lam: np.ndarray
    lam_prev: Optional[np.ndarray] = None

    def copy(self):
        return State(self.f.copy(), self.g.copy(), self.lam.copy(),
                     None if self.lam_prev is None else self.lam_prev.copy())


def init(P: Params, rho, ux, uy, T) -> State:
    N = P.nx * P.ny
    q = P.lattice
    rho, ux, uy, T = (_f64(a, (N,)) for a in (rho, ux, uy, T))
    f, g, lam = np.zeros((N, q)), np.zeros((N, q)), np.zeros((N, 3))
    nbad = lib().oracle_init_q(_q1(q), P.split, N, _d(rho), _d(ux), _d(uy), _d(T), P.gamma,
                               _d(f), _d(g), _d(lam))
    if nbad:
        raise ValueError(f"{nbad} nodes with rho <= 0, T <= 0 or non-finite values")
    return State(f, g, lam)


@dataclass
class StepStats:
    iters: np.ndarray      # gathers per node in the last step
    status: np.ndarray     # NONCONVERGED / NONPHYSICAL bits per node, last step
    total_iters: int       # gathers summed over nodes and steps
    nonconverged: int      # node-steps that hit the iteration cap
    nonphysical: int       # node-steps flagged non-physical


def step(P: Params, s: State, nsteps: int = 1):
    """Advance nsteps; returns (new State, StepStats)."""
    N = P.nx * P.ny
    q = P.lattice
    cur = s.copy()
    nxt = State(np.zeros((N, q)), np.zeros((N, q)), np.zeros((N, 3)))
    iters = np.zeros(N, dtype=np.int32)
    status = np.zeros(N, dtype=np.int32)
    tot = nonc = nbad = 0
    for _ in range(nsteps):
        bad = lib().oracle_step(ctypes.byref(P), _d(cur.f), _d(cur.g), _d(cur.lam),
                                _prev(cur), _d(nxt.f), _d(nxt.g), _d(nxt.lam), _i(iters),
                                _i(status))
        tot += int(iters.sum())
        nonc += int(((status & NONCONVERGED) != 0).sum())
        nbad += bad
        # the time-t frames become the new state's previous level (a fresh
        # array: nxt's buffers are reused for the step after)
        nxt.lam_prev = cur.lam.copy()
        cur, nxt = nxt, cur
        if bad:
            break
    return cur, StepStats(iters.copy(), status.copy(), tot, nonc, nbad)


def _prev(s: State):
    """The previous frames as a C pointer (NULL when the state has none)."""
    if s.lam_prev is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
    s.lam_prev = np.ascontiguousarray(s.lam_prev, dtype=np.float64)
    if s.lam_prev.shape != s.lam.shape:
        raise ValueError("lam_prev must have the shape of lam")
    return _d(s.lam_prev)


def step_nodes(P: Params, s: State, nodes):
    """One step evaluated only at the listed node indices (reading the full
    state).  Returns (f (k,Q), g (k,Q), lam (k,3), iters, status)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    k = len(nodes)
    q = P.lattice
    fo, go, lo = np.zeros((k, q)), np.zeros((k, q)), np.zeros((k, 3))
    iters = np.zeros(k, dtype=np.int32)
    status = np.zeros(k, dtype=np.int32)
    lib().oracle_step_nodes(ctypes.byref(P), _d(s.f), _d(s.g), _d(s.lam), _prev(s), k,
                            nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                            _d(fo), _d(go), _d(lo), _i(iters), _i(status))
    return fo, go, lo, iters, status


def moments(P: Params, s: State):
    """dict of rho, ux, uy, T, p, each of shape (ny, nx)."""
    N = P.nx * P.ny
    out = {k: np.zeros(N) for k in ("rho", "ux", "uy", "T", "p")}
    lib().oracle_moments_q(_q1(P.lattice), P.split, N, _d(s.f), _d(s.g), _d(s.lam), P.gamma,
                           _d(out["rho"]), _d(out["ux"]), _d(out["uy"]), _d(out["T"]),
                           _d(out["p"]))
    return {k: v.reshape(P.ny, P.nx) for k, v in out.items()}
