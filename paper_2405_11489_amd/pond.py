"""Thin ctypes binding of libpond.so (the C ABI of include/pond.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  Functions keep the C names; pointers may be numpy arrays (host)
or torch tensors (device memory of the context's GPU).  ``Solver`` wraps one
context with torch tensors for device memory and streams.

Importing this module loads the library; if it has not been built the import
fails loudly (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# POND_LIB_PATH selects another build of the library (e.g. one compiled with
# different tuning macros); the default is the in-tree build.
LIB_PATH = os.environ.get("POND_LIB_PATH") or os.path.join(HERE, "libpond.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NONPHYSICAL, ERR_STATE = range(7)
LATTICE_D2Q16, LATTICE_D2Q25 = 16, 25
SPLIT_TOTAL, SPLIT_INTERNAL, SPLIT_NONTRANS = 0, 1, 2
SERVE_ANY = -1  # server configuration: requests of any precision / stencil / split
PREC_FP64, PREC_FP32 = 0, 1
BC_PERIODIC, BC_CLAMP, BC_WALL = 0, 1, 2
ABI_VERSION = 3

EXPORTED = [
    "pond_abi_version", "pond_params_default", "pond_state_bytes", "pond_create",
    "pond_init_fields", "pond_step", "pond_moments", "pond_stats", "pond_synchronize",
    "pond_export_state", "pond_import_state", "pond_destroy", "pond_status_string",
    "pond_last_error", "pond_profile_enable", "pond_profile_read", "pond_get_tuning",
    "pond_set_tuning", "pond_batch_create", "pond_batch_step", "pond_batch_synchronize",
    "pond_batch_get_info", "pond_batch_member_tile_width", "pond_batch_destroy",
    "pond_autotune", "pond_tuning_cache_clear", "pond_server_config_default",
    "pond_server_create", "pond_server_submit", "pond_server_poll", "pond_server_wait",
    "pond_server_result", "pond_server_release", "pond_server_get_stats", "pond_server_destroy",
    "pond_step_noalloc", "pond_export_prev_frame", "pond_import_prev_frame",
]
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = range(4)
REQ_KEEP_MOMENTS, REQ_KEEP_STATE = 1, 2
KERNEL_TILED, KERNEL_GLOBAL = 0, 1
TILE_16x16, TILE_32x8, TILE_16x8, TILE_8x8, TILE_256x1, TILE_64x1, TILE_32x16 = range(7)


class pond_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("lattice", ctypes.c_int32),
        ("interp_points", ctypes.c_int32), ("split", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("pc_max_iter", ctypes.c_int32),
        ("tau", ctypes.c_double), ("prandtl", ctypes.c_double), ("gamma", ctypes.c_double),
        ("pc_tol", ctypes.c_double), ("wall_ux", ctypes.c_double * 2),
        ("wall_T", ctypes.c_double * 2),
    ]


class pond_stats_t(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("node_updates", ctypes.c_int64),
        ("pc_iterations", ctypes.c_int64), ("nonconverged", ctypes.c_int64),
        ("nonphysical", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class pond_profile_t(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("prepass_ms", ctypes.c_double),
                ("step_ms", ctypes.c_double)]


class pond_tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("lds_nodes", ctypes.c_int32), ("batch_tile_width", ctypes.c_int32)]


class pond_batch_info_t(ctypes.Structure):
    _fields_ = [("members", ctypes.c_int32), ("tiles", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("lds_nodes", ctypes.c_int32),
                ("nodes", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("graph_steps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class pond_server_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("interp_points", ctypes.c_int32), ("max_members", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("chunk_steps", ctypes.c_int64),
                ("fill_nodes", ctypes.c_int64), ("autotune_steps", ctypes.c_int64),
                ("split", ctypes.c_int32)]


class pond_request_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("error", ctypes.c_int32),
                ("steps_done", ctypes.c_int64), ("steps_total", ctypes.c_int64),
                ("state_bytes", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class pond_server_stats_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "submitted", "admitted", "completed", "failed", "admission_waits", "batch_builds",
        "batched_steps", "node_updates", "queued", "running", "used_bytes", "rounds",
        "ns_admit", "ns_build", "ns_step", "ns_retire")]


class PondError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first "
                      "(python -c 'import __graft_entry__ as g; g.build()')")

# torch ships its own HIP runtime under the same SONAME; importing it first makes
# libpond.so bind to that one, so the process holds a single HIP runtime.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_L = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_L.pond_abi_version.restype = ctypes.c_int
_L.pond_params_default.argtypes = [ctypes.POINTER(pond_params)]
_L.pond_state_bytes.argtypes = [ctypes.POINTER(pond_params)]
_L.pond_state_bytes.restype = ctypes.c_size_t
_L.pond_create.argtypes = [ctypes.POINTER(pond_params), _vp, _vp, ctypes.c_size_t,
                           ctypes.POINTER(_vp)]
_L.pond_init_fields.argtypes = [_vp, _vp, _vp, _vp, _vp]
_L.pond_step.argtypes = [_vp, ctypes.c_int64]
_L.pond_moments.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_L.pond_stats.argtypes = [_vp, ctypes.POINTER(pond_stats_t)]
_L.pond_synchronize.argtypes = [_vp]
_L.pond_export_state.argtypes = [_vp, _vp, _vp, _vp, _vp]
_L.pond_import_state.argtypes = [_vp, _vp, _vp, _vp, _vp]
_L.pond_export_prev_frame.argtypes = [_vp, _vp]
_L.pond_import_prev_frame.argtypes = [_vp, _vp]
_L.pond_destroy.argtypes = [_vp]
_L.pond_step_noalloc.argtypes = [ctypes.POINTER(pond_params), _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp, ctypes.c_int64, _vp, ctypes.POINTER(pond_stats_t)]
_L.pond_profile_enable.argtypes = [_vp, ctypes.c_int]
_L.pond_get_tuning.argtypes = [_vp, ctypes.POINTER(pond_tuning)]
_L.pond_set_tuning.argtypes = [_vp, ctypes.POINTER(pond_tuning)]
_L.pond_profile_read.argtypes = [_vp, ctypes.POINTER(pond_profile_t)]
_L.pond_batch_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _vp, ctypes.POINTER(_vp)]
_L.pond_batch_step.argtypes = [_vp, ctypes.c_int64]
_L.pond_batch_synchronize.argtypes = [_vp]
_L.pond_batch_get_info.argtypes = [_vp, ctypes.POINTER(pond_batch_info_t)]
_L.pond_batch_member_tile_width.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
_L.pond_batch_destroy.argtypes = [_vp]
_L.pond_autotune.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(pond_tuning)]
_L.pond_tuning_cache_clear.argtypes = []
_L.pond_server_config_default.argtypes = [ctypes.POINTER(pond_server_config)]
_L.pond_server_create.argtypes = [ctypes.POINTER(pond_server_config), ctypes.POINTER(_vp)]
_L.pond_server_submit.argtypes = [_vp, ctypes.POINTER(pond_params), _vp, _vp, _vp, _vp,
                                  ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
_L.pond_server_poll.argtypes = [_vp, ctypes.c_int64, ctypes.POINTER(pond_request_info)]
_L.pond_server_wait.argtypes = [_vp, ctypes.c_int64]
_L.pond_server_result.argtypes = [_vp, ctypes.c_int64, _vp, _vp]
_L.pond_server_release.argtypes = [_vp, ctypes.c_int64]
_L.pond_server_get_stats.argtypes = [_vp, ctypes.POINTER(pond_server_stats_t)]
_L.pond_server_destroy.argtypes = [_vp]
_L.pond_status_string.argtypes = [ctypes.c_int]
_L.pond_status_string.restype = ctypes.c_char_p
_L.pond_last_error.restype = ctypes.c_char_p
for _name in EXPORTED:
    if _name not in ("pond_abi_version", "pond_state_bytes", "pond_status_string",
                     "pond_last_error"):
        getattr(_L, _name).restype = ctypes.c_int
if _L.pond_abi_version() != ABI_VERSION:
    raise ImportError("libpond.so ABI version mismatch; rebuild")

lib = _L


def _check(status):
    if status != OK:
        raise PondError(status, _L.pond_last_error().decode() or
                        _L.pond_status_string(status).decode())


def _ptr(a):
    """Data pointer of a numpy array or torch tensor (contiguous float64), or None."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise TypeError("numpy arrays must be C-contiguous float64")
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        import torch
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise TypeError("tensors must be contiguous float64")
        return a.data_ptr()
    raise TypeError(f"unsupported array type {type(a)}")


# ------------------------------------------------------------- C names ----
def pond_abi_version() -> int:
    return _L.pond_abi_version()


def pond_params_default(**overrides) -> pond_params:
    p = pond_params()
    _check(_L.pond_params_default(ctypes.byref(p)))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def pond_state_bytes(p: pond_params) -> int:
    return int(_L.pond_state_bytes(ctypes.byref(p)))


def pond_create(p: pond_params, stream=None, device_mem=None, device_mem_bytes=0):
    ctx = _vp()
    _check(_L.pond_create(ctypes.byref(p), stream, device_mem, device_mem_bytes,
                          ctypes.byref(ctx)))
    return ctx


def pond_init_fields(ctx, rho, ux, uy, T):
    _check(_L.pond_init_fields(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T)))


def pond_step(ctx, nsteps: int):
    _check(_L.pond_step(ctx, int(nsteps)))


def pond_moments(ctx, rho=None, ux=None, uy=None, T=None, p=None):
    _check(_L.pond_moments(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(p)))


def pond_stats(ctx) -> pond_stats_t:
    s = pond_stats_t()
    _check(_L.pond_stats(ctx, ctypes.byref(s)))
    return s


def pond_synchronize(ctx):
    _check(_L.pond_synchronize(ctx))


def pond_export_state(ctx, f, g, frame, u_ref=None):
    _check(_L.pond_export_state(ctx, _ptr(f), _ptr(g), _ptr(frame), _ptr(u_ref)))


def pond_import_state(ctx, f, g, frame, u_ref=None):
    _check(_L.pond_import_state(ctx, _ptr(f), _ptr(g), _ptr(frame), _ptr(u_ref)))


def pond_export_prev_frame(ctx, prev):
    _check(_L.pond_export_prev_frame(ctx, _ptr(prev)))


def pond_import_prev_frame(ctx, prev):
    _check(_L.pond_import_prev_frame(ctx, _ptr(prev)))


def pond_destroy(ctx):
    _check(_L.pond_destroy(ctx))


def _dptr(a):
    """Data pointer of a contiguous torch tensor (any dtype), or an int address."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise TypeError("tensors must be contiguous")
        return a.data_ptr()
    raise TypeError(f"unsupported buffer type {type(a)}")


def pond_step_noalloc(p: pond_params, u_ref, f_a, g_a, frame_a, f_b, g_b, frame_b, nsteps: int,
                      stream=None, want_stats: bool = False):
    """pond_step_noalloc: buffers are device tensors (f, g in the precision's
    dtype, frames float64); u_ref a host sequence of 2 floats or None.  Returns
    the pond_stats_t of the steps when want_stats (the call then synchronises)."""
    ur = None if u_ref is None else (ctypes.c_double * 2)(float(u_ref[0]), float(u_ref[1]))
    st = pond_stats_t() if want_stats else None
    _check(_L.pond_step_noalloc(ctypes.byref(p), ur, _dptr(f_a), _dptr(g_a), _dptr(frame_a),
                                _dptr(f_b), _dptr(g_b), _dptr(frame_b), int(nsteps), stream,
                                ctypes.byref(st) if st is not None else None))
    return st


def pond_get_tuning(ctx) -> pond_tuning:
    t = pond_tuning()
    _check(_L.pond_get_tuning(ctx, ctypes.byref(t)))
    return t


def pond_set_tuning(ctx, kernel=None, tile=None, lds_nodes=None, batch_tile_width=None):
    t = pond_get_tuning(ctx)
    if kernel is not None:
        t.kernel = kernel
    if tile is not None:
        t.tile = tile
    if lds_nodes is not None:
        t.lds_nodes = lds_nodes
    if batch_tile_width is not None:
        t.batch_tile_width = batch_tile_width
    _check(_L.pond_set_tuning(ctx, ctypes.byref(t)))


def pond_batch_create(ctxs, stream=None):
    arr = (_vp * len(ctxs))(*[c.value if isinstance(c, _vp) else c for c in ctxs])
    b = _vp()
    _check(_L.pond_batch_create(arr, len(ctxs), stream, ctypes.byref(b)))
    return b


def pond_batch_step(b, nsteps: int):
    _check(_L.pond_batch_step(b, int(nsteps)))


def pond_batch_synchronize(b):
    _check(_L.pond_batch_synchronize(b))


def pond_batch_get_info(b) -> pond_batch_info_t:
    out = pond_batch_info_t()
    _check(_L.pond_batch_get_info(b, ctypes.byref(out)))
    return out


def pond_batch_member_tile_width(b, i: int) -> int:
    w = ctypes.c_int()
    _check(_L.pond_batch_member_tile_width(b, i, ctypes.byref(w)))
    return w.value


def pond_batch_destroy(b):
    _check(_L.pond_batch_destroy(b))


def pond_autotune(ctx, steps: int = 5) -> pond_tuning:
    t = pond_tuning()
    _check(_L.pond_autotune(ctx, int(steps), ctypes.byref(t)))
    return t


def pond_tuning_cache_clear():
    _check(_L.pond_tuning_cache_clear())


def pond_server_config_default(**overrides) -> pond_server_config:
    c = pond_server_config()
    _check(_L.pond_server_config_default(ctypes.byref(c)))
    for k, v in overrides.items():
        if not hasattr(c, k):
            raise AttributeError(k)
        setattr(c, k, v)
    return c


def pond_server_create(cfg: pond_server_config):
    s = _vp()
    _check(_L.pond_server_create(ctypes.byref(cfg), ctypes.byref(s)))
    return s


def pond_server_submit(srv, p: pond_params, rho, ux, uy, T, nsteps: int, flags: int = 0) -> int:
    """Fields: host float64 arrays of nx * ny values (copied before return)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (rho, ux, uy, T)]
    rid = ctypes.c_int64()
    _check(_L.pond_server_submit(srv, ctypes.byref(p), *[_ptr(a) for a in arrs], int(nsteps),
                                 int(flags), ctypes.byref(rid)))
    return rid.value


def pond_server_poll(srv, rid: int) -> pond_request_info:
    out = pond_request_info()
    _check(_L.pond_server_poll(srv, int(rid), ctypes.byref(out)))
    return out


def pond_server_wait(srv, rid: int = 0):
    _check(_L.pond_server_wait(srv, int(rid)))


def pond_server_result(srv, rid: int, moments=None, state=None):
    _check(_L.pond_server_result(srv, int(rid), _ptr(moments), _ptr(state)))


def pond_server_release(srv, rid: int):
    _check(_L.pond_server_release(srv, int(rid)))


def pond_server_get_stats(srv) -> pond_server_stats_t:
    out = pond_server_stats_t()
    _check(_L.pond_server_get_stats(srv, ctypes.byref(out)))
    return out


def pond_server_destroy(srv):
    _check(_L.pond_server_destroy(srv))


def pond_profile_enable(ctx, enable: bool):
    _check(_L.pond_profile_enable(ctx, 1 if enable else 0))


def pond_profile_read(ctx) -> pond_profile_t:
    out = pond_profile_t()
    _check(_L.pond_profile_read(ctx, ctypes.byref(out)))
    return out


def pond_status_string(status: int) -> str:
    return _L.pond_status_string(status).decode()


def pond_last_error() -> str:
    return _L.pond_last_error().decode()


# ----------------------------------------------------------- convenience ----
class Solver:
    """One context; host numpy in, host numpy out (device tensors also accepted)."""

    def __init__(self, nx, ny, *, tau, gamma=1.4, prandtl=1.0, bc_x=BC_PERIODIC,
                 bc_y=BC_PERIODIC, precision=PREC_FP32, interp_points=4, pc_tol=0.0,
                 pc_max_iter=32, split=SPLIT_TOTAL, lattice=LATTICE_D2Q16, wall_ux=(0.0, 0.0),
                 wall_T=(1.0, 1.0), stream=None, tuning=None):
        self.params = pond_params_default(nx=nx, ny=ny, tau=tau, gamma=gamma, prandtl=prandtl,
                                          bc_x=bc_x, bc_y=bc_y, precision=precision,
                                          interp_points=interp_points, pc_tol=pc_tol,
                                          pc_max_iter=pc_max_iter, split=split, lattice=lattice,
                                          wall_ux=(ctypes.c_double * 2)(*wall_ux),
                                          wall_T=(ctypes.c_double * 2)(*wall_T))
        self.nx, self.ny = nx, ny
        self.q = lattice
        self.ctx = pond_create(self.params, stream)
        if tuning:
            pond_set_tuning(self.ctx, **tuning)

    @classmethod
    def from_workload(cls, w, precision=PREC_FP32, **kw):
        if w.bc_y == BC_WALL:
            kw.setdefault("wall_ux", w.wall_ux)
            kw.setdefault("wall_T", w.wall_T)
        s = cls(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl, bc_x=w.bc_x,
                bc_y=w.bc_y, precision=precision, **kw)
        s.init_fields(w.rho, w.ux, w.uy, w.T)
        return s

    def init_fields(self, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).ravel() if isinstance(a, np.ndarray)
                else a for a in (rho, ux, uy, T)]
        pond_init_fields(self.ctx, *arrs)

    def step(self, n=1):
        pond_step(self.ctx, n)

    def moments(self):
        N = self.nx * self.ny
        out = {k: np.zeros(N) for k in ("rho", "ux", "uy", "T", "p")}
        pond_moments(self.ctx, out["rho"], out["ux"], out["uy"], out["T"], out["p"])
        return {k: v.reshape(self.ny, self.nx) for k, v in out.items()}

    def stats(self):
        return pond_stats(self.ctx)

    def export_state(self):
        """(f, g, frame, u_ref) with f, g of shape (Q, N) and frame (3, N)."""
        N = self.nx * self.ny
        f, g, fr, ur = np.zeros((self.q, N)), np.zeros((self.q, N)), np.zeros((3, N)), np.zeros(2)
        pond_export_state(self.ctx, f, g, fr, ur)
        return f, g, fr, ur

    def import_state(self, f, g, frame, u_ref=None):
        pond_import_state(self.ctx, np.ascontiguousarray(f, dtype=np.float64),
                          np.ascontiguousarray(g, dtype=np.float64),
                          np.ascontiguousarray(frame, dtype=np.float64),
                          None if u_ref is None else np.ascontiguousarray(u_ref, dtype=np.float64))

    def export_prev_frame(self):
        """Internal-energy split: the previous time level's frame velocities,
        shape (2, N) (u_x, u_y)."""
        prev = np.zeros((2, self.nx * self.ny))
        pond_export_prev_frame(self.ctx, prev)
        return prev

    def import_prev_frame(self, prev):
        pond_import_prev_frame(self.ctx, np.ascontiguousarray(prev, dtype=np.float64))

    def synchronize(self):
        pond_synchronize(self.ctx)

    def close(self):
        if self.ctx:
            pond_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
