"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/pond.h declares, and validates parameters before touching
the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pond.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"POND_API[^;{]*?\b(pond_\w+)\s*\(", text, re.S)))


@pytest.fixture(scope="module")
def pond():
    from paper_2405_11489_amd import pond as P
    return P


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("pond_create", "pond_init_fields", "pond_step", "pond_moments", "pond_destroy"):
        assert name in syms


def test_library_exports_every_declared_symbol(pond):
    lib = ctypes.CDLL(pond.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(pond.EXPORTED) == declared_symbols()


def test_abi_version_and_status_strings(pond):
    assert pond.pond_abi_version() == pond.ABI_VERSION
    for s in range(7):
        assert pond.pond_status_string(s)
    assert "unknown" in pond.pond_status_string(99)


def test_params_struct_size_matches_header(pond):
    # uint32 + 9 int32 = 40 bytes, then 4 doubles (8-aligned) and the two wall
    # pairs = 104 bytes
    assert ctypes.sizeof(pond.pond_params) == 104
    p = pond.pond_params_default()
    assert p.struct_size == 104 and p.lattice == 16 and p.interp_points == 4
    assert list(p.wall_T) == [1.0, 1.0] and list(p.wall_ux) == [0.0, 0.0]


def test_walls_add_ghost_rows_and_validate(pond):
    p = pond.pond_params_default(nx=4, ny=32, bc_y=pond.BC_WALL)
    q = pond.pond_params_default(nx=4, ny=32)
    # the moment planes gain 8 ghost rows per wall: 20 floats per node
    assert pond.pond_state_bytes(p) - pond.pond_state_bytes(q) >= 16 * 4 * 80
    # walls run every split on both lattices
    for lattice in (pond.LATTICE_D2Q16, pond.LATTICE_D2Q25):
        r = pond.pond_params_default(nx=4, ny=32, bc_y=pond.BC_WALL, lattice=lattice)
        r.split = pond.SPLIT_INTERNAL
        assert pond.pond_state_bytes(r) > 0
    r = pond.pond_params_default(nx=4, ny=32, bc_y=pond.BC_WALL)
    r.split = pond.SPLIT_INTERNAL
    # the internal split keeps the previous level's u_x, u_y in each buffer
    assert pond.pond_state_bytes(r) - pond.pond_state_bytes(p) >= 2 * 2 * 8 * 4 * 32
    for fields, status in (({"bc_x": pond.BC_WALL}, 1),):
        r = pond.pond_params_default(nx=4, ny=32, bc_y=pond.BC_WALL)
        for k, v in fields.items():
            setattr(r, k, v)
        assert pond.pond_state_bytes(r) == 0
        with pytest.raises(pond.PondError) as ei:
            pond.pond_create(r)
        assert ei.value.status == status
    r = pond.pond_params_default(nx=4, ny=32, bc_y=pond.BC_WALL)
    r.wall_T[1] = 0.0
    assert pond.pond_state_bytes(r) == 0


def test_state_bytes(pond):
    p = pond.pond_params_default(nx=512, ny=512, precision=pond.PREC_FP32)
    b32 = pond.pond_state_bytes(p)
    # two state buffers (16 + 16 float planes, 3 double frame planes) and the
    # moment planes of each (20 floats)
    assert 464 * 512 * 512 <= b32 < 464 * 512 * 512 + 16384
    p.precision = pond.PREC_FP64
    b64 = pond.pond_state_bytes(p)
    assert 880 * 512 * 512 <= b64 < 880 * 512 * 512 + 16384
    # the internal split: two more double planes per buffer
    p.precision = pond.PREC_FP32
    p.split = pond.SPLIT_INTERNAL
    assert 496 * 512 * 512 <= pond.pond_state_bytes(p) < 496 * 512 * 512 + 16384


def test_grid_size_limit(pond):
    """Node indices are 32-bit: nx * ny up to 2^31 - 1 is a valid grid (its
    state size is reported; nothing is allocated), one node more is refused
    before any device call."""
    p = pond.pond_params_default(nx=2**31 - 1, ny=1, precision=pond.PREC_FP32)
    n = 2**31 - 1
    assert 464 * n <= pond.pond_state_bytes(p) < 464 * n + 16384
    p = pond.pond_params_default(nx=46341, ny=46341)  # 2^31 + 4633 nodes
    assert pond.pond_state_bytes(p) == 0
    with pytest.raises(pond.PondError) as ei:
        pond.pond_create(p)
    assert ei.value.status == pond.ERR_INVALID_ARG


@pytest.mark.parametrize("field,value,status", [
    ("nx", 0, 1), ("ny", -3, 1), ("tau", 0.5, 1), ("tau", float("nan"), 1),
    ("prandtl", 0.0, 1), ("gamma", 1.0, 1), ("gamma", 2.5, 1), ("bc_x", 2, 1),
    ("interp_points", 5, 1), ("precision", 7, 1), ("lattice", 9, 2), ("lattice", 7, 1),
    ("split", 9, 1), ("struct_size", 64, 1),
])
def test_invalid_params_rejected_before_device(pond, field, value, status):
    p = pond.pond_params_default(nx=8, ny=8)
    setattr(p, field, value)
    assert pond.pond_state_bytes(p) == 0
    with pytest.raises(pond.PondError) as ei:
        pond.pond_create(p)
    assert ei.value.status == status
    assert pond.pond_last_error()


@pytest.mark.parametrize("fields", [
    {"split": 2, "prandtl": 0.71},                     # non-translational: BGK (Pr = 1) only
    {"lattice": 25, "interp_points": 3},               # D2Q25: cubic stencil
])
def test_unsupported_combinations_rejected_before_device(pond, fields):
    p = pond.pond_params_default(nx=8, ny=8)
    for k, v in fields.items():
        setattr(p, k, v)
    assert pond.pond_state_bytes(p) == 0
    with pytest.raises(pond.PondError) as ei:
        pond.pond_create(p)
    assert ei.value.status == pond.ERR_UNSUPPORTED


def test_d2q25_state_size(pond):
    p = pond.pond_params_default(nx=512, ny=512, lattice=25, precision=pond.PREC_FP32)
    b32 = pond.pond_state_bytes(p)
    # two buffers of 25 + 25 float planes and 3 double frame planes, and the
    # moment planes of each (32 floats)
    assert 704 * 512 * 512 <= b32 < 704 * 512 * 512 + 16384
    p.precision = pond.PREC_FP64
    b64 = pond.pond_state_bytes(p)
    assert 1328 * 512 * 512 <= b64 < 1328 * 512 * 512 + 16384
    p.split, p.prandtl = 2, 1.0
    assert pond.pond_state_bytes(p) == b64


def test_internal_split_accepted_with_the_previous_level(pond):
    """The internal split's buffers add the previous level's u_x, u_y (two
    double planes per buffer, each aligned to 256 bytes)."""
    p = pond.pond_params_default(nx=64, ny=32)
    b0 = pond.pond_state_bytes(p)
    p.split = pond.SPLIT_INTERNAL
    assert pond.pond_state_bytes(p) - b0 == 2 * 2 * 64 * 32 * 8 > 0


def test_caller_memory_too_small_rejected(pond):
    p = pond.pond_params_default(nx=8, ny=8)
    with pytest.raises(pond.PondError) as ei:
        pond.pond_create(p, None, 256, 16)      # never dereferenced: size check comes first
    assert ei.value.status == pond.ERR_OUT_OF_MEMORY


def test_null_context_calls(pond):
    assert pond.lib.pond_destroy(None) == pond.OK
    assert pond.lib.pond_step(None, 1) == pond.ERR_INVALID_ARG
    assert pond.lib.pond_synchronize(None) == pond.ERR_INVALID_ARG


def test_batch_and_server_structs_and_host_side_validation(pond):
    """Batch, autotune and server entry points validate their arguments before
    any device call (these calls need no GPU)."""
    assert ctypes.sizeof(pond.pond_tuning) == 16
    assert ctypes.sizeof(pond.pond_batch_info_t) == 40
    assert ctypes.sizeof(pond.pond_server_config) == 56
    assert ctypes.sizeof(pond.pond_request_info) == 56
    assert ctypes.sizeof(pond.pond_server_stats_t) == 128
    for call in (lambda: pond.pond_batch_create([]),
                 lambda: pond.pond_batch_step(None, 1),
                 lambda: pond.pond_batch_synchronize(None),
                 lambda: pond.pond_batch_get_info(None),
                 lambda: pond.pond_autotune(None, 1),
                 lambda: pond.pond_server_poll(None, 1),
                 lambda: pond.pond_server_wait(None, 0)):
        with pytest.raises(pond.PondError) as ei:
            call()
        assert ei.value.status == pond.ERR_INVALID_ARG
    pond.pond_batch_destroy(None)
    pond.pond_server_destroy(None)
    c = pond.pond_server_config_default()
    assert c.struct_size == 56 and c.hbm_budget_bytes == 64 << 30 and c.chunk_steps == 64
    assert c.fill_nodes == 1 << 19
    assert c.precision == pond.PREC_FP32 and c.interp_points == 4
    assert c.split == pond.SPLIT_TOTAL
    for bad in (dict(struct_size=12), dict(hbm_budget_bytes=0), dict(chunk_steps=-1),
                dict(precision=7), dict(interp_points=5), dict(split=3)):
        cfg = pond.pond_server_config_default(**bad)
        with pytest.raises(pond.PondError) as ei:
            pond.pond_server_create(cfg)
        assert ei.value.status == pond.ERR_INVALID_ARG
