// pond_api.hip -- host implementation of the C ABI declared in include/pond.h.
//
// A context owns (or adopts) one device allocation laid out as
//   [state buffer 0 | state buffer 1 | moment planes | counters | scratch]
// each region 256-byte aligned.  A state buffer holds 16 f planes and 16 g
// planes of P (float or double) followed by the frame planes u_x, u_y, T
// (double).  Steps ping-pong between the two buffers (Jacobi: every node of
// step t+1 reads only the state of step t).  The moment planes are rewritten
// at the start of every step and double as staging space for host-pointer
// transfers outside steps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pond_ctx.h"

using namespace pond;

namespace pond {

namespace {
thread_local std::string g_last_error;
}  // namespace

pond_status fail(pond_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

pond_status hip_fail(hipError_t e, const char *what) {
    return fail(POND_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const char *last_error() { return g_last_error.c_str(); }

Layout layout_for(long long N, size_t psize, int lattice, long long mom_nodes, int prev_planes) {
    Layout L;
    L.pop_bytes = align_up(size_t(N) * size_t(lattice) * psize);
    L.frame_bytes = align_up(size_t(N) * sizeof(double));
    L.buf_bytes = 2 * L.pop_bytes + size_t(3 + prev_planes) * L.frame_bytes;
    L.mom_bytes = align_up(size_t(mom_nodes) * moment_values(lattice, psize == 8) * psize);
    L.cnt_off = 2 * L.buf_bytes + 2 * L.mom_bytes;
    L.scratch_off = L.cnt_off + align_up(sizeof(DevCounters));
    L.total = L.scratch_off + align_up(kScratchDoubles * sizeof(double));
    return L;
}

int lds_nodes_for_blocks(int blocks_per_cu, bool dbl, int lattice) {
    // one KiB per block stays free for the kernels' static shared memory and
    // the allocation granularity
    if (blocks_per_cu < 1) blocks_per_cu = 1;
    const int bytes = 160 * 1024 / blocks_per_cu - 1024;
    return bytes / (lds_node_values(lattice, dbl) * (dbl ? 8 : 4));
}

pond_status check_ctx(const pond_ctx *c, bool need_init) {
    if (!c) return fail(POND_ERR_INVALID_ARG, "context is NULL");
    if (need_init && !c->initialized)
        return fail(POND_ERR_STATE, "context has no state (call pond_init_fields first)");
    return POND_OK;
}

pond_status read_counters(pond_ctx *c, DevCounters *out) {
    hipError_t e = hipMemcpyAsync(out, c->cnt, sizeof(DevCounters), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(counters)");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return POND_OK;
}

pond_status counters_status(pond_ctx *c, const DevCounters &h) {
    if (h.nonphysical) {
        c->failed = true;
        c->fail_status = POND_ERR_NONPHYSICAL;
        return fail(POND_ERR_NONPHYSICAL, "%llu node-steps produced rho <= 0, T <= 0 or NaN",
                    (unsigned long long)h.nonphysical);
    }
    if (h.ghost_overrun) {
        c->failed = true;
        c->fail_status = POND_ERR_UNSUPPORTED;
        return fail(POND_ERR_UNSUPPORTED,
                    "%llu node-steps had departure stencils beyond the %d ghost rows of a wall "
                    "(the flow near the wall became too hot or too fast for the wall closure)",
                    (unsigned long long)h.ghost_overrun, c->args.wall_h);
    }
    return POND_OK;
}

pond_status write_counters(pond_ctx *c, const DevCounters &in) {
    hipError_t e = hipMemcpyAsync(c->cnt, &in, sizeof(DevCounters), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(counters)");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return POND_OK;
}

// The step kernels are register-limited (two or three waves per SIMD in FP32,
// one in FP64 with the cubic stencil); the LDS of a CU is split between the
// blocks that fit by registers.  A 32 x 8 tile at T = 1, Mach 2 needs a
// 40 x 16 source region.
int default_lds_nodes(int tile, bool dbl, int np, int split, int lattice) {
    return lds_nodes_for_blocks(
        tiled_blocks_per_cu(lattice, dbl, np, split, static_cast<TileShape>(tile)), dbl, lattice);
}

// Compute units of the current device (0 if the query fails).
static int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

static long long tiles_of(const pond_params &p, int tx, int ty) {
    return (long long)((p.nx + tx - 1) / tx) * ((p.ny + ty - 1) / ty);
}

// Block shape: 64 x 1 rows for (quasi-)one-dimensional grids, else 32 x 8.
// D2Q16 takes the 512-lane 32 x 16 tile in FP64 when its tiles cover every CU
// (one block per CU holds the whole LDS, as one 32 x 8 block does, with twice
// the waves: 717 against 545 MLUPS at 512^2, Mach 2, 718 against 562 at
// 1024^2, 1157 against 864 on the 2048^2 quadrants; at 256^2 its 128 tiles
// leave half the CUs idle: 376 against 479), and in FP32 when the grid needs
// more than one round of 32 x 8 blocks but fits one round of 32 x 16 blocks (a
// kernel that runs more waves per SIMD with 512-lane blocks than with 256-lane
// ones).  The FP32 D2Q16 kernels with the shared x-pass run two waves per SIMD
// at either block size, so they keep 32 x 8 (2048^2 quadrants: 1.13 against
// 1.32 ms per step with 32 x 16; 512^2 Mach 2: 0.153 against 0.159 ms).
pond_tuning default_tuning(const pond_params &p) {
    pond_tuning t;
    t.kernel = POND_KERNEL_TILED;
    const bool dbl = p.precision == POND_PREC_FP64;
    if (p.ny < 8) {
        t.tile = POND_TILE_64x1;
    } else {
        t.tile = POND_TILE_32x8;
        if (p.lattice == POND_LATTICE_D2Q16 && p.ny >= 16) {
            const long long cus = device_cus();
            if (dbl) {
                if (cus > 0 && tiles_of(p, 32, 16) >= cus) t.tile = POND_TILE_32x16;
            } else {
                const long long cap8 =
                    cus * tiled_blocks_per_cu(p.lattice, false, p.interp_points, p.split,
                                              TileShape::T32x8);
                const long long cap16 =
                    cus * tiled_blocks_per_cu(p.lattice, false, p.interp_points, p.split,
                                              TileShape::T32x16);
                if (cus > 0 && tiles_of(p, 32, 8) > cap8 && tiles_of(p, 32, 16) <= cap16)
                    t.tile = POND_TILE_32x16;
            }
        }
    }
    // D2Q25: square tiles, whose source regions carry less halo per node (512^2
    // Mach 2: 545 against 495 MLUPS with 32 x 8)
    if (p.lattice == POND_LATTICE_D2Q25 && p.ny >= 16) t.tile = POND_TILE_16x16;
    t.lds_nodes =
        default_lds_nodes(t.tile, p.precision == POND_PREC_FP64, p.interp_points, p.split,
                          p.lattice);
    // FP64 moments take twice the LDS: measured at 512^2, Mach 2, one 32 x 8
    // block per CU holding its whole 40 x 16 source region beats two blocks
    // that fall back to HBM for part of the taps (527 vs 323 MLUPS); a 32 x 16
    // block fills one CU by its registers alone
    if (dbl && p.ny >= 8 && p.lattice == POND_LATTICE_D2Q16)
        t.lds_nodes = lds_nodes_for_blocks(1, true);
    t.batch_tile_width = 0;
    return t;
}

}  // namespace pond

pond_status pond::validate_params(const pond_params *p) {
    if (!p) return fail(POND_ERR_INVALID_ARG, "params is NULL");
    if (p->struct_size != sizeof(pond_params))
        return fail(POND_ERR_INVALID_ARG, "params.struct_size %u != %zu (ABI mismatch)",
                    p->struct_size, sizeof(pond_params));
    if (p->nx < 1 || p->ny < 1) return fail(POND_ERR_INVALID_ARG, "nx, ny must be >= 1");
    if ((long long)p->nx * p->ny > 0x7fffffffll)
        return fail(POND_ERR_INVALID_ARG, "nx * ny must stay below 2^31");
    if ((p->bc_x != POND_BC_PERIODIC && p->bc_x != POND_BC_CLAMP) ||
        (p->bc_y != POND_BC_PERIODIC && p->bc_y != POND_BC_CLAMP && p->bc_y != POND_BC_WALL))
        return fail(POND_ERR_INVALID_ARG,
                    "bc_x must be POND_BC_PERIODIC or POND_BC_CLAMP, bc_y also POND_BC_WALL");
    if (p->bc_y == POND_BC_WALL) {
        for (int k = 0; k < 2; ++k)
            if (!(p->wall_T[k] > 0.0) || !std::isfinite(p->wall_T[k]) ||
                !std::isfinite(p->wall_ux[k]))
                return fail(POND_ERR_INVALID_ARG, "wall_T must be finite and > 0, wall_ux finite");
    }
    if (p->lattice != POND_LATTICE_D2Q16 && p->lattice != POND_LATTICE_D2Q25) {
        if (p->lattice == 9)
            return fail(POND_ERR_UNSUPPORTED, "lattice 9 is not implemented (D2Q16, D2Q25)");
        return fail(POND_ERR_INVALID_ARG, "unknown lattice %d", p->lattice);
    }
    if (p->interp_points != 3 && p->interp_points != 4)
        return fail(POND_ERR_INVALID_ARG, "interp_points must be 3 or 4");
    if (p->split != POND_SPLIT_TOTAL && p->split != POND_SPLIT_INTERNAL &&
        p->split != POND_SPLIT_NONTRANS)
        return fail(POND_ERR_INVALID_ARG, "unknown split %d", p->split);
    if (p->precision != POND_PREC_FP64 && p->precision != POND_PREC_FP32)
        return fail(POND_ERR_INVALID_ARG, "unknown precision %d", p->precision);
    if (!(p->tau > 0.5) || !std::isfinite(p->tau))
        return fail(POND_ERR_INVALID_ARG, "tau must be finite and > 1/2");
    if (!(p->prandtl > 0.0) || !std::isfinite(p->prandtl))
        return fail(POND_ERR_INVALID_ARG, "prandtl must be finite and > 0");
    if (p->split == POND_SPLIT_NONTRANS && p->prandtl != 1.0)
        return fail(POND_ERR_UNSUPPORTED,
                    "the non-translational split is built with Pr = 1 (the paper's BGK) only");
    if (p->lattice == POND_LATTICE_D2Q25 && p->interp_points != 4)
        return fail(POND_ERR_UNSUPPORTED, "D2Q25 runs the cubic stencil (interp_points = 4)");
    if (!(p->gamma > 1.0) || !(p->gamma <= 2.0))
        return fail(POND_ERR_INVALID_ARG, "gamma must lie in (1, 2]");
    if (!std::isfinite(p->pc_tol)) return fail(POND_ERR_INVALID_ARG, "pc_tol must be finite");
    if (p->pc_max_iter > 10000) return fail(POND_ERR_INVALID_ARG, "pc_max_iter > 10000");
    return POND_OK;
}

void pond::fill_step_args(const pond_params &p, StepArgs &a) {
    a.nx = p.nx;
    a.ny = p.ny;
    a.bc_x = p.bc_x;
    a.bc_y = p.bc_y;
    a.N = (long long)p.nx * p.ny;
    a.interp_points = p.interp_points;
    a.pc_max_iter = p.pc_max_iter > 0 ? p.pc_max_iter : 32;
    a.pc_tol = p.pc_tol > 0 ? p.pc_tol : (p.precision == POND_PREC_FP64 ? 1e-13 : 1e-6);
    a.omega = 1.0 / p.tau;
    const double tau1 = 0.5 + (p.tau - 0.5) / p.prandtl;
    a.omega1 = 1.0 / tau1;
    a.unit_prandtl = p.prandtl == 1.0;
    a.split = p.split;
    a.lattice = p.lattice;
    a.wall_h = p.bc_y == POND_BC_WALL ? kWallGhostRows : 0;
    a.moff = (long long)a.wall_h * p.nx;
    a.mstride = moment_plane_nodes(p);
    for (int k = 0; k < 2; ++k) {
        a.wall_ux[k] = p.wall_ux[k];
        a.wall_T[k] = p.wall_T[k];
    }
    a.cv = 1.0 / (p.gamma - 1.0);
    a.uref_x = a.uref_y = 0.0;
}

namespace {

bool is_device_pointer(const void *ptr) {
    if (!ptr) return false;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace

namespace {

void fill_args(pond_ctx *c) { fill_step_args(c->p, c->args); }

bool fp64(const pond_ctx *c) { return c->p.precision == POND_PREC_FP64; }

int halo_for(int tile, int cap, bool single_row) {
    int tx, ty;
    tile_dims(static_cast<TileShape>(tile), tx, ty);
    return halo_for_dims(tx, ty, cap, single_row);
}

pond_status apply_tuning(pond_ctx *c, const pond_tuning &t) {
    if (t.kernel != POND_KERNEL_TILED && t.kernel != POND_KERNEL_GLOBAL)
        return fail(POND_ERR_INVALID_ARG, "unknown kernel %d", t.kernel);
    if (t.tile < POND_TILE_16x16 || t.tile > POND_TILE_32x16)
        return fail(POND_ERR_INVALID_ARG, "unknown tile %d", t.tile);
    if (t.tile == POND_TILE_32x16 && c->p.lattice != POND_LATTICE_D2Q16)
        return fail(POND_ERR_UNSUPPORTED, "the 32 x 16 tile is built for D2Q16 only");
    pond_tuning u = t;
    if (u.lds_nodes <= 0)
        u.lds_nodes =
            default_lds_nodes(u.tile, fp64(c), c->p.interp_points, c->p.split, c->p.lattice);
    const size_t bytes = size_t(u.lds_nodes) * lds_node_values(c->p.lattice, fp64(c)) * c->psize;
    if (bytes > 159 * 1024)  // one KiB stays for the static shared memory
        return fail(POND_ERR_INVALID_ARG, "lds_nodes %d needs %zu bytes of LDS (> 159 KiB)",
                    u.lds_nodes, bytes);
    const int h = halo_for(u.tile, u.lds_nodes, c->p.ny == 1);
    if (h < 0) return fail(POND_ERR_INVALID_ARG, "lds_nodes %d smaller than the tile", u.lds_nodes);
    if (u.batch_tile_width != 0 && u.batch_tile_width != 16 && u.batch_tile_width != 32 &&
        u.batch_tile_width != 64 && u.batch_tile_width != 128 && u.batch_tile_width != 256)
        return fail(POND_ERR_INVALID_ARG, "batch_tile_width %d not in {0, 16, 32, 64, 128, 256}",
                    u.batch_tile_width);
    c->tuning = u;
    c->tc.shape = static_cast<TileShape>(u.tile);
    c->tc.cap = u.lds_nodes;
    c->tc.halo_cap = h;
    return POND_OK;
}

pond_status sync_and_check(pond_ctx *c) {
    DevCounters h;
    pond_status s = read_counters(c, &h);
    if (s != POND_OK) return s;
    return counters_status(c, h);
}

// Copy n doubles from a caller pointer (host or device) into device memory.
pond_status stage_in(pond_ctx *c, const double *src, double *dst, long long n) {
    hipError_t e = hipMemcpyAsync(dst, src, size_t(n) * sizeof(double), hipMemcpyDefault, c->stream);
    return e == hipSuccess ? POND_OK : hip_fail(e, "hipMemcpyAsync(in)");
}

template <typename P>
hipError_t launch_init_t(pond_ctx *c, const double *r, const double *ux, const double *uy,
                         const double *T) {
    return launch_init<P>(c->args, r, ux, uy, T, c->buf[0], c->cnt, c->stream);
}

pond_status reset_counters(pond_ctx *c) {
    hipError_t e = hipMemsetAsync(c->cnt, 0, sizeof(DevCounters), c->stream);
    return e == hipSuccess ? POND_OK : hip_fail(e, "hipMemsetAsync(counters)");
}

// A frame loaded with walls whose departure stencils reach beyond the ghost rows.
pond_status ghost_band_refusal(pond_ctx *c, const DevCounters &h) {
    return fail(POND_ERR_UNSUPPORTED,
                "%llu nodes have departure stencils beyond the %d ghost rows of a wall: the "
                "wall closure needs c_out sqrt(T) + |u_y| small enough near the walls",
                (unsigned long long)h.ghost_overrun, c->args.wall_h);
}

// Operations that write the state or step it are refused while a batch owns the context.
pond_status check_unbatched(const pond_ctx *c) {
    if (c->batch) return fail(POND_ERR_STATE, "context is a member of a batch (destroy the batch first)");
    return POND_OK;
}

// Stencil reach of the frame just loaded (from cnt->partial[3]) and, unless the
// tuning was set explicitly, the autotuned configuration of the context's class.
pond_status finish_init(pond_ctx *c, const DevCounters &h) {
    const double r = std::ceil(h.partial[3]);
    c->reach = r > 1e6 ? 1000000 : int(r);
    pond_tuning t;
    if (!c->user_tuned && tuning_cache_lookup(c, &t)) return apply_tuning(c, t);
    return POND_OK;
}

pond_status set_reference_from_counters(pond_ctx *c) {
    DevCounters h;
    pond_status s = read_counters(c, &h);
    if (s != POND_OK) return s;
    if (!(h.partial[0] > 0.0)) return fail(POND_ERR_INVALID_ARG, "total mass is not positive");
    c->args.uref_x = h.partial[1] / h.partial[0];
    c->args.uref_y = h.partial[2] / h.partial[0];
    return POND_OK;
}

}  // namespace

// The entry points below take their C linkage from the declarations in pond.h.

int pond_abi_version(void) { return POND_ABI_VERSION; }

const char *pond_status_string(pond_status s) {
    switch (s) {
    case POND_OK: return "ok";
    case POND_ERR_INVALID_ARG: return "invalid argument";
    case POND_ERR_UNSUPPORTED: return "unsupported option";
    case POND_ERR_OUT_OF_MEMORY: return "out of device memory";
    case POND_ERR_DEVICE: return "device error";
    case POND_ERR_NONPHYSICAL: return "non-physical state (rho <= 0, T <= 0 or NaN)";
    case POND_ERR_STATE: return "invalid context state";
    }
    return "unknown status";
}

const char *pond_last_error(void) { return last_error(); }

pond_status pond_params_default(pond_params *p) {
    if (!p) return fail(POND_ERR_INVALID_ARG, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(pond_params);
    p->bc_x = p->bc_y = POND_BC_PERIODIC;
    p->lattice = POND_LATTICE_D2Q16;
    p->interp_points = 4;
    p->split = POND_SPLIT_TOTAL;
    p->precision = POND_PREC_FP32;
    p->pc_max_iter = 32;
    p->tau = 0.6;
    p->prandtl = 1.0;
    p->gamma = 1.4;
    p->pc_tol = 0.0;
    p->wall_T[0] = p->wall_T[1] = 1.0;
    return POND_OK;
}

size_t pond_state_bytes(const pond_params *p) {
    if (validate_params(p) != POND_OK) return 0;
    const size_t psize = p->precision == POND_PREC_FP64 ? sizeof(double) : sizeof(float);
    return layout_for((long long)p->nx * p->ny, psize, p->lattice, moment_plane_nodes(*p),
                      prev_frame_planes(p->split))
        .total;
}

pond_status pond_create(const pond_params *p, void *hip_stream, void *device_mem,
                        size_t device_mem_bytes, pond_ctx **out) {
    if (!out) return fail(POND_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    pond_status s = validate_params(p);
    if (s != POND_OK) return s;
    const size_t psize = p->precision == POND_PREC_FP64 ? sizeof(double) : sizeof(float);
    const long long N = (long long)p->nx * p->ny;
    Layout L = layout_for(N, psize, p->lattice, moment_plane_nodes(*p), prev_frame_planes(p->split));
    if (device_mem) {
        if (device_mem_bytes < L.total)
            return fail(POND_ERR_OUT_OF_MEMORY, "device_mem holds %zu bytes, %zu needed",
                        device_mem_bytes, L.total);
        if (reinterpret_cast<uintptr_t>(device_mem) % kAlign)
            return fail(POND_ERR_INVALID_ARG, "device_mem must be 256-byte aligned");
    }
    pond_ctx *c = new (std::nothrow) pond_ctx();
    if (!c) return fail(POND_ERR_OUT_OF_MEMORY, "host allocation failed");
    c->p = *p;
    c->psize = psize;
    c->L = L;
    c->own_stream = hip_stream == nullptr;
    if (c->own_stream) {
        hipError_t e = hipStreamCreate(&c->stream);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "hipStreamCreate");
        }
    } else {
        c->stream = static_cast<hipStream_t>(hip_stream);
    }
    c->own_mem = device_mem == nullptr;
    if (c->own_mem) {
        void *m = nullptr;
        hipError_t e = hipMalloc(&m, L.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return fail(POND_ERR_OUT_OF_MEMORY, "hipMalloc(%zu): %s", L.total, hipGetErrorString(e));
        }
        c->mem = static_cast<char *>(m);
    } else {
        c->mem = static_cast<char *>(device_mem);
    }
    for (int b = 0; b < 2; ++b) {
        char *base = c->mem + b * L.buf_bytes;
        c->buf[b].f = base;
        c->buf[b].g = base + L.pop_bytes;
        c->buf[b].ux = reinterpret_cast<double *>(base + 2 * L.pop_bytes);
        c->buf[b].uy = reinterpret_cast<double *>(base + 2 * L.pop_bytes + L.frame_bytes);
        c->buf[b].T = reinterpret_cast<double *>(base + 2 * L.pop_bytes + 2 * L.frame_bytes);
        const bool prev = prev_frame_planes(p->split) > 0;
        c->buf[b].uxp =
            prev ? reinterpret_cast<double *>(base + 2 * L.pop_bytes + 3 * L.frame_bytes) : nullptr;
        c->buf[b].uyp =
            prev ? reinterpret_cast<double *>(base + 2 * L.pop_bytes + 4 * L.frame_bytes) : nullptr;
    }
    c->mom[0] = c->mem + 2 * L.buf_bytes;
    c->mom[1] = c->mem + 2 * L.buf_bytes + L.mom_bytes;
    c->mom_fresh = false;
    c->cnt = reinterpret_cast<DevCounters *>(c->mem + L.cnt_off);
    c->scratch = reinterpret_cast<double *>(c->mem + L.scratch_off);
    c->cur = 0;
    c->mom_fresh = false;
    fill_args(c);
    c->initialized = false;
    c->failed = false;
    c->fail_status = POND_OK;
    c->steps = 0;
    c->profiling = false;
    c->prof_prepass_ms = c->prof_step_ms = 0.0;
    c->prof_launches = 0;
    c->batch = nullptr;
    c->reach = 0;
    c->user_tuned = false;
    s = apply_tuning(c, default_tuning(c->p));
    if (s == POND_OK) s = reset_counters(c);
    if (s != POND_OK) {
        pond_destroy(c);
        return s;
    }
    *out = c;
    return POND_OK;
}

pond_status pond_init_fields(pond_ctx *c, const double *rho, const double *ux, const double *uy,
                             const double *T) {
    pond_status s = check_ctx(c, false);
    if (s != POND_OK) return s;
    if ((s = check_unbatched(c)) != POND_OK) return s;
    if (!rho || !ux || !uy || !T) return fail(POND_ERR_INVALID_ARG, "field pointer is NULL");
    const long long N = c->args.N;
    // stage host inputs in the moment planes (>= 4 N doubles in either precision;
    // the moments are recomputed after initialisation)
    double *stg = static_cast<double *>(c->mom[0]);
    const double *in[4] = {rho, ux, uy, T};
    const double *dev[4];
    for (int k = 0; k < 4; ++k) {
        if (is_device_pointer(in[k])) {
            dev[k] = in[k];
        } else {
            s = stage_in(c, in[k], stg + k * N, N);
            if (s != POND_OK) return s;
            dev[k] = stg + k * N;
        }
    }
    c->initialized = false;
    c->failed = false;
    c->fail_status = POND_OK;
    c->cur = 0;
    c->mom_fresh = false;
    s = reset_counters(c);
    if (s != POND_OK) return s;
    hipError_t e = fp64(c) ? launch_init_t<double>(c, dev[0], dev[1], dev[2], dev[3])
                           : launch_init_t<float>(c, dev[0], dev[1], dev[2], dev[3]);
    if (e != hipSuccess) return hip_fail(e, "init kernel");
    e = launch_mean_velocity(N, dev[0], dev[1], dev[2], c->scratch, kScratchDoubles, c->cnt,
                             c->stream);
    if (e != hipSuccess) return hip_fail(e, "mean velocity");
    e = launch_frame_reach(N, dev[1], dev[2], dev[3], c->scratch, kScratchDoubles, c->cnt, c->stream);
    if (e != hipSuccess) return hip_fail(e, "frame reach");
    if (c->args.wall_h) {
        e = fp64(c) ? launch_ghost_check<double>(c->args, c->buf[0], c->cnt, c->stream)
                    : launch_ghost_check<float>(c->args, c->buf[0], c->cnt, c->stream);
        if (e != hipSuccess) return hip_fail(e, "ghost band check");
    }
    DevCounters h;
    s = read_counters(c, &h);
    if (s != POND_OK) return s;
    if (h.init_rejected)
        return fail(POND_ERR_INVALID_ARG, "%llu nodes with rho <= 0, T <= 0 or non-finite values",
                    (unsigned long long)h.init_rejected);
    if (h.ghost_overrun) return ghost_band_refusal(c, h);
    s = set_reference_from_counters(c);
    if (s == POND_OK) s = finish_init(c, h);
    if (s != POND_OK) return s;
    s = reset_counters(c);
    if (s != POND_OK) return s;
    c->steps = 0;
    c->initialized = true;
    return POND_OK;
}

namespace {

// Moments of buf[k] into mom[k] (and the wall ghost rows).
template <typename P>
hipError_t launch_prepass_t(pond_ctx *c, int k) {
    hipError_t e = launch_moments_prepass<P>(c->args, c->buf[k], static_cast<P *>(c->mom[k]),
                                             c->stream);
    if (e == hipSuccess && c->args.wall_h)
        e = launch_wall_ghosts<P>(c->args, c->buf[k], static_cast<P *>(c->mom[k]), c->stream);
    return e;
}

// Step buf[cur] -> buf[cur ^ 1]; the step kernel also writes the new state's
// moments into mom[cur ^ 1] (then the wall ghost rows are filled).
template <typename P>
hipError_t launch_step_t(pond_ctx *c) {
    const int k = c->cur;
    DevState src = c->buf[k], dst = c->buf[k ^ 1];
    const P *mom = static_cast<const P *>(c->mom[k]);
    P *mom_out = static_cast<P *>(c->mom[k ^ 1]);
    hipError_t e;
    if (c->tuning.kernel == POND_KERNEL_GLOBAL)
        e = launch_step<P>(c->args, src, mom, dst, mom_out, c->cnt, c->stream);
    else
        e = launch_step_tiled<P>(c->args, c->tc, src, mom, dst, mom_out, c->cnt, c->stream);
    if (e == hipSuccess && c->args.wall_h)
        e = launch_wall_ghosts<P>(c->args, dst, mom_out, c->stream);
    return e;
}

// One step: the moments pre-pass when mom[cur] is stale (after init, import or
// a restore), then the step kernel into the other buffer; with profiling on,
// events bracket each (three per step: pre-pass start, which stays null when
// no pre-pass runs, step start, step end).
hipError_t enqueue_step(pond_ctx *c) {
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    if (c->profiling) {
        for (int j = c->mom_fresh ? 1 : 0; j < 3 && e == hipSuccess; ++j)
            e = hipEventCreate(&ev[j]);
        for (int j = 0; j < 3; ++j) c->prof_events.push_back(ev[j]);
        if (e == hipSuccess && ev[0]) e = hipEventRecord(ev[0], c->stream);
    }
    if (e == hipSuccess && !c->mom_fresh)
        e = fp64(c) ? launch_prepass_t<double>(c, c->cur) : launch_prepass_t<float>(c, c->cur);
    if (e == hipSuccess && c->profiling) e = hipEventRecord(ev[1], c->stream);
    if (e == hipSuccess) e = fp64(c) ? launch_step_t<double>(c) : launch_step_t<float>(c);
    if (e == hipSuccess && c->profiling) e = hipEventRecord(ev[2], c->stream);
    return e;
}

}  // namespace

pond_status pond_step(pond_ctx *c, int64_t nsteps) {
    pond_status s = check_ctx(c, true);
    if (s != POND_OK) return s;
    if ((s = check_unbatched(c)) != POND_OK) return s;
    if (c->failed)
        return fail(POND_ERR_STATE, "context is in the error state (%s)",
                    pond_status_string(c->fail_status));
    if (nsteps < 0) return fail(POND_ERR_INVALID_ARG, "nsteps < 0");
    for (int64_t k = 0; k < nsteps; ++k) {
        hipError_t e = enqueue_step(c);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        c->cur ^= 1;
        c->mom_fresh = true;
        ++c->steps;
    }
    return POND_OK;
}

pond_status pond_moments(pond_ctx *c, double *rho, double *ux, double *uy, double *T, double *p) {
    pond_status s = check_ctx(c, true);
    if (s != POND_OK) return s;
    const long long N = c->args.N;
    double *outs[5] = {rho, ux, uy, T, p};
    double *dev[5];
    // staging: the other moment planes (rewritten by the next step), 5 N doubles
    double *stg = static_cast<double *>(c->mom[c->cur ^ 1]);
    for (int k = 0; k < 5; ++k)
        dev[k] = outs[k] ? (is_device_pointer(outs[k]) ? outs[k] : stg + k * N) : nullptr;
    hipError_t e = fp64(c) ? launch_macro<double>(c->args, c->buf[c->cur], dev[0], dev[1], dev[2],
                                                  dev[3], dev[4], c->stream)
                           : launch_macro<float>(c->args, c->buf[c->cur], dev[0], dev[1], dev[2],
                                                 dev[3], dev[4], c->stream);
    if (e != hipSuccess) return hip_fail(e, "moments kernel");
    for (int k = 0; k < 5; ++k)
        if (outs[k] && dev[k] != outs[k]) {
            e = hipMemcpyAsync(outs[k], dev[k], size_t(N) * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(out)");
        }
    return sync_and_check(c);
}

pond_status pond_stats(pond_ctx *c, pond_stats_t *out) {
    pond_status s = check_ctx(c, false);
    if (s != POND_OK) return s;
    if (!out) return fail(POND_ERR_INVALID_ARG, "out is NULL");
    DevCounters h;
    s = read_counters(c, &h);
    if (s != POND_OK) return s;
    out->steps = c->steps;
    out->node_updates = c->steps * c->args.N;
    out->pc_iterations = (int64_t)h.pc_iterations;
    out->nonconverged = (int64_t)h.nonconverged;
    out->nonphysical = h.nonphysical ? 1 : 0;
    out->reserved = 0;
    return counters_status(c, h);
}

pond_status pond_synchronize(pond_ctx *c) {
    pond_status s = check_ctx(c, false);
    if (s != POND_OK) return s;
    return sync_and_check(c);
}

pond_status pond_export_state(pond_ctx *c, double *f, double *g, double *frame, double *u_ref) {
    pond_status s = check_ctx(c, true);
    if (s != POND_OK) return s;
    if (!f || !g || !frame) return fail(POND_ERR_INVALID_ARG, "output pointer is NULL");
    const long long N = c->args.N;
    const long long Q = c->p.lattice;  // planes per distribution
    const bool dev = is_device_pointer(f) && is_device_pointer(g) && is_device_pointer(frame);
    hipError_t e;
    if (dev) {
        e = fp64(c) ? launch_export<double>(c->args, c->buf[c->cur], f, g, frame, c->stream)
                    : launch_export<float>(c->args, c->buf[c->cur], f, g, frame, c->stream);
        if (e != hipSuccess) return hip_fail(e, "export kernel");
    } else {
        // host destination: temporary device buffer (export is not on the hot path)
        double *tmp = nullptr;
        e = hipMalloc(&tmp, size_t(N) * (2 * Q + 3) * sizeof(double));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(POND_ERR_OUT_OF_MEMORY, "temporary export buffer");
        }
        e = fp64(c) ? launch_export<double>(c->args, c->buf[c->cur], tmp, tmp + Q * N,
                                            tmp + 2 * Q * N, c->stream)
                    : launch_export<float>(c->args, c->buf[c->cur], tmp, tmp + Q * N, tmp + 2 * Q * N,
                                           c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(f, tmp, size_t(N) * Q * sizeof(double), hipMemcpyDefault, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g, tmp + Q * N, size_t(N) * Q * sizeof(double), hipMemcpyDefault,
                               c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(frame, tmp + 2 * Q * N, size_t(N) * 3 * sizeof(double),
                               hipMemcpyDefault, c->stream);
        hipError_t e2 = hipStreamSynchronize(c->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return hip_fail(e, "export");
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamSynchronize");
    }
    if (u_ref) {
        u_ref[0] = c->args.uref_x;
        u_ref[1] = c->args.uref_y;
    }
    return sync_and_check(c);
}

pond_status pond_import_state(pond_ctx *c, const double *f, const double *g, const double *frame,
                              const double *u_ref) {
    pond_status s = check_ctx(c, false);
    if (s != POND_OK) return s;
    if ((s = check_unbatched(c)) != POND_OK) return s;
    if (!f || !g || !frame) return fail(POND_ERR_INVALID_ARG, "input pointer is NULL");
    const long long N = c->args.N;
    const long long Q = c->p.lattice;  // planes per distribution
    const bool dev = is_device_pointer(f) && is_device_pointer(g) && is_device_pointer(frame);
    double *tmp = nullptr;
    const double *df = f, *dg = g, *dfr = frame;
    hipError_t e;
    if (!dev) {
        e = hipMalloc(&tmp, size_t(N) * (2 * Q + 3) * sizeof(double));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(POND_ERR_OUT_OF_MEMORY, "temporary import buffer");
        }
        e = hipMemcpyAsync(tmp, f, size_t(N) * Q * sizeof(double), hipMemcpyDefault, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(tmp + Q * N, g, size_t(N) * Q * sizeof(double), hipMemcpyDefault,
                               c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(tmp + 2 * Q * N, frame, size_t(N) * 3 * sizeof(double),
                               hipMemcpyDefault, c->stream);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(c->stream);
            (void)hipFree(tmp);
            return hip_fail(e, "import copy");
        }
        df = tmp;
        dg = tmp + Q * N;
        dfr = tmp + 2 * Q * N;
    }
    c->initialized = false;
    c->failed = false;
    c->fail_status = POND_OK;
    c->cur = 0;
    c->mom_fresh = false;
    s = reset_counters(c);
    if (s == POND_OK) {
        e = fp64(c) ? launch_import<double>(c->args, df, dg, dfr, c->buf[0], c->stream)
                    : launch_import<float>(c->args, df, dg, dfr, c->buf[0], c->stream);
        if (e != hipSuccess) s = hip_fail(e, "import kernel");
    }
    if (s == POND_OK) {
        if (u_ref) {
            c->args.uref_x = u_ref[0];
            c->args.uref_y = u_ref[1];
        } else {
            e = fp64(c) ? launch_state_mean_velocity<double>(c->args, c->buf[0], c->scratch,
                                                             kScratchDoubles, c->cnt, c->stream)
                        : launch_state_mean_velocity<float>(c->args, c->buf[0], c->scratch,
                                                            kScratchDoubles, c->cnt, c->stream);
            s = e == hipSuccess ? set_reference_from_counters(c) : hip_fail(e, "mean velocity");
        }
    }
    if (s == POND_OK) {
        e = launch_frame_reach(N, c->buf[0].ux, c->buf[0].uy, c->buf[0].T, c->scratch,
                               kScratchDoubles, c->cnt, c->stream);
        if (e == hipSuccess && c->args.wall_h)
            e = fp64(c) ? launch_ghost_check<double>(c->args, c->buf[0], c->cnt, c->stream)
                        : launch_ghost_check<float>(c->args, c->buf[0], c->cnt, c->stream);
        DevCounters h;
        s = e == hipSuccess ? read_counters(c, &h) : hip_fail(e, "frame reach");
        if (s == POND_OK && h.ghost_overrun) s = ghost_band_refusal(c, h);
        if (s == POND_OK) s = finish_init(c, h);
    }
    if (tmp) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(tmp);
    }
    if (s != POND_OK) return s;
    s = reset_counters(c);
    if (s != POND_OK) return s;
    c->steps = 0;
    c->initialized = true;
    return POND_OK;
}

pond_status pond_export_prev_frame(pond_ctx *c, double *prev) {
    pond_status s = check_ctx(c, true);
    if (s != POND_OK) return s;
    if (!prev) return fail(POND_ERR_INVALID_ARG, "output pointer is NULL");
    const DevState &st = c->buf[c->cur];
    if (!st.uxp)
        return fail(POND_ERR_UNSUPPORTED,
                    "only the internal-energy split keeps the previous level's frames");
    const long long N = c->args.N;
    const size_t bytes = size_t(N) * sizeof(double);
    hipError_t e = hipMemcpyAsync(prev, st.uxp, bytes, hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(prev + N, st.uyp, bytes, hipMemcpyDefault, c->stream);
    if (e != hipSuccess) return hip_fail(e, "export of the previous frames");
    return sync_and_check(c);
}

pond_status pond_import_prev_frame(pond_ctx *c, const double *prev) {
    pond_status s = check_ctx(c, true);
    if (s != POND_OK) return s;
    if ((s = check_unbatched(c)) != POND_OK) return s;
    if (!prev) return fail(POND_ERR_INVALID_ARG, "input pointer is NULL");
    const DevState &st = c->buf[c->cur];
    if (!st.uxp)
        return fail(POND_ERR_UNSUPPORTED,
                    "only the internal-energy split keeps the previous level's frames");
    const long long N = c->args.N;
    const size_t bytes = size_t(N) * sizeof(double);
    hipError_t e = hipMemcpyAsync(st.uxp, prev, bytes, hipMemcpyDefault, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(st.uyp, prev + N, bytes, hipMemcpyDefault, c->stream);
    hipError_t e2 = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "import of the previous frames");
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamSynchronize");
    return POND_OK;
}

namespace {
void drop_events(pond_ctx *c) {
    for (hipEvent_t ev : c->prof_events)
        if (ev) (void)hipEventDestroy(ev);
    c->prof_events.clear();
}
}  // namespace

pond_status pond_get_tuning(pond_ctx *c, pond_tuning *out) {
    pond_status s = check_ctx(c, false);
    if (s != POND_OK) return s;
    if (!out) return fail(POND_ERR_INVALID_ARG, "out is NULL");
    *out = c->tuning;
    return POND_OK;
}

pond_status pond_set_tuning(pond_ctx *c, const pond_tuning *t) {
    pond_status s = check_ctx(c, false);
    if (s != POND_OK) return s;
    if (!t) return fail(POND_ERR_INVALID_ARG, "tuning is NULL");
    if ((s = check_unbatched(c)) != POND_OK) return s;
    s = apply_tuning(c, *t);
    if (s == POND_OK) c->user_tuned = true;
    return s;
}

pond_status pond_profile_enable(pond_ctx *c, int enable) {
    pond_status s = check_ctx(c, false);
    if (s != POND_OK) return s;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    drop_events(c);
    c->profiling = enable != 0;
    c->prof_prepass_ms = c->prof_step_ms = 0.0;
    c->prof_launches = 0;
    return POND_OK;
}

pond_status pond_profile_read(pond_ctx *c, pond_profile_t *out) {
    pond_status s = check_ctx(c, false);
    if (s != POND_OK) return s;
    if (!out) return fail(POND_ERR_INVALID_ARG, "out is NULL");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (size_t j = 0; j + 2 < c->prof_events.size(); j += 3) {
        float a = 0.f, b = 0.f;
        if (c->prof_events[j])
            e = hipEventElapsedTime(&a, c->prof_events[j], c->prof_events[j + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, c->prof_events[j + 1], c->prof_events[j + 2]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        c->prof_prepass_ms += a;
        c->prof_step_ms += b;
        ++c->prof_launches;
    }
    drop_events(c);
    out->launches = c->prof_launches;
    out->prepass_ms = c->prof_prepass_ms;
    out->step_ms = c->prof_step_ms;
    return POND_OK;
}

pond_status pond_destroy(pond_ctx *c) {
    if (!c) return POND_OK;
    if (c->batch) return fail(POND_ERR_STATE, "context is a member of a batch (destroy the batch first)");
    pond_status s = POND_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) s = hip_fail(e, "hipStreamSynchronize");
    drop_events(c);
    if (c->own_mem && c->mem) {
        e = hipFree(c->mem);
        if (e != hipSuccess && s == POND_OK) s = hip_fail(e, "hipFree");
    }
    if (c->own_stream) {
        e = hipStreamDestroy(c->stream);
        if (e != hipSuccess && s == POND_OK) s = hip_fail(e, "hipStreamDestroy");
    }
    delete c;
    return s;
}

