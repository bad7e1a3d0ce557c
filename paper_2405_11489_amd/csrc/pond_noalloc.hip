// pond_noalloc.hip -- pond_step_noalloc: the steps of pond_step on state
// buffers the caller owns, for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops that must not call hipMalloc).
//
// The only device memory the step needs beyond the caller's two state buffers
// -- the moment planes of the two states (the staged taps every step reads and
// writes, with the ghost rows of walls) and the counters -- lives in one
// fixed workspace: the file-scope device array `scratch` below.  Every GPU the
// library runs on holds its own copy of the array until the process ends.  Its
// device address is looked up once per device (hipGetSymbolAddress, on the
// entry point's first call on that device) and only that address is passed to
// kernels and copies: in host code the array's name is a host-side stand-in.
// Calls on one GPU share the array, so calls that overlap on one GPU (two
// streams, two threads) race; each call clears the counters it uses and
// rewrites the moment planes before reading them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "pond_ctx.h"

using namespace pond;

namespace {

// Workspace size: 64 MiB.  With the counters at its start, it holds the two
// sets of moment planes of up to ~419 000 nodes in FP32 on D2Q16 (80 B per
// node per set: e.g. 640 x 640), ~209 000 in FP64 (e.g. 456 x 456), ~262 000
// in FP32 on D2Q25 (128 B per node per set: 512 x 512).
constexpr size_t kWorkspaceBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kWorkspaceBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device).
pond_status workspace(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(POND_ERR_DEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(workspace)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return POND_OK;
}

// Zeroes the counters with a kernel (no memset node if the caller captures).
__global__ void clear_counters_kernel(DevCounters *c) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *c = DevCounters{};
}

bool device_pointer(const void *ptr) {
    if (!ptr) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

template <typename P>
hipError_t run_steps(const StepArgs &a, const TileConfig &tc, DevState st[2], P *mom[2],
                     DevCounters *cnt, int64_t nsteps, hipStream_t s) {
    hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(64), 0, s, cnt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_moments_prepass<P>(a, st[0], mom[0], s);
    if (e == hipSuccess && a.wall_h) e = launch_wall_ghosts<P>(a, st[0], mom[0], s);
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) {
        const int i = int(k & 1);
        e = launch_step_tiled<P>(a, tc, st[i], mom[i], st[i ^ 1], mom[i ^ 1], cnt, s);
        if (e == hipSuccess && a.wall_h) e = launch_wall_ghosts<P>(a, st[i ^ 1], mom[i ^ 1], s);
    }
    return e;
}

}  // namespace

pond_status pond_step_noalloc(const pond_params *p, const double *u_ref, void *f_a, void *g_a,
                              double *frame_a, void *f_b, void *g_b, double *frame_b,
                              int64_t nsteps, void *hip_stream, pond_stats_t *stats) {
    pond_status s = validate_params(p);
    if (s != POND_OK) return s;
    if (nsteps < 0) return fail(POND_ERR_INVALID_ARG, "nsteps < 0");
    const void *bufs[6] = {f_a, g_a, frame_a, f_b, g_b, frame_b};
    for (const void *b : bufs)
        if (!device_pointer(b))
            return fail(POND_ERR_INVALID_ARG,
                        "state buffers must be device memory of the current GPU");
    const bool dbl = p->precision == POND_PREC_FP64;
    const size_t psize = dbl ? sizeof(double) : sizeof(float);
    const size_t mom_bytes =
        align_up(size_t(moment_plane_nodes(*p)) * moment_values(p->lattice, dbl) * psize);
    const size_t need = align_up(sizeof(DevCounters)) + 2 * mom_bytes;
    if (need > kWorkspaceBytes)
        return fail(POND_ERR_OUT_OF_MEMORY,
                    "%d x %d nodes need %zu bytes of workspace; pond_step_noalloc has %zu "
                    "(use pond_create / pond_step for larger grids)",
                    p->nx, p->ny, need, kWorkspaceBytes);
    void *ws = nullptr;
    if ((s = workspace(&ws)) != POND_OK) return s;

    StepArgs a;
    fill_step_args(*p, a);
    if (u_ref) {
        if (!std::isfinite(u_ref[0]) || !std::isfinite(u_ref[1]))
            return fail(POND_ERR_INVALID_ARG, "u_ref must be finite");
        a.uref_x = u_ref[0];
        a.uref_y = u_ref[1];
    }
    const pond_tuning t = default_tuning(*p);
    TileConfig tc;
    tc.shape = static_cast<TileShape>(t.tile);
    tc.cap = t.lds_nodes;
    int tx = 0, ty = 0;
    tile_dims(tc.shape, tx, ty);
    tc.halo_cap = halo_for_dims(tx, ty, tc.cap, p->ny == 1);

    char *base = static_cast<char *>(ws);
    DevCounters *cnt = reinterpret_cast<DevCounters *>(base);
    void *mom[2] = {base + align_up(sizeof(DevCounters)),
                    base + align_up(sizeof(DevCounters)) + mom_bytes};
    const long long N = a.N;
    DevState st[2];
    // the internal split's frame buffers carry the previous level's u_x, u_y
    // after u_x, u_y, T
    const bool prev = prev_frame_planes(p->split) > 0;
    st[0] = DevState{f_a, g_a, frame_a, frame_a + N, frame_a + 2 * N,
                     prev ? frame_a + 3 * N : nullptr, prev ? frame_a + 4 * N : nullptr};
    st[1] = DevState{f_b, g_b, frame_b, frame_b + N, frame_b + 2 * N,
                     prev ? frame_b + 3 * N : nullptr, prev ? frame_b + 4 * N : nullptr};
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e;
    if (dbl) {
        double *m[2] = {static_cast<double *>(mom[0]), static_cast<double *>(mom[1])};
        e = run_steps<double>(a, tc, st, m, cnt, nsteps, stream);
    } else {
        float *m[2] = {static_cast<float *>(mom[0]), static_cast<float *>(mom[1])};
        e = run_steps<float>(a, tc, st, m, cnt, nsteps, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "pond_step_noalloc launch");
    if (!stats) return POND_OK;

    DevCounters h;
    e = hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "pond_step_noalloc counters");
    stats->steps = nsteps;
    stats->node_updates = nsteps * N;
    stats->pc_iterations = int64_t(h.pc_iterations);
    stats->nonconverged = int64_t(h.nonconverged);
    stats->nonphysical = h.nonphysical ? 1 : 0;
    stats->reserved = 0;
    if (h.nonphysical)
        return fail(POND_ERR_NONPHYSICAL, "%llu node-steps produced rho <= 0, T <= 0 or NaN",
                    (unsigned long long)h.nonphysical);
    if (h.ghost_overrun)
        return fail(POND_ERR_UNSUPPORTED,
                    "%llu node-steps had departure stencils beyond the %d ghost rows of a wall",
                    (unsigned long long)h.ghost_overrun, a.wall_h);
    return POND_OK;
}
