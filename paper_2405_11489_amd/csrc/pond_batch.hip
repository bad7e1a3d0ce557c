// pond_batch.hip -- many PonD instances advanced together, and the tile-shape
// autotuner.
//
// A batch steps its member contexts with one launch per step for all of them
// at once, replayed from captured HIP graphs: one step launch over the flat
// list of every member's tiles, one block per tile; the hardware dispatcher
// balances the tiles over the CUs, and the block -> tile map gives each XCD a
// contiguous range of the list.  The step writes the moments the next step
// reads; a flat moment pre-pass over every member's nodes (each 256-node block
// belongs to one member) runs only where a member's moments are stale (after
// its initialisation or an import).
// Which of a member's two state buffers is current alternates every step;
// the launches take that parity as an argument, so the batch keeps one graph
// per starting parity and needs no device-side step counter.
//
// (A persistent variant -- a fixed grid pulling tiles from per-XCD atomic
// queues -- ran 2.4x slower on one 512 x 512 instance: same-address
// device-scope atomics serialise, and the cost grew with the grid.  A fixed
// grid with static shares of the tile list and no atomics, the build option
// POND_BATCH_PERSISTENT, ran a 256-instance mixed batch 4.6 % slower than the
// flat launch: static shares do not follow the members' uneven tile costs.)
//
// Every node goes through the same per-node code as the single-instance
// kernels (tile_step / node_step with the member's own arguments), so a
// member's results do not depend on the batch it runs in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "pond_ctx.h"
#include "pond_tile.h"

namespace pond {
namespace {

constexpr int kBatchThreads = 256;

struct BatchMember {
    StepArgs a;
    DevState buf[2];
    void *mom[2];  // moments of buf[0] / buf[1]
    DevCounters *cnt;
    int parity0;   // current buffer of the member when the batch was built
    int lg;        // tile width 2^lg, height 256 >> lg
    int tiles_x;
    int tile_off;  // first tile of the member in the flat tile list
    int blk_off;   // first pre-pass block of the member
};

// Largest i in [0, n) with off[i] <= v (off strictly increasing, off[0] = 0).
__device__ __forceinline__ int find_member(const int *__restrict__ off, int n, int v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// flip: parity of the batched steps taken since the batch was built.
template <typename P, class L>
__global__ __launch_bounds__(kBatchThreads) void batch_moments_kernel(
    const BatchMember *__restrict__ mem, const int *__restrict__ blk_off, int nmem, int flip) {
    const int i = __builtin_amdgcn_readfirstlane(find_member(blk_off, nmem, int(blockIdx.x)));
    const StepArgs a = mem[i].a;
    const long long n = (long long)(int(blockIdx.x) - mem[i].blk_off) * kBatchThreads + threadIdx.x;
    if (n >= a.N) return;
    const int par = mem[i].parity0 ^ flip;
    node_moments<P, L>(a, mem[i].buf[par], static_cast<P *>(mem[i].mom[par]), n);
}

// Tile t of the flat list: its member's step on that tile.
template <typename P, int NP, int S, class L>
__device__ __forceinline__ void batch_tile(const BatchMember *__restrict__ mem,
                                           const int *__restrict__ tile_off, int nmem, int cap,
                                           int flip, int t, unsigned char *smem_raw, int *red) {
    const int i = __builtin_amdgcn_readfirstlane(find_member(tile_off, nmem, t));
    const StepArgs a = mem[i].a;
    const int lg = mem[i].lg, tiles_x = mem[i].tiles_x;
    const int lt = t - mem[i].tile_off;
    const int par = mem[i].parity0 ^ flip;
    tile_step<P, NP, S, L>(a, mem[i].buf[par], static_cast<const P *>(mem[i].mom[par]),
                               mem[i].buf[par ^ 1], static_cast<P *>(mem[i].mom[par ^ 1]),
                     mem[i].cnt, reinterpret_cast<P *>(smem_raw), cap, (lt % tiles_x) << lg,
                     (lt / tiles_x) * (kBatchThreads >> lg), Shape256{lg}, red);
}

// POND_BATCH_PERSISTENT=1: a fixed grid of the blocks the chip holds at once,
// block b (on XCD b % 8) stepping, in turn, a static share of its XCD's
// contiguous range of the tile list (no queue, no atomics).  Off by default
// (slower; see the note at the top of this file).
#ifndef POND_BATCH_PERSISTENT
#define POND_BATCH_PERSISTENT 0
#endif

template <typename P, int NP, int S, class L>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(
    step_min_waves<P, S, kBatchThreads, L>()))) void batch_step_kernel(
    const BatchMember *__restrict__ mem, const int *__restrict__ tile_off, int nmem, int cap,
    int flip, int ntiles) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int red[4 * red_slots<Shape256::kThreads>()];
#if POND_BATCH_PERSISTENT
    // the grid has at least 8 blocks, so every XCD has one
    const int b = int(blockIdx.x), nb = int(gridDim.x), x = b % 8;
    const int on_xcd = (nb - x + 7) / 8;
    const int lo = int((long long)x * ntiles / 8), hi = int((long long)(x + 1) * ntiles / 8);
    for (int t = lo + b / 8; t < hi; t += on_xcd) {
        batch_tile<P, NP, S, L>(mem, tile_off, nmem, cap, flip, t, smem_raw, red);
        __syncthreads();  // the next tile's staging overwrites the LDS
    }
#else
    (void)ntiles;
    batch_tile<P, NP, S, L>(mem, tile_off, nmem, cap, flip,
                            xcd_tile(int(blockIdx.x), int(gridDim.x)), smem_raw, red);
#endif
}

template <typename P, int NP, int S, class L>
const void *step_kernel_ptr() {
    return reinterpret_cast<const void *>(batch_step_kernel<P, NP, S, L>);
}

template <class L>
const void *batch_step_fn_l(bool dbl, int np, int split) {
    return with_variant(np, split, [&](auto n, auto sp) {
        return dbl ? step_kernel_ptr<double, n(), sp(), L>()
                   : step_kernel_ptr<float, n(), sp(), L>();
    });
}

const void *batch_step_fn(bool dbl, int np, int split, int lattice) {
    return lattice == POND_LATTICE_D2Q25 ? batch_step_fn_l<D2Q25>(dbl, np, split)
                                         : batch_step_fn_l<D2Q16>(dbl, np, split);
}

// ----------------------------------------------------- tuning cache ----
// Class of an instance: lattice, energy split, precision, stencil, boundary
// conditions, the rounded log2 of each axis (a single-row grid is its own
// class) and the stencil reach of its initial frame (the best tile shape
// depends on the halo).
using TuneKey = std::tuple<int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, pond_tuning> g_tune;

int log2_class(int n) { return n <= 1 ? -1 : int(std::lround(std::log2(double(n)))); }

TuneKey tune_key(const pond_ctx *c) {
    const pond_params &p = c->p;
    // lattices tune apart: a D2Q16 class may pick a tile D2Q25 does not run
    return TuneKey(p.lattice * 1024 + p.split * 64 + p.precision * 16 + p.interp_points,
                   p.bc_x * 2 + p.bc_y, log2_class(p.nx), log2_class(p.ny),
                   std::min(c->reach, 12));
}

int default_batch_width(const pond_params &p) {
    if (p.ny < 8) return 256;
    return p.precision == POND_PREC_FP64 ? 16 : 32;
}

int lg2(int w) {
    int l = 0;
    while ((1 << l) < w) ++l;
    return l;
}

}  // namespace

bool tuning_cache_lookup(const pond_ctx *c, pond_tuning *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(c));
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

}  // namespace pond

using namespace pond;

struct pond_batch {
    std::vector<pond_ctx *> members;
    std::vector<int> parity0;  // each member's current buffer when the batch was built
    std::vector<int> widths;
    bool dbl;
    int np, split;
    hipStream_t stream;
    bool own_stream;
    void *dev;  // [members | tile offsets | block offsets]
    BatchMember *d_mem;
    int *d_tile_off, *d_blk_off;
    int cap, tiles, blocks;
    int grid;     // blocks of the step launch
    int lattice;  // of every member
    long long nodes;
    long long steps;
    // [parity][0]: one step, [parity][1]: kGraphSteps steps, starting at that parity
    hipGraph_t graph[2][2];
    hipGraphExec_t exec[2][2];
    hipEvent_t done_ev;
    std::vector<hipStream_t> other_streams;  // member streams other than the batch's
    std::vector<hipEvent_t> other_ev;
};

namespace {

constexpr int kGraphSteps = 8;
static_assert(kGraphSteps % 2 == 0, "the long graph must leave the buffer parity unchanged");

// Moments of every member's current buffer (flip: batched steps taken so far).
// Ghost rows of the moment planes of every walled member, for the state in
// buffer parity0 ^ flip ^ next (next = 1: the state a batched step produces).
hipError_t enqueue_batch_wall_ghosts(pond_batch *b, int flip, int next) {
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < b->members.size() && e == hipSuccess; ++i) {
        const pond_ctx *c = b->members[i];
        if (c->args.bc_y != POND_BC_WALL) continue;
        const int par = b->parity0[i] ^ flip ^ next;
        e = b->dbl ? launch_wall_ghosts<double>(c->args, c->buf[par],
                                                static_cast<double *>(c->mom[par]), b->stream)
                   : launch_wall_ghosts<float>(c->args, c->buf[par],
                                               static_cast<float *>(c->mom[par]), b->stream);
    }
    return e;
}

template <class L>
void launch_batch_moments(pond_batch *b, int flip) {
    const int n = int(b->members.size());
    if (b->dbl)
        hipLaunchKernelGGL((batch_moments_kernel<double, L>), dim3(b->blocks), dim3(kBatchThreads),
                           0, b->stream, b->d_mem, b->d_blk_off, n, flip);
    else
        hipLaunchKernelGGL((batch_moments_kernel<float, L>), dim3(b->blocks), dim3(kBatchThreads),
                           0, b->stream, b->d_mem, b->d_blk_off, n, flip);
}

hipError_t enqueue_batch_moments(pond_batch *b, int flip) {
    if (b->lattice == POND_LATTICE_D2Q25)
        launch_batch_moments<D2Q25>(b, flip);
    else
        launch_batch_moments<D2Q16>(b, flip);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? enqueue_batch_wall_ghosts(b, flip, 0) : e;
}

// One batched step: every member's step kernel tiles, which also write the
// members' new moments (the moments of the current buffers must be fresh).
template <class L>
void launch_batch_step(pond_batch *b, int flip) {
    const int n = int(b->members.size());
    const size_t lds = size_t(b->cap) * lds_node_values(L::Q, b->dbl) *
                       (b->dbl ? sizeof(double) : sizeof(float));
    with_variant(b->np, b->split, [&](auto np, auto sp) {
        if (b->dbl)
            hipLaunchKernelGGL((batch_step_kernel<double, np(), sp(), L>), dim3(b->grid),
                               dim3(kBatchThreads), lds, b->stream, b->d_mem, b->d_tile_off, n,
                               b->cap, flip, b->tiles);
        else
            hipLaunchKernelGGL((batch_step_kernel<float, np(), sp(), L>), dim3(b->grid),
                               dim3(kBatchThreads), lds, b->stream, b->d_mem, b->d_tile_off, n,
                               b->cap, flip, b->tiles);
        return 0;
    });
}

hipError_t enqueue_batch_step(pond_batch *b, int flip) {
    if (b->lattice == POND_LATTICE_D2Q25)
        launch_batch_step<D2Q25>(b, flip);
    else
        launch_batch_step<D2Q16>(b, flip);
    hipError_t e = hipGetLastError();
    // walled members: the ghost rows of the moments the step wrote
    return e == hipSuccess ? enqueue_batch_wall_ghosts(b, flip, 1) : e;
}

hipError_t capture(pond_batch *b, int steps, int flip, hipGraph_t *g, hipGraphExec_t *x) {
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int k = 0; k < steps && le == hipSuccess; ++k) le = enqueue_batch_step(b, flip ^ (k & 1));
    e = hipStreamEndCapture(b->stream, g);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    return hipGraphInstantiate(x, *g, nullptr, nullptr, 0);
}

void release(pond_batch *b) {
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (int f = 0; f < 2; ++f)
        for (int k = 0; k < 2; ++k) {
            if (b->exec[f][k]) (void)hipGraphExecDestroy(b->exec[f][k]);
            if (b->graph[f][k]) (void)hipGraphDestroy(b->graph[f][k]);
        }
    if (b->done_ev) (void)hipEventDestroy(b->done_ev);
    for (hipEvent_t ev : b->other_ev) (void)hipEventDestroy(ev);
    if (b->dev) (void)hipFree(b->dev);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    for (pond_ctx *c : b->members)
        if (c && c->batch == b) c->batch = nullptr;
    delete b;
}

// Members' widths: explicit per-context width, else the tuning cache, else
// the default for the instance's shape.
int member_width(const pond_ctx *c) {
    if (c->tuning.batch_tile_width > 0) return c->tuning.batch_tile_width;
    pond_tuning t;
    if (tuning_cache_lookup(c, &t) && t.batch_tile_width > 0) return t.batch_tile_width;
    return default_batch_width(c->p);
}

}  // namespace

pond_status pond_batch_create(pond_ctx *const *ctxs, int n, void *hip_stream, pond_batch **out) {
    if (!out) return fail(POND_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ctxs || n < 1) return fail(POND_ERR_INVALID_ARG, "a batch needs at least one context");
    for (int i = 0; i < n; ++i) {
        const pond_ctx *c = ctxs[i];
        if (!c) return fail(POND_ERR_INVALID_ARG, "context %d is NULL", i);
        if (!c->initialized) return fail(POND_ERR_STATE, "context %d has no state", i);
        if (c->failed) return fail(POND_ERR_STATE, "context %d is in the error state", i);
        if (c->batch) return fail(POND_ERR_STATE, "context %d already belongs to a batch", i);
        if (c->p.precision != ctxs[0]->p.precision ||
            c->p.interp_points != ctxs[0]->p.interp_points || c->p.split != ctxs[0]->p.split ||
            c->p.lattice != ctxs[0]->p.lattice)
            return fail(POND_ERR_INVALID_ARG,
                        "context %d: members must share precision, interp_points, split and "
                        "lattice", i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return fail(POND_ERR_INVALID_ARG, "context %d appears twice", i);
    }
    pond_batch *b = new (std::nothrow) pond_batch();
    if (!b) return fail(POND_ERR_OUT_OF_MEMORY, "host allocation failed");
    b->members.assign(ctxs, ctxs + n);
    b->dbl = ctxs[0]->p.precision == POND_PREC_FP64;
    b->np = ctxs[0]->p.interp_points;
    b->split = ctxs[0]->p.split;
    b->lattice = ctxs[0]->p.lattice;
    b->own_stream = hip_stream == nullptr;
    hipError_t e = hipSuccess;
    if (b->own_stream)
        e = hipStreamCreate(&b->stream);
    else
        b->stream = static_cast<hipStream_t>(hip_stream);
    if (e != hipSuccess) {
        b->stream = nullptr;
        release(b);
        return hip_fail(e, "hipStreamCreate");
    }

    // LDS per block: the share of a CU of the blocks that fit by registers
    int per_cu = 0;
    const void *kern = batch_step_fn(b->dbl, b->np, b->split, b->lattice);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBatchThreads, 0);
    b->cap = lds_nodes_for_blocks(e == hipSuccess ? per_cu : 1, b->dbl, b->lattice);
    const size_t lds = size_t(b->cap) * lds_node_values(b->lattice, b->dbl) *
                       (b->dbl ? sizeof(double) : sizeof(float));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "batch launch configuration");
    }

    // descriptors
    std::vector<BatchMember> hm(n);
    std::vector<int> toff(n), boff(n);
    long long tiles = 0, blocks = 0, nodes = 0;
    for (int i = 0; i < n; ++i) {
        pond_ctx *c = ctxs[i];
        const int w = member_width(c), lg = lg2(w), h = kBatchThreads >> lg;
        const int tx = (c->p.nx + w - 1) / w, ty = (c->p.ny + h - 1) / h;
        const int halo = halo_for_dims(w, h, b->cap, c->p.ny == 1);
        if (halo < 0) {
            release(b);
            return fail(POND_ERR_INVALID_ARG, "context %d: tile %dx%d does not fit %d LDS nodes", i,
                        w, h, b->cap);
        }
        BatchMember &m = hm[i];
        m.a = c->args;
        m.buf[0] = c->buf[0];
        m.buf[1] = c->buf[1];
        m.mom[0] = c->mom[0];
        m.mom[1] = c->mom[1];
        m.cnt = c->cnt;
        m.parity0 = c->cur;
        b->parity0.push_back(c->cur);
        m.lg = lg;
        m.tiles_x = tx;
        m.tile_off = int(tiles);
        m.blk_off = int(blocks);
        toff[i] = int(tiles);
        boff[i] = int(blocks);
        tiles += (long long)tx * ty;
        blocks += (c->args.N + kBatchThreads - 1) / kBatchThreads;
        nodes += c->args.N;
        b->widths.push_back(w);
    }
    if (tiles > 0x7fffffffll || blocks > 0x7fffffffll) {
        release(b);
        return fail(POND_ERR_INVALID_ARG, "batch too large (%lld tiles)", tiles);
    }
    b->tiles = int(tiles);
    b->grid = b->tiles;
    if (POND_BATCH_PERSISTENT) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            per_cu > 0 && cus > 0)
            b->grid = std::max(8, (per_cu * cus + 7) / 8 * 8);
        else
            b->grid = std::max(8, b->tiles);
    }
    b->blocks = int(blocks);
    b->nodes = nodes;

    const size_t mem_bytes = align_up(sizeof(BatchMember) * n);
    const size_t off_bytes = align_up(sizeof(int) * n);
    e = hipMalloc(&b->dev, mem_bytes + 2 * off_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b->dev = nullptr;
        release(b);
        return fail(POND_ERR_OUT_OF_MEMORY, "batch descriptor allocation failed");
    }
    char *base = static_cast<char *>(b->dev);
    b->d_mem = reinterpret_cast<BatchMember *>(base);
    b->d_tile_off = reinterpret_cast<int *>(base + mem_bytes);
    b->d_blk_off = reinterpret_cast<int *>(base + mem_bytes + off_bytes);
    // members' pending work (initialisation, earlier steps) precedes the batch's
    for (pond_ctx *c : b->members)
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(b->d_mem, hm.data(), sizeof(BatchMember) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_tile_off, toff.data(), sizeof(int) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_blk_off, boff.data(), sizeof(int) * n, hipMemcpyHostToDevice);
    for (int f = 0; f < 2; ++f) {
        if (e == hipSuccess) e = capture(b, 1, f, &b->graph[f][0], &b->exec[f][0]);
        if (e == hipSuccess) e = capture(b, kGraphSteps, f, &b->graph[f][1], &b->exec[f][1]);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming);
    for (pond_ctx *c : b->members) {
        if (e != hipSuccess) break;
        if (c->stream == b->stream) continue;
        if (std::find(b->other_streams.begin(), b->other_streams.end(), c->stream) !=
            b->other_streams.end())
            continue;
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) {
            b->other_streams.push_back(c->stream);
            b->other_ev.push_back(ev);
        }
    }
    if (e != hipSuccess) {
        pond_status s = hip_fail(e, "batch set-up");
        release(b);
        return s;
    }
    for (pond_ctx *c : b->members) c->batch = b;
    b->steps = 0;
    *out = b;
    return POND_OK;
}

pond_status pond_batch_step(pond_batch *b, int64_t nsteps) {
    if (!b) return fail(POND_ERR_INVALID_ARG, "batch is NULL");
    if (nsteps < 0) return fail(POND_ERR_INVALID_ARG, "nsteps < 0");
    for (const pond_ctx *c : b->members)
        if (c->failed) return fail(POND_ERR_STATE, "a member is in the error state (non-physical)");
    if (nsteps == 0) return POND_OK;
    hipError_t e = hipSuccess;
    // work already queued on the members' own streams (e.g. moments read-outs) goes first
    for (size_t k = 0; k < b->other_streams.size() && e == hipSuccess; ++k) {
        e = hipEventRecord(b->other_ev[k], b->other_streams[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->other_ev[k], 0);
    }
    // kGraphSteps is even: the long graph leaves the parity unchanged
    const int f = int(b->steps & 1);
    // moments of the members' current buffers, once, if any member's are stale
    bool stale = false;
    for (const pond_ctx *c : b->members) stale = stale || !c->mom_fresh;
    if (stale && e == hipSuccess) e = enqueue_batch_moments(b, f);
    for (int64_t k = 0; k + kGraphSteps <= nsteps && e == hipSuccess; k += kGraphSteps)
        e = hipGraphLaunch(b->exec[f][1], b->stream);
    for (int64_t k = 0; k < nsteps % kGraphSteps && e == hipSuccess; ++k)
        e = hipGraphLaunch(b->exec[f ^ int(k & 1)][0], b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->done_ev, b->stream);
    for (size_t k = 0; k < b->other_streams.size() && e == hipSuccess; ++k)
        e = hipStreamWaitEvent(b->other_streams[k], b->done_ev, 0);
    if (e != hipSuccess) return hip_fail(e, "batch step launch");
    for (pond_ctx *c : b->members) {
        c->cur ^= int(nsteps & 1);
        c->steps += nsteps;
        c->mom_fresh = true;
    }
    b->steps += nsteps;
    return POND_OK;
}

pond_status pond_batch_synchronize(pond_batch *b) {
    if (!b) return fail(POND_ERR_INVALID_ARG, "batch is NULL");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int bad = 0;
    pond_status first = POND_OK;
    for (pond_ctx *c : b->members) {
        DevCounters h;
        pond_status s = read_counters(c, &h);
        if (s != POND_OK) return s;
        s = counters_status(c, h);
        if (s != POND_OK) {
            if (first == POND_OK) first = s;
            ++bad;
        }
    }
    if (bad)
        return fail(first, "%d member(s) failed: produced rho <= 0, T <= 0 or NaN, or reached "
                           "beyond a wall's ghost rows", bad);
    return POND_OK;
}

pond_status pond_batch_get_info(pond_batch *b, pond_batch_info_t *out) {
    if (!b || !out) return fail(POND_ERR_INVALID_ARG, "batch or out is NULL");
    out->members = int32_t(b->members.size());
    out->tiles = b->tiles;
    out->grid_blocks = b->grid;
    out->lds_nodes = b->cap;
    out->nodes = b->nodes;
    out->steps = b->steps;
    out->graph_steps = kGraphSteps;
    out->reserved = 0;
    return POND_OK;
}

pond_status pond_batch_member_tile_width(pond_batch *b, int i, int *width) {
    if (!b || !width) return fail(POND_ERR_INVALID_ARG, "batch or width is NULL");
    if (i < 0 || i >= int(b->members.size())) return fail(POND_ERR_INVALID_ARG, "member %d out of range", i);
    *width = b->widths[i];
    return POND_OK;
}

pond_status pond_batch_destroy(pond_batch *b) {
    if (!b) return POND_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    release(b);
    return e == hipSuccess ? POND_OK : hip_fail(e, "hipStreamSynchronize");
}

// ------------------------------------------------------------ autotune ----
namespace {

struct Saved {
    void *tmp = nullptr;
    int cur = 0;
    long long steps = 0;
    DevCounters cnt{};
    pond_tuning tuning{};
};

pond_status save_state(pond_ctx *c, Saved &s) {
    s.cur = c->cur;
    s.steps = c->steps;
    s.tuning = c->tuning;
    pond_status st = read_counters(c, &s.cnt);
    if (st != POND_OK) return st;
    hipError_t e = hipMalloc(&s.tmp, c->L.buf_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s.tmp = nullptr;
        return fail(POND_ERR_OUT_OF_MEMORY, "autotune state copy (%zu bytes)", c->L.buf_bytes);
    }
    e = hipMemcpyAsync(s.tmp, c->buf[s.cur].f, c->L.buf_bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? POND_OK : hip_fail(e, "autotune save");
}

pond_status restore_state(pond_ctx *c, const Saved &s) {
    hipError_t e = hipMemcpyAsync(c->buf[s.cur].f, s.tmp, c->L.buf_bytes, hipMemcpyDeviceToDevice,
                                  c->stream);
    if (e != hipSuccess) return hip_fail(e, "autotune restore");
    c->cur = s.cur;
    c->mom_fresh = false;
    c->steps = s.steps;
    c->failed = false;
    c->fail_status = POND_OK;
    return write_counters(c, s.cnt);
}

// Device time per step of c (single-instance path, or a one-member batch when
// batch_width > 0) over at least `steps` steps and at least kMinTuneMs of
// device time, after one untimed step; the state is restored afterwards.
constexpr double kMinTuneMs = 2.0;
constexpr int kMaxTuneSteps = 512;

pond_status time_candidate(pond_ctx *c, const Saved &sv, int steps, int batch_width, double *ms_per_step) {
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    pond_status s = e == hipSuccess ? POND_OK : hip_fail(e, "hipEventCreate");
    pond_batch *b = nullptr;
    if (s == POND_OK && batch_width > 0) {
        c->tuning.batch_tile_width = batch_width;
        s = pond_batch_create(&c, 1, c->stream, &b);
    }
    if (s == POND_OK) s = b ? pond_batch_step(b, 1) : pond_step(c, 1);
    int n = steps;
    for (;;) {
        if (s != POND_OK) break;
        e = hipEventRecord(ev[0], c->stream);
        if (e != hipSuccess) {
            s = hip_fail(e, "hipEventRecord");
            break;
        }
        s = b ? pond_batch_step(b, n) : pond_step(c, n);
        if (s != POND_OK) break;
        e = hipEventRecord(ev[1], c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
        if (e != hipSuccess) {
            s = hip_fail(e, "autotune timing");
            break;
        }
        *ms_per_step = t / n;
        if (t >= kMinTuneMs || n >= kMaxTuneSteps) break;
        n = std::min(kMaxTuneSteps, std::max(2 * n, int(n * kMinTuneMs / std::max(t, 1e-3f)) + 1));
    }
    if (b) {
        pond_status s2 = pond_batch_destroy(b);
        if (s == POND_OK) s = s2;
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    pond_status s3 = restore_state(c, sv);
    return s == POND_OK ? s3 : s;
}

// Index of the fastest candidate; the first (the default) unless another is
// faster by more than 3 %.
size_t pick(const std::vector<double> &t) {
    size_t best = 0;
    for (size_t k = 1; k < t.size(); ++k)
        if (t[k] < t[best] && t[k] < 0.97 * t[0]) best = k;
    return best;
}

}  // namespace

pond_status pond_autotune(pond_ctx *c, int steps, pond_tuning *out) {
    pond_status s = check_ctx(c, true);
    if (s != POND_OK) return s;
    if (c->batch) return fail(POND_ERR_STATE, "context is a member of a batch");
    if (c->failed) return fail(POND_ERR_STATE, "context is in the error state");
    if (steps < 1) return fail(POND_ERR_INVALID_ARG, "steps must be >= 1");
    const bool dbl = c->p.precision == POND_PREC_FP64, row = c->p.ny < 8;
    std::vector<int> tiles, widths;  // the context's default tile first
    if (row) {
        tiles = {POND_TILE_64x1, POND_TILE_256x1};
        widths = {256};
    } else {
        tiles = {default_tuning(c->p).tile, POND_TILE_32x8, POND_TILE_16x16, POND_TILE_16x8};
        if (c->p.lattice == POND_LATTICE_D2Q16) tiles.push_back(POND_TILE_32x16);
        // one-wave blocks: each wave frees its CU share as soon as it is done, which
        // pays where the predictor-corrector work varies from wave to wave (shocks:
        // 2048^2 quadrants 1.04 against 1.13 ms per step with 32 x 8)
        tiles.push_back(POND_TILE_8x8);
        for (size_t i = 1; i < tiles.size(); ++i)  // the default appears once
            if (tiles[i] == tiles[0]) tiles.erase(tiles.begin() + long(i--));
        widths = dbl ? std::vector<int>{16, 32, 64} : std::vector<int>{32, 16, 64};
    }
    Saved sv;
    s = save_state(c, sv);
    // two interleaved rounds; each candidate keeps its faster measurement
    // single-path candidates: each tile with the LDS share of the blocks that fit
    // by registers (lds 0 = default), and with the larger share of one block fewer
    struct Cand {
        int tile, lds;
    };
    std::vector<Cand> cands;
    for (int tile : tiles) {
        cands.push_back({tile, 0});
        const int blocks = tiled_blocks_per_cu(c->p.lattice, dbl, c->p.interp_points, c->p.split,
                                               static_cast<TileShape>(tile));
        if (blocks >= 2)
            cands.push_back({tile, lds_nodes_for_blocks(blocks - 1, dbl, c->p.lattice)});
    }
    std::vector<double> tt(cands.size(), 1e300), tw(widths.size(), 1e300);
    for (int round = 0; round < 2 && s == POND_OK; ++round) {
        for (size_t k = 0; k < cands.size() && s == POND_OK; ++k) {
            pond_tuning t = sv.tuning;
            t.kernel = POND_KERNEL_TILED;
            t.tile = cands[k].tile;
            t.lds_nodes = cands[k].lds;
            s = pond_set_tuning(c, &t);
            double ms = 0.0;
            if (s == POND_OK) s = time_candidate(c, sv, steps, 0, &ms);
            if (s == POND_OK) tt[k] = std::min(tt[k], ms);
        }
        for (size_t k = 0; k < widths.size() && widths.size() > 1 && s == POND_OK; ++k) {
            double ms = 0.0;
            s = time_candidate(c, sv, steps, widths[k], &ms);
            if (s == POND_OK) tw[k] = std::min(tw[k], ms);
        }
    }
    if (sv.tmp) (void)hipFree(sv.tmp);
    if (s != POND_OK) {
        c->tuning = sv.tuning;
        (void)pond_set_tuning(c, &sv.tuning);
        return s;
    }
    pond_tuning best = sv.tuning;
    best.kernel = POND_KERNEL_TILED;
    best.tile = cands[pick(tt)].tile;
    best.lds_nodes = cands[pick(tt)].lds;
    best.batch_tile_width = widths[widths.size() > 1 ? pick(tw) : 0];
    s = pond_set_tuning(c, &best);
    if (s != POND_OK) return s;
    best = c->tuning;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(c)] = best;
    }
    if (out) *out = best;
    return POND_OK;
}

pond_status pond_tuning_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return POND_OK;
}
