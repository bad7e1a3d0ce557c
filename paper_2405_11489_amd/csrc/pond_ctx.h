// pond_ctx.h -- the context object behind the opaque pond_ctx handle, and the
// host helpers shared by the single-instance ABI (pond_api.hip) and the
// batched / serving layer (pond_batch.hip, pond_server.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "pond.h"
#include "pond_internal.h"

namespace pond {

// Record a message for pond_last_error() on this thread and return s.
pond_status fail(pond_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
pond_status hip_fail(hipError_t e, const char *what);
const char *last_error();

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// One context's device allocation:
//   [state buffer 0 | state buffer 1 | moment planes 0 | moment planes 1 | counters | scratch]
// (moment planes k hold the moments of state buffer k).  A state buffer is
//   [Q f planes | Q g planes | u_x | u_y | T | (internal split) u_x, u_y of the previous level]
struct Layout {
    size_t pop_bytes;    // one set of Q planes (Q = 16 or 25)
    size_t frame_bytes;  // one frame plane
    size_t buf_bytes;    // one state buffer
    size_t mom_bytes;    // one set of moment planes (2 NM values per node, padded to the groups)
    size_t cnt_off, scratch_off, total;
};

// Frame planes of the previous time level per state buffer: 2 (u_x, u_y) for
// the internal-energy split, whose source extrapolates the velocity gradient
// along trajectories from the last two levels; 0 otherwise.
inline int prev_frame_planes(int split) { return split == POND_SPLIT_INTERNAL ? 2 : 0; }

constexpr int kScratchDoubles = 3 * 256;

// Values of a node's moment groups (2 NM moments, padded): 20 on D2Q16; on
// D2Q25 32 floats or 30 doubles.
inline int moment_values(int lattice, bool dbl) { return lattice == 25 ? (dbl ? 30 : 32) : 20; }

// Values (float or double) per node of an LDS tile: the moment groups (D2Q16:
// 20 floats or doubles; D2Q25: 32 floats, 30 doubles; FP32 D2Q16 tiles are
// node-major, the others grouped planes, neither padded).
inline int lds_node_values(int lattice, bool dbl) {
    return lattice == 25 ? (dbl ? 30 : 32) : 20;
}

// Ghost rows of the moment planes beyond each wall (bc_y == POND_BC_WALL).
constexpr int kWallGhostRows = 8;

// Nodes per moment plane: the grid, plus the ghost rows with walls.
inline long long moment_plane_nodes(const pond_params &p) {
    return (long long)p.nx * (p.ny + (p.bc_y == POND_BC_WALL ? 2 * kWallGhostRows : 0));
}

Layout layout_for(long long N, size_t psize, int lattice, long long mom_nodes, int prev_planes);

// LDS nodes per block (the moment groups of one node each) that let
// blocks_per_cu blocks share the 160 KiB of a CU.
int lds_nodes_for_blocks(int blocks_per_cu, bool dbl, int lattice = 16);
// LDS nodes per block of the tiled kernel's default share for a tile shape.
int default_lds_nodes(int tile, bool dbl, int np, int split, int lattice);
// Default launch configuration of a context with these parameters (on the
// current device).
pond_tuning default_tuning(const pond_params &p);

// POND_OK, or the status and message (pond_last_error) of the first invalid or
// unsupported parameter.  Touches no device.
pond_status validate_params(const pond_params *p);
// Kernel arguments of a validated parameter set (reference velocity zero).
void fill_step_args(const pond_params &p, StepArgs &a);

// Largest halo h of a tx x ty tile whose source region fits cap nodes:
// (tx + 2h)(ty + 2h) <= cap, or tx + 2h <= cap for a single-row grid (whose
// region is one row).  -1 if not even the tile fits.
inline int halo_for_dims(int tx, int ty, int cap, bool single_row) {
    if (single_row) return cap >= tx ? (cap - tx) / 2 : -1;
    int h = -1;
    while ((tx + 2 * (h + 1)) * (ty + 2 * (h + 1)) <= cap) ++h;
    return h;
}

}  // namespace pond

struct pond_ctx {
    pond_params p;
    size_t psize;
    pond::Layout L;
    hipStream_t stream;
    bool own_stream;
    char *mem;
    bool own_mem;
    pond::DevState buf[2];
    int cur;
    void *mom[2];     // moments of buf[0] / buf[1]
    bool mom_fresh;   // mom[cur] holds the moments of buf[cur]
    pond::DevCounters *cnt;
    double *scratch;
    pond::StepArgs args;
    bool initialized;
    bool failed;
    pond_status fail_status;  // why the context failed: POND_ERR_NONPHYSICAL or
                              // POND_ERR_UNSUPPORTED (wall ghost rows overrun)
    long long steps;
    pond_tuning tuning;
    pond::TileConfig tc;
    bool profiling;
    std::vector<hipEvent_t> prof_events;  // 3 per timed step
    double prof_prepass_ms, prof_step_ms;
    long long prof_launches;
    pond_batch *batch;  // batch that owns the stepping of this context, or NULL
    int reach;          // ceil of the largest stencil reach of the initial frame (nodes)
    bool user_tuned;    // tuning set explicitly: the tuning cache does not override it
};

namespace pond {

pond_status check_ctx(const pond_ctx *c, bool need_init);
pond_status read_counters(pond_ctx *c, DevCounters *out);
pond_status write_counters(pond_ctx *c, const DevCounters &in);
// Status of counters read after steps: POND_ERR_NONPHYSICAL (non-physical
// values) or POND_ERR_UNSUPPORTED (stencils beyond a wall's ghost rows) put the
// context into the error state; POND_OK otherwise.
pond_status counters_status(pond_ctx *c, const DevCounters &h);

// Autotuned launch configuration of c's class (size and stencil reach), if
// pond_autotune stored one.
bool tuning_cache_lookup(const pond_ctx *c, pond_tuning *out);

}  // namespace pond
