// pond_internal.h -- host-side interface between the C ABI (pond_api.hip) and
// the kernel launchers (pond_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pond {

// Device state of one instance.  Population planes: pop[i * N + n] for
// velocity i and node n = y * nx + x.  Frame planes: double ux, uy, T.  The
// internal-energy split also keeps the frame velocities of the previous time
// level (uxp, uyp: its source extrapolates the velocity gradient along
// trajectories from the last two levels); NULL for the other splits.
struct DevState {
    void *f, *g;          // Q planes each (float or double), Q = 16 or 25
    double *ux, *uy, *T;  // frame
    double *uxp, *uyp;    // frame velocities of the previous time level (internal split)
};

// Counters accumulated on the device (64-bit integer atomics only, so the sums
// do not depend on scheduling).
struct DevCounters {
    unsigned long long pc_iterations;
    unsigned long long nonconverged;
    unsigned long long nonphysical;
    unsigned long long init_rejected;
    // node-steps (or, at initialisation, nodes) whose departure stencil reached
    // beyond the ghost rows of a wall
    unsigned long long ghost_overrun;
    double partial[4];  // scratch for deterministic reductions
};

struct StepArgs {
    int nx, ny, bc_x, bc_y;
    long long N;
    int interp_points;   // 3 or 4
    int pc_max_iter;
    double pc_tol;
    double omega;        // 1 / tau
    double omega1;       // 1 / tau_1 (Fourier part of the energy flux)
    int unit_prandtl;    // 1: plain BGK for g
    int split;           // 0: total energy in g; 1: internal energy in g (plus its source);
                         // 2: non-translational energy in g
    int lattice;         // 16 (D2Q16) or 25 (D2Q25)
    long long mstride;   // nodes per moment plane: N, or (ny + 2 wall_h) nx with walls
    long long moff;      // node offset of grid row 0 in a moment plane (wall_h nx)
    int wall_h;          // ghost rows beyond each wall (bc_y == 2), else 0
    double wall_ux[2], wall_T[2];
    double cv;           // 1 / (gamma - 1)
    double uref_x, uref_y;
};

// Tiled step launch configuration: block shape, LDS capacity (nodes of the
// staged source region) and the largest halo that fits it.
enum class TileShape : int { T16x16 = 0, T32x8 = 1, T16x8 = 2, T8x8 = 3, T256x1 = 4, T64x1 = 5,
                             T32x16 = 6 };

struct TileConfig {
    TileShape shape;
    int cap;       // nodes of LDS per block
    int halo_cap;  // largest symmetric halo h with (TX + 2h)(TY + 2h) <= cap (>= 0: the tile fits)
};

inline void tile_dims(TileShape s, int &tx, int &ty) {
    switch (s) {
    case TileShape::T16x16: tx = 16; ty = 16; return;
    case TileShape::T32x8: tx = 32; ty = 8; return;
    case TileShape::T16x8: tx = 16; ty = 8; return;
    case TileShape::T8x8: tx = 8; ty = 8; return;
    case TileShape::T256x1: tx = 256; ty = 1; return;
    case TileShape::T64x1: tx = 64; ty = 1; return;
    case TileShape::T32x16: tx = 32; ty = 16; return;
    }
    tx = ty = 0;
}

// Blocks of the tiled step kernel (lattice, precision, stencil, energy split,
// shape) that fit one CU by registers and waves alone (no dynamic LDS).
int tiled_blocks_per_cu(int lattice, bool dbl, int np, int split, TileShape shape);

// Calls f(np, split) with both as std::integral_constant (np: 3 or 4 stencil
// points per axis, split: 0 total, 1 internal, 2 non-translational energy), so
// kernels can be picked by compile-time variant: the D2Q16 variants, of the
// single-instance and the batched paths alike.
template <class F>
inline auto with_variant(int np, int split, F &&f) {
    using std::integral_constant;
    if (np == 3) {
        if (split == 2) return f(integral_constant<int, 3>{}, integral_constant<int, 2>{});
        return split == 1 ? f(integral_constant<int, 3>{}, integral_constant<int, 1>{})
                          : f(integral_constant<int, 3>{}, integral_constant<int, 0>{});
    }
    if (split == 2) return f(integral_constant<int, 4>{}, integral_constant<int, 2>{});
    return split == 1 ? f(integral_constant<int, 4>{}, integral_constant<int, 1>{})
                      : f(integral_constant<int, 4>{}, integral_constant<int, 0>{});
}

// The single-instance variants of a lattice: D2Q16 takes both stencils and the
// three energy splits (0 total, 1 internal, 2 non-translational); D2Q25 the
// cubic stencil with the three splits (the API rejects other combinations
// before a launch).
template <class L, class F>
inline auto with_lattice_variant(int np, int split, F &&f) {
    using std::integral_constant;
    if constexpr (L::Q == 16) {
        return with_variant(np, split, static_cast<F &&>(f));
    } else {
        if (split == 2) return f(integral_constant<int, 4>{}, integral_constant<int, 2>{});
        return split == 1 ? f(integral_constant<int, 4>{}, integral_constant<int, 1>{})
                          : f(integral_constant<int, 4>{}, integral_constant<int, 0>{});
    }
}

template <typename P>
hipError_t launch_init(const StepArgs &a, const double *rho, const double *ux, const double *uy,
                       const double *T, DevState st, DevCounters *cnt, hipStream_t s);
template <typename P>
hipError_t launch_moments_prepass(const StepArgs &a, DevState st, P *mom, hipStream_t s);
// Ghost rows of the moment planes beyond walls (bc_y == 2), from the moments
// the pre-pass wrote; launched after it.
template <typename P>
hipError_t launch_wall_ghosts(const StepArgs &a, DevState st, P *mom, hipStream_t s);
// A step reads the moments of src (mom) and writes those of dst (mom_out).
template <typename P>
hipError_t launch_step(const StepArgs &a, DevState src, const P *mom, DevState dst, P *mom_out,
                       DevCounters *cnt, hipStream_t s);
template <typename P>
hipError_t launch_step_tiled(const StepArgs &a, const TileConfig &tc, DevState src, const P *mom,
                             DevState dst, P *mom_out, DevCounters *cnt, hipStream_t s);
// Walls (bc_y == 2): adds to cnt->ghost_overrun the nodes of st's frame whose
// departure stencil reaches beyond the ghost rows.
template <typename P>
hipError_t launch_ghost_check(const StepArgs &a, DevState st, DevCounters *cnt, hipStream_t s);
template <typename P>
hipError_t launch_macro(const StepArgs &a, DevState st, double *rho, double *ux, double *uy,
                        double *T, double *p, hipStream_t s);
template <typename P>
hipError_t launch_export(const StepArgs &a, DevState st, double *f, double *g, double *frame,
                         hipStream_t s);
template <typename P>
hipError_t launch_import(const StepArgs &a, const double *f, const double *g, const double *frame,
                         DevState st, hipStream_t s);
// Deterministic mass-weighted mean velocity of (rho, ux, uy) into cnt->partial[0..2]
// (sum rho, sum rho ux, sum rho uy), fixed summation order.
hipError_t launch_mean_velocity(long long N, const double *rho, const double *ux, const double *uy,
                                double *scratch, int scratch_len, DevCounters *cnt, hipStream_t s);
// Largest stencil reach max(|u_x|, |u_y|) + c_out sqrt(T) over the nodes of a
// frame, into cnt->partial[3].
hipError_t launch_frame_reach(long long N, const double *ux, const double *uy, const double *T,
                              double *scratch, int scratch_len, DevCounters *cnt, hipStream_t s);
// Mass-weighted mean velocity of a stored state (populations + frame).
template <typename P>
hipError_t launch_state_mean_velocity(const StepArgs &a, DevState st, double *scratch,
                                      int scratch_len, DevCounters *cnt, hipStream_t s);

}  // namespace pond
