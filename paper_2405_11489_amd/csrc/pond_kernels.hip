// pond_kernels.hip -- HIP kernels of the PonD f+g step for gfx950 (MI355X):
// the D2Q16 instantiation of the lattice-dependent kernels
// (pond_lattice_kernels.h; D2Q25 in pond_kernels25.hip), the launchers that
// pick the lattice, and the lattice-independent reductions.
//
// One kernel source, instantiated for P = double (FP64 mode) and P = float
// (FP32 mode: populations, moments, interpolation and frame transformation in
// float; conserved sums, temperature recovery and the predictor-corrector test
// in double).
#include "pond_lattice_kernels.h"

namespace pond {

template struct Launch<float, D2Q16>;
template struct Launch<double, D2Q16>;
extern template struct Launch<float, D2Q25>;
extern template struct Launch<double, D2Q25>;

namespace {

using lk::kBlock;
using lk::grid_for;
using lk::partial_sums_kernel;

// ------------------------------------------- deterministic reductions ----
constexpr int kRedBlocks = 256;

__global__ void final_sums_kernel(const double *scratch, int nblocks, DevCounters *cnt) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        s0 += scratch[b * 3];
        s1 += scratch[b * 3 + 1];
        s2 += scratch[b * 3 + 2];
    }
    cnt->partial[0] = s0;
    cnt->partial[1] = s1;
    cnt->partial[2] = s2;
}

// per-block maxima of max(|u_x|, |u_y|) + c_out sqrt(T) (the reach of a node's
// departure stencils, in nodes); non-finite values are skipped
__global__ __launch_bounds__(kBlock) void reach_partial_kernel(long long N, const double *ux,
                                                               const double *uy, const double *T,
                                                               double *scratch) {
    __shared__ double sh[kBlock];
    const long long chunk = (N + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < N ? lo + chunk : N;
    double m = 0.0;
    for (long long n = lo + threadIdx.x; n < hi; n += blockDim.x) {
        const double r = fmax(fabs(ux[n]), fabs(uy[n])) + c1(3) * sqrt(fmax(T[n], 0.0));
        if (isfinite(r)) m = fmax(m, r);
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scratch[blockIdx.x] = sh[0];
}

__global__ void reach_final_kernel(const double *scratch, int nblocks, DevCounters *cnt) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double m = 0.0;
    for (int b = 0; b < nblocks; ++b) m = fmax(m, scratch[b]);
    cnt->partial[3] = m;
}

struct FieldLoader {
    const double *rho, *ux, *uy;
    __device__ void operator()(long long n, double &r, double &jx, double &jy) const {
        r = rho[n];
        jx = rho[n] * ux[n];
        jy = rho[n] * uy[n];
    }
};

}  // namespace

template <typename P>
hipError_t launch_init(const StepArgs &a, const double *rho, const double *ux, const double *uy,
                       const double *T, DevState st, DevCounters *cnt, hipStream_t s) {
    return a.lattice == 25 ? Launch<P, D2Q25>::init(a, rho, ux, uy, T, st, cnt, s)
                           : Launch<P, D2Q16>::init(a, rho, ux, uy, T, st, cnt, s);
}

template <typename P>
hipError_t launch_moments_prepass(const StepArgs &a, DevState st, P *mom, hipStream_t s) {
    return a.lattice == 25 ? Launch<P, D2Q25>::moments(a, st, mom, s)
                           : Launch<P, D2Q16>::moments(a, st, mom, s);
}

template <typename P>
hipError_t launch_wall_ghosts(const StepArgs &a, DevState st, P *mom, hipStream_t s) {
    return a.lattice == 25 ? Launch<P, D2Q25>::wall_ghosts(a, st, mom, s)
                           : Launch<P, D2Q16>::wall_ghosts(a, st, mom, s);
}

template <typename P>
hipError_t launch_step(const StepArgs &a, DevState src, const P *mom, DevState dst, P *mom_out,
                       DevCounters *cnt, hipStream_t s) {
    return a.lattice == 25 ? Launch<P, D2Q25>::step(a, src, mom, dst, mom_out, cnt, s)
                           : Launch<P, D2Q16>::step(a, src, mom, dst, mom_out, cnt, s);
}

template <typename P>
hipError_t launch_step_tiled(const StepArgs &a, const TileConfig &tc, DevState src, const P *mom,
                             DevState dst, P *mom_out, DevCounters *cnt, hipStream_t s) {
    return a.lattice == 25 ? Launch<P, D2Q25>::step_tiled(a, tc, src, mom, dst, mom_out, cnt, s)
                           : Launch<P, D2Q16>::step_tiled(a, tc, src, mom, dst, mom_out, cnt, s);
}

int tiled_blocks_per_cu(int lattice, bool dbl, int np, int split, TileShape shape) {
    if (lattice == 25)
        return dbl ? Launch<double, D2Q25>::tiled_blocks_per_cu(np, split, shape)
                   : Launch<float, D2Q25>::tiled_blocks_per_cu(np, split, shape);
    return dbl ? Launch<double, D2Q16>::tiled_blocks_per_cu(np, split, shape)
               : Launch<float, D2Q16>::tiled_blocks_per_cu(np, split, shape);
}

template <typename P>
hipError_t launch_ghost_check(const StepArgs &a, DevState st, DevCounters *cnt, hipStream_t s) {
    return a.lattice == 25 ? Launch<P, D2Q25>::ghost_check(a, st, cnt, s)
                           : Launch<P, D2Q16>::ghost_check(a, st, cnt, s);
}

template <typename P>
hipError_t launch_macro(const StepArgs &a, DevState st, double *rho, double *ux, double *uy,
                        double *T, double *p, hipStream_t s) {
    return a.lattice == 25 ? Launch<P, D2Q25>::macro(a, st, rho, ux, uy, T, p, s)
                           : Launch<P, D2Q16>::macro(a, st, rho, ux, uy, T, p, s);
}

template <typename P>
hipError_t launch_export(const StepArgs &a, DevState st, double *f, double *g, double *frame,
                         hipStream_t s) {
    return a.lattice == 25 ? Launch<P, D2Q25>::exp(a, st, f, g, frame, s)
                           : Launch<P, D2Q16>::exp(a, st, f, g, frame, s);
}

template <typename P>
hipError_t launch_import(const StepArgs &a, const double *f, const double *g, const double *frame,
                         DevState st, hipStream_t s) {
    return a.lattice == 25 ? Launch<P, D2Q25>::imp(a, f, g, frame, st, s)
                           : Launch<P, D2Q16>::imp(a, f, g, frame, st, s);
}

hipError_t launch_mean_velocity(long long N, const double *rho, const double *ux, const double *uy,
                                double *scratch, int scratch_len, DevCounters *cnt,
                                hipStream_t s) {
    if (scratch_len < 3 * kRedBlocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(partial_sums_kernel<FieldLoader>, dim3(kRedBlocks), dim3(kBlock), 0, s, N,
                       FieldLoader{rho, ux, uy}, scratch);
    hipLaunchKernelGGL(final_sums_kernel, dim3(1), dim3(64), 0, s, scratch, kRedBlocks, cnt);
    return hipGetLastError();
}

hipError_t launch_frame_reach(long long N, const double *ux, const double *uy, const double *T,
                              double *scratch, int scratch_len, DevCounters *cnt, hipStream_t s) {
    if (scratch_len < kRedBlocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reach_partial_kernel, dim3(kRedBlocks), dim3(kBlock), 0, s, N, ux, uy, T,
                       scratch);
    hipLaunchKernelGGL(reach_final_kernel, dim3(1), dim3(64), 0, s, scratch, kRedBlocks, cnt);
    return hipGetLastError();
}

template <typename P>
hipError_t launch_state_mean_velocity(const StepArgs &a, DevState st, double *scratch,
                                      int scratch_len, DevCounters *cnt, hipStream_t s) {
    if (scratch_len < 3 * kRedBlocks) return hipErrorInvalidValue;
    hipError_t e = a.lattice == 25
                       ? Launch<P, D2Q25>::state_partial_sums(a, st, scratch, kRedBlocks, s)
                       : Launch<P, D2Q16>::state_partial_sums(a, st, scratch, kRedBlocks, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(final_sums_kernel, dim3(1), dim3(64), 0, s, scratch, kRedBlocks, cnt);
    return hipGetLastError();
}

#define POND_INSTANTIATE(P)                                                                        \
    template hipError_t launch_init<P>(const StepArgs &, const double *, const double *,           \
                                       const double *, const double *, DevState, DevCounters *,    \
                                       hipStream_t);                                               \
    template hipError_t launch_moments_prepass<P>(const StepArgs &, DevState, P *, hipStream_t);   \
    template hipError_t launch_wall_ghosts<P>(const StepArgs &, DevState, P *, hipStream_t);       \
    template hipError_t launch_step<P>(const StepArgs &, DevState, const P *, DevState, P *,       \
                                       DevCounters *, hipStream_t);                                \
    template hipError_t launch_step_tiled<P>(const StepArgs &, const TileConfig &, DevState,       \
                                             const P *, DevState, P *, DevCounters *,              \
                                             hipStream_t);                                         \
    template hipError_t launch_ghost_check<P>(const StepArgs &, DevState, DevCounters *,       \
                                              hipStream_t);                                        \
    template hipError_t launch_macro<P>(const StepArgs &, DevState, double *, double *, double *,  \
                                        double *, double *, hipStream_t);                          \
    template hipError_t launch_export<P>(const StepArgs &, DevState, double *, double *, double *, \
                                         hipStream_t);                                             \
    template hipError_t launch_import<P>(const StepArgs &, const double *, const double *,         \
                                         const double *, DevState, hipStream_t);                   \
    template hipError_t launch_state_mean_velocity<P>(const StepArgs &, DevState, double *, int,   \
                                                      DevCounters *, hipStream_t);

POND_INSTANTIATE(float)
POND_INSTANTIATE(double)

}  // namespace pond
