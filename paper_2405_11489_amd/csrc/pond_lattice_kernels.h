// pond_lattice_kernels.h -- the kernels of the PonD f+g step that depend on the
// lattice (D2Q16 or D2Q25), and their launchers, as templates over the
// arithmetic type P and the lattice L.  pond_kernels.hip instantiates them for
// D2Q16 and pond_kernels25.hip for D2Q25 (two translation units compiled in
// parallel); the launchers are reached through Launch<P, L>.
//
// Step = two launches on one stream:
//   1. moments pre-pass: per node, the moments of f and g up to the lattice's
//      Grad order (Eq. genericMomentUptoO3) about the instance's reference
//      velocity, written as grouped planes;
//   2. step: per destination node (one lane), the predictor-corrector loop
//      (gather -> conserved sums -> new frame -> convergence test, wave exits
//      when every lane has converged), then re-projection onto the frame of
//      the gathered moments and BGK relaxation in Grad-coefficient space, and
//      the store of f*, g* and the frame into the other state buffer.
// The gather evaluates Eq. propagationInterpolated through linearity: the
// moments of the stencil nodes are interpolated at the departure point and the
// frame transformation is applied once to the interpolated moments, instead of
// transforming every stencil node first (the two agree to rounding).
#pragma once

#include "pond_tile.h"

namespace pond {
namespace lk {

constexpr int kBlock = 256;

inline unsigned grid_for(long long N) { return unsigned((N + kBlock - 1) / kBlock); }

template <typename P>
__device__ __forceinline__ P *plane(void *base, int i, long long N) {
    return static_cast<P *>(base) + (long long)i * N;
}
template <typename P>
__device__ __forceinline__ const P *plane(const void *base, int i, long long N) {
    return static_cast<const P *>(base) + (long long)i * N;
}

// ---------------------------------------------------------------- init ----
// Equilibrium in each node's own frame: f_i = rho w_i; g_i = g_i^eq of the split
// (total: lab velocity C_i; internal: C_i - u; non-translational: U'/rho only).
template <typename P, class L>
__global__ __launch_bounds__(kBlock) void init_kernel(StepArgs a, const double *__restrict__ rho,
                                                      const double *__restrict__ ux,
                                                      const double *__restrict__ uy,
                                                      const double *__restrict__ T, DevState st,
                                                      DevCounters *cnt) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    const double r = rho[n], vx = ux[n], vy = uy[n], t = T[n];
    const bool ok = (r > 0.0) && (t > 0.0) && isfinite(r) && isfinite(t) && isfinite(vx) &&
                    isfinite(vy);
    if (!ok) {
        atomicAdd(&cnt->init_rejected, 1ull);
        return;
    }
    const double s = sqrt(t);
    // total split: g^eq uses the lab velocity C_i; internal split: C_i - u
    const double ox = a.split ? 0.0 : vx, oy = a.split ? 0.0 : vy;
    const double kin = a.split == 2 ? 0.0 : 0.5;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double w = L::w(i / L::Q1) * L::w(i % L::Q1);
        const double Cx = s * L::c(i / L::Q1) + ox, Cy = s * L::c(i % L::Q1) + oy;
        plane<P>(st.f, i, a.N)[n] = P(r * w);
        plane<P>(st.g, i, a.N)[n] = P(w * (r * (a.cv - 1.0) * t + kin * r * (Cx * Cx + Cy * Cy)));
    }
    st.ux[n] = vx;
    st.uy[n] = vy;
    st.T[n] = t;
    if (st.uxp) {
        // internal split: a fresh state's frames stand in for the previous level
        st.uxp[n] = vx;
        st.uyp[n] = vy;
    }
}

// ---------------------------------------------------- moments pre-pass ----
template <typename P, class L>
__global__ __launch_bounds__(kBlock) void moments_kernel(StepArgs a, DevState st,
                                                         P *__restrict__ mom) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    node_moments<P, L>(a, st, mom, n);
}

// ----------------------------------------------------- step (global taps) ----
// Reference step kernel: one lane per node in row-major order, taps read
// straight from the HBM moment planes.
template <typename P, int NP, int S, class L>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs a, DevState src,
                                                      const P *__restrict__ mom, DevState dst,
                                                      P *__restrict__ mom_out, DevCounters *cnt) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = n < a.N;
    int x = 0, y = 0;
    double l0 = 0.0, l1 = 0.0, l2 = 1.0;
    if (live) {
        x = int(n % a.nx);
        y = int(n / a.nx);
        l0 = src.ux[n];
        l1 = src.uy[n];
        l2 = src.T[n];
    }
    GlobalTaps<P, NP, L> taps{mom, a.mstride, a.nx, a.ny, a.bc_x, a.bc_y, a.moff, a.wall_h, {}};
    load_moments<P, nmom<L>()>(mom, a.mstride, a.moff + ref_node(x, y, a.nx), taps.ref);
    node_step<P, NP, S, L>(a, taps, x, y, n, live, l0, l1, l2, src, dst, mom_out, cnt);
}

// ------------------------------------------------------ step (LDS tiles) ----

// Minimum waves per SIMD requested from the register allocator for the tiled
// kernel (compile-time tuning; 0 keeps the defaults of step_min_waves).
#ifndef POND_TILED_WAVES_PER_EU
#define POND_TILED_WAVES_PER_EU 0
#endif
#define POND_TILED_ATTR(P, S, NT, L)                                                     \
    __attribute__((amdgpu_waves_per_eu(POND_TILED_WAVES_PER_EU > 0 ? POND_TILED_WAVES_PER_EU \
                                                                   : step_min_waves<P, S, NT, L>())))

template <typename P, int NP, int S, class L, int TX, int TY>
__global__ __launch_bounds__(TX *TY) POND_TILED_ATTR(P, S, TX *TY, L) void step_tiled_kernel(StepArgs a, DevState src,
                                                            const P *__restrict__ mom,
                                                            DevState dst, P *__restrict__ mom_out,
                                                            DevCounters *cnt, int cap, int tiles_x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int red[4 * red_slots<TX * TY>()];
    int tx, ty;
    band_tile<TX>(xcd_tile(blockIdx.x, gridDim.x), tiles_x, int(gridDim.x) / tiles_x, tx, ty);
    tile_step<P, NP, S, L>(a, src, mom, dst, mom_out, cnt, reinterpret_cast<P *>(smem_raw), cap,
                           tx * TX, ty * TY, FixedShape<TX, TY>{}, red);
}

// ------------------------------------------------------ wall ghosts ----
// Moments of the ghost rows beyond the walls (bc_y == 2): one lane per ghost
// node (column x, depth j, wall).  The ghost at row -1 - j (bottom) or ny + j
// (top) mirrors interior row m = j or ny - 1 - j (clamped): frame
// u_g = (2 U_w - u_mx, -u_my), T_g = max(2 T_w - T_m, T_w / 4), density
// rho_g = rho_m T_m / T_g (the mirror's pressure), moments
// M_g = M_m + M^eq(rho_g, lam_g) - M^eq(rho_m, lam_m) for f and g (the
// equilibrium moments from the split's equilibrium populations), about u_ref.
template <typename P, class L>
__global__ __launch_bounds__(kBlock) void wall_ghost_kernel(StepArgs a, DevState st,
                                                            P *__restrict__ mom) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per_wall = (long long)a.wall_h * a.nx;
    if (t >= 2 * per_wall) return;
    const int side = t >= per_wall ? 1 : 0;
    const long long r = t - side * per_wall;
    const int j = int(r / a.nx), x = int(r % a.nx);
    int m = side == 0 ? j : a.ny - 1 - j;
    m = m < 0 ? 0 : (m > a.ny - 1 ? a.ny - 1 : m);
    const int gy = side == 0 ? -1 - j : a.ny + j;
    const long long nm = (long long)m * a.nx + x;
    constexpr int NM = L::NM;
    constexpr int NPAD = nmom_padded<P, L>();
    P Mm[NPAD];
    load_moments<P, nmom<L>()>(mom, a.mstride, a.moff + nm, Mm);
    const double um0 = st.ux[nm], um1 = st.uy[nm], Tm = st.T[nm];
    const double rho_m = double(Mm[0]);
    double Tg = 2.0 * a.wall_T[side] - Tm;
    if (Tg < 0.25 * a.wall_T[side]) Tg = 0.25 * a.wall_T[side];
    const double ug0 = 2.0 * a.wall_ux[side] - um0, ug1 = -um1;
    const double rho_g = rho_m * Tm / Tg;
    const double sm = sqrt(Tm), sg = sqrt(Tg);
    double D[2 * NM];
#pragma unroll
    for (int k = 0; k < 2 * NM; ++k) D[k] = 0.0;
    const double kin = a.split == 2 ? 0.0 : 0.5;
    // the kinetic part of g^eq: lab velocity C (total split), peculiar C - u
    // (internal split), none (non-translational split)
    const double uk = a.split == 1 ? 0.0 : 1.0;
    for (int i = 0; i < L::Q; ++i) {
        const double w = L::w(i / L::Q1) * L::w(i % L::Q1);
        const double cx = L::c(i / L::Q1), cy = L::c(i % L::Q1);
        // ghost and mirror equilibria: f^eq = rho w, g^eq of the split
        const double Cgx = sg * cx + ug0, Cgy = sg * cy + ug1;
        const double Cmx = sm * cx + um0, Cmy = sm * cy + um1;
        const double Kgx = sg * cx + uk * ug0, Kgy = sg * cy + uk * ug1;
        const double Kmx = sm * cx + uk * um0, Kmy = sm * cy + uk * um1;
        const double fg = rho_g * w, fm = rho_m * w;
        const double gg = w * (rho_g * (a.cv - 1.0) * Tg + kin * rho_g * (Kgx * Kgx + Kgy * Kgy));
        const double gm = w * (rho_m * (a.cv - 1.0) * Tm + kin * rho_m * (Kmx * Kmx + Kmy * Kmy));
        const double Vgx = Cgx - a.uref_x, Vgy = Cgy - a.uref_y;
        const double Vmx = Cmx - a.uref_x, Vmy = Cmy - a.uref_y;
#pragma unroll
        for (int k = 0; k < NM; ++k) {
            const int p = mom_px(k), q = mom_py(k);
            double mg = 1.0, mm = 1.0;
            for (int e = 0; e < p; ++e) {
                mg *= Vgx;
                mm *= Vmx;
            }
            for (int e = 0; e < q; ++e) {
                mg *= Vgy;
                mm *= Vmy;
            }
            D[k] += fg * mg - fm * mm;
            D[NM + k] += gg * mg - gm * mm;
        }
    }
    P Mg[NPAD];
#pragma unroll
    for (int k = 0; k < NPAD; ++k) Mg[k] = P(0);
#pragma unroll
    for (int k = 0; k < 2 * NM; ++k) Mg[k] = P(double(Mm[k]) + D[k]);
    store_moments<P, nmom<L>()>(mom, a.mstride, a.moff + (long long)gy * a.nx + x, Mg);
}

// ------------------------------------------------------ ghost band ----
// Walls (bc_y == 2): counts the nodes of a frame whose departure stencil
// (every velocity, the stencil of NP points per axis) reaches beyond the
// wall_h ghost rows on either side of the grid.
template <int NP, class L>
__global__ __launch_bounds__(kBlock) void ghost_check_kernel(StepArgs a, const double *__restrict__ uy,
                                                             const double *__restrict__ T,
                                                             DevCounters *cnt) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool out = false;
    if (n < a.N) {
        const int y = int(n / a.nx);
        int lo, hi;
        stencil_extent<NP, L>(y, uy[n], sqrt(fmax(T[n], 0.0)), lo, hi);
        out = lo < -a.wall_h || hi > a.ny - 1 + a.wall_h;
    }
    const unsigned long long c = wave_sum((unsigned long long)out);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&cnt->ghost_overrun, c);
}

// ------------------------------------------------------ macroscopic ----
template <typename P, class L>
__global__ __launch_bounds__(kBlock) void macro_kernel(StepArgs a, DevState st, double *rho,
                                                       double *ux, double *uy, double *T,
                                                       double *p) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    const double s = sqrt(st.T[n]), vx = st.ux[n], vy = st.uy[n];
    double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double fi = double(plane<P>(st.f, i, a.N)[n]);
        const double Cx = s * L::c(i / L::Q1) + vx, Cy = s * L::c(i % L::Q1) + vy;
        r += fi;
        jx += fi * Cx;
        jy += fi * Cy;
        E += double(plane<P>(st.g, i, a.N)[n]);
        if (a.split == 2) E += 0.5 * fi * (Cx * Cx + Cy * Cy);
    }
    const double t = (a.split == 1 ? E : E - (jx * jx + jy * jy) / (2.0 * r)) / (r * a.cv);
    if (rho) rho[n] = r;
    if (ux) ux[n] = jx / r;
    if (uy) uy[n] = jy / r;
    if (T) T[n] = t;
    if (p) p[n] = r * t;
}

template <typename P, class L>
__global__ __launch_bounds__(kBlock) void export_kernel(StepArgs a, DevState st, double *f,
                                                        double *g, double *frame) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        f[(long long)i * a.N + n] = double(plane<P>(st.f, i, a.N)[n]);
        g[(long long)i * a.N + n] = double(plane<P>(st.g, i, a.N)[n]);
    }
    frame[n] = st.ux[n];
    frame[a.N + n] = st.uy[n];
    frame[2 * a.N + n] = st.T[n];
}

template <typename P, class L>
__global__ __launch_bounds__(kBlock) void import_kernel(StepArgs a, const double *f,
                                                        const double *g, const double *frame,
                                                        DevState st) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        plane<P>(st.f, i, a.N)[n] = P(f[(long long)i * a.N + n]);
        plane<P>(st.g, i, a.N)[n] = P(g[(long long)i * a.N + n]);
    }
    st.ux[n] = frame[n];
    st.uy[n] = frame[a.N + n];
    st.T[n] = frame[2 * a.N + n];
    if (st.uxp) {
        // internal split: the imported frames stand in for the previous level
        // (pond_import_prev_frame may load that level afterwards)
        st.uxp[n] = frame[n];
        st.uyp[n] = frame[a.N + n];
    }
}

// per-block sums of (rho, rho ux, rho uy) over a fixed contiguous chunk
template <typename Loader>
__global__ __launch_bounds__(kBlock) void partial_sums_kernel(long long N, Loader ld,
                                                              double *scratch) {
    __shared__ double sh[3][kBlock];
    const long long chunk = (N + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < N ? lo + chunk : N;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (long long n = lo + threadIdx.x; n < hi; n += blockDim.x) {
        double r, jx, jy;
        ld(n, r, jx, jy);
        s0 += r;
        s1 += jx;
        s2 += jy;
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    sh[2][threadIdx.x] = s2;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) scratch[blockIdx.x * 3 + c] = sh[c][0];
}

template <typename P, class L>
struct StateLoader {
    DevState st;
    long long N;
    __device__ void operator()(long long n, double &r, double &jx, double &jy) const {
        const double s = sqrt(st.T[n]);
        r = jx = jy = 0.0;
        for (int i = 0; i < L::Q; ++i) {
            const double fi = double(static_cast<const P *>(st.f)[(long long)i * N + n]);
            r += fi;
            jx += fi * (s * L::c(i / L::Q1) + st.ux[n]);
            jy += fi * (s * L::c(i % L::Q1) + st.uy[n]);
        }
    }
};

template <typename P, int NP, int S, class L>
const void *tiled_kernel_ptr(TileShape shape) {
    switch (shape) {
    case TileShape::T16x16: return reinterpret_cast<const void *>(step_tiled_kernel<P, NP, S, L, 16, 16>);
    case TileShape::T32x8: return reinterpret_cast<const void *>(step_tiled_kernel<P, NP, S, L, 32, 8>);
    case TileShape::T16x8: return reinterpret_cast<const void *>(step_tiled_kernel<P, NP, S, L, 16, 8>);
    case TileShape::T8x8: return reinterpret_cast<const void *>(step_tiled_kernel<P, NP, S, L, 8, 8>);
    case TileShape::T256x1: return reinterpret_cast<const void *>(step_tiled_kernel<P, NP, S, L, 256, 1>);
    case TileShape::T64x1: return reinterpret_cast<const void *>(step_tiled_kernel<P, NP, S, L, 64, 1>);
    case TileShape::T32x16:
        if constexpr (L::Q == 16)
            return reinterpret_cast<const void *>(step_tiled_kernel<P, NP, S, L, 32, 16>);
        else
            return nullptr;
    }
    return nullptr;
}

template <typename P, int NP, int S, class L, int TX, int TY>
hipError_t launch_tiled_t(const StepArgs &a, const TileConfig &tc, DevState src, const P *mom,
                          DevState dst, P *mom_out, DevCounters *cnt, hipStream_t s) {
    auto kern = step_tiled_kernel<P, NP, S, L, TX, TY>;
    const size_t lds = size_t(tc.cap) * lds_stride<P, L>() * (16 / sizeof(P)) * sizeof(P);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    const int tiles_x = (a.nx + TX - 1) / TX, tiles_y = (a.ny + TY - 1) / TY;
    hipLaunchKernelGGL(kern, dim3(tiles_x * tiles_y), dim3(TX * TY), lds, s, a, src, mom, dst,
                       mom_out, cnt, tc.cap, tiles_x);
    return hipGetLastError();
}

template <typename P, int NP, int S, class L>
hipError_t launch_tiled_v(const StepArgs &a, const TileConfig &tc, DevState src, const P *mom,
                          DevState dst, P *mo, DevCounters *cnt, hipStream_t s) {
    switch (tc.shape) {
    case TileShape::T16x16: return launch_tiled_t<P, NP, S, L, 16, 16>(a, tc, src, mom, dst, mo, cnt, s);
    case TileShape::T32x8: return launch_tiled_t<P, NP, S, L, 32, 8>(a, tc, src, mom, dst, mo, cnt, s);
    case TileShape::T16x8: return launch_tiled_t<P, NP, S, L, 16, 8>(a, tc, src, mom, dst, mo, cnt, s);
    case TileShape::T8x8: return launch_tiled_t<P, NP, S, L, 8, 8>(a, tc, src, mom, dst, mo, cnt, s);
    case TileShape::T256x1: return launch_tiled_t<P, NP, S, L, 256, 1>(a, tc, src, mom, dst, mo, cnt, s);
    case TileShape::T64x1: return launch_tiled_t<P, NP, S, L, 64, 1>(a, tc, src, mom, dst, mo, cnt, s);
    case TileShape::T32x16:  // D2Q16 only (the host refuses it on D2Q25)
        if constexpr (L::Q == 16)
            return launch_tiled_t<P, NP, S, L, 32, 16>(a, tc, src, mom, dst, mo, cnt, s);
        else
            return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

}  // namespace lk

// Launchers of the lattice-dependent kernels for arithmetic type P on lattice L
// (the variants a lattice supports: with_lattice_variant).  The members are
// defined out of the class, so an explicit instantiation declaration keeps a
// translation unit from instantiating another lattice's kernels.
template <typename P, class L>
struct Launch {
    static hipError_t init(const StepArgs &a, const double *rho, const double *ux,
                           const double *uy, const double *T, DevState st, DevCounters *cnt,
                           hipStream_t s);
    static hipError_t moments(const StepArgs &a, DevState st, P *mom, hipStream_t s);
    static hipError_t wall_ghosts(const StepArgs &a, DevState st, P *mom, hipStream_t s);
    static hipError_t step(const StepArgs &a, DevState src, const P *mom, DevState dst,
                           P *mom_out, DevCounters *cnt, hipStream_t s);
    static hipError_t step_tiled(const StepArgs &a, const TileConfig &tc, DevState src,
                                 const P *mom, DevState dst, P *mom_out, DevCounters *cnt,
                                 hipStream_t s);
    static hipError_t macro(const StepArgs &a, DevState st, double *rho, double *ux, double *uy,
                            double *T, double *p, hipStream_t s);
    static hipError_t exp(const StepArgs &a, DevState st, double *f, double *g, double *frame,
                          hipStream_t s);
    static hipError_t imp(const StepArgs &a, const double *f, const double *g, const double *frame,
                          DevState st, hipStream_t s);
    // per-block (rho, j) sums of a state into scratch[3 * nblocks]
    static hipError_t state_partial_sums(const StepArgs &a, DevState st, double *scratch,
                                         int nblocks, hipStream_t s);
    static int tiled_blocks_per_cu(int np, int split, TileShape shape);
    static hipError_t ghost_check(const StepArgs &a, DevState st, DevCounters *cnt, hipStream_t s);
};

template <typename P, class L>
hipError_t Launch<P, L>::init(const StepArgs &a, const double *rho, const double *ux,
                              const double *uy, const double *T, DevState st, DevCounters *cnt,
                              hipStream_t s) {
    hipLaunchKernelGGL((lk::init_kernel<P, L>), dim3(lk::grid_for(a.N)), dim3(lk::kBlock), 0, s,
                       a, rho, ux, uy, T, st, cnt);
    return hipGetLastError();
}

template <typename P, class L>
hipError_t Launch<P, L>::moments(const StepArgs &a, DevState st, P *mom, hipStream_t s) {
    hipLaunchKernelGGL((lk::moments_kernel<P, L>), dim3(lk::grid_for(a.N)), dim3(lk::kBlock), 0,
                       s, a, st, mom);
    return hipGetLastError();
}

template <typename P, class L>
hipError_t Launch<P, L>::wall_ghosts(const StepArgs &a, DevState st, P *mom, hipStream_t s) {
    const long long n = 2LL * a.wall_h * a.nx;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((lk::wall_ghost_kernel<P, L>), dim3(lk::grid_for(n)), dim3(lk::kBlock), 0,
                       s, a, st, mom);
    return hipGetLastError();
}

template <typename P, class L>
hipError_t Launch<P, L>::step(const StepArgs &a, DevState src, const P *mom, DevState dst,
                              P *mom_out, DevCounters *cnt, hipStream_t s) {
    return with_lattice_variant<L>(a.interp_points, a.split, [&](auto np, auto sp) {
        hipLaunchKernelGGL((lk::step_kernel<P, np(), sp(), L>), dim3(lk::grid_for(a.N)),
                           dim3(lk::kBlock), 0, s, a, src, mom, dst, mom_out, cnt);
        return hipGetLastError();
    });
}

template <typename P, class L>
hipError_t Launch<P, L>::step_tiled(const StepArgs &a, const TileConfig &tc, DevState src,
                                    const P *mom, DevState dst, P *mom_out, DevCounters *cnt,
                                    hipStream_t s) {
    return with_lattice_variant<L>(a.interp_points, a.split, [&](auto np, auto sp) {
        return lk::launch_tiled_v<P, np(), sp(), L>(a, tc, src, mom, dst, mom_out, cnt, s);
    });
}

template <typename P, class L>
hipError_t Launch<P, L>::macro(const StepArgs &a, DevState st, double *rho, double *ux,
                               double *uy, double *T, double *p, hipStream_t s) {
    hipLaunchKernelGGL((lk::macro_kernel<P, L>), dim3(lk::grid_for(a.N)), dim3(lk::kBlock), 0, s,
                       a, st, rho, ux, uy, T, p);
    return hipGetLastError();
}

template <typename P, class L>
hipError_t Launch<P, L>::exp(const StepArgs &a, DevState st, double *f, double *g, double *frame,
                             hipStream_t s) {
    hipLaunchKernelGGL((lk::export_kernel<P, L>), dim3(lk::grid_for(a.N)), dim3(lk::kBlock), 0, s,
                       a, st, f, g, frame);
    return hipGetLastError();
}

template <typename P, class L>
hipError_t Launch<P, L>::imp(const StepArgs &a, const double *f, const double *g,
                             const double *frame, DevState st, hipStream_t s) {
    hipLaunchKernelGGL((lk::import_kernel<P, L>), dim3(lk::grid_for(a.N)), dim3(lk::kBlock), 0, s,
                       a, f, g, frame, st);
    return hipGetLastError();
}

template <typename P, class L>
hipError_t Launch<P, L>::state_partial_sums(const StepArgs &a, DevState st, double *scratch,
                                            int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((lk::partial_sums_kernel<lk::StateLoader<P, L>>), dim3(nblocks),
                       dim3(lk::kBlock), 0, s, a.N, lk::StateLoader<P, L>{st, a.N}, scratch);
    return hipGetLastError();
}

template <typename P, class L>
hipError_t Launch<P, L>::ghost_check(const StepArgs &a, DevState st, DevCounters *cnt,
                                     hipStream_t s) {
    return with_lattice_variant<L>(a.interp_points, a.split, [&](auto np, auto) {
        hipLaunchKernelGGL((lk::ghost_check_kernel<np(), L>), dim3(lk::grid_for(a.N)),
                           dim3(lk::kBlock), 0, s, a, st.uy, st.T, cnt);
        return hipGetLastError();
    });
}

template <typename P, class L>
int Launch<P, L>::tiled_blocks_per_cu(int np, int split, TileShape shape) {
    const void *k = with_lattice_variant<L>(np, split, [&](auto n, auto sp) {
        return lk::tiled_kernel_ptr<P, n(), sp(), L>(shape);
    });
    int tx = 0, ty = 0;
    tile_dims(shape, tx, ty);
    int n = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, tx * ty, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n < 1 ? 1 : n;
}

}  // namespace pond
