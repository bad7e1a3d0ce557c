// pond_kernels.hip -- HIP kernels of the PonD f+g step for gfx950 (MI355X).
//
// One kernel source, instantiated for P = double (FP64 mode) and P = float
// (FP32 mode: populations, moments, interpolation and frame transformation in
// float; conserved sums, temperature recovery and the predictor-corrector test
// in double).
//
// Step = two launches on one stream:
//   1. moments pre-pass: per node, the 10 + 10 moments up to order three of f
//      and g (Eq. genericMomentUptoO3) about the instance's reference velocity,
//      written as 20 planes;
//   2. step: per destination node (one lane), the predictor-corrector loop
//      (gather -> conserved sums -> new frame -> convergence test, wave exits
//      when every lane has converged), then re-projection onto the frame of
//      the gathered moments and BGK relaxation in Grad-coefficient space, and
//      the store of f*, g* and the frame into the other state buffer.
// The gather evaluates Eq. propagationInterpolated through linearity: the
// moments of the stencil nodes are interpolated at the departure point and the
// frame transformation is applied once to the interpolated moments, instead of
// transforming every stencil node first (the two agree to rounding).
#include <utility>

#include "pond_device.h"
#include "pond_internal.h"

namespace pond {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename P>
__device__ __forceinline__ P *plane(void *base, int i, long long N) {
    return static_cast<P *>(base) + (long long)i * N;
}
template <typename P>
__device__ __forceinline__ const P *plane(const void *base, int i, long long N) {
    return static_cast<const P *>(base) + (long long)i * N;
}

// ---------------------------------------------------------------- init ----
template <typename P>
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
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const double w = w1(i / 4) * w1(i % 4);
        const double Cx = s * c1(i / 4) + vx, Cy = s * c1(i % 4) + vy;
        plane<P>(st.f, i, a.N)[n] = P(r * w);
        plane<P>(st.g, i, a.N)[n] = P(w * (r * (a.cv - 1.0) * t + 0.5 * r * (Cx * Cx + Cy * Cy)));
    }
    st.ux[n] = vx;
    st.uy[n] = vy;
    st.T[n] = t;
}

// ---------------------------------------------------- moments pre-pass ----
template <typename P>
__global__ __launch_bounds__(kBlock) void moments_kernel(StepArgs a, DevState st,
                                                         P *__restrict__ mom) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    const P s = P(sqrt(st.T[n]));
    const P dx = P(st.ux[n] - a.uref_x), dy = P(st.uy[n] - a.uref_y);
    P Mf[kNM], Mg[kNM];
#pragma unroll
    for (int k = 0; k < kNM; ++k) Mf[k] = Mg[k] = P(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const P fi = plane<P>(st.f, i, a.N)[n];
        const P gi = plane<P>(st.g, i, a.N)[n];
        const P Vx = s * P(c1(i / 4)) + dx, Vy = s * P(c1(i % 4)) + dy;
        const P mono[kNM] = {P(1),         Vx,          Vy,          Vx * Vx,     Vx * Vy,
                             Vy * Vy,      Vx * Vx * Vx, Vx * Vx * Vy, Vx * Vy * Vy, Vy * Vy * Vy};
#pragma unroll
        for (int k = 0; k < kNM; ++k) {
            Mf[k] += fi * mono[k];
            Mg[k] += gi * mono[k];
        }
    }
#pragma unroll
    for (int k = 0; k < kNM; ++k) {
        mom[(long long)k * a.N + n] = Mf[k];
        mom[(long long)(kNM + k) * a.N + n] = Mg[k];
    }
}

// ---------------------------------------------------------------- step ----
// Per-iteration gather geometry of one lane: interpolation weights and node
// offsets of the NP-point stencils along x (per a) and y (per b).
template <typename P, int NP>
struct Stencil {
    P wx[4][NP], wy[4][NP];
    int col[4][NP];   // x index
    int row[4][NP];   // y index * nx
};

template <typename P, int NP, int I>
__device__ __forceinline__ void gather_velocity(const StepArgs &a, const P *__restrict__ mom,
                                                const Stencil<P, NP> &S, P dux, P duy, P is,
                                                P *ft, P *gt) {
    constexpr int A = I / 4, B = I % 4;
    P Mf[kNM], Mg[kNM];
#pragma unroll
    for (int k = 0; k < kNM; ++k) Mf[k] = Mg[k] = P(0);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const P W = S.wx[A][p] * S.wy[B][q];
            const long long idx = (long long)S.row[B][q] + S.col[A][p];
#pragma unroll
            for (int k = 0; k < kNM; ++k) {
                Mf[k] += W * mom[(long long)k * a.N + idx];
                Mg[k] += W * mom[(long long)(kNM + k) * a.N + idx];
            }
        }
    }
    P m[kNM];
    central_normalised(Mf, dux, duy, is, m);
    ft[I] = pop_from_central<P, A, B>(m);
    central_normalised(Mg, dux, duy, is, m);
    gt[I] = pop_from_central<P, A, B>(m);
}

template <typename P, int NP, int... Is>
__device__ __forceinline__ void gather_all(std::integer_sequence<int, Is...>, const StepArgs &a,
                                           const P *__restrict__ mom, const Stencil<P, NP> &S,
                                           P dux, P duy, P is, P *ft, P *gt) {
    (gather_velocity<P, NP, Is>(a, mom, S, dux, duy, is, ft, gt), ...);
}

template <typename P, int I>
__device__ __forceinline__ void store_velocity(const StepArgs &a, DevState dst, long long n,
                                               const P *af, const P *ag, bool bad) {
    constexpr int A = I / 4, B = I % 4;
    P fv = pop_from_hermite<P, A, B>(af);
    P gv = pop_from_hermite<P, A, B>(ag);
    if (bad) fv = gv = P(NAN);
    plane<P>(dst.f, I, a.N)[n] = fv;
    plane<P>(dst.g, I, a.N)[n] = gv;
}

template <typename P, int... Is>
__device__ __forceinline__ void store_all(std::integer_sequence<int, Is...>, const StepArgs &a,
                                          DevState dst, long long n, const P *af, const P *ag,
                                          bool bad) {
    (store_velocity<P, Is>(a, dst, n, af, ag, bad), ...);
}

template <typename P, int NP>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs a, DevState src,
                                                      const P *__restrict__ mom, DevState dst,
                                                      DevCounters *cnt) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = n < a.N;
    int x = 0, y = 0;
    double lg0 = 0.0, lg1 = 0.0, lg2 = 1.0;  // frame of the current gather
    if (live) {
        x = int(n % a.nx);
        y = int(n / a.nx);
        lg0 = src.ux[n];
        lg1 = src.uy[n];
        lg2 = src.T[n];
    }
    double ln0 = lg0, ln1 = lg1, ln2 = lg2;  // frame of the gathered moments
    double rho = 1.0;
    P ft[kQ], gt[kQ];
    bool done = !live, conv = false, bad = false;
    int used = 0;
    Stencil<P, NP> S;

    for (int k = 0; k < a.pc_max_iter; ++k) {
        if (!done) {
            const double s = sqrt(lg2);
            // departure points y_i = x - C_i(lam_bar) dt, split per axis
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double dep_x = double(x) - (s * c1(c) + lg0);
                const double dep_y = double(y) - (s * c1(c) + lg1);
                const int bx = lagrange<NP>(dep_x, S.wx[c]);
                const int by = lagrange<NP>(dep_y, S.wy[c]);
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    S.col[c][j] = wrap_index(bx + j, a.nx, a.bc_x);
                    S.row[c][j] = wrap_index(by + j, a.ny, a.bc_y) * a.nx;
                }
            }
            const P dux = P(lg0 - a.uref_x), duy = P(lg1 - a.uref_y), is = P(1.0 / s);
            gather_all<P, NP>(std::make_integer_sequence<int, kQ>{}, a, mom, S, dux, duy, is, ft, gt);

            // conserved moments (FP64) and the frame they imply
            double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const double fi = double(ft[i]);
                r += fi;
                jx += fi * (s * c1(i / 4) + lg0);
                jy += fi * (s * c1(i % 4) + lg1);
                E += double(gt[i]);
            }
            rho = r;
            ln0 = jx / r;
            ln1 = jy / r;
            ln2 = (E - (jx * jx + jy * jy) / (2.0 * r)) / (r * a.cv);
            used = k + 1;
            if (!(r > 0.0) || !(ln2 > 0.0) || !isfinite(ln0) || !isfinite(ln1) || !isfinite(ln2) ||
                !isfinite(E)) {
                bad = true;
                done = true;
            } else {
                const double du = fmax(fabs(ln0 - lg0), fabs(ln1 - lg1)) / sqrt(ln2);
                const double dT = fabs(ln2 - lg2) / ln2;
                if (fmax(du, dT) <= a.pc_tol) {
                    conv = true;
                    done = true;
                } else if (k + 1 < a.pc_max_iter) {
                    lg0 = ln0;
                    lg1 = ln1;
                    lg2 = ln2;
                }
            }
        }
        if (__all(done)) break;  // wave-uniform exit once every lane has converged
    }

    if (live) {
        // lab moments of the gathered populations (frame lg) about u_ref
        const P s = P(sqrt(lg2));
        const P dx = P(lg0 - a.uref_x), dy = P(lg1 - a.uref_y);
        P Mf[kNM], Mg[kNM];
#pragma unroll
        for (int k = 0; k < kNM; ++k) Mf[k] = Mg[k] = P(0);
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const P Vx = s * P(c1(i / 4)) + dx, Vy = s * P(c1(i % 4)) + dy;
            const P mono[kNM] = {P(1),        Vx,           Vy,           Vx * Vx,      Vx * Vy,
                                 Vy * Vy,     Vx * Vx * Vx, Vx * Vx * Vy, Vx * Vy * Vy, Vy * Vy * Vy};
#pragma unroll
            for (int k = 0; k < kNM; ++k) {
                Mf[k] += ft[i] * mono[k];
                Mg[k] += gt[i] * mono[k];
            }
        }
        // re-projection onto lam* = (ln0, ln1, ln2): Grad coefficients there
        const double sT = sqrt(ln2);
        const P is = P(1.0 / sT);
        const P tx = P(ln0 - a.uref_x), ty = P(ln1 - a.uref_y);
        P m[kNM], af[kNM], ag[kNM];
        central_normalised(Mf, tx, ty, is, m);
        hermite_from_central(m, af);
        central_normalised(Mg, tx, ty, is, m);
        hermite_from_central(m, ag);

        // BGK collision in lam*, on the Grad coefficients.
        // f: f^eq = rho w_i has only a0; every higher coefficient decays by (1 - omega).
        // g: g^eq = w_i [rho (c_v - 1) T + rho |C_i|^2 / 2] has
        //    a0 = rho c_v T + rho |u|^2 / 2, a1 = rho sqrt(T) u, a2 = rho T I, a3 = 0.
        const double om = a.omega;
        double geq[kNM];
        geq[0] = rho * (a.cv - 1.0) * ln2 + 0.5 * rho * (2.0 * ln2 + ln0 * ln0 + ln1 * ln1);
        geq[1] = rho * sT * ln0;
        geq[2] = rho * sT * ln1;
        geq[3] = rho * ln2;
        geq[4] = 0.0;
        geq[5] = rho * ln2;
        geq[6] = geq[7] = geq[8] = geq[9] = 0.0;
        if (a.unit_prandtl) {
#pragma unroll
            for (int k = 0; k < kNM; ++k) ag[k] = ag[k] + P(om) * (P(geq[k]) - ag[k]);
        } else {
            // quasi-equilibrium: energy flux of g^eq plus the viscous heating u . P^neq,
            // P^neq = T a2(f) + sqrt(T) (u a1(f) + a1(f) u) in lam*.
            const double a1x = double(af[1]), a1y = double(af[2]);
            const double Pxx = ln2 * double(af[3]) + sT * 2.0 * ln0 * a1x;
            const double Pxy = ln2 * double(af[4]) + sT * (ln0 * a1y + a1x * ln1);
            const double Pyy = ln2 * double(af[5]) + sT * 2.0 * ln1 * a1y;
            const double dqx = ln0 * Pxx + ln1 * Pxy;
            const double dqy = ln0 * Pxy + ln1 * Pyy;
            double gqe[kNM];
#pragma unroll
            for (int k = 0; k < kNM; ++k) gqe[k] = geq[k];
            gqe[1] += dqx / sT;
            gqe[2] += dqy / sT;
            const double om1 = a.omega1;
#pragma unroll
            for (int k = 0; k < kNM; ++k)
                ag[k] = ag[k] + P(om1) * (P(gqe[k]) - ag[k]) + P(om) * (P(geq[k]) - P(gqe[k]));
        }
        const P decay = P(1.0 - om);
#pragma unroll
        for (int k = 1; k < kNM; ++k) af[k] *= decay;

        store_all<P>(std::make_integer_sequence<int, kQ>{}, a, dst, n, af, ag, bad);
        dst.ux[n] = bad ? NAN : ln0;
        dst.uy[n] = bad ? NAN : ln1;
        dst.T[n] = bad ? NAN : ln2;
    }

    // counters: one atomic per wave
    const unsigned long long it = wave_sum((unsigned long long)used);
    const unsigned long long nc = wave_sum((unsigned long long)(live && !conv && !bad));
    const unsigned long long nb = wave_sum((unsigned long long)(live && bad));
    if ((threadIdx.x & 63) == 0) {
        if (it) atomicAdd(&cnt->pc_iterations, it);
        if (nc) atomicAdd(&cnt->nonconverged, nc);
        if (nb) atomicAdd(&cnt->nonphysical, nb);
    }
}

// ------------------------------------------------------ macroscopic ----
template <typename P>
__global__ __launch_bounds__(kBlock) void macro_kernel(StepArgs a, DevState st, double *rho,
                                                       double *ux, double *uy, double *T,
                                                       double *p) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    const double s = sqrt(st.T[n]), vx = st.ux[n], vy = st.uy[n];
    double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const double fi = double(plane<P>(st.f, i, a.N)[n]);
        r += fi;
        jx += fi * (s * c1(i / 4) + vx);
        jy += fi * (s * c1(i % 4) + vy);
        E += double(plane<P>(st.g, i, a.N)[n]);
    }
    const double t = (E - (jx * jx + jy * jy) / (2.0 * r)) / (r * a.cv);
    if (rho) rho[n] = r;
    if (ux) ux[n] = jx / r;
    if (uy) uy[n] = jy / r;
    if (T) T[n] = t;
    if (p) p[n] = r * t;
}

template <typename P>
__global__ __launch_bounds__(kBlock) void export_kernel(StepArgs a, DevState st, double *f,
                                                        double *g, double *frame) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        f[(long long)i * a.N + n] = double(plane<P>(st.f, i, a.N)[n]);
        g[(long long)i * a.N + n] = double(plane<P>(st.g, i, a.N)[n]);
    }
    frame[n] = st.ux[n];
    frame[a.N + n] = st.uy[n];
    frame[2 * a.N + n] = st.T[n];
}

template <typename P>
__global__ __launch_bounds__(kBlock) void import_kernel(StepArgs a, const double *f,
                                                        const double *g, const double *frame,
                                                        DevState st) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        plane<P>(st.f, i, a.N)[n] = P(f[(long long)i * a.N + n]);
        plane<P>(st.g, i, a.N)[n] = P(g[(long long)i * a.N + n]);
    }
    st.ux[n] = frame[n];
    st.uy[n] = frame[a.N + n];
    st.T[n] = frame[2 * a.N + n];
}

// ------------------------------------------- deterministic reductions ----
constexpr int kRedBlocks = 256;

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

struct FieldLoader {
    const double *rho, *ux, *uy;
    __device__ void operator()(long long n, double &r, double &jx, double &jy) const {
        r = rho[n];
        jx = rho[n] * ux[n];
        jy = rho[n] * uy[n];
    }
};

template <typename P>
struct StateLoader {
    DevState st;
    long long N;
    __device__ void operator()(long long n, double &r, double &jx, double &jy) const {
        const double s = sqrt(st.T[n]);
        r = jx = jy = 0.0;
        for (int i = 0; i < kQ; ++i) {
            const double fi = double(static_cast<const P *>(st.f)[(long long)i * N + n]);
            r += fi;
            jx += fi * (s * c1(i / 4) + st.ux[n]);
            jy += fi * (s * c1(i % 4) + st.uy[n]);
        }
    }
};

unsigned grid_for(long long N) { return unsigned((N + kBlock - 1) / kBlock); }

}  // namespace

template <typename P>
hipError_t launch_init(const StepArgs &a, const double *rho, const double *ux, const double *uy,
                       const double *T, DevState st, DevCounters *cnt, hipStream_t s) {
    hipLaunchKernelGGL(init_kernel<P>, dim3(grid_for(a.N)), dim3(kBlock), 0, s, a, rho, ux, uy, T,
                       st, cnt);
    return hipGetLastError();
}

template <typename P>
hipError_t launch_moments_prepass(const StepArgs &a, DevState st, P *mom, hipStream_t s) {
    hipLaunchKernelGGL(moments_kernel<P>, dim3(grid_for(a.N)), dim3(kBlock), 0, s, a, st, mom);
    return hipGetLastError();
}

template <typename P>
hipError_t launch_step(const StepArgs &a, DevState src, const P *mom, DevState dst,
                       DevCounters *cnt, hipStream_t s) {
    if (a.interp_points == 3)
        hipLaunchKernelGGL((step_kernel<P, 3>), dim3(grid_for(a.N)), dim3(kBlock), 0, s, a, src,
                           mom, dst, cnt);
    else
        hipLaunchKernelGGL((step_kernel<P, 4>), dim3(grid_for(a.N)), dim3(kBlock), 0, s, a, src,
                           mom, dst, cnt);
    return hipGetLastError();
}

template <typename P>
hipError_t launch_macro(const StepArgs &a, DevState st, double *rho, double *ux, double *uy,
                        double *T, double *p, hipStream_t s) {
    hipLaunchKernelGGL(macro_kernel<P>, dim3(grid_for(a.N)), dim3(kBlock), 0, s, a, st, rho, ux,
                       uy, T, p);
    return hipGetLastError();
}

template <typename P>
hipError_t launch_export(const StepArgs &a, DevState st, double *f, double *g, double *frame,
                         hipStream_t s) {
    hipLaunchKernelGGL(export_kernel<P>, dim3(grid_for(a.N)), dim3(kBlock), 0, s, a, st, f, g,
                       frame);
    return hipGetLastError();
}

template <typename P>
hipError_t launch_import(const StepArgs &a, const double *f, const double *g, const double *frame,
                         DevState st, hipStream_t s) {
    hipLaunchKernelGGL(import_kernel<P>, dim3(grid_for(a.N)), dim3(kBlock), 0, s, a, f, g, frame,
                       st);
    return hipGetLastError();
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

template <typename P>
hipError_t launch_state_mean_velocity(const StepArgs &a, DevState st, double *scratch,
                                      int scratch_len, DevCounters *cnt, hipStream_t s) {
    if (scratch_len < 3 * kRedBlocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(partial_sums_kernel<StateLoader<P>>, dim3(kRedBlocks), dim3(kBlock), 0, s,
                       a.N, StateLoader<P>{st, a.N}, scratch);
    hipLaunchKernelGGL(final_sums_kernel, dim3(1), dim3(64), 0, s, scratch, kRedBlocks, cnt);
    return hipGetLastError();
}

#define POND_INSTANTIATE(P)                                                                        \
    template hipError_t launch_init<P>(const StepArgs &, const double *, const double *,           \
                                       const double *, const double *, DevState, DevCounters *,    \
                                       hipStream_t);                                               \
    template hipError_t launch_moments_prepass<P>(const StepArgs &, DevState, P *, hipStream_t);   \
    template hipError_t launch_step<P>(const StepArgs &, DevState, const P *, DevState,            \
                                       DevCounters *, hipStream_t);                                \
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
