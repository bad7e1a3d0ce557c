// pond_step_common.h -- per-node body of the PonD step shared by the step
// kernels: departure stencils, the predictor-corrector loop over a tap source,
// re-projection, collision in Grad-coefficient space and the store.
//
// Moment storage ("grouped planes"): the 2 NM moments of a node (f moments
// 0..NM-1, g moments NM..2NM-1, ordering of pond_device.h; NM = 10 on D2Q16,
// 15 on D2Q25) are held as G vector groups (float: float4, the last padded;
// double: double2); in the HBM moment planes group k of node idx sits at
// base[k * stride + idx] (stride = nodes per plane: lanes of a wave read
// consecutive vectors); the LDS tiles hold a node's groups contiguously
// (lds_stride below).
#pragma once

#include <utility>

// Stencil rows interpolated per loop trip in the HBM tap gather.
#ifndef POND_ROW_UNROLL
#define POND_ROW_UNROLL 1
#endif

#include "pond_device.h"
#include "pond_internal.h"

namespace pond {

template <typename P, int NMOM>
struct MomVec;
template <int NMOM>
struct MomVec<float, NMOM> {
    using V = float4;
    static constexpr int W = 4;
    static constexpr int G = (NMOM + 3) / 4;
};
template <int NMOM>
struct MomVec<double, NMOM> {
    using V = double2;
    static constexpr int W = 2;
    static constexpr int G = (NMOM + 1) / 2;
};

constexpr int kNMom = 2 * kNM;  // 20 moments per node on D2Q16

// Moments per node of a lattice, and the values a node's groups hold (padded).
template <class L>
constexpr int nmom() { return 2 * L::NM; }
template <typename P, class L>
constexpr int nmom_padded() {
    return MomVec<P, nmom<L>()>::G * MomVec<P, nmom<L>()>::W;
}

template <typename P, int NMOM = kNMom>
__device__ __forceinline__ void load_moments(const P *__restrict__ base, long long stride,
                                             long long idx, P *M) {
    using MV = MomVec<P, NMOM>;
    using V = typename MV::V;
    const V *b = reinterpret_cast<const V *>(base);
    if constexpr (MV::W == 4) {
#pragma unroll
        for (int k = 0; k < MV::G; ++k) {
            const V v = b[k * stride + idx];
            M[4 * k] = v.x;
            M[4 * k + 1] = v.y;
            M[4 * k + 2] = v.z;
            M[4 * k + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < MV::G; ++k) {
            const V v = b[k * stride + idx];
            M[2 * k] = v.x;
            M[2 * k + 1] = v.y;
        }
    }
}

// Stores of the step's outputs in HBM.  This step never reads what it writes,
// so they may stream past the caches (non-temporal stores), leaving L2 to the
// halo moments that neighbouring tiles re-read.  POND_STREAM_STORE is a mask
// of the streams stored that way: 1 the populations, 2 the frame, 4 the
// moment planes.  Off by default: on the 2048^2 quadrants streaming the moment
// planes (and the frame) cut the read bytes by 3 % (7.5 %) at the same step
// time, and streamed population stores (one dword per lane) raised the written
// bytes by half and slowed the step.
#ifndef POND_STREAM_STORE
#define POND_STREAM_STORE 0
#endif
typedef float pond_f4v __attribute__((ext_vector_type(4)));
typedef double pond_d2v __attribute__((ext_vector_type(2)));

template <int Stream, typename T>
__device__ __forceinline__ void out_store(T *p, T v) {
    if constexpr ((POND_STREAM_STORE & Stream) != 0)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
template <int Stream>
__device__ __forceinline__ void out_store(float4 *p, float4 v) {
    if constexpr ((POND_STREAM_STORE & Stream) != 0)
        __builtin_nontemporal_store(pond_f4v{v.x, v.y, v.z, v.w}, reinterpret_cast<pond_f4v *>(p));
    else
        *p = v;
}
template <int Stream>
__device__ __forceinline__ void out_store(double2 *p, double2 v) {
    if constexpr ((POND_STREAM_STORE & Stream) != 0)
        __builtin_nontemporal_store(pond_d2v{v.x, v.y}, reinterpret_cast<pond_d2v *>(p));
    else
        *p = v;
}
constexpr int kStreamPops = 1, kStreamFrame = 2, kStreamMoments = 4;

template <typename P, int NMOM = kNMom>
__device__ __forceinline__ void store_moments_out(P *__restrict__ base, long long stride,
                                                  long long idx, const P *M) {
    using MV = MomVec<P, NMOM>;
    using V = typename MV::V;
    V *b = reinterpret_cast<V *>(base);
    if constexpr (MV::W == 4) {
#pragma unroll
        for (int k = 0; k < MV::G; ++k)
            out_store<kStreamMoments>(&b[k * stride + idx],
                                      V{M[4 * k], M[4 * k + 1], M[4 * k + 2], M[4 * k + 3]});
    } else {
#pragma unroll
        for (int k = 0; k < MV::G; ++k) out_store<kStreamMoments>(&b[k * stride + idx], V{M[2 * k], M[2 * k + 1]});
    }
}

template <typename P, int NMOM = kNMom>
__device__ __forceinline__ void store_moments(P *__restrict__ base, long long stride,
                                              long long idx, const P *M) {
    using MV = MomVec<P, NMOM>;
    using V = typename MV::V;
    V *b = reinterpret_cast<V *>(base);
    if constexpr (MV::W == 4) {
#pragma unroll
        for (int k = 0; k < MV::G; ++k)
            b[k * stride + idx] = V{M[4 * k], M[4 * k + 1], M[4 * k + 2], M[4 * k + 3]};
    } else {
#pragma unroll
        for (int k = 0; k < MV::G; ++k) b[k * stride + idx] = V{M[2 * k], M[2 * k + 1]};
    }
}

// LDS tiles of the FP32 D2Q16 kernels hold the moment groups of a node
// contiguously (node-major, 5 float4 = 80 B per node), so every tap and group of
// a stencil row is reached from one address with immediate offsets; lanes
// reading neighbouring nodes then touch disjoint banks (a stride of 20 banks).
// The per-velocity gather (FP64, D2Q25) stages the region as grouped planes
// instead: group k of staged node idx at vector k * cap + idx, so the lanes of
// a wave, which read neighbouring nodes, read neighbouring vectors.  Node-major
// tiles of those variants either share banks between lanes (D2Q25 FP32, 128 B
// per node: 161 against 495 MLUPS on the 512^2 Mach-2 modes) or, padded by a
// group against that, hold fewer nodes (365 MLUPS; FP64 D2Q16 at 512^2: 528
// against 657).  The staged values are the same in either layout, only their
// addresses differ.
template <typename P, class L>
constexpr bool lds_planar() {
    return !(sizeof(P) == 4 && L::Q == 16);
}

// Vectors (float4 / double2) per node of the LDS array: the node's groups.
template <typename P, class L>
constexpr int lds_stride() {
    return MomVec<P, nmom<L>()>::G;
}

// Bytes of one node in the LDS array.
template <typename P, class L>
constexpr unsigned lds_node_bytes() {
    return unsigned(lds_stride<P, L>() * sizeof(typename MomVec<P, nmom<L>()>::V));
}

template <typename P, class L>
__device__ __forceinline__ void load_node_lds(const P *lds, int idx, P *M) {
    using MV = MomVec<P, nmom<L>()>;
    using V = typename MV::V;
    const V *b = reinterpret_cast<const V *>(lds) + idx * lds_stride<P, L>();
#pragma unroll
    for (int k = 0; k < MV::G; ++k) {
        const V v = b[k];
        if constexpr (MV::W == 4) {
            M[4 * k] = v.x;
            M[4 * k + 1] = v.y;
            M[4 * k + 2] = v.z;
            M[4 * k + 3] = v.w;
        } else {
            M[2 * k] = v.x;
            M[2 * k + 1] = v.y;
        }
    }
}

// The same from the node's byte offset in the LDS array.
template <typename P, class L>
__device__ __forceinline__ void load_node_lds_at(const P *lds, unsigned off, P *M) {
    using MV = MomVec<P, nmom<L>()>;
    using V = typename MV::V;
    const V *b = reinterpret_cast<const V *>(reinterpret_cast<const char *>(lds) + off);
#pragma unroll
    for (int k = 0; k < MV::G; ++k) {
        const V v = b[k];
        if constexpr (MV::W == 4) {
            M[4 * k] = v.x;
            M[4 * k + 1] = v.y;
            M[4 * k + 2] = v.z;
            M[4 * k + 3] = v.w;
        } else {
            M[2 * k] = v.x;
            M[2 * k + 1] = v.y;
        }
    }
}

template <typename P, class L>
__device__ __forceinline__ void store_node_lds(P *lds, int idx, int cap, const P *M) {
    if constexpr (lds_planar<P, L>()) {
        store_moments<P, nmom<L>()>(lds, cap, idx, M);
        return;
    }
    using MV = MomVec<P, nmom<L>()>;
    using V = typename MV::V;
    V *b = reinterpret_cast<V *>(lds) + idx * lds_stride<P, L>();
#pragma unroll
    for (int k = 0; k < MV::G; ++k) {
        if constexpr (MV::W == 4)
            b[k] = V{M[4 * k], M[4 * k + 1], M[4 * k + 2], M[4 * k + 3]};
        else
            b[k] = V{M[2 * k], M[2 * k + 1]};
    }
}

template <typename P>
__device__ __forceinline__ P *pop_plane(void *base, int i, long long N) {
    return static_cast<P *>(base) + (long long)i * N;
}
template <typename P>
__device__ __forceinline__ const P *pop_plane(const void *base, int i, long long N) {
    return static_cast<const P *>(base) + (long long)i * N;
}

static __constant__ VelocityTablesP<float> kTabF = make_velocity_tables_p<float>();
static __constant__ VelocityTablesP<double> kTabD = make_velocity_tables_p<double>();
static __constant__ LatticeTablesP<float, D2Q25> kTab25F = make_lattice_tables_p<float, D2Q25>();
static __constant__ LatticeTablesP<double, D2Q25> kTab25D = make_lattice_tables_p<double, D2Q25>();

template <typename P>
__device__ __forceinline__ const VelocityTablesP<P> &vtab();
template <>
__device__ __forceinline__ const VelocityTablesP<float> &vtab<float>() {
    return kTabF;
}
template <>
__device__ __forceinline__ const VelocityTablesP<double> &vtab<double>() {
    return kTabD;
}

// Reconstruction tables of lattice L (recon, herm; see pond_device.h).
template <typename P, class L>
__device__ __forceinline__ const auto &ltab() {
    if constexpr (L::Q == 16)
        return vtab<P>();
    else if constexpr (sizeof(P) == 4)
        return kTab25F;
    else
        return kTab25D;
}

// Lattice monomials c(a)^p c(b)^q of every velocity i = Q1 a + b (exponents
// of moment k), for the lattice sums of the per-velocity gather.
template <typename P, class L>
struct LatticeMonomials {
    P m[L::Q][L::NM];
};
template <typename P, class L>
constexpr LatticeMonomials<P, L> make_lattice_monomials() {
    LatticeMonomials<P, L> t{};
    for (int i = 0; i < L::Q; ++i) {
        const double ca = L::c(i / L::Q1), cb = L::c(i % L::Q1);
        for (int k = 0; k < L::NM; ++k) {
            double v = 1.0;
            for (int p = 0; p < mom_px(k); ++p) v *= ca;
            for (int q = 0; q < mom_py(k); ++q) v *= cb;
            t.m[i][k] = P(v);
        }
    }
    return t;
}
static __constant__ LatticeMonomials<float, D2Q16> kMono16F = make_lattice_monomials<float, D2Q16>();
static __constant__ LatticeMonomials<double, D2Q16> kMono16D = make_lattice_monomials<double, D2Q16>();
static __constant__ LatticeMonomials<float, D2Q25> kMono25F = make_lattice_monomials<float, D2Q25>();
static __constant__ LatticeMonomials<double, D2Q25> kMono25D = make_lattice_monomials<double, D2Q25>();

template <typename P, class L>
__device__ __forceinline__ const LatticeMonomials<P, L> &lmono() {
    if constexpr (L::Q == 16) {
        if constexpr (sizeof(P) == 4)
            return kMono16F;
        else
            return kMono16D;
    } else if constexpr (sizeof(P) == 4) {
        return kMono25F;
    } else {
        return kMono25D;
    }
}

// Tap source reading the HBM moment planes with periodic / clamp wrapping.
// gather() accumulates sum_{p,q} wx[p] wy[q] M(bx + p, by + q) for the NP x NP
// stencil whose first node is (bx, by) in unwrapped grid coordinates.
// Moment-plane row of the (unwrapped) grid row y: periodic wrap, clamp, or with
// walls (bc 2) the ghost rows -wall_h .. -1 and ny .. ny + wall_h - 1 around
// the grid (rows further out read the last ghost row).
__device__ __forceinline__ int mom_row(int y, int ny, int bc, int wall_h) {
    if (bc == 2) return min(max(y, -wall_h), ny + wall_h - 1);
    return wrap_index(y, ny, bc);
}

// Reference blocks.  The gather interpolates the deviations M - M_ref of the
// taps' moments from those of a reference node and starts its sums at M_ref:
// equal to interpolating M itself (the weights sum to 1), but the rounding of
// the weights -- whose sum differs from 1 by ~1e-8 in FP32, the same way at
// every node of a uniform flow -- then scales only the deviation.  (Otherwise a
// uniform flow at rest gains or loses ~2e-8 of its mass every step, 7e-8 at
// T = 0.04.)  The reference node of a destination node is the first node of
// the aligned kRefBlockX x kRefBlockY block holding it: every tile shape
// divides the block, so a tile has one reference, and every kernel and tile
// shape interpolate the same deviations.
constexpr int kRefBlockX = 256, kRefBlockY = 16;
__device__ __forceinline__ long long ref_node(int x, int y, int nx) {
    return (long long)(y / kRefBlockY * kRefBlockY) * nx + (x / kRefBlockX * kRefBlockX);
}

template <typename P, int NP, class L = D2Q16>
struct GlobalTaps {
    const P *mom;
    long long N;  // nodes per moment plane
    int nx, ny, bc_x, bc_y;
    long long moff;  // node offset of grid row 0
    int wall_h;
    P ref[nmom_padded<P, L>()];  // moments of the reference node

    // the interpolation sums start at the reference moments
    __device__ __forceinline__ void init(P Mf[L::NM], P Mg[L::NM]) const {
#pragma unroll
        for (int k = 0; k < L::NM; ++k) {
            Mf[k] = ref[k];
            Mg[k] = ref[L::NM + k];
        }
    }

    __device__ __forceinline__ P ref_at(int k) const { return ref[k]; }

    // Stencil rows r0 .. r0 + n - 1 (unwrapped) of the column stencil bx .. bx +
    // NP - 1: for each row r, in ascending order, X = sum_p wx[p] (M(bx + p, r) -
    // M_ref) over the 2 NM moments (the x-pass), handed to visit(r, seg, X).
    template <class Visit>
    __device__ __forceinline__ void rows(int bx, const P wx[NP], int r0, int n, int seg,
                                         Visit &visit) const {
        int col[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) col[j] = wrap_index(bx + j, nx, bc_x);
#pragma unroll 1
        for (int t = 0; t < n; ++t) {
            const long long row = moff + (long long)mom_row(r0 + t, ny, bc_y, wall_h) * nx;
            P X[2 * L::NM];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                P M[nmom_padded<P, L>()];
                load_moments<P, nmom<L>()>(mom, N, row + col[p], M);
#pragma unroll
                for (int k = 0; k < 2 * L::NM; ++k) {
                    const P dv = M[k] - ref[k];
                    X[k] = p == 0 ? wx[p] * dv : X[k] + wx[p] * dv;
                }
            }
            visit(r0 + t, seg, X);
        }
    }

    // adds sum_{p,q} wx[p] wy[q] (M(bx + p, by + q) - M_ref)
    __device__ __forceinline__ void gather(int bx, int by, const P wx[NP], const P wy[NP],
                                           P Mf[L::NM], P Mg[L::NM]) const {
        int col[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) col[j] = wrap_index(bx + j, nx, bc_x);
#pragma unroll POND_ROW_UNROLL
        for (int q = 0; q < NP; ++q) {
            const long long row = moff + (long long)mom_row(by + q, ny, bc_y, wall_h) * nx;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const P W = wx[p] * wy[q];
                P M[nmom_padded<P, L>()];
                load_moments<P, nmom<L>()>(mom, N, row + col[p], M);
#pragma unroll
                for (int k = 0; k < L::NM; ++k) {
                    Mf[k] += W * (M[k] - ref[k]);
                    Mg[k] += W * (M[L::NM + k] - ref[L::NM + k]);
                }
            }
        }
    }
};

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Lanes of the wave for which c holds (a ballot and a scalar bit count).
__device__ __forceinline__ unsigned long long wave_count(bool c) {
    return (unsigned long long)__popcll(__ballot(c));
}

// Coefficients B with pop_i = sum_j B_j M_j for raw moments M (about u_ref):
// the reconstruction weights r of velocity i on the normalised central
// moments about d = (dx, dy) (frame velocity - u_ref) with scale is = 1/sqrt(T),
// composed with that shift and scaling (the transpose of central_normalised).
// One coefficient vector serves both f and g.
//
// Each coefficient is the table weight plus the terms of the shift: the shift
// terms are summed first and the weight added last, in one rounding.  Added
// one by one onto the weight, each term would round at the weight's ulp, and
// over the sixteen velocities the coefficients of m00 (the mass) would sum to
// 1 + 7e-9 on average for frames within 1e-3 of u_ref -- a mass drift of that
// size every step in FP32.  Summed first, the single rounding is unbiased.
template <typename P>
__device__ __forceinline__ void pop_coeffs(const P r[kNM], P dx, P dy, P is, P B[kNM]) {
    const P is2 = is * is, is3 = is2 * is;
    const P r00 = r[0], r10 = r[1] * is, r01 = r[2] * is;
    const P r20 = r[3] * is2, r11 = r[4] * is2, r02 = r[5] * is2;
    const P r30 = r[6] * is3, r21 = r[7] * is3, r12 = r[8] * is3, r03 = r[9] * is3;
    const P ex = -dx, ey = -dy, exx = ex * ex, eyy = ey * ey, exy = ex * ey;
    B[9] = r03;
    B[8] = r12;
    B[7] = r21;
    B[6] = r30;
    B[5] = r02 + (ex * r12 + P(3) * ey * r03);
    B[4] = r11 + (P(2) * ex * r21 + P(2) * ey * r12);
    B[3] = r20 + (P(3) * ex * r30 + ey * r21);
    B[2] = r01 + (ex * r11 + P(2) * ey * r02 + exx * r21 + P(2) * exy * r12 + P(3) * eyy * r03);
    B[1] = r10 + (P(2) * ex * r20 + ey * r11 + P(3) * exx * r30 + P(2) * exy * r21 + eyy * r12);
    B[0] = r00 + (ex * r10 + ey * r01 + exx * r20 + exy * r11 + eyy * r02 + exx * ex * r30 +
                  exx * ey * r21 + ex * eyy * r12 + eyy * ey * r03);
}

// pop_coeffs for any order: B_rt = sum_{p >= r, q >= t} r_pq is^(p+q) C(p,r) C(q,t)
// (-dx)^(p-r) (-dy)^(q-t), the shift applied in y, then in x.
template <class L, typename P>
__device__ __forceinline__ void pop_coeffs_n(const P r[L::NM], P dx, P dy, P is, P B[L::NM]) {
    constexpr int N = L::N;
    P ex[N + 1], ey[N + 1], sc[N + 1];
    ex[0] = ey[0] = sc[0] = P(1);
#pragma unroll
    for (int j = 1; j <= N; ++j) {
        ex[j] = ex[j - 1] * (-dx);
        ey[j] = ey[j - 1] * (-dy);
        sc[j] = sc[j - 1] * is;
    }
    P R[L::NM], T[L::NM];
#pragma unroll
    for (int k = 0; k < L::NM; ++k) R[k] = r[k] * sc[mom_px(k) + mom_py(k)];
    // each stage sums its shift terms first and adds the leading term last (see
    // pop_coeffs)
#pragma unroll
    for (int k = 0; k < L::NM; ++k) {
        const int p = mom_px(k), t = mom_py(k);
        P acc = P(0);
#pragma unroll
        for (int q = t + 1; q <= N - p; ++q)
            acc += P(binom_c(q, t)) * ey[q - t] * R[mom_index(p, q)];
        T[k] = R[k] + acc;
    }
#pragma unroll
    for (int k = 0; k < L::NM; ++k) {
        const int rr = mom_px(k), t = mom_py(k);
        P acc = P(0);
#pragma unroll
        for (int p = rr + 1; p <= N - t; ++p)
            acc += P(binom_c(p, rr)) * ex[p - rr] * T[mom_index(p, t)];
        B[k] = T[k] + acc;
    }
}

// Moments sum_i f_i V_ix^p V_iy^q of Q populations at the velocities V_i =
// s c_i + d (c_i = (c(a), c(b)) for i = Q1 a + b; one scale s and offset d for
// all i) through the lattice sums C_pq = sum_i f_i c(a)^p c(b)^q, which the
// x-components build in turn: column_add takes population (a, b) into S_q =
// sum_b f_(a,b) c(b)^q, column_flush adds c(a)^p S_q to C_pq once the
// x-component is done, and moments_from_lattice_sums expands (s c + d)^p by
// the binomial theorem at the end.  (Q1 operations per population and NM per
// x-component, where the monomials of each V_i and their products with f_i
// cost about 3 NM.)
template <class L, typename P>
__device__ __forceinline__ void column_add(P S[L::N + 1], int b, P f) {
    const P cb = P(L::c(b));
    S[0] += f;
    if (cb == P(0)) return;  // the zero abscissa of an odd lattice
    P cq = cb;
#pragma unroll
    for (int q = 1; q <= L::N; ++q) {
        S[q] += f * cq;
        cq *= cb;
    }
}

template <class L, typename P>
__device__ __forceinline__ void column_flush(P C[L::NM], P S[L::N + 1], int a) {
    const P ca = P(L::c(a));
    P cp = P(1);
#pragma unroll
    for (int p = 0; p <= L::N; ++p) {
#pragma unroll
        for (int q = 0; p + q <= L::N; ++q) C[mom_index(p, q)] += p == 0 ? S[q] : cp * S[q];
        cp *= ca;
    }
#pragma unroll
    for (int q = 0; q <= L::N; ++q) S[q] = P(0);
}

template <class L, typename P>
__device__ __forceinline__ void moments_from_lattice_sums(const P C[L::NM], P s, P dx, P dy,
                                                          P M[L::NM]) {
    constexpr int N = L::N, NM = L::NM;
    P ex[N + 1], ey[N + 1], sc[N + 1];
    ex[0] = ey[0] = sc[0] = P(1);
#pragma unroll
    for (int j = 1; j <= N; ++j) {
        ex[j] = ex[j - 1] * dx;
        ey[j] = ey[j - 1] * dy;
        sc[j] = sc[j - 1] * s;
    }
    // U_rt = s^(r+t) C_rt; then T[p][t] = sum_r C(p,r) dx^(p-r) U[r][t] and
    // M[p][q] = sum_t C(q,t) dy^(q-t) T[p][t], each sum starting at its unit term
    P U[NM], T[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        const int o = mom_px(k) + mom_py(k);
        U[k] = o == 0 ? C[k] : C[k] * sc[o];
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        const int p = mom_px(k), t = mom_py(k);
        P acc = U[k];
#pragma unroll
        for (int r = p - 1; r >= 0; --r) acc += (P(binom_c(p, r)) * ex[p - r]) * U[mom_index(r, t)];
        T[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        const int p = mom_px(k), q = mom_py(k);
        P acc = T[k];
#pragma unroll
        for (int t = q - 1; t >= 0; --t) acc += (P(binom_c(q, t)) * ey[q - t]) * T[mom_index(p, t)];
        M[k] = acc;
    }
}

// Unwrapped index range [lo, hi] of the stencils of every velocity of a node at
// coordinate x with frame velocity u and sqrt(T) = s along one axis.
template <int NP, class L = D2Q16>
__device__ __forceinline__ void stencil_extent(int x, double u, double s, int &lo, int &hi) {
    // departure coordinates x - (s c + u) for c = +-c_out bound all stencils
    const double dlo = double(x) - (s * L::c(L::Q1 - 1) + u), dhi = double(x) - (s * L::c(0) + u);
    const double clo = fmin(fmax(dlo, double(x) - 4096.0), double(x) + 4096.0);
    const double chi = fmin(fmax(dhi, double(x) - 4096.0), double(x) + 4096.0);
    if (NP == 4) {
        lo = int(floor(clo)) - 1;
        hi = int(floor(chi)) + 2;
    } else {
        lo = int(floor(clo + 0.5)) - 1;
        hi = int(floor(chi + 0.5)) + 1;
    }
}

// Velocity gradient of frame velocities (ux, uy) at grid node (x, y), for the
// internal-energy split: central differences of the four neighbours' velocities
// (wrapped or clamped like the stencil; with walls a neighbour row beyond a wall
// takes the ghost frame velocity of the wall closure, the mirror node -- here
// the node itself -- reflected about the wall velocity).
// g = (d_x u_x, d_x u_y, d_y u_x, d_y u_y).
__device__ __forceinline__ void node_gradient(const StepArgs &a, const double *__restrict__ ux,
                                              const double *__restrict__ uy, int x, int y,
                                              double g[4]) {
    const long long row = (long long)y * a.nx;
    const long long xm = row + wrap_index(x - 1, a.nx, a.bc_x);
    const long long xp = row + wrap_index(x + 1, a.nx, a.bc_x);
    const long long ym = (long long)wrap_index(y - 1, a.ny, a.bc_y) * a.nx + x;
    const long long yp = (long long)wrap_index(y + 1, a.ny, a.bc_y) * a.nx + x;
    double uxm = ux[ym], uym = uy[ym], uxp = ux[yp], uyp = uy[yp];
    if (a.bc_y == 2 && y == 0) {
        uxm = 2.0 * a.wall_ux[0] - ux[row + x];
        uym = -uy[row + x];
    }
    if (a.bc_y == 2 && y == a.ny - 1) {
        uxp = 2.0 * a.wall_ux[1] - ux[row + x];
        uyp = -uy[row + x];
    }
    g[0] = 0.5 * (ux[xp] - ux[xm]);
    g[1] = 0.5 * (uy[xp] - uy[xm]);
    g[2] = 0.5 * (uxp - uxm);
    g[3] = 0.5 * (uyp - uym);
}

// Velocity gradient of frame velocities (ux, uy) at the point (px, py): the
// bilinear interpolation of node_gradient over the four nodes around it
// (columns and rows wrapped or clamped like the stencil; with walls a row
// beyond them is the last row).  The point is clamped to a finite range first,
// so a non-physical frame still indexes inside the grid.
__device__ __forceinline__ void point_gradient(const StepArgs &a, const double *__restrict__ ux,
                                               const double *__restrict__ uy, double px, double py,
                                               double g[4]) {
    px = fmin(fmax(px, -1.0e8), 1.0e8);
    py = fmin(fmax(py, -1.0e8), 1.0e8);
    const double fx = floor(px), fy = floor(py);
    const double ax = px - fx, ay = py - fy;
    const int x0 = int(fx), y0 = int(fy);
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = 0.0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int yj = wrap_index(y0 + j, a.ny, a.bc_y);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int xi = wrap_index(x0 + i, a.nx, a.bc_x);
            const double w = (i ? ax : 1.0 - ax) * (j ? ay : 1.0 - ay);
            double gn[4];
            node_gradient(a, ux, uy, xi, yj, gn);
#pragma unroll
            for (int k = 0; k < 4; ++k) g[k] += w * gn[k];
        }
    }
}

// The internal-energy split's velocity gradient for destination node (x, y)
// with time-t frame velocity (u0, u1): taken at the end of the step, where the
// collision and the source act, by linear extrapolation along the node's
// trajectory from the last two time levels, 2 G_t(x - u) - G_{t-1}(x - 2u)
// (G_t: point_gradient of the time-t frames, G_{t-1}: of the previous level's;
// exact for a velocity field advected with the flow).
__device__ __forceinline__ void source_gradient(const StepArgs &a, const DevState &src, int x,
                                                int y, double u0, double u1, double g[4]) {
    double ga[4], gb[4];
    point_gradient(a, src.ux, src.uy, double(x) - u0, double(y) - u1, ga);
    point_gradient(a, src.uxp, src.uyp, double(x) - 2.0 * u0, double(y) - 2.0 * u1, gb);
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = 2.0 * ga[k] - gb[k];
}

// FP32 D2Q25 shares its x-pass too (gather_shared_rows_transformed; 0: the
// per-velocity gather).
#ifndef POND_D2Q25_SHARED
#define POND_D2Q25_SHARED 1
#endif

// Velocities per shared x-pass of the FP32 D2Q16 gather (4: the Q1 velocities
// of one x-component; 2: half of them; 1: no sharing, every velocity gathers its
// own NP x NP taps).  FP64 and D2Q25 gather per velocity.
#ifndef POND_VEL_GROUP
#define POND_VEL_GROUP 4
#endif
template <typename P, class L>
constexpr int vel_group() {
    return (L::Q == 16 && sizeof(P) == 4) ? POND_VEL_GROUP : 1;
}

// The gather of every velocity of a D2Q16 node in the iterate frame (departure
// offsets xu = x - u, yu = y - u relative to the node, scale sc = sqrt(T),
// frame shift (dux, duy) from u_ref and 1 / sqrt(T) = is), with the
// x-interpolation shared: the VG velocities of a group have the same x-component
// c(ia), so the same departure abscissa and column stencil, and differ only in
// their rows.  Each row of the union of their row stencils is interpolated along
// x once (taps.rows); every velocity whose stencil holds the row takes that
// x-pass with its row weight, through its frame-transformation coefficients
// (the scalar f_i = B_i . I_i distributes over the rows).  When the union is
// longer than the separate stencils (hot flows), each velocity's rows are
// visited on their own; the sums are the same either way.  take(b, cx, cy,
// f_i, g_i) receives each gathered population pair (i = Q1 ia + b), and
// column(ia) follows the last of an x-component's.
//
// The populations handed over are those of the interpolated deviations from
// the reference moments only: the reference's own share, B_i . M_ref, is the
// same reconstruction of one moment vector for every velocity, and the
// reconstruction keeps the moments up to order three (the quadrature is exact
// to degree seven), so its share of every sum that take forms -- mass,
// momentum, energy, the lab moments -- follows from M_ref itself; the caller
// adds it once after the gather.  (The share then enters the sums exactly,
// with no rounding of the coefficients B_i.)
template <typename P, int NP, class L, int VG, class Taps, class Take, class Column>
__device__ __forceinline__ void gather_shared_rows(const Taps &taps, const VelocityTablesP<P> &tab,
                                                   double xu, double yu, double sc, P dux, P duy,
                                                   P is, Take &take, Column &column) {
    constexpr int NM = L::NM;
    static_assert(L::Q1 % VG == 0, "velocity groups split the x-component's velocities");
#pragma unroll 1
    for (int ia = 0; ia < L::Q1; ++ia) {
        const double cx = L::c(ia);
        P wx[NP];
        const int bx = lagrange<NP>(fma(-sc, cx, xu), wx);
#pragma unroll 1
        for (int g = 0; g < L::Q1 / VG; ++g) {
            // rows and weights of the group's velocities b = g VG + v: their
            // departure ordinates y - u - sqrt(T) c(b) descend with b, and so do
            // their first stencil rows by[v]
            int by[VG];
            P wq[VG][NP];  // row weights, consumed first to last
            P B[VG][NM];
            P af[VG], ag[VG];
#pragma unroll
            for (int v = 0; v < VG; ++v) {
                const int b = g * VG + v;
                by[v] = lagrange<NP>(fma(-sc, L::c(b), yu), wq[v]);
                pop_coeffs(tab.recon[L::Q1 * ia + b], dux, duy, is, B[v]);
                af[v] = ag[v] = P(0);
            }
            auto visit = [&](int r, int seg, const P (&X)[2 * NM]) {
#pragma unroll
                for (int v = 0; v < VG; ++v) {
                    const bool mine = seg < 0 ? unsigned(r - by[v]) < unsigned(NP) : seg == v;
                    if (mine) {
                        const P w = wq[v][0];
#pragma unroll
                        for (int q = 0; q + 1 < NP; ++q) wq[v][q] = wq[v][q + 1];
                        P df = P(0), dg = P(0);
#pragma unroll
                        for (int k = 0; k < NM; ++k) {
                            df += B[v][k] * X[k];
                            dg += B[v][k] * X[NM + k];
                        }
                        af[v] += w * df;
                        ag[v] += w * dg;
                    }
                }
            };
            const int span = by[0] - by[VG - 1] + NP;
            if (span <= VG * NP) {
                taps.rows(bx, wx, by[VG - 1], span, -1, visit);
            } else {
#pragma unroll 1
                for (int v = 0; v < VG; ++v) {
                    int r0 = by[0];
#pragma unroll
                    for (int u = 1; u < VG; ++u) r0 = v == u ? by[u] : r0;
                    taps.rows(bx, wx, r0, NP, v, visit);
                }
            }
#pragma unroll
            for (int v = 0; v < VG; ++v) {
                const int b = g * VG + v;
                take(b, cx, L::c(b), af[v], ag[v]);
            }
        }
        column(ia);
    }
}

// D2Q25 in FP32 shares the x-pass between the five velocities of an
// x-component too, in a form that holds no per-velocity coefficients (their 75
// registers do not fit beside the 30-moment rows): each row of the union of the
// row stencils is interpolated along x once and turned into the normalised
// central moments of the iterate frame once (central_normalised_n: a linear
// map, so it commutes with the row weights), and each velocity whose stencil
// holds the row adds its row weight times the reconstruction weights (the
// lattice tables, uniform across lanes) dotted with those moments.  As in
// gather_shared_rows, the populations handed over are those of the deviations
// from the reference moments; the order-4 reconstruction keeps the moments up
// to order four (D1Q5 integrates exactly to degree nine), so the reference's
// share of the sums is added by the caller, once.
template <typename P, class L>
constexpr bool shared_rows_transformed() {
    return L::Q == 25 && sizeof(P) == 4 && POND_D2Q25_SHARED != 0;
}

template <typename P, int NP, class L, class Taps, class Tab, class Take, class Column>
__device__ __forceinline__ void gather_shared_rows_transformed(const Taps &taps, const Tab &tab,
                                                               double xu, double yu, double sc,
                                                               P dux, P duy, P is, Take &take,
                                                               Column &column) {
    constexpr int NM = L::NM, Q1 = L::Q1;
#pragma unroll 1
    for (int ia = 0; ia < Q1; ++ia) {
        const double cx = L::c(ia);
        P wx[NP];
        const int bx = lagrange<NP>(fma(-sc, cx, xu), wx);
        int by[Q1];
        P wq[Q1][NP];  // row weights, consumed first to last
        P af[Q1], ag[Q1];
#pragma unroll
        for (int b = 0; b < Q1; ++b) {
            by[b] = lagrange<NP>(fma(-sc, L::c(b), yu), wq[b]);
            af[b] = ag[b] = P(0);
        }
        auto visit = [&](int row, int seg, const P (&X)[2 * NM]) {
            P Zf[NM], Zg[NM];
            central_normalised_n<L>(X, dux, duy, is, Zf);
            central_normalised_n<L>(X + NM, dux, duy, is, Zg);
#pragma unroll
            for (int b = 0; b < Q1; ++b) {
                const bool mine = seg < 0 ? unsigned(row - by[b]) < unsigned(NP) : seg == b;
                if (mine) {
                    const P w = wq[b][0];
#pragma unroll
                    for (int q = 0; q + 1 < NP; ++q) wq[b][q] = wq[b][q + 1];
                    // the velocity's weights are read from the constant table at
                    // each visit (a scalar load): the x-component's 75 weights held
                    // across the row loop would not fit the scalar registers and
                    // would be spilled into vector-register lanes
                    int row_tab = Q1 * ia + b;
                    asm volatile("" : "+s"(row_tab));
                    const P *r = tab.recon[row_tab];
                    P df = P(0), dg = P(0);
#pragma unroll
                    for (int k = 0; k < NM; ++k) {
                        df += r[k] * Zf[k];
                        dg += r[k] * Zg[k];
                    }
                    af[b] += w * df;
                    ag[b] += w * dg;
                }
            }
        };
        const int span = by[0] - by[Q1 - 1] + NP;
        if (span <= Q1 * NP) {
            taps.rows(bx, wx, by[Q1 - 1], span, -1, visit);
        } else {
#pragma unroll 1
            for (int b = 0; b < Q1; ++b) {
                int r0 = by[0];
#pragma unroll
                for (int u = 1; u < Q1; ++u) r0 = b == u ? by[u] : r0;
                taps.rows(bx, wx, r0, NP, b, visit);
            }
        }
#pragma unroll
        for (int b = 0; b < Q1; ++b) take(b, cx, L::c(b), af[b], ag[b]);
        column(ia);
    }
}

// The whole step of one destination node (x, y) = node n whose time-t frame
// is (l0, l1, l2), for the energy split S (0: total energy, 1: internal
// energy, 2: non-translational energy) on lattice L; src is the time-t state
// (its frames feed the velocity gradient of the internal-energy split).  The
// node's moments of the new state (those the next step interpolates) go to
// mom_out, computed from the stored populations and frame exactly as the
// moments pre-pass computes them.  Lanes with live == false take part in the
// wave-level predictor-corrector exit and the counter reduction only.
//
// Per predictor-corrector gather, for each velocity i: departure point and
// Lagrange weights, interpolation of the 2 NM moments, frame transformation of
// the interpolated moments into the iterate frame (population i of f and g);
// the FP64 sums rho, j, E and the lattice sums of the gathered populations
// (their lab moments follow once, from the last gather's) are accumulated on
// the fly, so no population array is kept.
template <typename P, int NP, int S, class L, class Taps>
__device__ __forceinline__ void node_step(const StepArgs &a, const Taps &taps, int x, int y,
                                          long long n, bool live, double l0, double l1, double l2,
                                          const DevState &src, DevState dst,
                                          P *__restrict__ mom_out, DevCounters *cnt) {
    constexpr int NM = L::NM;
    const auto &tab = ltab<P, L>();
    double lg0 = l0, lg1 = l1, lg2 = l2;     // frame of the current gather
    double ln0 = lg0, ln1 = lg1, ln2 = lg2;  // frame of the gathered moments
    double rho = 1.0, gsum = 0.0;  // FP64 sums of the last gather's f and g
    P Mf[NM], Mg[NM];  // lab moments (about u_ref) of the last gather's populations
    P Cf[NM], Cg[NM];  // their lattice sums (column_add), in the gather's frame
#pragma unroll
    for (int k = 0; k < NM; ++k) Mf[k] = Mg[k] = Cf[k] = Cg[k] = P(0);
    bool done = !live, conv = false, bad = false, overrun = false;
    unsigned long long itc = 0;  // gathers of the wave's lanes
    // internal split: the source's velocity gradient (the same for every
    // iterate), in the arithmetic's precision
    P gxx = P(0), gxy = P(0), gyx = P(0), gyy = P(0);
    if constexpr (S == 1) {
        if (live) {
            double gr[4];
            source_gradient(a, src, x, y, l0, l1, gr);
            gxx = P(gr[0]);
            gxy = P(gr[1]);
            gyx = P(gr[2]);
            gyy = P(gr[3]);
        }
    }

    // lab moments of a gather's populations from its lattice sums (frame scale sP,
    // offset (dux, duy) from u_ref); the shared gathers sum the deviations from
    // the reference moments, whose share is added here
    auto lab_moments = [&](P sP, P dux, P duy) {
        moments_from_lattice_sums<L>(Cf, sP, dux, duy, Mf);
        moments_from_lattice_sums<L>(Cg, sP, dux, duy, Mg);
        if constexpr (vel_group<P, L>() > 1 || shared_rows_transformed<P, L>()) {
#pragma unroll
            for (int k = 0; k < NM; ++k) {
                Mf[k] += taps.ref_at(k);
                Mg[k] += taps.ref_at(NM + k);
            }
        }
    };

    for (int it = 0; it < a.pc_max_iter; ++it) {
        itc += wave_count(!done);
        if (!done) {
            const double s = sqrt(lg2);
            if (a.bc_y == 2) {
                // walls: every stencil row must lie within the ghost rows
                int lo, hi;
                stencil_extent<NP, L>(y, lg1, s, lo, hi);
                if (lo < -a.wall_h || hi > a.ny - 1 + a.wall_h) overrun = true;
            }
            const P sP = P(s), dux = P(lg0 - a.uref_x), duy = P(lg1 - a.uref_y), is = P(1.0 / s);
            // departure coordinates x - (s c + u) = (x - u) - s c, from the iterate
            // frame clamped to a finite range (a non-physical iterate, which the
            // test below flags, must still index inside the grid)
            const double sc = fmin(fmax(s, 0.0), 1.0e6);
            const double xu = double(x) - fmin(fmax(lg0, -1.0e8), 1.0e8);
            const double yu = double(y) - fmin(fmax(lg1, -1.0e8), 1.0e8);
            double r = 0.0, jx = 0.0, jy = 0.0, E = 0.0, Eg = 0.0;
            P Sf[L::N + 1], Sg[L::N + 1];
#pragma unroll
            for (int k = 0; k < NM; ++k) Cf[k] = Cg[k] = P(0);
#pragma unroll
            for (int q = 0; q <= L::N; ++q) Sf[q] = Sg[q] = P(0);
            // population i = Q1 ia + b of f and g gathered in the iterate frame: the
            // FP64 sums rho, j, E (sums) and the lattice sums of the gathered
            // populations (take: through the column sums)
            auto sums = [&](double cx, double cy, P fi, P gi) {
                // conserved moments in FP64
                const double fd = double(fi);
                r += fd;
                jx += fd * (s * cx + lg0);
                jy += fd * (s * cy + lg1);
                E += double(gi);
                if constexpr (S == 2) {
                    // non-translational split: f carries the translational energy
                    Eg += double(gi);
                    const double Cx = s * cx + lg0, Cy = s * cy + lg1;
                    E += 0.5 * fd * (Cx * Cx + Cy * Cy);
                }
            };
            auto take = [&](int b, double cx, double cy, P fi, P gi) {
                sums(cx, cy, fi, gi);
                column_add<L>(Sf, b, fi);
                column_add<L>(Sg, b, gi);
            };
            auto column = [&](int ia) {
                column_flush<L>(Cf, Sf, ia);
                column_flush<L>(Cg, Sg, ia);
            };
            if constexpr (vel_group<P, L>() > 1 || shared_rows_transformed<P, L>()) {
                if constexpr (vel_group<P, L>() > 1)
                    gather_shared_rows<P, NP, L, vel_group<P, L>()>(taps, tab, xu, yu, sc, dux,
                                                                     duy, is, take, column);
                else
                    gather_shared_rows_transformed<P, NP, L>(taps, tab, xu, yu, sc, dux, duy, is,
                                                             take, column);
                // the reference moments' share of the sums (moments about u_ref;
                // the lab velocity is V + u_ref), added once after the deviations'
                const double m00 = double(taps.ref_at(0));
                const double m10 = double(taps.ref_at(mom_index(1, 0)));
                const double m01 = double(taps.ref_at(mom_index(0, 1)));
                r += m00;
                jx += m10 + a.uref_x * m00;
                jy += m01 + a.uref_y * m00;
                E += double(taps.ref_at(NM));
                if constexpr (S == 2) {
                    Eg += double(taps.ref_at(NM));
                    const double m20 = double(taps.ref_at(mom_index(2, 0)));
                    const double m02 = double(taps.ref_at(mom_index(0, 2)));
                    E += 0.5 * (m20 + m02) + a.uref_x * m10 + a.uref_y * m01 +
                         0.5 * (a.uref_x * a.uref_x + a.uref_y * a.uref_y) * m00;
                }
            } else {
                // velocity i = Q1 ia + ib has x-component c(ia) and y-component c(ib):
                // the x-stencil serves the Q1 velocities of one ia
#pragma unroll 1
                for (int ia = 0; ia < L::Q1; ++ia) {
                    const double cx = L::c(ia);
                    // departure point x - C_i(lam_bar) dt and its stencil, x then y
                    P wx[NP];
                    const int bx = lagrange<NP>(fma(-sc, cx, xu), wx);
#pragma unroll 1
                    for (int ib = 0; ib < L::Q1; ++ib) {
                        const int i = L::Q1 * ia + ib;
                        const double cy = L::c(ib);
                        P wy[NP];
                        const int by = lagrange<NP>(fma(-sc, cy, yu), wy);
                        P If[NM], Ig[NM];
                        taps.init(If, Ig);
                        taps.gather(bx, by, wx, wy, If, Ig);
                        // frame transformation of the interpolated moments: population i
                        P B[NM];
                        if constexpr (L::Q == 16)
                            pop_coeffs(tab.recon[i], dux, duy, is, B);
                        else
                            pop_coeffs_n<L>(tab.recon[i], dux, duy, is, B);
                        P fi = P(0), gi = P(0);
#pragma unroll
                        for (int k = 0; k < NM; ++k) {
                            fi += B[k] * If[k];
                            gi += B[k] * Ig[k];
                        }
                        // lattice sums with the velocity's monomials from the
                        // table: column sums held across this loop would take
                        // registers the FP64 kernels do not have
                        sums(cx, cy, fi, gi);
                        const P *mi = lmono<P, L>().m[i];
#pragma unroll
                        for (int k = 0; k < NM; ++k) {
                            Cf[k] += fi * mi[k];
                            Cg[k] += gi * mi[k];
                        }
                    }
                }
            }
            rho = r;
            gsum = S == 2 ? Eg : E;
            ln0 = jx / r;
            ln1 = jy / r;
            // total split: sum g = E = rho c_v T + |j|^2 / (2 rho); internal: sum g = rho c_v T;
            // non-translational: E = sum g + sum f |C|^2 / 2 = rho c_v T + |j|^2 / (2 rho)
            if constexpr (S == 1) lab_moments(sP, dux, duy);
            if constexpr (S == 1) {
                // the energy of the step's middle, U = sum g + (sum G) / 2, with the
                // source's sum G = -(omega / 2) rho T div u - (1 - omega / 2) P : grad u
                // (P the pressure tensor of the gathered f about u, from its moments
                // about u_ref): rho c_v T = U solved for T
                const double dx = ln0 - a.uref_x, dy = ln1 - a.uref_y;
                const double m00 = double(Mf[mom_index(0, 0)]), m10 = double(Mf[mom_index(1, 0)]);
                const double m01 = double(Mf[mom_index(0, 1)]), m20 = double(Mf[mom_index(2, 0)]);
                const double m11 = double(Mf[mom_index(1, 1)]), m02 = double(Mf[mom_index(0, 2)]);
                const double Pxx = m20 - 2.0 * dx * m10 + dx * dx * m00;
                const double Pxy = m11 - dx * m01 - dy * m10 + dx * dy * m00;
                const double Pyy = m02 - 2.0 * dy * m01 + dy * dy * m00;
                const double PdU = Pxx * double(gxx) + Pxy * (double(gxy) + double(gyx)) +
                                   Pyy * double(gyy);
                ln2 = (E - 0.5 * (1.0 - 0.5 * a.omega) * PdU) /
                      (r * (a.cv + 0.25 * a.omega * (double(gxx) + double(gyy))));
            } else
                ln2 = (E - (jx * jx + jy * jy) / (2.0 * r)) / (r * a.cv);
            if (!(r > 0.0) || !(ln2 > 0.0) || !isfinite(ln0) || !isfinite(ln1) || !isfinite(ln2) ||
                !isfinite(E)) {
                bad = true;
                done = true;
            } else {
                const double du = fmax(fabs(ln0 - lg0), fabs(ln1 - lg1)) / sqrt(ln2);
                // FP64: the change of T relative to T.  FP32: relative to the scale of
                // the energy T is recovered from, E / (rho c_v) (T itself in the internal
                // split, T + |u|^2 / (2 c_v) in the total split): single-precision
                // populations resolve E, and so T, only to a fraction of that scale
                double Tscale = ln2;
                if constexpr (sizeof(P) == 4) Tscale = E / (r * a.cv);
                const double dT = fabs(ln2 - lg2) / Tscale;
                if (fmax(du, dT) <= a.pc_tol) {
                    conv = true;
                    done = true;
                } else if (it + 1 < a.pc_max_iter) {
                    lg0 = ln0;
                    lg1 = ln1;
                    lg2 = ln2;
                }
            }
        }
        if (__all(done)) break;  // wave-uniform exit once every lane has converged
    }

    if (live) {
        if constexpr (S != 1) {
            // the last gather's frame (lam is only advanced when another gather follows)
            const double s = sqrt(lg2);
            lab_moments(P(s), P(lg0 - a.uref_x), P(lg1 - a.uref_y));
        }
        // re-projection onto lam* = (ln0, ln1, ln2): Grad coefficients there
        const double sT = sqrt(ln2);
        const P is = P(1.0 / sT);
        const P tx = P(ln0 - a.uref_x), ty = P(ln1 - a.uref_y);
        P m[NM], af[NM], ag[NM];
        // the zeroth moments are the exact FP64 sums of the gathered populations,
        // rounded once: a float sum of the Q populations loses ~1e-7 of the mass
        // in a way that repeats from step to step in a near-uniform flow (a
        // drift); in FP64 the two are the same sums
        Mf[0] = P(rho);
        Mg[0] = P(gsum);
        if constexpr (L::Q == 16) {
            central_normalised(Mf, tx, ty, is, m);
            hermite_from_central(m, af);
            central_normalised(Mg, tx, ty, is, m);
            hermite_from_central(m, ag);
        } else {
            central_normalised_n<L>(Mf, tx, ty, is, m);
            hermite_from_central_n<L>(m, af);
            central_normalised_n<L>(Mg, tx, ty, is, m);
            hermite_from_central_n<L>(m, ag);
        }

        // BGK collision in lam*, on the Grad coefficients.
        // f: f^eq = rho w_i has only a0; every higher coefficient decays by (1 - omega).
        // g, total split: g^eq = w_i [rho (c_v - 1) T + rho |C_i|^2 / 2] has
        //    a0 = rho c_v T + rho |u|^2 / 2, a1 = rho sqrt(T) u, a2 = rho T I, a3 = 0;
        // g, internal split: C_i - u in place of C_i, so a0 = rho c_v T, a1 = 0;
        // g, non-translational split: g^eq = w_i rho (c_v - 1) T, a0 only.
        const double om = a.omega;
        double geq[NM];
#pragma unroll
        for (int k = 0; k < NM; ++k) geq[k] = 0.0;
        if constexpr (S == 1) {
            geq[0] = rho * a.cv * ln2;
            geq[1] = geq[2] = 0.0;
        } else if constexpr (S == 2) {
            geq[0] = rho * (a.cv - 1.0) * ln2;
        } else {
            geq[0] = rho * (a.cv - 1.0) * ln2 + 0.5 * rho * (2.0 * ln2 + ln0 * ln0 + ln1 * ln1);
            geq[1] = rho * sT * ln0;
            geq[2] = rho * sT * ln1;
        }
        if constexpr (S != 2) {
            geq[3] = rho * ln2;
            geq[4] = 0.0;
            geq[5] = rho * ln2;
            geq[6] = geq[7] = geq[8] = geq[9] = 0.0;
        }
        if (S == 1 || S == 2 || a.unit_prandtl) {
            // internal split: the flux of g is the heat flux alone, relaxed at omega_1
            // (omega at Pr = 1); the non-translational split runs at Pr = 1 only
            const double og = a.unit_prandtl ? om : a.omega1;
#pragma unroll
            for (int k = 0; k < NM; ++k) ag[k] = ag[k] + P(og) * (P(geq[k]) - ag[k]);
        } else {
            // quasi-equilibrium: energy flux of g^eq plus the viscous heating u . P^neq,
            // P^neq = T a2(f) + sqrt(T) (u a1(f) + a1(f) u) in lam*.
            const double a1x = double(af[1]), a1y = double(af[2]);
            const double Pxx = ln2 * double(af[3]) + sT * 2.0 * ln0 * a1x;
            const double Pxy = ln2 * double(af[4]) + sT * (ln0 * a1y + a1x * ln1);
            const double Pyy = ln2 * double(af[5]) + sT * 2.0 * ln1 * a1y;
            const double dqx = ln0 * Pxx + ln1 * Pxy;
            const double dqy = ln0 * Pxy + ln1 * Pyy;
            double gqe[NM];
#pragma unroll
            for (int k = 0; k < NM; ++k) gqe[k] = geq[k];
            gqe[1] += dqx / sT;
            gqe[2] += dqy / sT;
            const double om1 = a.omega1;
#pragma unroll
            for (int k = 0; k < NM; ++k)
                ag[k] = ag[k] + P(om1) * (P(gqe[k]) - ag[k]) + P(om) * (P(geq[k]) - P(gqe[k]));
        }
        // internal split: source of the g-equation, S_i = -f_i (C_i - u) . (a + C_i . grad u)
        // with f the step's time-centred population (the mean of the re-projected
        // pre-collision and the collided f: a0 and (1 - omega / 2) times the higher
        // coefficients, whose stress is the physical one), a = d_t u = u* - u(t),
        // grad u from source_gradient; g receives (1 - omega_g / 2) S, omega_g its
        // relaxation rate (its equilibrium already holds the other half of sum S)
        P afp[NM];
        P ax = P(0), ay = P(0), src_w = P(0);
        if constexpr (S == 1) {
            const P half_decay = P(1.0 - 0.5 * om);
            afp[0] = af[0];
#pragma unroll
            for (int k = 1; k < NM; ++k) afp[k] = af[k] * half_decay;
            // the time-t velocity is read again rather than kept live across the loop
            ax = P(ln0 - src.ux[n]);
            ay = P(ln1 - src.uy[n]);
            src_w = P(1.0 - 0.5 * (a.unit_prandtl ? om : a.omega1));
        }
        const P decay = P(1.0 - om);
#pragma unroll
        for (int k = 1; k < NM; ++k) af[k] *= decay;

        // reconstruct and store the post-collision populations, and accumulate the
        // moments of the stored values about u_ref (the next step's taps)
        const P sTP = P(sT), u0 = P(ln0), u1 = P(ln1);
        const double Tst = bad ? NAN : ln2, uxst = bad ? NAN : ln0, uyst = bad ? NAN : ln1;
        const P sM = P(sqrt(Tst)), dxM = P(uxst - a.uref_x), dyM = P(uyst - a.uref_y);
        P MM[nmom_padded<P, L>()];
#pragma unroll
        for (int k = 0; k < nmom_padded<P, L>(); ++k) MM[k] = P(0);
        P Nf[NM], Ng[NM], Sf[L::N + 1], Sg[L::N + 1];  // lattice sums (column_add)
#pragma unroll
        for (int k = 0; k < NM; ++k) Nf[k] = Ng[k] = P(0);
#pragma unroll
        for (int q = 0; q <= L::N; ++q) Sf[q] = Sg[q] = P(0);
        double mass = 0.0, gzero = 0.0;  // zeroth moments summed in FP64 (see above)
#pragma unroll 1
        for (int ia = 0; ia < L::Q1; ++ia) {
#pragma unroll
            for (int b = 0; b < L::Q1; ++b) {
                const int i = L::Q1 * ia + b;
                P fv = P(0), gv = P(0);
#pragma unroll
                for (int k = 0; k < NM; ++k) {
                    fv += tab.herm[i][k] * af[k];
                    gv += tab.herm[i][k] * ag[k];
                }
                if constexpr (S == 1) {
                    P ft = P(0);
#pragma unroll
                    for (int k = 0; k < NM; ++k) ft += tab.herm[i][k] * afp[k];
                    const P ex = sTP * P(L::c(ia)), ey = sTP * P(L::c(b));
                    const P Cx = ex + u0, Cy = ey + u1;
                    gv -= src_w * ft * (ex * (ax + Cx * gxx + Cy * gyx) + ey * (ay + Cx * gxy + Cy * gyy));
                }
                if (bad) fv = gv = P(NAN);
                out_store<kStreamPops>(&pop_plane<P>(dst.f, i, a.N)[n], fv);
                out_store<kStreamPops>(&pop_plane<P>(dst.g, i, a.N)[n], gv);
                column_add<L>(Sf, b, fv);
                column_add<L>(Sg, b, gv);
                mass += double(fv);
                gzero += double(gv);
            }
            column_flush<L>(Nf, Sf, ia);
            column_flush<L>(Ng, Sg, ia);
        }
        moments_from_lattice_sums<L>(Nf, sM, dxM, dyM, MM);
        moments_from_lattice_sums<L>(Ng, sM, dxM, dyM, MM + NM);
        MM[0] = P(mass);
        MM[NM] = P(gzero);
        out_store<kStreamFrame>(&dst.ux[n], uxst);
        out_store<kStreamFrame>(&dst.uy[n], uyst);
        out_store<kStreamFrame>(&dst.T[n], Tst);
        if constexpr (S == 1) {
            // the time-t frame becomes the new state's previous level (read again
            // rather than kept live across the loop)
            out_store<kStreamFrame>(&dst.uxp[n], src.ux[n]);
            out_store<kStreamFrame>(&dst.uyp[n], src.uy[n]);
        }
        store_moments_out<P, nmom<L>()>(mom_out, a.mstride, a.moff + n, MM);
    }

    // counters: one atomic per wave
    const unsigned long long nc = wave_count(live && !conv && !bad);
    const unsigned long long nb = wave_count(live && bad);
    const unsigned long long no = wave_count(live && overrun);
    if ((threadIdx.x & 63) == 0) {
        if (itc) atomicAdd(&cnt->pc_iterations, itc);
        if (nc) atomicAdd(&cnt->nonconverged, nc);
        if (nb) atomicAdd(&cnt->nonphysical, nb);
        if (no) atomicAdd(&cnt->ghost_overrun, no);
    }
}

}  // namespace pond
