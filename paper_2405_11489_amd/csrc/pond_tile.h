// pond_tile.h -- one block's share of the PonD step: a rectangular tile of
// destination nodes whose source moments are staged in LDS.  Shared by the
// single-instance tiled kernel (tile shape fixed at compile time) and the
// batched kernel (shape chosen per instance at run time).
#pragma once

#include "pond_step_common.h"

// Taps of a stencil row whose LDS loads are issued together; the row's later
// taps are loaded only after these are consumed (0: the whole row at once).
// Fewer loads in flight per lane -> fewer live registers -> more waves per
// SIMD: FP32 165 VGPRs (3 waves) with groups of 2, FP64 238 (2 waves) with 1.
// The four-wave FP32 kernel (512-lane blocks) loads one tap at a time: its
// 128 VGPRs then spill 17 registers instead of 30.
#ifndef POND_TAP_GROUP_F32
#define POND_TAP_GROUP_F32 2
#endif
#ifndef POND_TAP_GROUP_F64
#define POND_TAP_GROUP_F64 1
#endif

#ifndef POND_D2Q25_SHARED_WAVES
#define POND_D2Q25_SHARED_WAVES 2
#endif

namespace pond {

// Tap source of a tile: the moments of the block's source region (unwrapped
// rectangle [X0, X1] x [Y0, Y1], W wide, row-major) staged in LDS node-major
// (lds_stride), cap nodes at most; a velocity whose stencil leaves the region
// reads HBM.  With a
// single grid row (flat_y) every stencil row is row 0, so the region is one
// row and all NP stencil rows read it (same arithmetic as the HBM gather).
// G: taps per group of LDS loads (the arithmetic does not depend on it).
template <typename P, int NP, class L = D2Q16,
          int G = sizeof(P) == 8 ? POND_TAP_GROUP_F64 : POND_TAP_GROUP_F32>
struct TileTaps {
    const P *lds;
    int cap, X0, Y0, X1, Y1, W;
    bool flat_y;
    GlobalTaps<P, NP, L> glob;

    __device__ __forceinline__ void init(P Mf[L::NM], P Mg[L::NM]) const { glob.init(Mf, Mg); }
    __device__ __forceinline__ P ref_at(int k) const { return glob.ref[k]; }

    // The x-pass over stencil rows r0 .. r0 + n - 1 (see GlobalTaps::rows): from
    // LDS when the rows' stencil lies in the staged region, else from HBM (the
    // staged moments are the deviations from the reference node, rounded as
    // GlobalTaps rounds them, so both give the same bits).
    template <class Visit>
    __device__ __forceinline__ void rows(int bx, const P wx[NP], int r0, int n, int seg,
                                         Visit &visit) const {
        const bool inside =
            bx >= X0 && bx + NP - 1 <= X1 && (flat_y || (r0 >= Y0 && r0 + n - 1 <= Y1));
        if (inside && lds_planar<P, L>()) {
            // grouped planes: group k of node idx at vector k * cap + idx, so the NP
            // taps of a row are consecutive vectors of each group plane
            using MV = MomVec<P, nmom<L>()>;
            using V = typename MV::V;
            const int rs = flat_y ? 0 : W;
            int idx = (flat_y ? 0 : r0 - Y0) * W + (bx - X0);
#pragma unroll 1
            for (int t = 0; t < n; ++t) {
                const V *b = reinterpret_cast<const V *>(lds) + idx;
                P X[2 * L::NM];
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if (G > 0 && p > 0 && p % G == 0) asm volatile("" ::: "memory");
                    P M[nmom_padded<P, L>()];
#pragma unroll
                    for (int k = 0; k < MV::G; ++k) {
                        const V v = b[k * cap + p];
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
#pragma unroll
                    for (int k = 0; k < 2 * L::NM; ++k)
                        X[k] = p == 0 ? wx[p] * M[k] : X[k] + wx[p] * M[k];
                }
                visit(r0 + t, seg, X);
                idx += rs;
            }
        } else if (inside) {
            constexpr unsigned NB = lds_node_bytes<P, L>();
            const unsigned rowb = flat_y ? 0u : unsigned(W) * NB;
            unsigned off = __umul24(unsigned(flat_y ? 0 : r0 - Y0), rowb) +
                           __umul24(unsigned(bx - X0), NB);
#pragma unroll 1
            for (int t = 0; t < n; ++t) {
                P X[2 * L::NM];
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if (G > 0 && p > 0 && p % G == 0) asm volatile("" ::: "memory");
                    P M[nmom_padded<P, L>()];
                    load_node_lds_at<P, L>(lds, off + unsigned(p) * NB, M);
#pragma unroll
                    for (int k = 0; k < 2 * L::NM; ++k)
                        X[k] = p == 0 ? wx[p] * M[k] : X[k] + wx[p] * M[k];
                }
                visit(r0 + t, seg, X);
                off += rowb;
            }
        } else {
            int bxv = bx;
            asm volatile("" : "+v"(bxv));
            glob.rows(bxv, wx, r0, n, seg, visit);
        }
    }

    // the staged moments are the deviations from the tile's reference node
    __device__ __forceinline__ void gather(int bx, int by, const P wx[NP], const P wy[NP],
                                           P Mf[L::NM], P Mg[L::NM]) const {
        const bool inside =
            bx >= X0 && bx + NP - 1 <= X1 && (flat_y || (by >= Y0 && by + NP - 1 <= Y1));
        if (inside && lds_planar<P, L>()) {
            // grouped planes (node idx, group k at vector k * cap + idx)
            const int rs = flat_y ? 0 : W;
            const int base = (flat_y ? 0 : by - Y0) * W + (bx - X0);
#pragma unroll POND_ROW_UNROLL
            for (int q = 0; q < NP; ++q) {
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if (G > 0 && p > 0 && p % G == 0) asm volatile("" ::: "memory");
                    const P Wt = wx[p] * wy[q];
                    P M[nmom_padded<P, L>()];
                    load_moments<P, nmom<L>()>(lds, cap, base + q * rs + p, M);
#pragma unroll
                    for (int k = 0; k < L::NM; ++k) {
                        Mf[k] += Wt * M[k];
                        Mg[k] += Wt * M[L::NM + k];
                    }
                }
            }
        } else if (inside) {
            // byte offsets: the region is under 2^24 bytes, so the products are
            // 24-bit multiplies (full rate, where 32-bit ones take four cycles)
            constexpr unsigned NB = lds_node_bytes<P, L>();
            const unsigned rowb = flat_y ? 0u : unsigned(W) * NB;
            unsigned row = __umul24(unsigned(flat_y ? 0 : by - Y0), rowb) +
                           __umul24(unsigned(bx - X0), NB);
            // every stencil row unrolled (its weight wy[q] is a register); a
            // compiler barrier after each G taps bounds the loads in flight
#pragma unroll
            for (int q = 0; q < NP; ++q) {
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if (G > 0 && (q > 0 || p > 0) && (q * NP + p) % G == 0)
                        asm volatile("" ::: "memory");
                    const P Wt = wx[p] * wy[q];
                    P M[nmom_padded<P, L>()];
                    load_node_lds_at<P, L>(lds, row + unsigned(p) * NB, M);
#pragma unroll
                    for (int k = 0; k < L::NM; ++k) {
                        Mf[k] += Wt * M[k];
                        Mg[k] += Wt * M[L::NM + k];
                    }
                }
                row += rowb;
            }
        } else {
            // the HBM gather's column indices depend on bx alone; the empty asm
            // keeps the compiler from hoisting them out of the velocity loop into
            // the path every lane runs
            int bxv = bx;
            asm volatile("" : "+v"(bxv));
            glob.gather(bxv, by, wx, wy, Mf, Mg);
        }
    }
};

// Ints of shared memory per block_min of a block of NT lanes: one per wave, at
// least four (blocks of up to 256 lanes keep a 16-int array; a larger static
// array moves the dynamic LDS and costs the step kernel a register).
template <int NT>
constexpr int red_slots() {
    return NT > 256 ? (NT + 63) / 64 : 4;
}

// Minimum over the block (at most 8 waves); red holds one int per wave.
__device__ __forceinline__ int block_min(int v, int *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    const int w = threadIdx.x / 64, nw = (blockDim.x + 63) / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    int r = red[0];
    for (int i = 1; i < nw; ++i) r = min(r, red[i]);
    return r;
}

// Minimum waves per SIMD asked of the register allocator for the step kernels
// of NT lanes per block (168 VGPRs allow three, 128 four).  FP32 asks for three:
// the allocation sits at that boundary, and one register more halves the
// waves that hide the LDS latency.  FP32 blocks of 512 lanes ask for four: two
// such blocks share a CU's LDS, half of it each, which holds the source region
// of a 32 x 16 tile of an advected flow, and a grid of 4096 waves (512^2
// nodes) then runs in a single round.  FP64 holds two unforced (the internal
// split, whose frame temperature takes the source's work, asks); D2Q25 keeps
// the compiler's choice (two waves in FP32, one in FP64: more would spill).
template <typename P, int S, int NT = 256, class L = D2Q16>
constexpr int step_min_waves() {
    if (L::Q != 16) return shared_rows_transformed<P, L>() ? POND_D2Q25_SHARED_WAVES : 1;
    if (sizeof(P) == 4) {
        // the shared x-pass holds the coefficients and sums of a velocity group
        // (250 VGPRs with groups of four): two waves
        if (vel_group<P, L>() > 1) return 2;
        return NT == 512 ? 4 : 3;
    }
    return S == 1 ? 2 : 1;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8);
// give each XCD a contiguous range of tiles so that neighbouring tiles, which
// share halo moments, share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb / 8, r = nb % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// Order of the tiles within the range: column bands about POND_BAND_NODES
// nodes wide (0: plain row-major order), each walked row by row.  The blocks an
// XCD holds at once take consecutive tiles, so in row-major order they form a
// strip one tile high across the grid (8 x 2048 nodes for 8 x 8 tiles on
// 2048^2), whose source region carries halo rows above and below every tile;
// in a band they form a square of about POND_BAND_NODES^2 nodes, whose halo is
// only its perimeter.  (The halo rows shared with the previous set of tiles are
// gone from L2 by then either way: each set writes more than L2 holds.)  Off by
// default: on the 2048^2 quadrants bands of 128 (256) nodes cut the step's HBM
// reads by 21 % (25 %) but lengthened it by 6 % (a band's set of tiles spans
// 128 rows of every plane where a strip spans 8); on 512^2 the order made no
// difference.
#ifndef POND_BAND_NODES
#define POND_BAND_NODES 0
#endif
template <int TX>
__device__ __forceinline__ void band_tile(int t, int tiles_x, int tiles_y, int &tx, int &ty) {
    constexpr int bw = POND_BAND_NODES / TX > 1 ? POND_BAND_NODES / TX : 1;  // tiles per band
    if constexpr (POND_BAND_NODES == 0 || bw == 1) {
        tx = t % tiles_x;
        ty = t / tiles_x;
    } else {
        const int full = tiles_x / bw, per = bw * tiles_y;  // full bands, tiles per band
        if (t < full * per) {
            const int band = t / per, r = t - band * per;
            ty = r / bw;
            tx = band * bw + (r - ty * bw);
        } else {
            // the last band, narrower (tiles_x is no multiple of bw)
            const int w = tiles_x - full * bw, r = t - full * per;
            ty = r / w;
            tx = full * bw + (r - ty * w);
        }
    }
}

// Tile shapes: TX x TY destination nodes, one lane each, lane t at (t % TX, t / TX).
template <int TX, int TY>
struct FixedShape {
    static constexpr int kThreads = TX * TY;
    __device__ __forceinline__ int tx() const { return TX; }
    __device__ __forceinline__ int ty() const { return TY; }
    __device__ __forceinline__ int lx(int t) const { return t % TX; }
    __device__ __forceinline__ int ly(int t) const { return t / TX; }
};
// 256 lanes, TX = 2^lg, TY = 256 / TX.
struct Shape256 {
    static constexpr int kThreads = 256;
    int lg;
    __device__ __forceinline__ int tx() const { return 1 << lg; }
    __device__ __forceinline__ int ty() const { return 256 >> lg; }
    __device__ __forceinline__ int lx(int t) const { return t & ((1 << lg) - 1); }
    __device__ __forceinline__ int ly(int t) const { return t >> lg; }
};

// Source region of a tile: the union [X0, X1] x [Y0, Y1] of its lanes'
// predictor stencils.  When that exceeds cap nodes, the parts sticking out of
// the tile are cut to at most h nodes per side, with the largest h whose
// region fits (h = 0, the tile itself, always fits); an asymmetric halo (the
// upwind side of an advected flow) is kept whole when it fits.  A single-row
// grid stages one row.
__device__ __forceinline__ void clip_region(int tx0, int ty0, int tx, int ty, int cap, bool flat_y,
                                            int &X0, int &X1, int &Y0, int &Y1) {
    if (flat_y) Y0 = Y1 = 0;
    if (X1 < X0 || Y1 < Y0) return;  // no live lane
    const int tx1 = tx0 + tx - 1, ty1 = ty0 + ty - 1;
    auto area = [&](int h) {
        const long long w = (long long)min(X1, tx1 + h) - max(X0, tx0 - h) + 1;
        const long long v = flat_y ? 1 : (long long)min(Y1, ty1 + h) - max(Y0, ty0 - h) + 1;
        return w * v;
    };
    int hi = max(max(tx0 - X0, X1 - tx1), flat_y ? 0 : max(ty0 - Y0, Y1 - ty1));
    if (hi <= 0 || area(hi) <= cap) return;
    int lo = 0;  // area(lo) <= cap < area(hi)
    while (hi - lo > 1) {
        const int mid = lo + (hi - lo) / 2;
        if (area(mid) <= cap)
            lo = mid;
        else
            hi = mid;
    }
    X0 = max(X0, tx0 - lo);
    X1 = min(X1, tx1 + lo);
    if (!flat_y) {
        Y0 = max(Y0, ty0 - lo);
        Y1 = min(Y1, ty1 + lo);
    }
}

// The tile with first node (tx0, ty0): load the time-t frames, bound the
// source region (clip_region), stage the region's moments, then run every
// lane's node step (energy split S, lattice L).  Every thread of the block must
// call it (it synchronises the block).  red: 4 red_slots<Shape::kThreads>()
// ints of shared memory.
template <typename P, int NP, int S, class L, class Shape>
__device__ __forceinline__ void tile_step(const StepArgs &a, DevState src, const P *__restrict__ mom,
                                          DevState dst, P *__restrict__ mom_out, DevCounters *cnt,
                                          P *lds, int cap, int tx0, int ty0, Shape sh, int *red) {
    const int nthreads = sh.tx() * sh.ty();
    const int x = tx0 + sh.lx(int(threadIdx.x)), y = ty0 + sh.ly(int(threadIdx.x));
    const bool live = x < a.nx && y < a.ny;
    const long long n = live ? (long long)y * a.nx + x : 0;
    double l0 = 0.0, l1 = 0.0, l2 = 1.0;
    if (live) {
        l0 = src.ux[n];
        l1 = src.uy[n];
        l2 = src.T[n];
    }

    constexpr int kFar = 1 << 30;
    int lx = kFar, hx = -kFar, ly = kFar, hy = -kFar;
    if (live && isfinite(l0) && isfinite(l1) && l2 > 0.0 && isfinite(l2)) {
        const double s = sqrt(l2);
        stencil_extent<NP, L>(x, l0, s, lx, hx);
        stencil_extent<NP, L>(y, l1, s, ly, hy);
    }
    const bool flat_y = a.ny == 1 && a.bc_y != 2;  // walls: the ghost rows differ
    constexpr int RS = red_slots<Shape::kThreads>();
    int X0 = block_min(lx, red);
    int X1 = -block_min(-hx, red + RS);
    int Y0 = block_min(ly, red + 2 * RS);
    int Y1 = -block_min(-hy, red + 3 * RS);
    clip_region(tx0, ty0, sh.tx(), sh.ty(), cap, flat_y, X0, X1, Y0, Y1);
    const int W = X1 >= X0 ? X1 - X0 + 1 : 0;
    const int H = Y1 >= Y0 ? Y1 - Y0 + 1 : 0;

    // the tile's reference moments (every node of the tile shares its block)
    GlobalTaps<P, NP, L> glob{mom, a.mstride, a.nx, a.ny, a.bc_x, a.bc_y, a.moff, a.wall_h, {}};
    load_moments<P, nmom<L>()>(mom, a.mstride, a.moff + ref_node(tx0, ty0, a.nx), glob.ref);

    for (int idx = threadIdx.x; idx < W * H; idx += nthreads) {
        const int gx = wrap_index(X0 + idx % W, a.nx, a.bc_x);
        const int gy = mom_row(Y0 + idx / W, a.ny, a.bc_y, a.wall_h);
        P M[nmom_padded<P, L>()];
        load_moments<P, nmom<L>()>(mom, a.mstride, a.moff + (long long)gy * a.nx + gx, M);
#pragma unroll
        for (int k = 0; k < nmom<L>(); ++k) M[k] -= glob.ref[k];
        store_node_lds<P, L>(lds, idx, cap, M);
    }
    __syncthreads();

    constexpr int G = sizeof(P) == 4 && Shape::kThreads == 512 ? 1
                      : (sizeof(P) == 8 ? POND_TAP_GROUP_F64 : POND_TAP_GROUP_F32);
    const TileTaps<P, NP, L, G> taps{lds, cap, X0, Y0, X1, Y1, W, flat_y, glob};
    node_step<P, NP, S, L>(a, taps, x, y, n, live, l0, l1, l2, src, dst, mom_out, cnt);
}

// Moments up to the lattice's Grad order (three on D2Q16, four on D2Q25) of
// f and g of node n (Eq. genericMomentUptoO3), about u_ref, stored as grouped
// planes.
template <typename P, class L = D2Q16>
__device__ __forceinline__ void node_moments(const StepArgs &a, DevState st, P *__restrict__ mom,
                                             long long n) {
    const P s = P(sqrt(st.T[n]));
    const P dx = P(st.ux[n] - a.uref_x), dy = P(st.uy[n] - a.uref_y);
    constexpr int NM = L::NM;
    P M[nmom_padded<P, L>()];
#pragma unroll
    for (int k = 0; k < nmom_padded<P, L>(); ++k) M[k] = P(0);
    // through the lattice sums, in the order the step forms them (the same bits)
    P Cf[NM], Cg[NM], Sf[L::N + 1], Sg[L::N + 1];
#pragma unroll
    for (int k = 0; k < NM; ++k) Cf[k] = Cg[k] = P(0);
#pragma unroll
    for (int q = 0; q <= L::N; ++q) Sf[q] = Sg[q] = P(0);
    double mass = 0.0, gzero = 0.0;  // zeroth moments summed in FP64, as the step does
#pragma unroll
    for (int ia = 0; ia < L::Q1; ++ia) {
#pragma unroll
        for (int b = 0; b < L::Q1; ++b) {
            const int i = L::Q1 * ia + b;
            const P fi = pop_plane<P>(st.f, i, a.N)[n];
            const P gi = pop_plane<P>(st.g, i, a.N)[n];
            mass += double(fi);
            gzero += double(gi);
            column_add<L>(Sf, b, fi);
            column_add<L>(Sg, b, gi);
        }
        column_flush<L>(Cf, Sf, ia);
        column_flush<L>(Cg, Sg, ia);
    }
    moments_from_lattice_sums<L>(Cf, s, dx, dy, M);
    moments_from_lattice_sums<L>(Cg, s, dx, dy, M + NM);
    M[0] = P(mass);
    M[NM] = P(gzero);
    store_moments<P, nmom<L>()>(mom, a.mstride, a.moff + n, M);
}

}  // namespace pond
