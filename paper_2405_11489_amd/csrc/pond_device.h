// pond_device.h -- device-side lattice constants and per-node arithmetic of the
// PonD f+g step (lattices D2Q16 and D2Q25 of Table I).
//
// Moment ordering used everywhere on the device (10 per distribution on D2Q16,
// orders 0..3; 15 on D2Q25, orders 0..4):
//   k : 0    1    2    3    4    5    6    7    8    9    10   11   12   13   14
//  pq : 00   10   01   20   11   02   30   21   12   03   40   31   22   13   04
// where M_pq = sum_i pop_i V_ix^p V_iy^q (order n starts at k = n(n+1)/2, p
// descending).  Device moments are taken about a
// fixed per-instance reference velocity u_ref (V = C - u_ref), which keeps the
// float planes free of the cancellation a Mach-2 background would cause; any
// fixed origin gives the same transform.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pond {

// Table I, D1Q4 (rT_L = 1): ascending abscissae -c_out, -c_in, c_in, c_out with
// c_in = sqrt(3 - sqrt 6), c_out = sqrt(3 + sqrt 6); weights (3 + sqrt 6)/12 on
// the inner pair, (3 - sqrt 6)/12 on the outer pair.
constexpr double kCin = 0.741963784302726;
constexpr double kCout = 2.3344142183389773;
constexpr double kWin = 0.4541241452319315;
constexpr double kWout = 0.04587585476806851;

__host__ __device__ constexpr double c1(int a) {
    return a == 0 ? -kCout : (a == 1 ? -kCin : (a == 2 ? kCin : kCout));
}
__host__ __device__ constexpr double w1(int a) { return (a == 0 || a == 3) ? kWout : kWin; }

constexpr int kQ = 16;       // D2Q16 velocities, i = 4a + b, c_i = (c1(a), c1(b))
constexpr int kNM = 10;      // moments / Grad coefficients per distribution

// Per-velocity constants, i = 4a + b with c_i = (c1(a), c1(b)).
//  recon[i][k]: weights of the N = 3 Grad reconstruction (Eq.
//    gradGeneralTransform with rT_L = 1) on the normalised central moments m_k
//    (same ordering as the moments): pop_i = sum_k recon[i][k] m_k, from the
//    Hermite coefficients a0 = m00, a1 = m10|m01, a2 = m20 - m00 | m11 |
//    m02 - m00, a3 = m30 - 3 m10 | m21 - m01 | m12 - m10 | m03 - 3 m01 written
//    into w_i sum_n a_(n) : H_(n)(c_i) / n!.
//  herm[i][k]: the same reconstruction on the Hermite coefficients a_k:
//    pop_i = sum_k herm[i][k] a_k = w_i (a0 + a1.H1 + a2:H2/2 + a3:H3/6).
struct VelocityTables {
    double recon[kQ][kNM];
    double herm[kQ][kNM];
};

constexpr VelocityTables make_velocity_tables() {
    VelocityTables t{};
    for (int i = 0; i < kQ; ++i) {
        const double cx = c1(i / 4), cy = c1(i % 4), w = w1(i / 4) * w1(i % 4);
        const double Hxx = cx * cx - 1.0, Hyy = cy * cy - 1.0, Hxy = cx * cy;
        const double Hxxx = cx * cx * cx - 3.0 * cx, Hyyy = cy * cy * cy - 3.0 * cy;
        const double Hxxy = Hxx * cy, Hxyy = cx * Hyy;
        const double r[kNM] = {1.0 - 0.5 * Hxx - 0.5 * Hyy, cx - 0.5 * Hxxx - 0.5 * Hxyy,
                               cy - 0.5 * Hxxy - 0.5 * Hyyy, 0.5 * Hxx, Hxy, 0.5 * Hyy,
                               Hxxx / 6.0, 0.5 * Hxxy, 0.5 * Hxyy, Hyyy / 6.0};
        const double h[kNM] = {1.0, cx, cy, 0.5 * Hxx, Hxy, 0.5 * Hyy,
                               Hxxx / 6.0, 0.5 * Hxxy, 0.5 * Hxyy, Hyyy / 6.0};
        for (int k = 0; k < kNM; ++k) {
            t.recon[i][k] = w * r[k];
            t.herm[i][k] = w * h[k];
        }
    }
    return t;
}

// ---------------------------------------------------------------- lattices
// Table I, D1Q5 (rT_L = 1): abscissae -c_out, -c_in, 0, c_in, c_out with
// c_in = sqrt(5 - sqrt 10), c_out = sqrt(5 + sqrt 10); weights 8/15 at 0,
// (7 + 2 sqrt 10)/60 on the inner pair, (7 - 2 sqrt 10)/60 on the outer pair.
constexpr double kC5in = 1.3556261799742657;
constexpr double kC5out = 2.8569700138728056;
constexpr double kW5zero = 0.53333333333333333;
constexpr double kW5in = 0.22207592200561266;
constexpr double kW5out = 0.011257411327720682;

// Lattice traits: Q1 points per axis, Q = Q1^2 velocities (i = Q1 a + b,
// c_i = (c(a), c(b))), Grad order N = Q1 - 1 with NM = (N + 1)(N + 2)/2
// moments / coefficients per distribution.
struct D2Q16 {
    static constexpr int Q1 = 4, Q = 16, N = 3, NM = 10;
    __host__ __device__ static constexpr double c(int a) { return c1(a); }
    __host__ __device__ static constexpr double w(int a) { return w1(a); }
};
struct D2Q25 {
    static constexpr int Q1 = 5, Q = 25, N = 4, NM = 15;
    __host__ __device__ static constexpr double c(int a) {
        return a == 0 ? -kC5out : (a == 1 ? -kC5in : (a == 2 ? 0.0 : (a == 3 ? kC5in : kC5out)));
    }
    __host__ __device__ static constexpr double w(int a) {
        return (a == 0 || a == 4) ? kW5out : (a == 2 ? kW5zero : kW5in);
    }
};

// Index k of the moment with exponents (p, q) (orders up to 4), and back.
__host__ __device__ constexpr int mom_index(int p, int q) {
    return (p + q) * (p + q + 1) / 2 + q;
}
__host__ __device__ constexpr int mom_order(int k) {
    return k < 1 ? 0 : (k < 3 ? 1 : (k < 6 ? 2 : (k < 10 ? 3 : 4)));
}
__host__ __device__ constexpr int mom_py(int k) {
    return k - mom_order(k) * (mom_order(k) + 1) / 2;
}
__host__ __device__ constexpr int mom_px(int k) { return mom_order(k) - mom_py(k); }

// Coefficient of x^p in the probabilists' Hermite polynomial He_n(x), n <= 4:
// He_0 = 1, He_1 = x, He_2 = x^2 - 1, He_3 = x^3 - 3x, He_4 = x^4 - 6x^2 + 3.
__host__ __device__ constexpr double he_coef(int n, int p) {
    return p == n ? 1.0
         : (n == 2 && p == 0) ? -1.0
         : (n == 3 && p == 1) ? -3.0
         : (n == 4 && p == 2) ? -6.0
         : (n == 4 && p == 0) ? 3.0
         : 0.0;
}
__host__ __device__ constexpr double he_value(int n, double x) {
    return he_coef(n, 0) + x * (he_coef(n, 1) + x * (he_coef(n, 2) + x * (he_coef(n, 3) +
                                                                            x * he_coef(n, 4))));
}
// n! and C(n, k) for n <= 4
__host__ __device__ constexpr double factorial_c(int n) {
    return n <= 1 ? 1.0 : (n == 2 ? 2.0 : (n == 3 ? 6.0 : 24.0));
}
__host__ __device__ constexpr double binom_c(int n, int k) {
    return factorial_c(n) / (factorial_c(k) * factorial_c(n - k));
}

// Reconstruction tables of a lattice (the D2Q16 tables above, written for any
// order): herm[i][k(a,b)] = w_i He_a(c_ix) He_b(c_iy) / (a! b!), so that
// pop_i = sum_k herm[i][k] A_k for Hermite coefficients A_ab; recon[i][k(p,q)]
// = sum_{a >= p, b >= q} herm[i][k(a,b)] he_a[p] he_b[q], the same
// reconstruction on the normalised central moments m_pq.
template <class L>
struct LatticeTables {
    double recon[L::Q][L::NM];
    double herm[L::Q][L::NM];
};

template <class L>
constexpr LatticeTables<L> make_lattice_tables() {
    LatticeTables<L> t{};
    for (int i = 0; i < L::Q; ++i) {
        const double cx = L::c(i / L::Q1), cy = L::c(i % L::Q1);
        const double w = L::w(i / L::Q1) * L::w(i % L::Q1);
        for (int k = 0; k < L::NM; ++k) {
            const int a = mom_px(k), b = mom_py(k);
            t.herm[i][k] = w * he_value(a, cx) * he_value(b, cy) / (factorial_c(a) * factorial_c(b));
        }
        for (int k = 0; k < L::NM; ++k) {
            const int p = mom_px(k), q = mom_py(k);
            double r = 0.0;
            for (int j = 0; j < L::NM; ++j) {
                const int a = mom_px(j), b = mom_py(j);
                if (a >= p && b >= q) r += t.herm[i][j] * he_coef(a, p) * he_coef(b, q);
            }
            t.recon[i][k] = r;
        }
    }
    return t;
}

template <typename P, class L>
struct LatticeTablesP {
    P recon[L::Q][L::NM];
    P herm[L::Q][L::NM];
};

// ------------------------------------------------ mass-exact float tables
// Rounding every table entry to the nearest float leaves the column that
// carries the mass -- the weights w_i of a0 in the reconstruction, the weights
// of m00 in the transformation -- summing to 1 only up to a few ulps (D2Q16:
// the sixteen weights sum to 1 - 1.96e-8).  That deficit is the same at every
// node and every step, so FP32 steps would lose (or gain) that fraction of
// mass and energy each step: 4e-5 of the density over 2000 steps.  The column
// is therefore rounded so that its float entries sum to 1 exactly: after
// rounding to nearest, the entries of one symmetry class (equal |c_x|, |c_y|
// up to exchange of the axes, which keeps the lattice's symmetries) move
// together by whole ulps, the class with the largest step first.

// ulp of the float nearest to v (|v| normal)
__host__ __device__ constexpr double ulp_of_float(double v) {
    v = v < 0 ? -v : v;
    double u = 1.0;
    if (v >= 1.0) {
        while (u * 2.0 <= v) u *= 2.0;
    } else {
        while (u > v) u *= 0.5;
    }
    return u / 8388608.0;  // 2^-23
}

// Rounds column col of the Q x NM table d into f (float) so that the float
// entries sum exactly to target; returns the deficit left (0 when exact).
template <int Q1, int NM>
constexpr double round_column_to_sum(const double (&d)[Q1 * Q1][NM], float (&f)[Q1 * Q1][NM],
                                     int col, double target) {
    constexpr int Q = Q1 * Q1;
    double sum = 0.0;  // exact: a few dozen floats within a dozen binades
    for (int i = 0; i < Q; ++i) {
        f[i][col] = float(d[i][col]);
        sum += double(f[i][col]);
    }
    double deficit = target - sum;
    // symmetry classes, keyed by the sorted distances of (a, b) from the centre
    int key[Q] = {};
    for (int i = 0; i < Q; ++i) {
        const int da = 2 * (i / Q1) - (Q1 - 1), db = 2 * (i % Q1) - (Q1 - 1);
        const int ua = da < 0 ? -da : da, ub = db < 0 ? -db : db;
        key[i] = ua < ub ? ua * 64 + ub : ub * 64 + ua;
    }
    bool done[Q] = {};
    for (int pass = 0; pass < Q && deficit != 0.0; ++pass) {
        // the unprocessed class with the largest step (members x ulp)
        int best = -1;
        double best_step = 0.0;
        for (int i = 0; i < Q; ++i) {
            if (done[i] || f[i][col] == 0.0f) continue;
            int m = 0;
            for (int j = 0; j < Q; ++j) m += key[j] == key[i] ? 1 : 0;
            const double step = m * ulp_of_float(double(f[i][col]));
            if (step > best_step) {
                best_step = step;
                best = i;
            }
        }
        if (best < 0) break;
        const double q = deficit / best_step;
        const long long n = (long long)(q < 0 ? -q : q) * (q < 0 ? -1 : 1);  // toward zero
        for (int j = 0; j < Q; ++j)
            if (key[j] == key[best]) {
                done[j] = true;
                if (n != 0) {
                    const double nv = double(f[j][col]) + double(n) * ulp_of_float(double(f[j][col]));
                    deficit -= nv - double(f[j][col]);
                    f[j][col] = float(nv);
                }
            }
    }
    return deficit;
}

template <typename P, class L>
constexpr LatticeTablesP<P, L> make_lattice_tables_p() {
    const LatticeTables<L> d = make_lattice_tables<L>();
    LatticeTablesP<P, L> t{};
    for (int i = 0; i < L::Q; ++i)
        for (int k = 0; k < L::NM; ++k) {
            t.recon[i][k] = P(d.recon[i][k]);
            t.herm[i][k] = P(d.herm[i][k]);
        }
    if constexpr (sizeof(P) == 4) {
        round_column_to_sum<L::Q1, L::NM>(d.recon, t.recon, 0, 1.0);
        round_column_to_sum<L::Q1, L::NM>(d.herm, t.herm, 0, 1.0);
    }
    return t;
}

// Exact float sum of a column (for the static checks below).
template <int Q, int NM>
constexpr double float_column_sum(const float (&f)[Q][NM], int col) {
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += double(f[i][col]);
    return s;
}

// Generic order-N versions of central_normalised / hermite_from_central (the
// D2Q16 ones below are written out for N = 3).
// m_pq = is^(p+q) sum_{r<=p, t<=q} C(p,r) C(q,t) (-dx)^(p-r) (-dy)^(q-t) M_rt.
template <class L, typename P>
__device__ __forceinline__ void central_normalised_n(const P M[L::NM], P dx, P dy, P is,
                                                     P m[L::NM]) {
    constexpr int N = L::N;
    P ex[N + 1], ey[N + 1], sc[N + 1];
    ex[0] = ey[0] = sc[0] = P(1);
#pragma unroll
    for (int j = 1; j <= N; ++j) {
        ex[j] = ex[j - 1] * (-dx);
        ey[j] = ey[j - 1] * (-dy);
        sc[j] = sc[j - 1] * is;
    }
    // shift in x: T[p][t] = sum_r C(p,r) ex^(p-r) M[r][t]; each sum starts at
    // its unit term (r = p), so it takes p multiply-adds
    P T[L::NM];
#pragma unroll
    for (int k = 0; k < L::NM; ++k) {
        const int p = mom_px(k), t = mom_py(k);
        P acc = M[k];
#pragma unroll
        for (int r = p - 1; r >= 0; --r) acc += (P(binom_c(p, r)) * ex[p - r]) * M[mom_index(r, t)];
        T[k] = acc;
    }
    // shift in y, then the scale is^(p+q)
#pragma unroll
    for (int k = 0; k < L::NM; ++k) {
        const int p = mom_px(k), q = mom_py(k);
        P acc = T[k];
#pragma unroll
        for (int t = q - 1; t >= 0; --t) acc += (P(binom_c(q, t)) * ey[q - t]) * T[mom_index(p, t)];
        m[k] = p + q == 0 ? acc : acc * sc[p + q];
    }
}

// A_ab = sum_{p<=a, q<=b} he_a[p] he_b[q] m_pq.
template <class L, typename P>
__device__ __forceinline__ void hermite_from_central_n(const P m[L::NM], P A[L::NM]) {
#pragma unroll
    for (int k = 0; k < L::NM; ++k) {
        const int a = mom_px(k), b = mom_py(k);
        P acc = P(0);
#pragma unroll
        for (int j = 0; j < L::NM; ++j) {
            const int p = mom_px(j), q = mom_py(j);
            if (p <= a && q <= b && he_coef(a, p) != 0.0 && he_coef(b, q) != 0.0)
                acc += P(he_coef(a, p) * he_coef(b, q)) * m[j];
        }
        A[k] = acc;
    }
}

template <typename P>
struct VelocityTablesP {
    P recon[kQ][kNM];
    P herm[kQ][kNM];
};

template <typename P>
constexpr VelocityTablesP<P> make_velocity_tables_p() {
    const VelocityTables d = make_velocity_tables();
    VelocityTablesP<P> t{};
    for (int i = 0; i < kQ; ++i)
        for (int k = 0; k < kNM; ++k) {
            t.recon[i][k] = P(d.recon[i][k]);
            t.herm[i][k] = P(d.herm[i][k]);
        }
    if constexpr (sizeof(P) == 4) {  // mass-exact float tables (see above)
        round_column_to_sum<4, kNM>(d.recon, t.recon, 0, 1.0);
        round_column_to_sum<4, kNM>(d.herm, t.herm, 0, 1.0);
    }
    return t;
}

static_assert(float_column_sum(make_velocity_tables_p<float>().herm, 0) == 1.0,
              "D2Q16 float weights must sum to 1 exactly");
static_assert(float_column_sum(make_velocity_tables_p<float>().recon, 0) == 1.0,
              "D2Q16 float m00 transform weights must sum to 1 exactly");
static_assert(float_column_sum(make_lattice_tables_p<float, D2Q25>().herm, 0) == 1.0,
              "D2Q25 float weights must sum to 1 exactly");
static_assert(float_column_sum(make_lattice_tables_p<float, D2Q25>().recon, 0) == 1.0,
              "D2Q25 float m00 transform weights must sum to 1 exactly");

// Central moments about d = (dx, dy), scaled by 1/s^(p+q): the normalised
// moments m_pq of xi = (V - d)/s, from raw moments M about the same origin.
template <typename P>
__device__ __forceinline__ void central_normalised(const P M[kNM], P dx, P dy, P is, P m[kNM]) {
    const P dx2 = dx * dx, dy2 = dy * dy, dxy = dx * dy;
    const P c00 = M[0];
    const P c10 = M[1] - dx * M[0];
    const P c01 = M[2] - dy * M[0];
    const P c20 = M[3] - P(2) * dx * M[1] + dx2 * M[0];
    const P c11 = M[4] - dx * M[2] - dy * M[1] + dxy * M[0];
    const P c02 = M[5] - P(2) * dy * M[2] + dy2 * M[0];
    const P c30 = M[6] - P(3) * dx * M[3] + P(3) * dx2 * M[1] - dx2 * dx * M[0];
    const P c21 = M[7] - P(2) * dx * M[4] - dy * M[3] + dx2 * M[2] + P(2) * dxy * M[1] - dx2 * dy * M[0];
    const P c12 = M[8] - P(2) * dy * M[4] - dx * M[5] + dy2 * M[1] + P(2) * dxy * M[2] - dx * dy2 * M[0];
    const P c03 = M[9] - P(3) * dy * M[5] + P(3) * dy2 * M[2] - dy2 * dy * M[0];
    const P is2 = is * is, is3 = is2 * is;
    m[0] = c00;
    m[1] = c10 * is;
    m[2] = c01 * is;
    m[3] = c20 * is2;
    m[4] = c11 * is2;
    m[5] = c02 * is2;
    m[6] = c30 * is3;
    m[7] = c21 * is3;
    m[8] = c12 * is3;
    m[9] = c03 * is3;
}

// Hermite (Grad) coefficients a0..a3 from normalised central moments.
template <typename P>
__device__ __forceinline__ void hermite_from_central(const P m[kNM], P a[kNM]) {
    a[0] = m[0];
    a[1] = m[1];
    a[2] = m[2];
    a[3] = m[3] - m[0];
    a[4] = m[4];
    a[5] = m[5] - m[0];
    a[6] = m[6] - P(3) * m[1];
    a[7] = m[7] - m[2];
    a[8] = m[8] - m[1];
    a[9] = m[9] - P(3) * m[2];
}

// Lagrange interpolation weights for a departure coordinate y (node units).
// NP = 4: nodes floor(y)-1 .. floor(y)+2 (cubic); NP = 3: nodes m-1, m, m+1 with
// m = floor(y + 1/2) (quadratic).  Returns the first node.
// y must be finite and within the int range (the step clamps the frame it
// computes departure points from).
template <int NP, typename P>
__device__ __forceinline__ int lagrange(double y, P w[NP]) {
    if constexpr (NP == 4) {
        const double fl = floor(y);
        const P d = P(y - fl);
        const P dm1 = d - P(1), dm2 = d - P(2), dp1 = d + P(1);
        if constexpr (sizeof(P) == 4) {
            // 1/6 is no float: fl(1/6) exceeds it by 3e-8, which would scale both
            // outer weights, and so the weights' sum, the same way at every node
            // and every step (a mass drift of -5e-9 per step on average); the
            // product with 1/6 is taken as x hi + x lo with a single rounding
            constexpr float kHi = float(1.0 / 6.0);
            constexpr float kLo = float(1.0 / 6.0 - double(kHi));
            const P a0 = -d * dm1 * dm2, a3 = dp1 * d * dm1;
            w[0] = fmaf(a0, kHi, a0 * kLo);
            w[3] = fmaf(a3, kHi, a3 * kLo);
        } else {
            w[0] = -d * dm1 * dm2 * P(1.0 / 6.0);
            w[3] = dp1 * d * dm1 * P(1.0 / 6.0);
        }
        w[1] = dp1 * dm1 * dm2 * P(0.5);
        w[2] = -dp1 * d * dm2 * P(0.5);
        return int(fl) - 1;
    } else {
        const double m = floor(y + 0.5);
        const P d = P(y - m);
        w[0] = d * (d - P(1)) * P(0.5);
        w[1] = (P(1) - d) * (P(1) + d);
        w[2] = (d + P(1)) * d * P(0.5);
        return int(m) - 1;
    }
}

__device__ __forceinline__ int wrap_index(int i, int n, int bc) {
    if (bc == 0) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

}  // namespace pond
