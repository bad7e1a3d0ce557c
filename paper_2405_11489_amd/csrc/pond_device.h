// pond_device.h -- device-side lattice constants and per-node arithmetic of the
// PonD f+g step (D2Q16, total-energy split).
//
// Moment ordering used everywhere on the device (10 per distribution):
//   k : 0    1    2    3    4    5    6    7    8    9
//  pq : 00   10   01   20   11   02   30   21   12   03
// where M_pq = sum_i pop_i V_ix^p V_iy^q.  Device moments are taken about a
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
    return t;
}

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
template <int NP, typename P>
__device__ __forceinline__ int lagrange(double y, P w[NP]) {
    y = fmin(fmax(y, -1.0e9), 1.0e9);  // keeps the node index representable
    if constexpr (NP == 4) {
        const double fl = floor(y);
        const P d = P(y - fl);
        const P dm1 = d - P(1), dm2 = d - P(2), dp1 = d + P(1);
        w[0] = -d * dm1 * dm2 * P(1.0 / 6.0);
        w[1] = dp1 * dm1 * dm2 * P(0.5);
        w[2] = -dp1 * d * dm2 * P(0.5);
        w[3] = dp1 * d * dm1 * P(1.0 / 6.0);
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
