/*
 * pond_oracle.c -- plain FP64 CPU oracle of the particles-on-demand (PonD)
 * stream-and-collide step of the double-distribution-function BGK model:
 * total-energy, internal-energy and non-translational energy splits, on the
 * D2Q16 and D2Q25 lattices of Table I.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or constant with the GPU library, and the GPU library never calls it.
 *
 * Source: S. A. Hosseini, A. Bhadauria, I. V. Karlin, "Probing double
 * distribution function models in the lattice Boltzmann method for highly
 * compressible flows", arXiv:2405.11489.  Each function cites the passage it
 * follows.  The step is written the slow, literal way:
 *   for every destination node, every predictor-corrector iterate, every
 *   discrete velocity and every stencil node, the stencil node's populations
 *   are transformed into the iterate's frame (frame transformation, Sec.
 *   "Frame transformation") and only then weighted by the interpolation kernel
 *   (Eq. propagationInterpolated).
 * No blocking, fusion or reordering beyond that.
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - interpolation: Lagrange polynomial stencil; 4 points (cubic) by default,
 *     3 points (the paper's "2nd-order" stencil) on request;
 *   - the gather is evaluated at the departure point x - C_i(lambda_bar) dt,
 *     with C_i in the destination frame;
 *   - the destination frame is found by a predictor-corrector fixed-point
 *     iteration (predictor: the node's own frame at time t), which the paper
 *     takes from its PonD reference; the converged populations are re-projected
 *     onto the frame of their own moments before the collision;
 *   - Grad order N = 3 for both f and g on D2Q16, N = 4 on D2Q25 (the order
 *     the non-translational split needs for f's fourth moment, Sec. II); the
 *     order-4 coefficients follow the same definition as the printed a0..a3,
 *     the Hermite projection in the destination frame;
 *   - the collision sign is -(1/tau)(f - f^eq) (Eq. boltz_eq carries a
 *     typo'd sign; the g-equations of Sec. II have the correct one);
 *   - discrete relaxation time: nu = (tau - 1/2) T, omega = 1/tau;
 *   - Prandtl number != 1: quasi-equilibrium with the Fourier part of the
 *     energy flux relaxed at omega_1 = 1/tau_1, tau_1 = 1/2 + (tau - 1/2)/Pr,
 *     and the viscous-heating part u . P^neq at omega (Sec. II points to the
 *     quasi-equilibrium approach without giving its form); in the internal-
 *     energy split g carries no viscous-heating flux, so g relaxes at omega_1;
 *   - internal-energy split source G = -f (v - u).(d_t u + v.grad u), taken
 *     to second order in the time step the way a BGK source is: g relaxes to
 *     the equilibrium of U = sum g + (sum G)/2 and receives (1 - omega_g/2) G
 *     after the collision (omega_g its relaxation rate), so the energy gains
 *     sum G per step; f in G is the time-centred population, the mean of the
 *     re-projected gathered f and the collided f (with the gathered f alone
 *     the viscous heating came out 2 tau / (2 tau - 1) times too large),
 *     whose pressure tensor is rho T I + (1 - omega/2) P~neq, so that
 *     sum G = -(omega/2) rho T div u - (1 - omega/2) P~ : grad u and the frame
 *     temperature solves rho c_v T = sum g + (sum G)/2 in closed form (see
 *     conserved()); u the new frame velocity, d_t u the difference between
 *     the new and the time-t frame velocity of the node; grad u is taken at
 *     the end of the step, where the collision and the source act, by linear
 *     extrapolation along the node's trajectory: 2 G_t(x - u) - G_{t-1}(x - 2u)
 *     with u the node's time-t frame velocity and G_t the velocity gradient
 *     of the time-t frames at a point, the bilinear interpolation of the
 *     nodal central differences (four neighbours, wrapped or clamped like the
 *     stencil; a neighbour row beyond a wall takes the ghost frame velocity
 *     of the wall closure, 2 U_wall - u of the mirror node along x, -u along
 *     y; a point beyond the wall rows is taken on the last row).  Without
 *     the frames of t - 1 (the first step after initialisation) the time-t
 *     frames stand in for them.  Advected with the flow,
 *     the extrapolation is exact; at rest it is 2 grad u(t) - grad u(t - 1).
 *     The time-t gradient alone lags the collision by a step and left
 *     acoustic waves under-damped by (gamma - 1) T k^2 / 2;
 *   - non-translational split: the paper's single-relaxation BGK only (Pr = 1;
 *     its quasi-equilibrium form is not given and not built here);
 *   - walls (the thermal Couette flow of Sec. "Measuring viscous heating"; the
 *     paper gives no boundary scheme): ghost nodes beyond the wall mirror the
 *     interior, see ghost_node().
 *
 * Units: lattice units, dx = dt = 1, r = 1, T_L = 1 (Table I column rT_L).
 * Layout (oracle only): node n = y*nx + x; populations pop[n*Q + i] with
 * Q = 16 or 25; frame lam[n*3 + {0,1,2}] = (u_x, u_y, T).  Velocity
 * i = q1*a + b (q1 = 4 or 5) has c_i = (c_a, c_b) with the one-dimensional
 * abscissae in ascending order.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_ABI 5
#define Q1 4      /* D1Q4 */
#define Q 16      /* D2Q16 */
#define QMAX 25   /* D2Q25 */

typedef struct {
    int nx, ny;
    int bc_x, bc_y;        /* 0 = periodic, 1 = clamp (zero-gradient); bc_y = 2: walls */
    int interp_points;     /* 4 = cubic Lagrange, 3 = quadratic Lagrange */
    int pc_max_iter;       /* predictor-corrector iteration cap (>= 1) */
    double tau;            /* discrete relaxation time, > 1/2 */
    double prandtl;        /* > 0; 1 = the paper's plain BGK */
    double gamma;          /* adiabatic exponent, c_v = 1/(gamma - 1) */
    double pc_tol;         /* predictor-corrector tolerance */
    int split;             /* 0 = total energy (Eq. total_energy_g), 1 = internal energy
                              (Eq. int_energy_g), 2 = non-translational energy
                              (Eq. nt_energy_g) */
    int lattice;           /* 16 = D2Q16 (D1Q4 x D1Q4), 25 = D2Q25 (D1Q5 x D1Q5) */
    double wall_ux[2];     /* bc_y = 2: x-velocity of the bottom / top wall */
    double wall_T[2];      /* bc_y = 2: temperature of the bottom / top wall */
} oracle_params;

/* status bits per node written by oracle_step */
#define ORACLE_NONCONVERGED 1
#define ORACLE_NONPHYSICAL 2

int oracle_abi_version(void) { return ORACLE_ABI; }

/* Threads the OpenMP loops of this library use. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads of the following OpenMP loops (n >= 1). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Table I, row D1Q4 (rT_L = 1): abscissae +-sqrt(3 -+ sqrt 6) with weights
 * (3 +- sqrt 6)/12, the inner pair carrying the larger weight. */
void oracle_lattice_1d(double c[Q1], double w[Q1])
{
    double s6 = sqrt(6.0);
    double c_in = sqrt(3.0 - s6), c_out = sqrt(3.0 + s6);
    double w_in = (3.0 + s6) / 12.0, w_out = (3.0 - s6) / 12.0;
    c[0] = -c_out; c[1] = -c_in; c[2] = c_in; c[3] = c_out;
    w[0] = w_out;  w[1] = w_in;  w[2] = w_in; w[3] = w_out;
}

/* Table I, D2Q16 = D1Q4 x D1Q4: velocity i = 4a + b. */
void oracle_lattice_2d(double cx[Q], double cy[Q], double w[Q])
{
    double c[Q1], w1[Q1];
    oracle_lattice_1d(c, w1);
    for (int a = 0; a < Q1; a++)
        for (int b = 0; b < Q1; b++) {
            cx[4 * a + b] = c[a];
            cy[4 * a + b] = c[b];
            w[4 * a + b] = w1[a] * w1[b];
        }
}

/* Table I, row D1Q5 (rT_L = 1): abscissae 0, +-sqrt(5 -+ sqrt 10) with weights
 * 8/15 at the origin, (7 + 2 sqrt 10)/60 on the inner pair, (7 - 2 sqrt 10)/60
 * on the outer pair. */
void oracle_lattice_1d_q5(double c[5], double w[5])
{
    double s10 = sqrt(10.0);
    double c_in = sqrt(5.0 - s10), c_out = sqrt(5.0 + s10);
    double w_in = (7.0 + 2.0 * s10) / 60.0, w_out = (7.0 - 2.0 * s10) / 60.0;
    c[0] = -c_out; c[1] = -c_in; c[2] = 0.0; c[3] = c_in; c[4] = c_out;
    w[0] = w_out;  w[1] = w_in;  w[2] = 8.0 / 15.0; w[3] = w_in; w[4] = w_out;
}

/* One-dimensional rule of the lattice with q1 = 4 (D1Q4) or 5 (D1Q5) points;
 * returns q1, or 0 for any other value. */
int oracle_lattice_1d_q(int q1, double *c, double *w)
{
    if (q1 == 4)
        oracle_lattice_1d(c, w);
    else if (q1 == 5)
        oracle_lattice_1d_q5(c, w);
    else
        return 0;
    return q1;
}

/* Tensor-product lattice D1Qq1 x D1Qq1: velocity i = q1*a + b has
 * c_i = (c_a, c_b), w_i = w_a w_b.  Returns Q = q1^2, or 0. */
int oracle_lattice_2d_q(int q1, double *cx, double *cy, double *w)
{
    double c[5], w1[5];
    if (!oracle_lattice_1d_q(q1, c, w1))
        return 0;
    for (int a = 0; a < q1; a++)
        for (int b = 0; b < q1; b++) {
            cx[q1 * a + b] = c[a];
            cy[q1 * a + b] = c[b];
            w[q1 * a + b] = w1[a] * w1[b];
        }
    return q1 * q1;
}

/* q1 of a lattice given by its velocity count (16 or 25), else 0. */
static int q1_of(int lattice) { return lattice == 16 ? 4 : (lattice == 25 ? 5 : 0); }

static double kron(int a, int b) { return a == b ? 1.0 : 0.0; }

/*
 * Frame transformation M_{lam_src -> lam_dst} (Sec. "Frame transformation").
 *   1. Lab-frame moments up to order three of the populations, with the
 *      particle velocities of the source frame C_i = sqrt(T_src) c_i + u_src
 *      (Eq. genericMomentUptoO3).
 *   2. Grad coefficients a_0..a_3 in the destination frame (the four equations
 *      that follow Eq. gradGeneralTransform), with theta = T_dst / T_L and the
 *      overline read as the sum over the distinct index permutations.
 *   3. Populations f_i = w_i sum_{n<=3} (1/n!) a_(n) : H_(n)(c_i)
 *      (Eq. gradGeneralTransform; with rT_L = 1 the normalisation is 1/n!).
 * Full rank-2 and rank-3 tensors are used, contracted index by index.
 * out may alias pop.
 */
void oracle_transform(const double *pop, const double *lam_src, const double *lam_dst, double *out)
{
    double cx[Q], cy[Q], w[Q];
    oracle_lattice_2d(cx, cy, w);

    double M0 = 0.0, M1[2] = {0.0, 0.0}, M2[2][2] = {{0.0}}, M3[2][2][2] = {{{0.0}}};
    double sTs = sqrt(lam_src[2]);
    for (int i = 0; i < Q; i++) {
        double V[2] = {sTs * cx[i] + lam_src[0], sTs * cy[i] + lam_src[1]};
        M0 += pop[i];
        for (int a = 0; a < 2; a++) {
            M1[a] += pop[i] * V[a];
            for (int b = 0; b < 2; b++) {
                M2[a][b] += pop[i] * V[a] * V[b];
                for (int g = 0; g < 2; g++)
                    M3[a][b][g] += pop[i] * V[a] * V[b] * V[g];
            }
        }
    }

    double th = lam_dst[2];
    double sq = sqrt(th);
    double u[2] = {lam_dst[0], lam_dst[1]};
    double a0 = M0, a1[2], a2[2][2], a3[2][2][2];
    for (int a = 0; a < 2; a++)
        a1[a] = (M1[a] - M0 * u[a]) / sq;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            a2[a][b] = (M2[a][b] - M0 * th * kron(a, b)
                        - sq * (u[a] * a1[b] + a1[a] * u[b])
                        - M0 * u[a] * u[b]) / th;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int g = 0; g < 2; g++) {
                double sym_u_S = u[a] * (M0 * kron(b, g) + a2[b][g])
                               + u[b] * (M0 * kron(a, g) + a2[a][g])
                               + u[g] * (M0 * kron(a, b) + a2[a][b]);
                double sym_a1_I = a1[a] * kron(b, g) + a1[b] * kron(a, g) + a1[g] * kron(a, b);
                double sym_a1_uu = a1[a] * u[b] * u[g] + a1[b] * u[a] * u[g] + a1[g] * u[a] * u[b];
                a3[a][b][g] = (M3[a][b][g] - th * sym_u_S - th * sq * sym_a1_I
                               - sq * sym_a1_uu - M0 * u[a] * u[b] * u[g]) / (th * sq);
            }

    double res[Q];
    for (int i = 0; i < Q; i++) {
        double c[2] = {cx[i], cy[i]};
        double s = a0;
        for (int a = 0; a < 2; a++)
            s += a1[a] * c[a];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                s += 0.5 * a2[a][b] * (c[a] * c[b] - kron(a, b));
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int g = 0; g < 2; g++) {
                    double H3 = c[a] * c[b] * c[g]
                              - (c[a] * kron(b, g) + c[b] * kron(a, g) + c[g] * kron(a, b));
                    s += a3[a][b][g] * H3 / 6.0;
                }
        res[i] = w[i] * s;
    }
    memcpy(out, res, sizeof res);
}

/* Probabilists' Hermite polynomial He_n(x) from the three-term recurrence
 * He_{n+1} = x He_n - n He_{n-1}, He_0 = 1, He_1 = x. */
static double hermite(int n, double x)
{
    if (n == 0)
        return 1.0;
    double h0 = 1.0, h1 = x;
    for (int k = 1; k < n; k++) {
        double h2 = x * h1 - k * h0;
        h0 = h1;
        h1 = h2;
    }
    return h1;
}

static double factorial(int n)
{
    double r = 1.0;
    for (int k = 2; k <= n; k++)
        r *= k;
    return r;
}

/*
 * Frame transformation as the Hermite projection of order N = order in the
 * destination frame (Sec. "Frame transformation", Eq. gradGeneralTransform).
 * The Grad coefficient tensors a_(n) of the destination frame are the Hermite
 * moments of the populations in the reduced velocity
 * xi_i = (C_i(lam_src) - u_dst) / sqrt(T_dst): a rank-n component with k
 * indices x and n - k indices y is
 *   A_{k, n-k} = sum_i pop_i He_k(xi_ix) He_{n-k}(xi_iy)
 * (the printed a0..a3 are this projection written through the source-frame
 * moments).  Reconstruction: a_(n) : H_(n)(c_i) / n! counts each component
 * once per ordering of its indices, C(n, k) times, so
 *   out_i = w_i sum_{k + l <= N} A_{k,l} He_k(c_ix) He_l(c_iy) / (k! l!).
 * Only moments of the populations up to order N enter.  Needs the Hermite
 * polynomials up to order N to be orthogonal on the lattice (N <= q1 - 1,
 * N <= 4); returns -1 otherwise, 0 on success.  out may alias pop.
 */
int oracle_transform_hermite(int q1, int order, const double *pop, const double *lam_src,
                             const double *lam_dst, double *out)
{
    double cx[QMAX], cy[QMAX], w[QMAX];
    int q = oracle_lattice_2d_q(q1, cx, cy, w);
    if (!q || order < 0 || order > 4 || order > q1 - 1)
        return -1;
    double A[5][5] = {{0.0}};
    double sTs = sqrt(lam_src[2]), sTd = sqrt(lam_dst[2]);
    for (int i = 0; i < q; i++) {
        double xi_x = (sTs * cx[i] + lam_src[0] - lam_dst[0]) / sTd;
        double xi_y = (sTs * cy[i] + lam_src[1] - lam_dst[1]) / sTd;
        for (int k = 0; k <= order; k++)
            for (int l = 0; k + l <= order; l++)
                A[k][l] += pop[i] * hermite(k, xi_x) * hermite(l, xi_y);
    }
    double res[QMAX];
    for (int i = 0; i < q; i++) {
        double s = 0.0;
        for (int k = 0; k <= order; k++)
            for (int l = 0; k + l <= order; l++)
                s += A[k][l] * hermite(k, cx[i]) * hermite(l, cy[i]) /
                     (factorial(k) * factorial(l));
        res[i] = w[i] * s;
    }
    memcpy(out, res, sizeof(double) * q);
    return 0;
}

/* The frame transformation of a lattice: the printed a0..a3 (oracle_transform)
 * on D2Q16 (q1 = 4), the order-4 Hermite projection on D2Q25 (q1 = 5). */
void oracle_transform_q(int q1, const double *pop, const double *lam_src, const double *lam_dst,
                        double *out)
{
    if (q1 == 4)
        oracle_transform(pop, lam_src, lam_dst, out);
    else
        oracle_transform_hermite(q1, 4, pop, lam_src, lam_dst, out);
}

/*
 * Local equilibria in the frame (u, T) (Sec. "Discrete velocity solver ...:
 * PonD"): f_i^eq = rho w_i, and the g^eq of Sec. II with v -> C_i =
 * sqrt(T) c_i + u and U' = U - rho D T / 2 = rho T (c_v - 1) for D = 2,
 * c_v = 1/(gamma - 1):
 *   split 0 (total energy):             g^eq = (U'/rho + v^2/2) f^eq;
 *   split 1 (internal energy):          g^eq = (U'/rho + (v - u)^2/2) f^eq;
 *   split 2 (non-translational energy): g^eq = (U'/rho) f^eq.
 * Lattice D1Qq1 x D1Qq1, q1 = 4 or 5.
 */
void oracle_equilibrium_q(int q1, int split, double rho, double ux, double uy, double T,
                          double gamma, double *feq, double *geq)
{
    double cx[QMAX], cy[QMAX], w[QMAX];
    int q = oracle_lattice_2d_q(q1, cx, cy, w);
    double cv = 1.0 / (gamma - 1.0);
    double sT = sqrt(T);
    for (int i = 0; i < q; i++) {
        double Cx = sT * cx[i] + ux, Cy = sT * cy[i] + uy;
        if (split == 1) {
            Cx -= ux;
            Cy -= uy;
        }
        feq[i] = rho * w[i];
        if (split == 2)
            geq[i] = w[i] * rho * (cv - 1.0) * T;
        else
            geq[i] = w[i] * (rho * (cv - 1.0) * T + 0.5 * rho * (Cx * Cx + Cy * Cy));
    }
}

void oracle_equilibrium_split(int split, double rho, double ux, double uy, double T,
                              double gamma, double *feq, double *geq)
{
    oracle_equilibrium_q(4, split, rho, ux, uy, T, gamma, feq, geq);
}

void oracle_equilibrium(double rho, double ux, double uy, double T, double gamma,
                        double *feq, double *geq)
{
    oracle_equilibrium_split(0, rho, ux, uy, T, gamma, feq, geq);
}

/*
 * BGK collision of f and g in the frame lam = (u, T) of their own moments.
 * f*_i = f_i + omega (f_i^eq - f_i) with omega = 1/tau.
 * Pr = 1 (and the non-translational split): g*_i = g_i + omega (g_i^eq - g_i),
 * the paper's model.
 * Pr != 1 (quasi-equilibrium reading): with P^neq = sum_i C_i C_i (f_i - f_i^eq)
 * and dq = u . P^neq, g^qe_i = g^eq_i + w_i (c_i . dq)/sqrt(T) carries the
 * equilibrium energy flux plus the viscous-heating flux; then
 * g*_i = g_i + omega_1 (g^qe_i - g_i) + omega (g^eq_i - g^qe_i).
 * The Fourier part of the energy flux relaxes at omega_1, the viscous-heating
 * part at omega; the zeroth moment (total energy) is untouched by either.
 */
void oracle_collide_q(int q1, int split, const double *ft, const double *gt, const double *lam,
                      double tau, double prandtl, double gamma, double *fo, double *go)
{
    double cx[QMAX], cy[QMAX], w[QMAX], feq[QMAX], geq[QMAX];
    int q = oracle_lattice_2d_q(q1, cx, cy, w);
    double rho = 0.0;
    for (int i = 0; i < q; i++)
        rho += ft[i];
    double ux = lam[0], uy = lam[1], T = lam[2];
    oracle_equilibrium_q(q1, split, rho, ux, uy, T, gamma, feq, geq);
    double omega = 1.0 / tau;
    double fin[QMAX], gin[QMAX];
    memcpy(fin, ft, sizeof(double) * q);
    memcpy(gin, gt, sizeof(double) * q);
    for (int i = 0; i < q; i++)
        fo[i] = fin[i] + omega * (feq[i] - fin[i]);
    if (prandtl == 1.0 || split == 2) {
        /* the non-translational split is taken with the paper's BGK only */
        for (int i = 0; i < q; i++)
            go[i] = gin[i] + omega * (geq[i] - gin[i]);
        return;
    }
    double tau1 = 0.5 + (tau - 0.5) / prandtl;
    double omega1 = 1.0 / tau1;
    if (split == 1) {
        /* internal energy: the flux of g is the heat flux alone */
        for (int i = 0; i < q; i++)
            go[i] = gin[i] + omega1 * (geq[i] - gin[i]);
        return;
    }
    double sT = sqrt(T);
    double P[2][2] = {{0.0}};
    for (int i = 0; i < q; i++) {
        double C[2] = {sT * cx[i] + ux, sT * cy[i] + uy};
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                P[a][b] += C[a] * C[b] * (fin[i] - feq[i]);
    }
    double u[2] = {ux, uy};
    double dq[2];
    for (int a = 0; a < 2; a++)
        dq[a] = u[0] * P[0][a] + u[1] * P[1][a];
    for (int i = 0; i < q; i++) {
        double gqe = geq[i] + w[i] * (cx[i] * dq[0] + cy[i] * dq[1]) / sT;
        go[i] = gin[i] + omega1 * (gqe - gin[i]) + omega * (geq[i] - gqe);
    }
}

void oracle_collide_split(int split, const double *ft, const double *gt, const double *lam,
                          double tau, double prandtl, double gamma, double *fo, double *go)
{
    oracle_collide_q(4, split, ft, gt, lam, tau, prandtl, gamma, fo, go);
}

void oracle_collide(const double *ft, const double *gt, const double *lam,
                    double tau, double prandtl, double gamma, double *fo, double *go)
{
    oracle_collide_split(0, ft, gt, lam, tau, prandtl, gamma, fo, go);
}

/*
 * Source of the internal-energy g-equation (Eq. int_g_evolution), one time
 * step: S_i = -f_i (C_i - u) . (a + C_i . grad u), with C_i = sqrt(T) c_i + u
 * in the frame lam = (u, T) of the populations f, a = d_t u and
 * grad[alpha][beta] = d_alpha u_beta.
 */
void oracle_internal_source_q(int q1, const double *f, const double *lam, const double a[2],
                              const double grad[2][2], double *S)
{
    double cx[QMAX], cy[QMAX], w[QMAX];
    int q = oracle_lattice_2d_q(q1, cx, cy, w);
    double sT = sqrt(lam[2]);
    for (int i = 0; i < q; i++) {
        double C[2] = {sT * cx[i] + lam[0], sT * cy[i] + lam[1]};
        double dv[2] = {sT * cx[i], sT * cy[i]};
        double s = 0.0;
        for (int b = 0; b < 2; b++)
            s += dv[b] * (a[b] + C[0] * grad[0][b] + C[1] * grad[1][b]);
        S[i] = -f[i] * s;
    }
}

void oracle_internal_source(const double *f, const double *lam, const double a[2],
                            const double grad[2][2], double *S)
{
    oracle_internal_source_q(4, f, lam, a, grad, S);
}

/*
 * Lagrange interpolation stencil for a departure coordinate y (in node
 * units).  npts = 4: nodes floor(y)-1 .. floor(y)+2 (cubic).  npts = 3: nodes
 * m-1, m, m+1 with m = floor(y + 1/2) (quadratic, ties to the upper node).
 * The weights are the Lagrange basis polynomials, written as the textbook
 * product prod_{m != j} (y - y_m)/(y_j - y_m).  *base receives the first node.
 */
int oracle_lagrange(int npts, double y, int *base, double *wts)
{
    int first;
    if (npts == 4)
        first = (int)floor(y) - 1;
    else if (npts == 3)
        first = (int)floor(y + 0.5) - 1;
    else
        return -1;
    for (int j = 0; j < npts; j++) {
        double l = 1.0;
        for (int m = 0; m < npts; m++)
            if (m != j)
                l *= (y - (double)(first + m)) / (double)(j - m);
        wts[j] = l;
    }
    *base = first;
    return 0;
}

static int node_index(int i, int n, int bc)
{
    if (bc == 0) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/*
 * Streaming with interpolated reconstruction, gather form
 * (Eq. propagationInterpolated): for each velocity i, the departure point is
 * y_i = x - C_i(lam_bar) dt (dt = 1), and
 *   {f_i, g_i}(x) = sum_s W(y_i - x_s) [M_{lam_s -> lam_bar} {f, g}(x_s)]_i,
 * every stencil node transformed from its own frame lam_s.
 */
/*
 * Wall boundary (bc_y = 2).  Walls at y = -1/2 (bottom, index 0) and
 * y = ny - 1/2 (top, index 1) move along x at wall_ux and are held at wall_T.
 * The stencil node at row y = -1 - j (bottom) or ny + j (top), j >= 0, is a
 * ghost mirroring interior row m = j or ny - 1 - j (clamped to the grid) of
 * the same column:
 *   - its frame continues the mirror node's through the wall linearly:
 *     u_gx = 2 U_w - u_mx, u_gy = -u_my, T_g = 2 T_w - T_m (at least T_w / 4);
 *   - its density keeps the mirror node's pressure: rho_g = rho_m T_m / T_g;
 *   - its populations are the equilibrium of that state plus the mirror
 *     node's non-equilibrium part carried into the ghost frame,
 *       f_g = f^eq(rho_g, lam_g) + M_{lam_m -> lam_g}(f_m - f^eq(rho_m, lam_m)),
 *     and g likewise with the split's g^eq.
 */
static void ghost_node(const oracle_params *P, const double *f, const double *g,
                       const double *lam, int jx, int jy, double *fo, double *go, double *lo)
{
    double cx[QMAX], cy[QMAX], w[QMAX];
    int q1 = q1_of(P->lattice);
    int q = oracle_lattice_2d_q(q1, cx, cy, w);
    int side = jy < 0 ? 0 : 1;
    int m = side == 0 ? -1 - jy : 2 * P->ny - 1 - jy;
    if (m < 0)
        m = 0;
    if (m > P->ny - 1)
        m = P->ny - 1;
    long s = (long)m * P->nx + jx;
    const double *fm = f + (long)q * s, *gm = g + (long)q * s, *lm = lam + 3 * s;
    double rho_m = 0.0;
    for (int i = 0; i < q; i++)
        rho_m += fm[i];
    double Tg = 2.0 * P->wall_T[side] - lm[2];
    if (Tg < 0.25 * P->wall_T[side])
        Tg = 0.25 * P->wall_T[side];
    lo[0] = 2.0 * P->wall_ux[side] - lm[0];
    lo[1] = -lm[1];
    lo[2] = Tg;
    double rho_g = rho_m * lm[2] / Tg;
    double feq[QMAX], geq[QMAX], fn[QMAX], gn[QMAX];
    oracle_equilibrium_q(q1, P->split, rho_m, lm[0], lm[1], lm[2], P->gamma, feq, geq);
    for (int i = 0; i < q; i++) {
        fn[i] = fm[i] - feq[i];
        gn[i] = gm[i] - geq[i];
    }
    oracle_transform_q(q1, fn, lm, lo, fn);
    oracle_transform_q(q1, gn, lm, lo, gn);
    oracle_equilibrium_q(q1, P->split, rho_g, lo[0], lo[1], lo[2], P->gamma, feq, geq);
    for (int i = 0; i < q; i++) {
        fo[i] = feq[i] + fn[i];
        go[i] = geq[i] + gn[i];
    }
}

/* Time-t frame velocity at column x of row jy, for the central differences of
 * the internal-energy split's source: a row beyond a wall takes the ghost
 * frame velocity of ghost_node() (the mirror node's, reflected about the wall
 * velocity); other rows wrap or clamp like the stencil. */
static void row_velocity(const oracle_params *P, const double *lam, int x, int jy, double u[2])
{
    if (P->bc_y == 2 && (jy < 0 || jy >= P->ny)) {
        int side = jy < 0 ? 0 : 1;
        int m = side == 0 ? -1 - jy : 2 * P->ny - 1 - jy;
        if (m < 0)
            m = 0;
        if (m > P->ny - 1)
            m = P->ny - 1;
        const double *lm = lam + 3 * ((long)m * P->nx + x);
        u[0] = 2.0 * P->wall_ux[side] - lm[0];
        u[1] = -lm[1];
        return;
    }
    const double *l = lam + 3 * ((long)node_index(jy, P->ny, P->bc_y) * P->nx + x);
    u[0] = l[0];
    u[1] = l[1];
}

/* grad u of the frames lam at node (x, y): central differences of the four
 * neighbours' frame velocities, grad[alpha][beta] = d_alpha u_beta. */
static void node_gradient(const oracle_params *P, const double *lam, int x, int y,
                          double grad[2][2])
{
    long xm = (long)y * P->nx + node_index(x - 1, P->nx, P->bc_x);
    long xp = (long)y * P->nx + node_index(x + 1, P->nx, P->bc_x);
    double uym[2], uyp[2];
    row_velocity(P, lam, x, y - 1, uym);
    row_velocity(P, lam, x, y + 1, uyp);
    for (int b = 0; b < 2; b++) {
        grad[0][b] = 0.5 * (lam[3 * xp + b] - lam[3 * xm + b]);
        grad[1][b] = 0.5 * (uyp[b] - uym[b]);
    }
}

/* grad u of the frames lam at the point (px, py): bilinear interpolation of
 * node_gradient over the four nodes around it (columns and rows wrapped or
 * clamped like the stencil; with walls a row beyond them is the last row). */
static void point_gradient(const oracle_params *P, const double *lam, double px, double py,
                           double grad[2][2])
{
    double fx = floor(px), fy = floor(py);
    double ax = px - fx, ay = py - fy;
    int x0 = (int)fx, y0 = (int)fy;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            grad[a][b] = 0.0;
    for (int j = 0; j < 2; j++) {
        int yj = y0 + j;
        if (P->bc_y == 2)
            yj = yj < 0 ? 0 : (yj > P->ny - 1 ? P->ny - 1 : yj);
        else
            yj = node_index(yj, P->ny, P->bc_y);
        for (int i = 0; i < 2; i++) {
            int xi = node_index(x0 + i, P->nx, P->bc_x);
            double w = (i ? ax : 1.0 - ax) * (j ? ay : 1.0 - ay);
            double gn[2][2];
            node_gradient(P, lam, xi, yj, gn);
            for (int a = 0; a < 2; a++)
                for (int b = 0; b < 2; b++)
                    grad[a][b] += w * gn[a][b];
        }
    }
}

/* The internal-energy split's grad u for destination node (x, y): the end of
 * the step along the node's trajectory, 2 G_t(x - u) - G_{t-1}(x - 2u), u the
 * node's time-t frame velocity; without lam_prev, lam stands in for it. */
static void source_gradient(const oracle_params *P, const double *lam, const double *lam_prev,
                            int x, int y, double grad[2][2])
{
    if (!lam_prev)
        lam_prev = lam;
    const double *l = lam + 3 * ((long)y * P->nx + x);
    double ga[2][2], gb[2][2];
    point_gradient(P, lam, x - l[0], y - l[1], ga);
    point_gradient(P, lam_prev, x - 2.0 * l[0], y - 2.0 * l[1], gb);
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            grad[a][b] = 2.0 * ga[a][b] - gb[a][b];
}

static void gather(const oracle_params *P, const double *f, const double *g, const double *lam,
                   int x, int y, const double *lam_bar, double *ft, double *gt)
{
    double cx[QMAX], cy[QMAX], w[QMAX];
    int q1 = q1_of(P->lattice);
    int q = oracle_lattice_2d_q(q1, cx, cy, w);
    int np = P->interp_points;
    double sT = sqrt(lam_bar[2]);
    double tf[QMAX], tg[QMAX], wx[4], wy[4];
    for (int i = 0; i < q; i++) {
        double Cx = sT * cx[i] + lam_bar[0];
        double Cy = sT * cy[i] + lam_bar[1];
        double yx = (double)x - Cx, yy = (double)y - Cy;
        int bx, by;
        oracle_lagrange(np, yx, &bx, wx);
        oracle_lagrange(np, yy, &by, wy);
        double sf = 0.0, sg = 0.0;
        for (int sy = 0; sy < np; sy++) {
            int ry = by + sy;
            int wall = P->bc_y == 2 && (ry < 0 || ry >= P->ny);
            int jy = wall ? 0 : node_index(ry, P->ny, P->bc_y);
            for (int sx = 0; sx < np; sx++) {
                int jx = node_index(bx + sx, P->nx, P->bc_x);
                long s = (long)jy * P->nx + jx;
                if (wall) {
                    double fgh[QMAX], ggh[QMAX], lgh[3];
                    ghost_node(P, f, g, lam, jx, ry, fgh, ggh, lgh);
                    oracle_transform_q(q1, fgh, lgh, lam_bar, tf);
                    oracle_transform_q(q1, ggh, lgh, lam_bar, tg);
                } else {
                    oracle_transform_q(q1, f + (long)q * s, lam + 3 * s, lam_bar, tf);
                    oracle_transform_q(q1, g + (long)q * s, lam + 3 * s, lam_bar, tg);
                }
                double W = wx[sx] * wy[sy];
                sf += W * tf[i];
                sg += W * tg[i];
            }
        }
        ft[i] = sf;
        gt[i] = sg;
    }
}

/*
 * Conserved moments of (f, g) living in frame lam (Sec. II): density and
 * momentum of f, and the frame they imply: u = j/rho and
 *   total-energy split:    E = sum g,     T = (E - |j|^2/(2 rho)) / (rho c_v);
 *   internal-energy split: rho c_v T = sum g + (sum G)/2 with the step's
 *     source sum G = -(omega/2) rho T div u - (1 - omega/2) P : grad u (P the
 *     pressure tensor of f about u; zero grad: T = sum g / (rho c_v));
 *   non-translational split: E = sum (g + |C_i|^2 f / 2) (Eq. nt_energy_g),
 *                          T = (E - |j|^2/(2 rho)) / (rho c_v).
 * *E receives the split's energy sum (sum g, or E of the non-translational
 * split).
 */
static void conserved(int q1, int split, const double *ft, const double *gt, const double *lam,
                      double cv, double omega, const double grad[2][2], double *rho, double *jx,
                      double *jy, double *E, double *lam_new)
{
    double cx[QMAX], cy[QMAX], w[QMAX];
    int q = oracle_lattice_2d_q(q1, cx, cy, w);
    double sT = sqrt(lam[2]);
    double r = 0.0, px = 0.0, py = 0.0, e = 0.0, sxx = 0.0, sxy = 0.0, syy = 0.0;
    for (int i = 0; i < q; i++) {
        double Cx = sT * cx[i] + lam[0], Cy = sT * cy[i] + lam[1];
        r += ft[i];
        px += ft[i] * Cx;
        py += ft[i] * Cy;
        e += gt[i];
        sxx += ft[i] * Cx * Cx;
        sxy += ft[i] * Cx * Cy;
        syy += ft[i] * Cy * Cy;
        if (split == 2)
            e += 0.5 * (Cx * Cx + Cy * Cy) * ft[i];
    }
    *rho = r; *jx = px; *jy = py; *E = e;
    lam_new[0] = px / r;
    lam_new[1] = py / r;
    if (split == 1) {
        double ux = px / r, uy = py / r;
        double Pxx = sxx - r * ux * ux, Pxy = sxy - r * ux * uy, Pyy = syy - r * uy * uy;
        double PdU = Pxx * grad[0][0] + Pxy * (grad[0][1] + grad[1][0]) + Pyy * grad[1][1];
        double div = grad[0][0] + grad[1][1];
        lam_new[2] = (e - 0.5 * (1.0 - 0.5 * omega) * PdU) / (r * (cv + 0.25 * omega * div));
    } else {
        lam_new[2] = (e - (px * px + py * py) / (2.0 * r)) / (r * cv);
    }
}

/*
 * One time step of destination node n, reading only the time-t state (Jacobi).
 *   lam^0 = its own frame at time t;  for k = 0, 1, ...:
 *     gather (f~, g~) in lam^k; lam^{k+1} = frame of their conserved moments;
 *     stop when max(|u^{k+1} - u^k|_inf / sqrt(T^{k+1}), |T^{k+1} - T^k| / T^{k+1})
 *     <= pc_tol, or after pc_max_iter gathers (node counted non-converged);
 *   re-project (f~, g~) from the last gather frame onto lam* = lam^{k+1};
 *   collide in lam* (internal-energy split: then add the g source);
 *   write f*, g*, lam* (16, 16 and 3 values).
 * *iters receives the number of gathers, *status the ORACLE_* bits.
 * Returns 1 if the node is non-physical (rho <= 0, T <= 0 or non-finite; the
 * outputs are then NaN), else 0.
 */
static int node_step(const oracle_params *P, const double *f, const double *g, const double *lam,
                     const double *lam_prev, long n, double *fo, double *go, double *lamo,
                     int *iters, int *status)
{
    double cv = 1.0 / (P->gamma - 1.0);
    int q1 = q1_of(P->lattice), q = q1 * q1;
    int x = (int)(n % P->nx), y = (int)(n / P->nx);
    double lg[3] = {lam[3 * n], lam[3 * n + 1], lam[3 * n + 2]};
    double ln[3] = {lg[0], lg[1], lg[2]};
    double ft[QMAX], gt[QMAX];
    double gradu[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    if (P->split == 1)
        source_gradient(P, lam, lam_prev, x, y, gradu);
    int k, conv = 0, bad = 0, used = 0;
    for (k = 0; k < P->pc_max_iter; k++) {
        double rho, jx, jy, E;
        gather(P, f, g, lam, x, y, lg, ft, gt);
        conserved(q1, P->split, ft, gt, lg, cv, 1.0 / P->tau, gradu, &rho, &jx, &jy, &E, ln);
        used = k + 1;
        if (!(rho > 0.0) || !(ln[2] > 0.0) || !isfinite(ln[0]) || !isfinite(ln[1]) ||
            !isfinite(ln[2]) || !isfinite(E)) {
            bad = 1;
            break;
        }
        double du = fmax(fabs(ln[0] - lg[0]), fabs(ln[1] - lg[1])) / sqrt(ln[2]);
        double dT = fabs(ln[2] - lg[2]) / ln[2];
        if (fmax(du, dT) <= P->pc_tol) {
            conv = 1;
            break;
        }
        if (k + 1 < P->pc_max_iter)
            memcpy(lg, ln, sizeof lg);
    }
    *iters = used;
    *status = (conv ? 0 : ORACLE_NONCONVERGED) | (bad ? ORACLE_NONPHYSICAL : 0);
    if (bad) {
        for (int i = 0; i < q; i++)
            fo[i] = go[i] = NAN;
        lamo[0] = lamo[1] = lamo[2] = NAN;
        return 1;
    }
    oracle_transform_q(q1, ft, lg, ln, ft);
    oracle_transform_q(q1, gt, lg, ln, gt);
    oracle_collide_q(q1, P->split, ft, gt, ln, P->tau, P->prandtl, P->gamma, fo, go);
    if (P->split == 1) {
        /* d_t u: new minus time-t frame velocity of the node; grad u: the
           source gradient of the iteration (source_gradient) */
        const double *l0 = lam + 3 * n;
        double a[2] = {ln[0] - l0[0], ln[1] - l0[1]};
        /* the source's f is the step's time-centred population, the mean of
           the gathered (pre-collision) and the collided f: its stress is the
           physical one, (1 - omega/2) times the pre-collision non-equilibrium
           stress, the same midpoint rule that makes nu = (tau - 1/2) T */
        double fmid[QMAX], S[QMAX];
        for (int i = 0; i < q; i++)
            fmid[i] = 0.5 * (ft[i] + fo[i]);
        oracle_internal_source_q(q1, fmid, ln, a, gradu, S);
        double tau_g = P->prandtl == 1.0 ? P->tau : 0.5 + (P->tau - 0.5) / P->prandtl;
        for (int i = 0; i < q; i++)
            go[i] += (1.0 - 0.5 / tau_g) * S[i];
    }
    lamo[0] = ln[0];
    lamo[1] = ln[1];
    lamo[2] = ln[2];
    return 0;
}

/* One step for every node (node-major outputs).  lam_prev: the frames of the
 * previous time level (internal-energy split; NULL on the first step after
 * initialisation and for the other splits).  Returns the number of
 * non-physical nodes. */
int oracle_step(const oracle_params *P, const double *f, const double *g, const double *lam,
                const double *lam_prev, double *fo, double *go, double *lamo, int *iters,
                int *status)
{
    long N = (long)P->nx * P->ny;
    long q = (long)P->lattice;
    if (!q1_of(P->lattice))
        return -1;
    int nbad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nbad)
    for (long n = 0; n < N; n++)
        nbad += node_step(P, f, g, lam, lam_prev, n, fo + q * n, go + q * n, lamo + 3 * n,
                          iters + n, status + n);
    return nbad;
}

/* One step for the listed nodes only (outputs packed in list order), reading
 * the full time-t state; lets a large state be checked node by node. */
int oracle_step_nodes(const oracle_params *P, const double *f, const double *g, const double *lam,
                      const double *lam_prev, long count, const long *nodes, double *fo,
                      double *go, double *lamo, int *iters, int *status)
{
    long q = (long)P->lattice;
    if (!q1_of(P->lattice))
        return -1;
    int nbad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : nbad)
    for (long k = 0; k < count; k++)
        nbad += node_step(P, f, g, lam, lam_prev, nodes[k], fo + q * k, go + q * k, lamo + 3 * k,
                          iters + k, status + k);
    return nbad;
}

/*
 * Initial state: equilibrium populations in each node's own frame
 * (f_i = rho w_i, g_i = g_i^eq of the split), frame = (u, T).  Returns the
 * number of rejected nodes (rho <= 0, T <= 0 or non-finite input); nothing is
 * written for those.
 */
int oracle_init_q(int q1, int split, long N, const double *rho, const double *ux,
                  const double *uy, const double *T, double gamma, double *f, double *g,
                  double *lam)
{
    long q = (long)q1 * q1;
    int nbad = 0;
    for (long n = 0; n < N; n++) {
        if (!(rho[n] > 0.0) || !(T[n] > 0.0) || !isfinite(rho[n]) || !isfinite(T[n]) ||
            !isfinite(ux[n]) || !isfinite(uy[n])) {
            nbad++;
            continue;
        }
        oracle_equilibrium_q(q1, split, rho[n], ux[n], uy[n], T[n], gamma, f + q * n, g + q * n);
        lam[3 * n] = ux[n];
        lam[3 * n + 1] = uy[n];
        lam[3 * n + 2] = T[n];
    }
    return nbad;
}

int oracle_init_split(int split, long N, const double *rho, const double *ux, const double *uy,
                      const double *T, double gamma, double *f, double *g, double *lam)
{
    return oracle_init_q(4, split, N, rho, ux, uy, T, gamma, f, g, lam);
}

int oracle_init(long N, const double *rho, const double *ux, const double *uy, const double *T,
                double gamma, double *f, double *g, double *lam)
{
    return oracle_init_split(0, N, rho, ux, uy, T, gamma, f, g, lam);
}

/*
 * Macroscopic fields from the stored state (Sec. II): rho = sum f,
 * rho u = sum f C_i, T from sum g as in conserved(), p = rho T.
 */
void oracle_moments_q(int q1, int split, long N, const double *f, const double *g,
                      const double *lam, double gamma, double *rho, double *ux, double *uy,
                      double *T, double *p)
{
    double cv = 1.0 / (gamma - 1.0);
    long q = (long)q1 * q1;
    for (long n = 0; n < N; n++) {
        double r, jx, jy, E, ln[3];
        const double nograd[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        conserved(q1, split, f + q * n, g + q * n, lam + 3 * n, cv, 0.0, nograd, &r, &jx, &jy,
                  &E, ln);
        rho[n] = r;
        ux[n] = ln[0];
        uy[n] = ln[1];
        T[n] = ln[2];
        if (p)
            p[n] = r * ln[2];
    }
}

void oracle_moments_split(int split, long N, const double *f, const double *g, const double *lam,
                          double gamma, double *rho, double *ux, double *uy, double *T, double *p)
{
    oracle_moments_q(4, split, N, f, g, lam, gamma, rho, ux, uy, T, p);
}

void oracle_moments(long N, const double *f, const double *g, const double *lam, double gamma,
                    double *rho, double *ux, double *uy, double *T, double *p)
{
    oracle_moments_split(0, N, f, g, lam, gamma, rho, ux, uy, T, p);
}
