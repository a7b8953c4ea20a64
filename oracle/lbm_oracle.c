/*
 * lbm_oracle.c -- FP64 CPU reference for the rectangular-lattice central
 * moment LBM (RC-LBM) and its raw-moment special case (RNR-LBM) of
 * E. Yahia & K. N. Premnath, "Central Moment Lattice Boltzmann Method on a
 * Rectangular Lattice" (arXiv 2103.02119).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the CPU
 * baseline of the benchmark.  The product path never calls it.
 *
 * Written from the definitions, in the opposite form to the GPU path's
 * component form (the paper recommends the component form for speed,
 * Sec. 3): the raw and central moments of a node are direct sums of the
 * basis monomials of Eq. 3 over its populations, evaluated at e_i (raw) or
 * e_i - u (central, Eq. 43); after relaxation the post-collision populations
 * are the solution of the 9 x 9 linear system "these populations have these
 * moments", solved by Gaussian elimination.  The equilibrium populations are
 * found the same way from the central equilibria of Eq. 49.  The matrices
 * the paper prints for the transforms (T^{-1}, App. A; F(u), Eq. 53) are
 * kept only as functions the tests pin against the printed values; the
 * scheme does not use them.  Each step follows the order of Sec. 3 / Sec. 4:
 * moments, relaxation, back to populations, stream, update of the
 * hydrodynamic fields.
 *
 * Readings taken where the printed text is garbled or silent (each one is
 * listed with its justification in the design notes of the repository):
 *   - velocity ordering from Eq. 2 (Eq. 1 is garbled);
 *   - T is built from the basis definition Eq. 3; Eq. 4 row 7 prints "a"
 *     where e_x e_y^2 of (1, a) is a^2;
 *   - T^{-1} (App. A) row 0 column 8 is +1/a^2 (printed -1/a^2);
 *   - Eq. 12, m_8: coefficient of rho cs^2 (ux^2 + uy^2) is 1, as the
 *     binomial transform of the central equilibria (Eq. 49) requires;
 *   - dt = 1 multiplies the corrections; d rho by central differences at the
 *     same time level as f, with y spacing a; at a wall the missing
 *     neighbour's density is the node's own density;
 *   - the non-equilibrium moments in Eq. 37-38 are the raw ones of
 *     Eq. 34-35 (m - m^{eq,r}), with no forcing term;
 *   - bounce-back: f_i(x_f, t+1) = ft_ibar(x_f, t) - (feq_ibar - feq_i)(rho_w, u_w)
 *     with rho_w = rho0; a link that crosses a moving wall uses that wall.
 *
 * Parity unpinned: the conventions the paper leaves open have no value in
 * the paper or the mathematics that fixes them, so the GPU path agrees with
 * this file on them but nothing independent checks them -- the wall
 * neighbour's density in the gradient, rho_w = rho0, the corner rule for a
 * link that crosses two faces, and the initial state f = feq(rho, u) with no
 * non-equilibrium part.  (The lid and the corner rule together are checked
 * only indirectly, by the primary-vortex centres the paper prints.)
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Eq. 2: e_x = CX, e_y = a * CY for i = 0..8. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* e_ibar = -e_i */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Eq. 3: T = [|1>, |ex>, |ey>, |ex^2+ey^2>, |ex^2-ey^2>, |ex ey>, |ex^2 ey>,
 * |ex ey^2>, |ex^2 ey^2>] as rows, evaluated on the velocity set of Eq. 2. */
void orc_T(double a, double *T)
{
    for (int k = 0; k < 9; ++k) {
        const double ex = CX[k], ey = a * CY[k];
        T[0 * 9 + k] = 1.0;
        T[1 * 9 + k] = ex;
        T[2 * 9 + k] = ey;
        T[3 * 9 + k] = ex * ex + ey * ey;
        T[4 * 9 + k] = ex * ex - ey * ey;
        T[5 * 9 + k] = ex * ey;
        T[6 * 9 + k] = ex * ex * ey;
        T[7 * 9 + k] = ex * ey * ey;
        T[8 * 9 + k] = ex * ex * ey * ey;
    }
}

/* The nine monomials of the moment basis of Eq. 3 at a velocity (vx, vy):
 * 1, vx, vy, vx^2 + vy^2, vx^2 - vy^2, vx vy, vx^2 vy, vx vy^2, vx^2 vy^2. */
static void basis9(double vx, double vy, double *phi)
{
    phi[0] = 1.0;
    phi[1] = vx;
    phi[2] = vy;
    phi[3] = vx * vx + vy * vy;
    phi[4] = vx * vx - vy * vy;
    phi[5] = vx * vy;
    phi[6] = vx * vx * vy;
    phi[7] = vx * vy * vy;
    phi[8] = vx * vx * vy * vy;
}

/* Moments of a node's populations about the velocity (ux, uy):
 * m_j = sum_i f_i phi_j(e_i - u).  With u = 0 these are the raw moments of
 * Eq. 3; with the node's own velocity, the central moments of Eq. 43. */
static void moments_about(double a, double ux, double uy, const double *f9, double *m)
{
    for (int j = 0; j < 9; ++j)
        m[j] = 0.0;
    for (int i = 0; i < 9; ++i) {
        double phi[9];
        basis9(CX[i] - ux, a * CY[i] - uy, phi);
        for (int j = 0; j < 9; ++j)
            m[j] += f9[i] * phi[j];
    }
}

/* The populations f whose moments about (ux, uy) are m: the 9 x 9 system
 * sum_i phi_j(e_i - u) f_i = m_j, solved by LU factorisation with partial
 * pivoting and one step of iterative refinement (the residual of the first
 * solution, solved with the same factors and added), so that each solution
 * is accurate to about one rounding of its components. */
static void populations_with_moments(double a, double ux, double uy, const double *m,
                                     double *f9)
{
    double A[9][9], LU[9][9], x[9] = {0}, r[9] = {0};
    int perm[9];
    for (int i = 0; i < 9; ++i) {
        double phi[9];
        basis9(CX[i] - ux, a * CY[i] - uy, phi);
        for (int j = 0; j < 9; ++j)
            A[j][i] = LU[j][i] = phi[j];
    }
    for (int j = 0; j < 9; ++j)
        perm[j] = j;
    for (int c = 0; c < 9; ++c) {
        int piv = c;
        for (int q = c + 1; q < 9; ++q)
            if (fabs(LU[q][c]) > fabs(LU[piv][c]))
                piv = q;
        if (piv != c) {
            for (int q = 0; q < 9; ++q) {
                const double t = LU[c][q];
                LU[c][q] = LU[piv][q];
                LU[piv][q] = t;
            }
            const int t = perm[c];
            perm[c] = perm[piv];
            perm[piv] = t;
        }
        for (int q = c + 1; q < 9; ++q) {
            LU[q][c] /= LU[c][c];
            for (int w = c + 1; w < 9; ++w)
                LU[q][w] -= LU[q][c] * LU[c][w];
        }
    }
    /* solve L U x = P b, for b = m and then for the residual */
    for (int pass = 0; pass < 2; ++pass) {
        double y[9];
        for (int j = 0; j < 9; ++j) {
            double v = pass == 0 ? m[perm[j]] : r[perm[j]];
            for (int q = 0; q < j; ++q)
                v -= LU[j][q] * y[q];
            y[j] = v;
        }
        for (int j = 8; j >= 0; --j) {
            double v = y[j];
            for (int q = j + 1; q < 9; ++q)
                v -= LU[j][q] * y[q];
            y[j] = v / LU[j][j];
        }
        if (pass == 0) {
            for (int j = 0; j < 9; ++j)
                x[j] = y[j];
            for (int j = 0; j < 9; ++j) {
                double v = m[j];
                for (int i = 0; i < 9; ++i)
                    v -= A[j][i] * x[i];
                r[j] = v;
            }
        } else {
            for (int j = 0; j < 9; ++j)
                f9[j] = x[j] + y[j];
        }
    }
}

/* App. A, Eq. (Tinverse), with r1, r2 as defined there and the sign of
 * row 0 / column 8 read as +1/a^2.  Not used by the scheme (which solves for
 * the populations); kept for the tests that pin the printed matrix. */
void orc_Tinv(double a, double *Ti)
{
    const double a2 = a * a;
    const double r1 = -0.5 * (1.0 + 1.0 / a2);
    const double r2 = -0.5 * (1.0 - 1.0 / a2);
    const double h = 0.5, q = 0.25;
    const double M[9][9] = {
        {1, 0, 0, r1, r2, 0, 0, 0, 1.0 / a2},
        {0, h, 0, q, q, 0, 0, -h / a2, -h / a2},
        {0, 0, h / a, q / a2, -q / a2, 0, -h / a, 0, -h / a2},
        {0, -h, 0, q, q, 0, 0, h / a2, -h / a2},
        {0, 0, -h / a, q / a2, -q / a2, 0, h / a, 0, -h / a2},
        {0, 0, 0, 0, 0, q / a, q / a, q / a2, q / a2},
        {0, 0, 0, 0, 0, -q / a, q / a, -q / a2, q / a2},
        {0, 0, 0, 0, 0, q / a, -q / a, -q / a2, q / a2},
        {0, 0, 0, 0, 0, -q / a, -q / a, q / a2, q / a2},
    };
    memcpy(Ti, M, sizeof(M));
}

/* App. B, Eq. 53: frame transformation F(u) from raw to central moments.
 * Its inverse is F(-u) (Eq. 55).  Not used by the scheme (which sums the
 * central moments directly); kept for the tests that pin the printed
 * matrix. */
void orc_F(double ux, double uy, double *F)
{
    const double ux2 = ux * ux, uy2 = uy * uy;
    const double M[9][9] = {
        {1, 0, 0, 0, 0, 0, 0, 0, 0},
        {-ux, 1, 0, 0, 0, 0, 0, 0, 0},
        {-uy, 0, 1, 0, 0, 0, 0, 0, 0},
        {ux2 + uy2, -2 * ux, -2 * uy, 1, 0, 0, 0, 0, 0},
        {ux2 - uy2, -2 * ux, 2 * uy, 0, 1, 0, 0, 0, 0},
        {ux * uy, -uy, -ux, 0, 0, 1, 0, 0, 0},
        {-ux2 * uy, 2 * ux * uy, ux2, -0.5 * uy, -0.5 * uy, -2 * ux, 1, 0, 0},
        {-ux * uy2, uy2, 2 * ux * uy, -0.5 * ux, 0.5 * ux, -2 * uy, 0, 1, 0},
        {ux2 * uy2, -2 * ux * uy2, -2 * ux2 * uy, 0.5 * (ux2 + uy2), 0.5 * (uy2 - ux2),
         4 * ux * uy, -2 * uy, -2 * ux, 1},
    };
    memcpy(F, M, sizeof(M));
}

/* Sec. 3 / Sec. 4, "update hydrodynamic fields":
 * rho = sum f, rho u = sum f e + F/2 (dt = 1). */
void orc_macro(const orc_params *p, const double *f9, double *rho, double *ux, double *uy)
{
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int k = 0; k < 9; ++k) {
        r += f9[k];
        jx += f9[k] * CX[k];
        jy += f9[k] * (p->a * CY[k]);
    }
    *rho = r;
    *ux = (jx + 0.5 * p->force[0]) / r;
    *uy = (jy + 0.5 * p->force[1]) / r;
}

/* Equilibrium populations: the populations whose central moments are the
 * central equilibria of Eq. 49 without the corrections,
 * (rho, 0, 0, 2 rho cs^2, 0, 0, 0, 0, rho cs^4) about the velocity u. */
void orc_feq(const orc_params *p, double rho, double ux, double uy, double *feq9)
{
    const double s = p->cs2;
    const double mceq[9] = {rho, 0, 0, 2 * rho * s, 0, 0, 0, 0, rho * s * s};
    populations_with_moments(p->a, ux, uy, mceq, feq9);
}

/* Eq. 12 (square-lattice raw equilibria), m_8 coefficient read as 1. */
static void raw_equilibria(double rho, double ux, double uy, double s, double *meq)
{
    meq[0] = rho;
    meq[1] = rho * ux;
    meq[2] = rho * uy;
    meq[3] = 2 * rho * s + rho * (ux * ux + uy * uy);
    meq[4] = rho * (ux * ux - uy * uy);
    meq[5] = rho * ux * uy;
    meq[6] = s * rho * uy + rho * ux * ux * uy;
    meq[7] = s * rho * ux + rho * ux * uy * uy;
    meq[8] = rho * s * s + rho * s * (ux * ux + uy * uy) + rho * ux * ux * uy * uy;
}

/* Eq. 13 (raw source moments). */
static void raw_sources(double Fx, double Fy, double ux, double uy, double *phi)
{
    phi[0] = 0.0;
    phi[1] = Fx;
    phi[2] = Fy;
    phi[3] = 2 * (Fx * ux + Fy * uy);
    phi[4] = 2 * (Fx * ux - Fy * uy);
    phi[5] = Fx * uy + Fy * ux;
    phi[6] = Fy * ux * ux + 2 * Fx * ux * uy;
    phi[7] = Fx * uy * uy + 2 * Fy * uy * ux;
    phi[8] = 2 * (Fx * ux * uy * uy + Fy * uy * ux * ux);
}

/* Eq. 37-38 with the coefficients of Eq. 40; the bracketed non-equilibrium
 * moments are eta - m^{eq,r} of Eq. 34-35. */
static void strain_rate_from(const orc_params *p, const double *m, double rho, double ux,
                             double uy, double gx, double gy, double *X, double *Y)
{
    const double s = p->cs2, a2 = p->a * p->a;
    const double w3 = p->omega[3], w4 = p->omega[4];
    const double m3eqr = 2 * rho * s + rho * (ux * ux + uy * uy);
    const double m4eqr = rho * (ux * ux - uy * uy);

    const double B1 = rho * (-2 * s / w3 - (-3 * s + 1) / 2 + 3 * ux * ux / 2);
    const double B2 = rho * (-2 * s / w3 - (-3 * s + a2) / 2 + 3 * uy * uy / 2);
    const double B3 = ((3 * s - 1) / 2) * ux;
    const double B4 = ((3 * s - a2) / 2) * uy;
    const double C1 = rho * (-2 * s / w4 - (-3 * s + 1) / 2 + 3 * ux * ux / 2);
    const double C2 = rho * (2 * s / w4 - (3 * s - a2) / 2 - 3 * uy * uy / 2);
    const double C3 = ((3 * s - 1) / 2) * ux;
    const double C4 = ((-3 * s + a2) / 2) * uy;

    const double M3 = m[3] - m3eqr - B3 * gx - B4 * gy;
    const double M4 = m[4] - m4eqr - C3 * gx - C4 * gy;
    *X = (C2 * M3 - B2 * M4) / (C2 * B1 - C1 * B2);
    *Y = (C1 * M3 - B1 * M4) / (C1 * B2 - C2 * B1);
}

/* Eq. 23-26 (with Eq. 27: no correction on m_5), dt = 1. */
static void corrections_from(const orc_params *p, double rho, double ux, double uy, double gx,
                             double gy, double X, double Y, double *d3, double *d4)
{
    if (!p->corrections) {
        *d3 = 0.0;
        *d4 = 0.0;
        return;
    }
    const double s = p->cs2, a2 = p->a * p->a;
    const double k3 = 1.0 / p->omega[3] - 0.5;
    const double k4 = 1.0 / p->omega[4] - 0.5;
    const double m3s = k3 * ((-3 * s + 1) * rho * X + (-3 * s + a2) * rho * Y +
                             (-3 * s + 1) * ux * gx + (-3 * s + a2) * uy * gy);
    const double m4s = k4 * ((-3 * s + 1) * rho * X + (3 * s - a2) * rho * Y +
                             (-3 * s + 1) * ux * gx + (3 * s - a2) * uy * gy);
    const double m3G = -3 * rho * k3 * (ux * ux * X + uy * uy * Y);
    const double m4G = -3 * rho * k4 * (ux * ux * X - uy * uy * Y);
    *d3 = m3s + m3G;
    *d4 = m4s + m4G;
}

void orc_strain_rate(const orc_params *p, const double *f9, double drho_dx, double drho_dy,
                     double *dux_dx, double *duy_dy)
{
    double m[9], rho, ux, uy;
    moments_about(p->a, 0.0, 0.0, f9, m);
    orc_macro(p, f9, &rho, &ux, &uy);
    strain_rate_from(p, m, rho, ux, uy, drho_dx, drho_dy, dux_dx, duy_dy);
}

void orc_corrections(const orc_params *p, const double *f9, double drho_dx, double drho_dy,
                     double *delta3, double *delta4)
{
    double m[9], rho, ux, uy, X, Y;
    moments_about(p->a, 0.0, 0.0, f9, m);
    orc_macro(p, f9, &rho, &ux, &uy);
    strain_rate_from(p, m, rho, ux, uy, drho_dx, drho_dy, &X, &Y);
    corrections_from(p, rho, ux, uy, drho_dx, drho_dy, X, Y, delta3, delta4);
}

/* One node's collision. */
static void collide_with(const orc_params *p, const double *f9, double gx, double gy,
                         double *out9)
{
    const double s = p->cs2;
    const double *w = p->omega;
    const double Fx = p->force[0], Fy = p->force[1];
    double rho, ux, uy, X, Y, d3, d4;
    double m[9];

    /* hydrodynamic fields and the raw moments (Eq. 3) */
    orc_macro(p, f9, &rho, &ux, &uy);
    moments_about(p->a, 0.0, 0.0, f9, m);
    /* local strain rate (Eq. 37-38) and corrections (Eq. 23-27) */
    strain_rate_from(p, m, rho, ux, uy, gx, gy, &X, &Y);
    corrections_from(p, rho, ux, uy, gx, gy, X, Y, &d3, &d4);

    if (p->collision == ORC_RC) {
        /* Sec. 4: central moments (Eq. 43) relaxed toward Eq. 49 with the
         * central sources (0, Fx, Fy, 0, ...); the post-collision populations
         * are those with the relaxed central moments. */
        double mc[9], mct[9];
        const double mceq[9] = {rho, 0, 0, 2 * rho * s + d3, d4, 0.0, 0, 0, rho * s * s};
        const double phic[9] = {0, Fx, Fy, 0, 0, 0, 0, 0, 0};
        moments_about(p->a, ux, uy, f9, mc);
        for (int j = 0; j < 9; ++j)
            mct[j] = mc[j] + w[j] * (mceq[j] - mc[j]) + (1 - w[j] / 2) * phic[j];
        populations_with_moments(p->a, ux, uy, mct, out9);
    } else {
        /* Sec. 3: raw moments relaxed toward m^{eq,r} + corrections (Eq. 10,
         * Eq. 12) with the sources of Eq. 13; the post-collision populations
         * are those with the relaxed raw moments. */
        double meq[9], phi[9], mt[9];
        raw_equilibria(rho, ux, uy, s, meq);
        meq[3] += d3;
        meq[4] += d4;
        raw_sources(Fx, Fy, ux, uy, phi);
        for (int j = 0; j < 9; ++j)
            mt[j] = m[j] + w[j] * (meq[j] - m[j]) + (1 - w[j] / 2) * phi[j];
        populations_with_moments(p->a, 0.0, 0.0, mt, out9);
    }
}

void orc_collide_node(const orc_params *p, const double *f9, double drho_dx, double drho_dy,
                      double *out9)
{
    collide_with(p, f9, drho_dx, drho_dy, out9);
}

/* ---------------------------------------------------------------- fields */

#define IDX(p, j, i) ((size_t)(j) * (size_t)(p)->nx + (size_t)(i))
#define FIDX(p, k, j, i) ((size_t)(k) * (size_t)(p)->nx * (size_t)(p)->ny + IDX(p, j, i))

static int is_solid(const orc_params *p, int i, int j)
{
    return p->solid != NULL && p->solid[IDX(p, j, i)] != 0;
}

static void gather9(const orc_params *p, const double *f, int i, int j, double *f9)
{
    for (int k = 0; k < 9; ++k)
        f9[k] = f[FIDX(p, k, j, i)];
}

/* Lattices below this many nodes run on one thread: for them the cost of
 * starting a parallel region every step exceeds the work.  Every node is
 * computed independently, so the results do not depend on the threads. */
static int threaded(const orc_params *p) { return (long)p->nx * p->ny >= 8192; }

void orc_init(const orc_params *p, const double *rho, const double *ux, const double *uy,
              double *f)
{
#pragma omp parallel for schedule(static) if (threaded(p))
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            double feq[9];
            const size_t n = IDX(p, j, i);
            if (is_solid(p, i, j))
                orc_feq(p, p->rho0, 0.0, 0.0, feq);
            else
                orc_feq(p, rho ? rho[n] : p->rho0, ux ? ux[n] : 0.0, uy ? uy[n] : 0.0, feq);
            for (int k = 0; k < 9; ++k)
                f[FIDX(p, k, j, i)] = feq[k];
        }
}

void orc_density(const orc_params *p, const double *f, double *rho)
{
#pragma omp parallel for schedule(static) if (threaded(p))
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            double r = 0.0;
            for (int k = 0; k < 9; ++k)
                r += f[FIDX(p, k, j, i)];
            rho[IDX(p, j, i)] = r;
        }
}

/* Neighbour of node (i, j) used by the density gradient: across a periodic
 * face it wraps, across a wall or onto a solid node it is the node itself. */
static int nb_x(const orc_params *p, int i, int j, int d)
{
    int n = i + d;
    if (n < 0) {
        if (p->bc_type[0] != ORC_PERIODIC) return i;
        n = p->nx - 1;
    } else if (n >= p->nx) {
        if (p->bc_type[1] != ORC_PERIODIC) return i;
        n = 0;
    }
    return is_solid(p, n, j) ? i : n;
}

static int nb_y(const orc_params *p, int i, int j, int d)
{
    int n = j + d;
    if (n < 0) {
        if (p->bc_type[2] != ORC_PERIODIC) return j;
        n = p->ny - 1;
    } else if (n >= p->ny) {
        if (p->bc_type[3] != ORC_PERIODIC) return j;
        n = 0;
    }
    return is_solid(p, i, n) ? j : n;
}

/* Central differences (the paper computes the density gradient "using a
 * central difference approach"); x spacing 1, y spacing a. */
void orc_density_gradient(const orc_params *p, const double *rho, double *gx, double *gy)
{
    const int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static) if (threaded(p))
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            gx[IDX(p, j, i)] =
                (rho[IDX(p, j, nb_x(p, i, j, 1))] - rho[IDX(p, j, nb_x(p, i, j, -1))]) / 2.0;
            gy[IDX(p, j, i)] =
                (rho[IDX(p, nb_y(p, i, j, 1), i)] - rho[IDX(p, nb_y(p, i, j, -1), i)]) /
                (2.0 * p->a);
        }
}

/* Post-collision populations of every node (f -> f~). */
void orc_collide(const orc_params *p, const double *f, double *ft)
{
    const size_t n = (size_t)p->nx * p->ny;
    double *rho = malloc(n * sizeof(double));
    double *gx = malloc(n * sizeof(double));
    double *gy = malloc(n * sizeof(double));
    orc_density(p, f, rho);
    orc_density_gradient(p, rho, gx, gy);
#pragma omp parallel for schedule(static) if (threaded(p))
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            double f9[9], o9[9];
            gather9(p, f, i, j, f9);
            collide_with(p, f9, gx[IDX(p, j, i)], gy[IDX(p, j, i)], o9);
            for (int k = 0; k < 9; ++k)
                ft[FIDX(p, k, j, i)] = o9[k];
        }
    free(rho);
    free(gx);
    free(gy);
}

/* Source of the link k that arrives at node (i, j) under perfect-shift
 * streaming f_i(x, t+1) = f~_i(x - e_i, t).  Returns -1 and the (periodically
 * wrapped) source node, or the index of the wall face the link crosses
 * (half-way bounce-back), or ORC_OBSTACLE when the source is a solid node.
 * A link crossing two wall faces takes the moving one if exactly one of them
 * moves, else the y face; a link that leaves the domain never sees the mask. */
#define ORC_OBSTACLE 4
static int link_source(const orc_params *p, int i, int j, int k, int *si_out, int *sj_out)
{
    const int nx = p->nx, ny = p->ny;
    int si = i - CX[k], sj = j - CY[k];
    const int fx = (si < 0) ? 0 : (si >= nx) ? 1 : -1;
    const int fy = (sj < 0) ? 2 : (sj >= ny) ? 3 : -1;
    const int wx = (fx >= 0 && p->bc_type[fx] != ORC_PERIODIC) ? fx : -1;
    const int wy = (fy >= 0 && p->bc_type[fy] != ORC_PERIODIC) ? fy : -1;
    if (wx >= 0 && wy >= 0)
        return (p->bc_type[wx] == ORC_MOVING_WALL && p->bc_type[wy] != ORC_MOVING_WALL) ? wx : wy;
    if (wy >= 0) return wy;
    if (wx >= 0) return wx;
    if (si < 0) si += nx;
    if (si >= nx) si -= nx;
    if (sj < 0) sj += ny;
    if (sj >= ny) sj -= ny;
    if (is_solid(p, si, sj)) return ORC_OBSTACLE;
    *si_out = si;
    *sj_out = sj;
    return -1;
}

/* (feq_ibar - feq_i)(rho_w, u_w) of every face; rho_w = rho0.  For a wall
 * at rest the difference is zero (the equilibrium at u = 0 is symmetric
 * under e -> -e) and is set so, exactly. */
static void wall_terms(const orc_params *p, double dwall[5][9])
{
    for (int face = 0; face < 4; ++face) {
        double feq[9];
        const int mv = p->bc_type[face] == ORC_MOVING_WALL;
        orc_feq(p, p->rho0, mv ? p->u_wall[face][0] : 0.0, mv ? p->u_wall[face][1] : 0.0, feq);
        for (int k = 0; k < 9; ++k)
            dwall[face][k] = mv ? feq[OPP[k]] - feq[k] : 0.0;
    }
    for (int k = 0; k < 9; ++k)
        dwall[ORC_OBSTACLE][k] = 0.0;  /* obstacles are at rest */
}

/* Streaming by perfect shift with periodic wrap or half-way bounce-back
 * (moving-wall form of Sec. 5.2) where the source node lies outside. */
void orc_stream(const orc_params *p, const double *ft, double *f)
{
    double dwall[5][9], rest[9];
    wall_terms(p, dwall);
    orc_feq(p, p->rho0, 0.0, 0.0, rest);
#pragma omp parallel for schedule(static) if (threaded(p))
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i)
            for (int k = 0; k < 9; ++k) {
                if (is_solid(p, i, j)) {
                    f[FIDX(p, k, j, i)] = rest[k];
                    continue;
                }
                int si = 0, sj = 0;
                const int face = link_source(p, i, j, k, &si, &sj);
                if (face >= 0)
                    f[FIDX(p, k, j, i)] = ft[FIDX(p, OPP[k], j, i)] - dwall[face][k];
                else
                    f[FIDX(p, k, j, i)] = ft[FIDX(p, k, sj, si)];
            }
}

static double node_density(const orc_params *p, const double *f, int i, int j)
{
    double r = 0.0;
    for (int k = 0; k < 9; ++k)
        r += f[FIDX(p, k, j, i)];
    return r;
}

/* One node's populations after one collide + stream step, evaluated from the
 * whole pre-step field f without touching any other node's output: the
 * sources of its nine links are collided one by one (each with its own
 * central-difference density gradient) and streamed as in orc_stream. */
void orc_step_node(const orc_params *p, const double *f, int i, int j, double *out9)
{
    double dwall[5][9];
    wall_terms(p, dwall);
    if (is_solid(p, i, j)) {
        orc_feq(p, p->rho0, 0.0, 0.0, out9);
        return;
    }
    for (int k = 0; k < 9; ++k) {
        int si = i, sj = j;
        const int face = link_source(p, i, j, k, &si, &sj);
        const int comp = face >= 0 ? OPP[k] : k;
        double f9[9], o9[9];
        gather9(p, f, si, sj, f9);
        const double gx = (node_density(p, f, nb_x(p, si, sj, 1), sj) -
                           node_density(p, f, nb_x(p, si, sj, -1), sj)) / 2.0;
        const double gy = (node_density(p, f, si, nb_y(p, si, sj, 1)) -
                           node_density(p, f, si, nb_y(p, si, sj, -1))) / (2.0 * p->a);
        collide_with(p, f9, gx, gy, o9);
        out9[k] = o9[comp] - (face >= 0 ? dwall[face][k] : 0.0);
    }
}

/* nsteps of collide + stream; f holds the populations at the current time
 * level on entry and on exit.  work (9*nx*ny doubles) may be NULL. */
void orc_run(const orc_params *p, double *f, double *work, long nsteps)
{
    const size_t n9 = (size_t)9 * p->nx * p->ny;
    double *ft = work ? work : malloc(n9 * sizeof(double));
    for (long s = 0; s < nsteps; ++s) {
        orc_collide(p, f, ft);
        orc_stream(p, ft, f);
    }
    if (!work)
        free(ft);
}

/* Local viscous stress of every node (Sec. 4 stress output): the strain
 * rate of Eq. 37-38 (d_x u_x, d_y u_y) and Eq. 39 read as
 * d_y u_x + d_x u_y = (eta_xy - m_5^{eq,r}) / D_1, D_1 = -rho cs2 / omega_5,
 * with the raw non-equilibrium moments of Eq. 34-36; then the viscous terms
 * of Eq. 30-31: tau_xx = rho [nu (2 d_x u_x - div u) + zeta div u], tau_yy
 * likewise, tau_xy = rho nu (d_y u_x + d_x u_y), nu from omega_4 / omega_5
 * (Eq. 32), zeta from omega_3 (Eq. 33).  Solid nodes get 0. */
void orc_stress(const orc_params *p, const double *f, double *sxx, double *syy, double *sxy)
{
    const size_t n = (size_t)p->nx * p->ny;
    double *rho = malloc(n * sizeof(double));
    double *gx = malloc(n * sizeof(double));
    double *gy = malloc(n * sizeof(double));
    orc_density(p, f, rho);
    orc_density_gradient(p, rho, gx, gy);
    const double s = p->cs2;
    const double nu4 = s * (1.0 / p->omega[4] - 0.5), nu5 = s * (1.0 / p->omega[5] - 0.5);
    const double zeta = s * (1.0 / p->omega[3] - 0.5);
#pragma omp parallel for schedule(static) if (threaded(p))
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            const size_t q = IDX(p, j, i);
            if (is_solid(p, i, j)) {
                sxx[q] = syy[q] = sxy[q] = 0.0;
                continue;
            }
            double f9[9], m[9], r, ux, uy, X, Y;
            gather9(p, f, i, j, f9);
            moments_about(p->a, 0.0, 0.0, f9, m);
            orc_macro(p, f9, &r, &ux, &uy);
            strain_rate_from(p, m, r, ux, uy, gx[q], gy[q], &X, &Y);
            const double S = (m[5] - r * ux * uy) / (-r * s / p->omega[5]);
            const double div = X + Y;
            sxx[q] = r * (nu4 * (2 * X - div) + zeta * div);
            syy[q] = r * (nu4 * (2 * Y - div) + zeta * div);
            sxy[q] = r * nu5 * S;
        }
    free(rho);
    free(gx);
    free(gy);
}

void orc_moments(const orc_params *p, const double *f, double *rho, double *ux, double *uy)
{
#pragma omp parallel for schedule(static) if (threaded(p))
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            double f9[9], r, vx, vy;
            gather9(p, f, i, j, f9);
            orc_macro(p, f9, &r, &vx, &vy);
            const size_t n = IDX(p, j, i);
            if (rho) rho[n] = r;
            if (ux) ux[n] = vx;
            if (uy) uy[n] = vy;
        }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
