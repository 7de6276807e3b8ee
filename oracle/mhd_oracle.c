/*
 * Plain FP64 CPU oracle for the fused MHD right-hand side and the
 * low-storage RK3 substep.  TEST INFRASTRUCTURE ONLY: it exists so the
 * tests, the smoke check and the CPU-baseline leg of the benchmark can
 * check the GPU path against a slow, obviously correct implementation.
 * Nothing in the product path may call it.  It shares no code, header,
 * table or helper with the HIP library.
 *
 * What it follows (Pekkila et al., "Scalable communication for high-order
 * stencil computations using CUDA-aware MPI"):
 *   - Section 2: a grid of n cells per axis; the stencil radius r is the
 *     largest Chebyshev distance of a stencil point (Eq. 1).  Section 4
 *     lists 2nd-, 4th-, 6th- and 8th-order stencils (k = 2r, r = 1..4);
 *     r is a parameter here, 3 by default.
 *   - Section 3.3: on a periodic domain a halo index s maps to the interior
 *     index ((s - r) mod n) + r.  The oracle keeps no halo at all; it reads
 *     the neighbour at offset m of interior cell i as cell (i + m) mod n,
 *     which is the same value the halo holds.
 *   - Section 4, Eq. (stencil-fd): order-2r central differences whose
 *     stencil holds only points z(x +- y), |z| <= r, with x, y standard
 *     basis vectors or 0 -- the three axis lines and the planar diagonals.
 *     Hence mixed derivatives use the diagonal points only (see d_mixed).
 *   - Section 4: time integration by Williamson's third-order low-storage
 *     (2N) Runge-Kutta scheme.
 *   - Appendix B, Eqs. B.1-B.4 and Tables B.1-B.2: the non-ideal MHD system
 *     for ln(rho), u, s and A, in non-conservative form.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - derivative weights: the standard central weights of order 2r (the
 *     unique ones exact on polynomials of degree 2r on the 2r+1 points);
 *   - mixed derivative: difference of the second derivatives along the
 *     two diagonals of the plane, each with the pure second-derivative
 *     weights, divided by 4 h_a h_b;
 *   - RK3 coefficients: alpha = (0, -5/9, -153/128), beta = (1/3, 15/16, 8/15);
 *   - equation of state: ideal gas, cs^2 = cs0^2 exp(gamma s/cp
 *     + (gamma - 1)(ln rho - ln rho0)), and cp (gamma - 1) T = cs^2;
 *   - K constant; the explicit heating H and cooling C, for which the
 *     paper gives no model, spatially uniform constants (0 by default), so
 *     B.3 divided by rho T reads
 *     Ds/Dt = (K/rho)(lap lnT + |grad lnT|^2)
 *             + (1/T)((H - C)/rho + eta mu0 j.j / rho + 2 nu S:S
 *                     + zeta (div u)^2);
 *   - j = (grad(div A) - lap A)/mu0, built from second derivatives (the
 *     radius-r form of mu0^-1 curl curl A);
 *   - B = curl A + B_ext with an optional uniform B_ext (zero by default);
 *   - S_ij = (d_j u_i + d_i u_j)/2 - delta_ij div(u)/3.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp, no fast-math.
 * Layout: field-major, f[q][k][j][i] with i (x) fastest, unpadded
 * nx*ny*nz cells per field, 8 fields in the order of Table B.1:
 * lnrho, ux, uy, uz, ss, Ax, Ay, Az.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 8
enum { Q_LNRHO = 0, Q_UX, Q_UY, Q_UZ, Q_SS, Q_AX, Q_AY, Q_AZ };

typedef struct {
    int32_t nx, ny, nz, radius; /* radius r = 1..4: order 2r */
    double lx, ly, lz;
    double cs0, gamma, cp, lnrho0, mu0, nu, zeta, eta, K;
    double bext[3];
    double heat, cool; /* H and C of Eq. B.3, uniform */
} oracle_params;

#define RMAX 4

/* Central weights of order 2r for offsets m = -r..r, stored at [r-1][m+4]
 * (zero outside |m| <= r), written as integer numerators over one
 * denominator per row:
 *   first derivative:  f'(0)  ~ (1/h)   * sum_m A1[r-1][m+4] f(m)
 *   second derivative: f''(0) ~ (1/h^2) * sum_m A2[r-1][m+4] f(m)       */
static const double A1[RMAX][2 * RMAX + 1] = {
    {0, 0, 0, -1.0 / 2.0, 0.0, 1.0 / 2.0, 0, 0, 0},
    {0, 0, 1.0 / 12.0, -8.0 / 12.0, 0.0, 8.0 / 12.0, -1.0 / 12.0, 0, 0},
    {0, -1.0 / 60.0, 9.0 / 60.0, -45.0 / 60.0, 0.0, 45.0 / 60.0, -9.0 / 60.0, 1.0 / 60.0, 0},
    {3.0 / 840.0, -32.0 / 840.0, 168.0 / 840.0, -672.0 / 840.0, 0.0, 672.0 / 840.0,
     -168.0 / 840.0, 32.0 / 840.0, -3.0 / 840.0}};
static const double A2[RMAX][2 * RMAX + 1] = {
    {0, 0, 0, 1.0, -2.0, 1.0, 0, 0, 0},
    {0, 0, -1.0 / 12.0, 16.0 / 12.0, -30.0 / 12.0, 16.0 / 12.0, -1.0 / 12.0, 0, 0},
    {0, 2.0 / 180.0, -27.0 / 180.0, 270.0 / 180.0, -490.0 / 180.0, 270.0 / 180.0,
     -27.0 / 180.0, 2.0 / 180.0, 0},
    {-9.0 / 5040.0, 128.0 / 5040.0, -1008.0 / 5040.0, 8064.0 / 5040.0, -14350.0 / 5040.0,
     8064.0 / 5040.0, -1008.0 / 5040.0, 128.0 / 5040.0, -9.0 / 5040.0}};

/* Williamson 2N third-order coefficients: per substep s,
 *   w <- alpha_s w + dt F(f);  f <- f + beta_s w.                       */
static const double RK_ALPHA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK_BETA[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

static inline int64_t wrap(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

typedef struct {
    int64_t n[3];
    const double *f; /* one field */
} field_view;

/* Value at cell (i, j, k) + offset (o[0], o[1], o[2]), periodic. */
static inline double at(const field_view *v, int64_t i, int64_t j, int64_t k,
                        int64_t ox, int64_t oy, int64_t oz)
{
    int64_t ii = wrap(i + ox, v->n[0]);
    int64_t jj = wrap(j + oy, v->n[1]);
    int64_t kk = wrap(k + oz, v->n[2]);
    return v->f[(kk * v->n[1] + jj) * v->n[0] + ii];
}

/* Unit offset vectors for axes 0 (x), 1 (y), 2 (z). */
static const int64_t E[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

/* First derivative along axis a at cell (i, j, k), radius r. */
static double d_first(const field_view *v, const double h[3], int r, int a,
                      int64_t i, int64_t j, int64_t k)
{
    double acc = 0.0;
    for (int m = -r; m <= r; ++m)
        acc += A1[r - 1][m + RMAX] * at(v, i, j, k, m * E[a][0], m * E[a][1], m * E[a][2]);
    return acc / h[a];
}

/* Pure second derivative along axis a at cell (i, j, k), radius r. */
static double d_second(const field_view *v, const double h[3], int r, int a,
                       int64_t i, int64_t j, int64_t k)
{
    double acc = 0.0;
    for (int m = -r; m <= r; ++m)
        acc += A2[r - 1][m + RMAX] * at(v, i, j, k, m * E[a][0], m * E[a][1], m * E[a][2]);
    return acc / (h[a] * h[a]);
}

/* Mixed second derivative d^2 f / (d x_a d x_b), a != b, from the planar
 * diagonal points only.  Along the diagonal e_a + e_b, the curve
 * g(t) = f(x + t(h_a e_a + h_b e_b)) has
 *   g'' = h_a^2 f_aa + 2 h_a h_b f_ab + h_b^2 f_bb,
 * and along e_a - e_b, q'' = h_a^2 f_aa - 2 h_a h_b f_ab + h_b^2 f_bb,
 * so f_ab = (g'' - q'') / (4 h_a h_b).  g'' and q'' use the pure
 * second-derivative weights with unit step along their diagonal.         */
static double d_mixed(const field_view *v, const double h[3], int r, int a, int b,
                      int64_t i, int64_t j, int64_t k)
{
    double gpp = 0.0, qpp = 0.0;
    for (int m = -r; m <= r; ++m) {
        int64_t ox_p = m * (E[a][0] + E[b][0]);
        int64_t oy_p = m * (E[a][1] + E[b][1]);
        int64_t oz_p = m * (E[a][2] + E[b][2]);
        int64_t ox_q = m * (E[a][0] - E[b][0]);
        int64_t oy_q = m * (E[a][1] - E[b][1]);
        int64_t oz_q = m * (E[a][2] - E[b][2]);
        gpp += A2[r - 1][m + RMAX] * at(v, i, j, k, ox_p, oy_p, oz_p);
        qpp += A2[r - 1][m + RMAX] * at(v, i, j, k, ox_q, oy_q, oz_q);
    }
    return (gpp - qpp) / (4.0 * h[a] * h[b]);
}

static void grid_spacing(const oracle_params *p, double h[3])
{
    h[0] = p->lx / p->nx;
    h[1] = p->ly / p->ny;
    h[2] = p->lz / p->nz;
}

/* Right-hand side of Eqs. B.1-B.4 at one cell.  Every field gets its
 * full gradient and full Hessian; the physics below then reads only what
 * the equations use.                                                     */
static void rhs_cell(const oracle_params *p, const double *f, int64_t i, int64_t j,
                     int64_t k, double out[NQ])
{
    double h[3];
    grid_spacing(p, h);
    const int64_t cells = (int64_t)p->nx * p->ny * p->nz;
    const int r = p->radius;

    double c[NQ];        /* centre values */
    double g[NQ][3];     /* g[q][a] = d f_q / d x_a */
    double H[NQ][3][3];  /* H[q][a][b] = d^2 f_q / (d x_a d x_b) */
    for (int q = 0; q < NQ; ++q) {
        field_view v = {{p->nx, p->ny, p->nz}, f + q * cells};
        c[q] = at(&v, i, j, k, 0, 0, 0);
        for (int a = 0; a < 3; ++a) {
            g[q][a] = d_first(&v, h, r, a, i, j, k);
            H[q][a][a] = d_second(&v, h, r, a, i, j, k);
        }
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b) {
                H[q][a][b] = d_mixed(&v, h, r, a, b, i, j, k);
                H[q][b][a] = H[q][a][b];
            }
    }

    const double lnrho = c[Q_LNRHO], ss = c[Q_SS];
    const double u[3] = {c[Q_UX], c[Q_UY], c[Q_UZ]};
    const double *glnrho = g[Q_LNRHO];
    const double *gss = g[Q_SS];

    /* G[a][b] = d u_a / d x_b; A_grad[a][b] = d A_a / d x_b */
    double G[3][3], GA[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            G[a][b] = g[Q_UX + a][b];
            GA[a][b] = g[Q_AX + a][b];
        }

    /* Thermodynamics (ideal gas). */
    const double gamma = p->gamma, cp = p->cp;
    const double rho = exp(lnrho);
    const double cs2 = p->cs0 * p->cs0 *
                       exp(gamma * ss / cp + (gamma - 1.0) * (lnrho - p->lnrho0));
    const double inv_T = cp * (gamma - 1.0) / cs2;

    /* Velocity gradient, divergence, traceless rate of shear. */
    const double divu = G[0][0] + G[1][1] + G[2][2];
    double S[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            S[a][b] = 0.5 * (G[a][b] + G[b][a]) - (a == b ? divu / 3.0 : 0.0);

    /* Magnetic field B = curl A + B_ext. */
    double B[3];
    B[0] = GA[2][1] - GA[1][2] + p->bext[0];
    B[1] = GA[0][2] - GA[2][0] + p->bext[1];
    B[2] = GA[1][0] - GA[0][1] + p->bext[2];

    /* Laplacians and gradient of divergence. */
    double lapu[3], graddivu[3], lapA[3], graddivA[3];
    for (int a = 0; a < 3; ++a) {
        lapu[a] = H[Q_UX + a][0][0] + H[Q_UX + a][1][1] + H[Q_UX + a][2][2];
        lapA[a] = H[Q_AX + a][0][0] + H[Q_AX + a][1][1] + H[Q_AX + a][2][2];
        graddivu[a] = H[Q_UX][a][0] + H[Q_UY][a][1] + H[Q_UZ][a][2];
        graddivA[a] = H[Q_AX][a][0] + H[Q_AY][a][1] + H[Q_AZ][a][2];
    }
    const double laplnrho = H[Q_LNRHO][0][0] + H[Q_LNRHO][1][1] + H[Q_LNRHO][2][2];
    const double lapss = H[Q_SS][0][0] + H[Q_SS][1][1] + H[Q_SS][2][2];

    /* Current density j = (grad div A - lap A) / mu0. */
    double jc[3];
    for (int a = 0; a < 3; ++a)
        jc[a] = (graddivA[a] - lapA[a]) / p->mu0;

    /* Cross products. */
    double jxB[3], uxB[3];
    jxB[0] = jc[1] * B[2] - jc[2] * B[1];
    jxB[1] = jc[2] * B[0] - jc[0] * B[2];
    jxB[2] = jc[0] * B[1] - jc[1] * B[0];
    uxB[0] = u[1] * B[2] - u[2] * B[1];
    uxB[1] = u[2] * B[0] - u[0] * B[2];
    uxB[2] = u[0] * B[1] - u[1] * B[0];

    /* B.1: continuity for ln rho. */
    double u_dot_glnrho = 0.0;
    for (int b = 0; b < 3; ++b)
        u_dot_glnrho += u[b] * glnrho[b];
    out[Q_LNRHO] = -u_dot_glnrho - divu;

    /* B.2: momentum. */
    for (int a = 0; a < 3; ++a) {
        double adv = 0.0, S_glnrho = 0.0;
        for (int b = 0; b < 3; ++b) {
            adv += u[b] * G[a][b];
            S_glnrho += S[a][b] * glnrho[b];
        }
        const double pressure = -cs2 * (gss[a] / cp + glnrho[a]);
        const double lorentz = jxB[a] / rho;
        const double visc = p->nu * (lapu[a] + graddivu[a] / 3.0 + 2.0 * S_glnrho);
        const double bulk = p->zeta * graddivu[a];
        out[Q_UX + a] = -adv + pressure + lorentz + visc + bulk;
    }

    /* B.3: entropy, divided by rho T. */
    double glnT[3];
    for (int a = 0; a < 3; ++a)
        glnT[a] = gamma * gss[a] / cp + (gamma - 1.0) * glnrho[a];
    const double laplnT = gamma * lapss / cp + (gamma - 1.0) * laplnrho;
    double glnT2 = 0.0, u_dot_gss = 0.0, jj = 0.0, SS = 0.0;
    for (int a = 0; a < 3; ++a) {
        glnT2 += glnT[a] * glnT[a];
        u_dot_gss += u[a] * gss[a];
        jj += jc[a] * jc[a];
        for (int b = 0; b < 3; ++b)
            SS += S[a][b] * S[a][b];
    }
    const double conduction = (p->K / rho) * (laplnT + glnT2);
    const double heating = inv_T * ((p->heat - p->cool) / rho + p->eta * p->mu0 * jj / rho +
                                    2.0 * p->nu * SS + p->zeta * divu * divu);
    out[Q_SS] = -u_dot_gss + conduction + heating;

    /* B.4: induction in the resistive gauge as printed. */
    for (int a = 0; a < 3; ++a)
        out[Q_AX + a] = uxB[a] + p->eta * lapA[a];
}

/* ---------------------------------------------------------------- API */

/* Derivative operator codes for oracle_deriv. */
enum {
    OP_D1X = 0, OP_D1Y, OP_D1Z, OP_D2X, OP_D2Y, OP_D2Z, OP_DXY, OP_DXZ, OP_DYZ
};

/* Apply one derivative operator of radius r to one periodic field of
 * nx*ny*nz cells.  Returns 0, or -1 on a bad operator code, radius or size. */
int oracle_deriv(int32_t nx, int32_t ny, int32_t nz, double lx, double ly, double lz,
                 int32_t r, const double *f, int32_t op, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || op < 0 || op > OP_DYZ || r < 1 || r > RMAX)
        return -1;
    const double h[3] = {lx / nx, ly / ny, lz / nz};
    field_view v = {{nx, ny, nz}, f};
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double d;
                switch (op) {
                case OP_D1X: d = d_first(&v, h, r, 0, i, j, k); break;
                case OP_D1Y: d = d_first(&v, h, r, 1, i, j, k); break;
                case OP_D1Z: d = d_first(&v, h, r, 2, i, j, k); break;
                case OP_D2X: d = d_second(&v, h, r, 0, i, j, k); break;
                case OP_D2Y: d = d_second(&v, h, r, 1, i, j, k); break;
                case OP_D2Z: d = d_second(&v, h, r, 2, i, j, k); break;
                case OP_DXY: d = d_mixed(&v, h, r, 0, 1, i, j, k); break;
                case OP_DXZ: d = d_mixed(&v, h, r, 0, 2, i, j, k); break;
                default:     d = d_mixed(&v, h, r, 1, 2, i, j, k); break;
                }
                out[(k * ny + j) * nx + i] = d;
            }
    return 0;
}

/* The weights the oracle uses at radius r, for the tests that check them
 * against an independent derivation: a1[2r+1], a2[2r+1] for offsets -r..r.
 * Returns 0, or -1 on a bad radius.                                     */
int oracle_weights(int32_t r, double *a1, double *a2)
{
    if (r < 1 || r > RMAX)
        return -1;
    for (int m = -r; m <= r; ++m) {
        a1[m + r] = A1[r - 1][m + RMAX];
        a2[m + r] = A2[r - 1][m + RMAX];
    }
    return 0;
}

void oracle_rk3_coeffs(double alpha[3], double beta[3])
{
    memcpy(alpha, RK_ALPHA, sizeof RK_ALPHA);
    memcpy(beta, RK_BETA, sizeof RK_BETA);
}

/* RHS of all 8 fields at every cell: f and rhs are 8*nx*ny*nz doubles. */
int oracle_rhs(const oracle_params *p, const double *f, double *rhs)
{
    if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1 || p->radius < 1 || p->radius > RMAX)
        return -1;
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz, cells = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double out[NQ];
                rhs_cell(p, f, i, j, k, out);
                const int64_t c = (k * ny + j) * nx + i;
                for (int q = 0; q < NQ; ++q)
                    rhs[q * cells + c] = out[q];
            }
    return 0;
}

/* The 2N update of one value for substep s: w <- alpha_s w + dt rhs,
 * f <- f + beta_s w.  For s = 0 the old w is not read (alpha_0 = 0), so an
 * uninitialised w cannot leak into the result.                          */
static void rk_update_one(int32_t s, double f_old, double w_old, double rhs, double dt,
                          double *f_new, double *w_new)
{
    const double wn = (s == 0) ? dt * rhs : RK_ALPHA[s] * w_old + dt * rhs;
    *w_new = wn;
    *f_new = f_old + RK_BETA[s] * wn;
}

/* One 2N update of n values for substep s, in place on f and w. */
int oracle_rk3_update(int64_t n, int32_t s, double *f, double *w, const double *rhs,
                      double dt)
{
    if (s < 0 || s > 2 || n < 0)
        return -1;
    for (int64_t c = 0; c < n; ++c)
        rk_update_one(s, f[c], s == 0 ? 0.0 : w[c], rhs[c], dt, &f[c], &w[c]);
    return 0;
}

/* Substep s evaluated at selected cells only, for spot checks of large
 * grids.  cells[t] is a flat interior index (k*ny + j)*nx + i.  Reads the
 * whole state f (8 fields) and, for s > 0, w; writes out_f[q*ncells + t]
 * and out_w[q*ncells + t].  Returns 0, or -1 on bad arguments.          */
int oracle_substep_at(const oracle_params *p, int32_t s, const double *f, const double *w,
                      double dt, int64_t ncells, const int64_t *cells, double *out_f,
                      double *out_w)
{
    if (!p || s < 0 || s > 2 || (s > 0 && !w) || ncells < 0 || p->radius < 1 ||
        p->radius > RMAX)
        return -1;
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz, n = nx * ny * nz;
    for (int64_t t = 0; t < ncells; ++t)
        if (cells[t] < 0 || cells[t] >= n)
            return -1;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < ncells; ++t) {
        const int64_t c = cells[t];
        const int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        double r[NQ];
        rhs_cell(p, f, i, j, k, r);
        for (int q = 0; q < NQ; ++q)
            rk_update_one(s, f[q * n + c], s == 0 ? 0.0 : w[q * n + c], r[q], dt,
                          &out_f[q * ncells + t], &out_w[q * ncells + t]);
    }
    return 0;
}

/* One substep: rhs = F(f), then the 2N update in place on f and w.
 * scratch holds 8*nx*ny*nz doubles.                                     */
int oracle_substep(const oracle_params *p, int32_t s, double *f, double *w, double dt,
                   double *scratch)
{
    if (oracle_rhs(p, f, scratch) != 0)
        return -1;
    const int64_t n = (int64_t)NQ * p->nx * p->ny * p->nz;
    return oracle_rk3_update(n, s, f, w, scratch, dt);
}

/* nsteps full RK3 steps (three substeps each) in place on f; w is the
 * 8*nx*ny*nz-double 2N register (its contents on entry are not read).   */
int oracle_step(const oracle_params *p, double *f, double *w, double dt, int32_t nsteps)
{
    if (!p || nsteps < 0)
        return -1;
    const int64_t n = (int64_t)NQ * p->nx * p->ny * p->nz;
    double *scratch = (double *)malloc((size_t)n * sizeof(double));
    if (!scratch)
        return -2;
    int rc = 0;
    for (int32_t t = 0; t < nsteps && rc == 0; ++t)
        for (int32_t s = 0; s < 3 && rc == 0; ++s)
            rc = oracle_substep(p, s, f, w, dt, scratch);
    free(scratch);
    return rc;
}
