/*
 * FP64 CPU oracle of the hybrid central-moments / BGK lattice Boltzmann step for the
 * coupled Cahn-Hilliard--Navier-Stokes equations (De Rosis, Saito, Kaneko, Abe,
 * "Central-moments-based lattice Boltzmann scheme for coupled Cahn-Hilliard--Navier-Stokes
 * equations", arXiv:1803.11345).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, literal reference that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may build, load or call it; the GPU library neither links nor includes it, and it
 * shares no header, table or helper with the GPU code.
 *
 * It follows the paper's steps in the paper's order and notation, in plain double precision:
 *   1. phi = sum_i g_i for every node first (macroscopic variables, paragraph after Eq. (14));
 *   2. the isotropic 9-point gradient and Laplacian of phi (Eq. (12));
 *   3. mu = a(-phi + phi^3) - gamma Lap phi (chemical potential in the introduction),
 *      rho = sum f, v = sum f c / rho, p0 (Eq. (13)), p~ (Eq. (14)), the relaxation
 *      frequencies (paragraph after Eq. (14));
 *   4. f: the explicit 9x9 matrix Tbar^T of the shifted basis (Eq. (15)), pre-collision
 *      central moments k = Tbar^T f, the printed equilibrium central moments (list before and
 *      including Eq. (16)), relaxation (Eq. (17)) with omega_4 = omega_5 = omega_rho and
 *      omega_6..8 = 1, and f* = (Tbar^T)^{-1} k* by a generic LU solve;
 *   5. g: BGK relaxation (Eq. (7)) to the equilibrium of Eqs. (9)-(10);
 *   6. streaming in the push form of Eqs. (4)-(5) into a second buffer.
 *
 * Readings where the paper is silent or its printed text is inconsistent (each one is listed
 * with its reason in the design notes of the repository):
 *   - w^yy_4 is taken as +1/3 (printed -1/3 in Eq. (11)); with -1/3 the equilibrium carries a
 *     spurious y momentum and the second moment no longer matches the pressure tensor.
 *   - k8^eq: the definition k^eq = Tbar^T f^eq gives -(c_s^2/2) gamma |grad phi|^2 where
 *     Eq. (16) prints -(c_s^2/2) gamma Lap phi.  Default: the definition (k8_printed = 0);
 *     k8_printed = 1 keeps the printed term for sensitivity runs.
 *   - omega_3 (bulk) is not given; it is a parameter (default 1).
 *   - a body force F (not in the paper) enters with Guo's half-step: v = (sum f c + F/2)/rho,
 *     and the central moments R = Tbar^T F^Guo are added with weight (1 - omega_i/2).
 *   - walls (bc 1): half-way bounce-back of both f and g at y = -1/2 and y = ny - 1/2.  The
 *     ghost row behind a wall holds phi of the first (last) row minus the wall gradient
 *     d_perp phi_w of the contact-angle test (taken along the normal into the fluid, one node
 *     spacing across the wall; 0 gives the mirrored, zero-gradient row).
 *   - moving walls (the shear test): a wall moving along x with speed U returns a link j with
 *     the momentum correction 2 w_j s (c_j . U) / c_s^2 of the half-way bounce-back, s = 1 (the
 *     reference density) for f and s = phi of the node for g, so that the wall drags phi as the
 *     fluid does.
 *   - initial populations are the equilibria of the initial (phi, rho, v).
 *
 * Layout of every population array: P[i][y][x], i = 0..8, x fastest, planes of nx*ny values.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny;
    int walls;        /* 0: periodic in y; 1: half-way bounce-back walls in y */
    double a, gamma;  /* free-energy constants */
    double mobility;  /* M */
    double Gamma;     /* Gamma in the g equilibrium and the mobility relation */
    double nu_l;      /* viscosity where phi = +1 */
    double nu_g;      /* viscosity where phi = -1 */
    double omega3;    /* bulk-viscosity rate of k3 */
    double force_x, force_y;
    double wall_ux_bottom, wall_ux_top; /* x velocities of the walls (walls = 1) */
    double wall_gradient;             /* d_perp phi_w at both walls, along the inward normal */
    int k8_printed;   /* 1: k8 equilibrium with the printed gamma*Lap(phi) term */
    int collision;    /* 0: central moments (the method); 1: central moments with every rate
                         equal to omega_rho; 2: double BGK (Eq. (6)) */
    int nthreads;     /* OpenMP threads, 0 = runtime default */
} orc_params;

/* D2Q9 velocities and weights (paragraph before Eq. (4); weights after Eq. (14)). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const double CS2 = 1.0 / 3.0;

/* Surface-tension weights, Eq. (11), with w^yy_4 = +1/3. */
static const double WXX[9] = {0, 1.0 / 3, -1.0 / 6, 1.0 / 3, -1.0 / 6,
                              -1.0 / 24, -1.0 / 24, -1.0 / 24, -1.0 / 24};
static const double WYY[9] = {0, -1.0 / 6, 1.0 / 3, -1.0 / 6, 1.0 / 3,
                              -1.0 / 24, -1.0 / 24, -1.0 / 24, -1.0 / 24};
static const double WXY[9] = {0, 0, 0, 0, 0, 1.0 / 4, -1.0 / 4, 1.0 / 4, -1.0 / 4};

/* Stencils of Eq. (12): coefficient i multiplies phi at x + c_i. */
static const double SX[9] = {0, 4.0 / 12, 0, -4.0 / 12, 0, 1.0 / 12, -1.0 / 12, -1.0 / 12, 1.0 / 12};
static const double SY[9] = {0, 0, 4.0 / 12, 0, -4.0 / 12, 1.0 / 12, 1.0 / 12, -1.0 / 12, -1.0 / 12};
static const double SL[9] = {-20.0 / 6, 4.0 / 6, 4.0 / 6, 4.0 / 6, 4.0 / 6,
                             1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};

#ifdef _OPENMP
#include <omp.h>
#else
static int omp_get_max_threads(void) { return 1; }
#endif

static int nthr(const orc_params *p) { return p->nthreads > 0 ? p->nthreads : omp_get_max_threads(); }

static int opposite(int i)
{
    for (int j = 0; j < 9; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i]) return j;
    return -1;
}

static int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

int orc_check(const orc_params *p)
{
    if (!p || p->nx < 1 || p->ny < 1) return -1;
    if (p->walls != 0 && p->walls != 1) return -1;
    if (!(p->nu_l > 0) || !(p->nu_g > 0) || !(p->mobility > 0) || !(p->Gamma > 0)) return -1;
    if (!isfinite(p->wall_ux_bottom) || !isfinite(p->wall_ux_top) || !isfinite(p->wall_gradient)) return -1;
    if (p->collision < 0 || p->collision > 2) return -1;
    return 0;
}

/* phi at (x, y) where x may be any integer (periodic) and y may be -1 or ny with walls
   (ghost row: the first / last row minus the wall gradient) or any integer when periodic. */
static double phi_at(const orc_params *p, const double *phi, int x, int y)
{
    x = wrap(x, p->nx);
    if (p->walls) {
        if (y < 0) return phi[x] - p->wall_gradient;
        if (y >= p->ny) return phi[(size_t)(p->ny - 1) * p->nx + x] - p->wall_gradient;
    } else {
        y = wrap(y, p->ny);
    }
    return phi[(size_t)y * p->nx + x];
}

/* Eq. (12) applied to a phi plane. */
void orc_stencil(const orc_params *p, const double *phi, double *dx, double *dy, double *lap)
{
    const int nx = p->nx, ny = p->ny;
#pragma omp parallel for num_threads(nthr(p))
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double sx = 0, sy = 0, sl = 0;
            for (int i = 0; i < 9; ++i) {
                double v = phi_at(p, phi, x + CX[i], y + CY[i]);
                sx += SX[i] * v;
                sy += SY[i] * v;
                sl += SL[i] * v;
            }
            size_t n = (size_t)y * nx + x;
            if (dx) dx[n] = sx;
            if (dy) dy[n] = sy;
            if (lap) lap[n] = sl;
        }
}

/* Chemical potential (introduction), bulk pressure Eq. (13), modified pressure Eq. (14). */
double orc_mu(double a, double gamma, double phi, double lap)
{
    return a * (-phi + phi * phi * phi) - gamma * lap;
}

double orc_p0(double a, double rho, double phi)
{
    return rho * CS2 + a * (-0.5 * phi * phi + 0.75 * phi * phi * phi * phi);
}

double orc_ptilde(double a, double gamma, double rho, double phi, double lap)
{
    return orc_p0(a, rho, phi) - gamma * phi * lap;
}

/* Relaxation frequencies (paragraph after Eq. (14)). */
double orc_omega_rho(const orc_params *p, double phi)
{
    double wl = 1.0 / (p->nu_l / CS2 + 0.5);
    double wg = 1.0 / (p->nu_g / CS2 + 0.5);
    return wg + 0.5 * (phi + 1.0) * (wl - wg);
}

double orc_omega_phi(const orc_params *p)
{
    /* M = (1/omega_phi - 1/2) Gamma c_s^2 */
    return 1.0 / (p->mobility / (p->Gamma * CS2) + 0.5);
}

/* Eq. (8) for i = 1..8 and Eq. (10) for i = 0. */
void orc_feq(double rho, double ux, double uy, double pt, double gamma, double dpx, double dpy,
             double out[9])
{
    double sum = 0;
    double u2 = ux * ux + uy * uy;
    for (int i = 1; i < 9; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        out[i] = W[i] * (pt / CS2 + rho * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - u2 / (2 * CS2))) +
                 gamma * (WXX[i] * dpx * dpx + WYY[i] * dpy * dpy + WXY[i] * dpx * dpy);
        sum += out[i];
    }
    out[0] = rho - sum;
}

/* Eq. (9) for i = 1..8 and Eq. (10) for i = 0. */
void orc_geq(double phi, double mu, double ux, double uy, double Gamma, double out[9])
{
    double sum = 0;
    double u2 = ux * ux + uy * uy;
    for (int i = 1; i < 9; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        out[i] = W[i] * (Gamma * mu + phi * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - u2 / (2 * CS2)));
        sum += out[i];
    }
    out[0] = phi - sum;
}

/* Tbar^T of Eq. (15): row j holds basis vector Tbar_j evaluated at cbar_i = c_i - u, so that
   k = M f. */
void orc_tmatrix(double ux, double uy, double M[81])
{
    for (int i = 0; i < 9; ++i) {
        double bx = CX[i] - ux, by = CY[i] - uy;
        M[0 * 9 + i] = 1.0;
        M[1 * 9 + i] = bx;
        M[2 * 9 + i] = by;
        M[3 * 9 + i] = bx * bx + by * by;
        M[4 * 9 + i] = bx * bx - by * by;
        M[5 * 9 + i] = bx * by;
        M[6 * 9 + i] = bx * bx * by;
        M[7 * 9 + i] = bx * by * by;
        M[8 * 9 + i] = bx * bx * by * by;
    }
}

/* Equilibrium central moments as listed in the paper (list ending in Eq. (16)).  k8 carries
   -(c_s^2/2) gamma |grad phi|^2 unless k8_printed, which uses the printed Lap(phi). */
void orc_keq(double rho, double ux, double uy, double pt, double gamma, double dpx, double dpy,
             double lap, int k8_printed, double k[9])
{
    k[0] = rho;
    k[1] = 0;
    k[2] = 0;
    k[3] = 2 * pt;
    k[4] = gamma * (dpx * dpx - dpy * dpy);
    k[5] = gamma * dpx * dpy;
    k[6] = -0.5 * uy * k[4] - 2 * ux * k[5] + rho * uy * (CS2 - ux * ux) - pt * uy;
    k[7] = 0.5 * ux * k[4] - 2 * uy * k[5] + rho * ux * (CS2 - uy * uy) - pt * ux;
    double surf = k8_printed ? lap : (dpx * dpx + dpy * dpy);
    k[8] = pt * (CS2 + ux * ux + uy * uy) - rho * CS2 * (ux * ux + uy * uy) +
           rho / CS2 * ux * ux * uy * uy - 0.5 * CS2 * gamma * surf +
           0.5 * k[4] * (uy * uy - ux * ux) + 4 * ux * uy * k[5];
}

/* Guo's forcing populations F_i = w_i [ (c_i - u)/c_s^2 + (c_i . u) c_i / c_s^4 ] . F. */
void orc_guo(double ux, double uy, double Fx, double Fy, double out[9])
{
    for (int i = 0; i < 9; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        double cf = CX[i] * Fx + CY[i] * Fy;
        out[i] = W[i] * (((CX[i] - ux) * Fx + (CY[i] - uy) * Fy) / CS2 + cu * cf / (CS2 * CS2));
    }
}

/* Solve A x = b for a 9x9 system by Gaussian elimination with partial pivoting. */
static void solve9(const double Ain[81], const double bin[9], double x[9])
{
    double A[81], b[9];
    memcpy(A, Ain, sizeof A);
    memcpy(b, bin, sizeof b);
    for (int c = 0; c < 9; ++c) {
        int piv = c;
        for (int r = c + 1; r < 9; ++r)
            if (fabs(A[r * 9 + c]) > fabs(A[piv * 9 + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < 9; ++k) {
                double t = A[c * 9 + k];
                A[c * 9 + k] = A[piv * 9 + k];
                A[piv * 9 + k] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < 9; ++r) {
            double m = A[r * 9 + c] / A[c * 9 + c];
            if (m == 0) continue;
            for (int k = c; k < 9; ++k) A[r * 9 + k] -= m * A[c * 9 + k];
            b[r] -= m * b[c];
        }
    }
    for (int r = 8; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < 9; ++k) s -= A[r * 9 + k] * x[k];
        x[r] = s / A[r * 9 + r];
    }
}

/* Post-collision f at one node, given its pre-collision f and the phi data of the node.
   Also returns the velocity used (out_u, may be NULL). */
void orc_collide_f(const orc_params *p, const double f[9], double phi, double dpx, double dpy,
                   double lap, double fstar[9], double out_u[2])
{
    double rho = 0, jx = 0, jy = 0;
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += f[i] * CX[i];
        jy += f[i] * CY[i];
    }
    const double Fx = p->force_x, Fy = p->force_y;
    double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
    if (out_u) {
        out_u[0] = ux;
        out_u[1] = uy;
    }
    double pt = orc_ptilde(p->a, p->gamma, rho, phi, lap);
    double wr = orc_omega_rho(p, phi);
    double F[9];
    orc_guo(ux, uy, Fx, Fy, F);

    if (p->collision == 2) { /* double BGK, Eq. (6) (+ Guo force) */
        double feq[9];
        orc_feq(rho, ux, uy, pt, p->gamma, dpx, dpy, feq);
        for (int i = 0; i < 9; ++i) fstar[i] = f[i] + wr * (feq[i] - f[i]) + (1 - 0.5 * wr) * F[i];
        return;
    }

    double M[81], k[9], keq[9], R[9], ks[9], om[9];
    orc_tmatrix(ux, uy, M);
    for (int j = 0; j < 9; ++j) {
        double s = 0, r = 0;
        for (int i = 0; i < 9; ++i) {
            s += M[j * 9 + i] * f[i];
            r += M[j * 9 + i] * F[i];
        }
        k[j] = s;
        R[j] = r;
    }
    orc_keq(rho, ux, uy, pt, p->gamma, dpx, dpy, lap, p->k8_printed, keq);
    /* Eq. (17): omega_4 = omega_5 = omega_rho, omega_3 bulk, omega_6..8 = 1; the conserved
       k0..k2 take their equilibrium (plus the force) which equals a unit rate. */
    if (p->collision == 1) {
        for (int j = 0; j < 9; ++j) om[j] = wr;
    } else {
        om[0] = om[1] = om[2] = 1.0;
        om[3] = p->omega3;
        om[4] = om[5] = wr;
        om[6] = om[7] = om[8] = 1.0;
    }
    for (int j = 0; j < 9; ++j) ks[j] = k[j] + om[j] * (keq[j] - k[j]) + (1 - 0.5 * om[j]) * R[j];
    solve9(M, ks, fstar);
}

/* Post-collision g at one node, Eq. (7) with Eqs. (9)-(10). */
void orc_collide_g(const orc_params *p, const double g[9], double phi, double lap, double ux,
                   double uy, double gstar[9])
{
    double mu = orc_mu(p->a, p->gamma, phi, lap);
    double geq[9];
    orc_geq(phi, mu, ux, uy, p->Gamma, geq);
    double wp = orc_omega_phi(p);
    for (int i = 0; i < 9; ++i) gstar[i] = g[i] + wp * (geq[i] - g[i]);
}

/* Streaming in the push form of Eqs. (4)-(5): P_out[i](x + c_i) = Pstar[i](x); a link that
   leaves the lattice through a wall returns to the same node in the opposite direction. */
static void stream_push(const orc_params *p, const double *star, double *out)
{
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
#pragma omp parallel for num_threads(nthr(p))
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < 9; ++i) {
                int xd = wrap(x + CX[i], nx);
                int yd = y + CY[i];
                double v = star[(size_t)i * N + (size_t)y * nx + x];
                if (p->walls && (yd < 0 || yd >= ny)) {
                    out[(size_t)opposite(i) * N + (size_t)y * nx + x] = v;
                } else {
                    yd = wrap(yd, ny);
                    out[(size_t)i * N + (size_t)yd * nx + xd] = v;
                }
            }
}

/* Moving walls: the links that returned from a wall at this step gain 2 w_j s (c_j . U) / c_s^2
   (U the wall's x velocity; s = 1 for f, phi = sum of the node's g for g). */
static void wall_motion(const orc_params *p, double *out, int is_g)
{
    if (!p->walls || (p->wall_ux_bottom == 0 && p->wall_ux_top == 0)) return;
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    for (int x = 0; x < nx; ++x) {
        for (int side = 0; side < 2; ++side) {
            const int y = side == 0 ? 0 : ny - 1;
            const double U = side == 0 ? p->wall_ux_bottom : p->wall_ux_top;
            const int cy = side == 0 ? 1 : -1; /* links coming back from the wall */
            const size_t n = (size_t)y * nx + x;
            double s = 1.0;
            if (is_g) {
                s = 0;
                for (int i = 0; i < 9; ++i) s += out[(size_t)i * N + n];
            }
            for (int j = 0; j < 9; ++j)
                if (CY[j] == cy) out[(size_t)j * N + n] += 2.0 * W[j] * s * CX[j] * U / CS2;
        }
    }
}

/* Initial populations: equilibria of (phi0, rho0, u0).  NULL rho0/ux0/uy0 mean 1, 0, 0.
   Velocity passed in is the physical v (with a force the same v is used in f^eq). */
int orc_init(const orc_params *p, const double *phi0, const double *rho0, const double *ux0,
             const double *uy0, double *f, double *g)
{
    if (orc_check(p) || !phi0 || !f || !g) return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    double *dx = malloc(N * sizeof(double)), *dy = malloc(N * sizeof(double)),
           *lap = malloc(N * sizeof(double));
    if (!dx || !dy || !lap) {
        free(dx);
        free(dy);
        free(lap);
        return -2;
    }
    orc_stencil(p, phi0, dx, dy, lap);
#pragma omp parallel for num_threads(nthr(p))
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            double phi = phi0[n];
            double rho = rho0 ? rho0[n] : 1.0;
            double ux = ux0 ? ux0[n] : 0.0, uy = uy0 ? uy0[n] : 0.0;
            double pt = orc_ptilde(p->a, p->gamma, rho, phi, lap[n]);
            double mu = orc_mu(p->a, p->gamma, phi, lap[n]);
            double fe[9], ge[9];
            orc_feq(rho, ux, uy, pt, p->gamma, dx[n], dy[n], fe);
            orc_geq(phi, mu, ux, uy, p->Gamma, ge);
            for (int i = 0; i < 9; ++i) {
                f[(size_t)i * N + n] = fe[i];
                g[(size_t)i * N + n] = ge[i];
            }
        }
    free(dx);
    free(dy);
    free(lap);
    return 0;
}

/* One time step t -> t+1 (f, g -> f_out, g_out; the buffers must not overlap). */
int orc_step(const orc_params *p, const double *f, const double *g, double *f_out, double *g_out)
{
    if (orc_check(p) || !f || !g || !f_out || !g_out) return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    double *phi = malloc(N * sizeof(double)), *dx = malloc(N * sizeof(double)),
           *dy = malloc(N * sizeof(double)), *lap = malloc(N * sizeof(double)),
           *fs = malloc(9 * N * sizeof(double)), *gs = malloc(9 * N * sizeof(double));
    if (!phi || !dx || !dy || !lap || !fs || !gs) {
        free(phi);
        free(dx);
        free(dy);
        free(lap);
        free(fs);
        free(gs);
        return -2;
    }
    /* 1. phi = sum_i g_i at every node before any collision. */
#pragma omp parallel for num_threads(nthr(p))
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            double s = 0;
            for (int i = 0; i < 9; ++i) s += g[(size_t)i * N + n];
            phi[n] = s;
        }
    /* 2. gradient and Laplacian. */
    orc_stencil(p, phi, dx, dy, lap);
    /* 3.-5. collisions. */
#pragma omp parallel for num_threads(nthr(p))
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            double fl[9], gl[9], fo[9], go[9], u[2];
            for (int i = 0; i < 9; ++i) {
                fl[i] = f[(size_t)i * N + n];
                gl[i] = g[(size_t)i * N + n];
            }
            orc_collide_f(p, fl, phi[n], dx[n], dy[n], lap[n], fo, u);
            orc_collide_g(p, gl, phi[n], lap[n], u[0], u[1], go);
            for (int i = 0; i < 9; ++i) {
                fs[(size_t)i * N + n] = fo[i];
                gs[(size_t)i * N + n] = go[i];
            }
        }
    /* 6. streaming, and the momentum the moving walls give back. */
    stream_push(p, fs, f_out);
    stream_push(p, gs, g_out);
    wall_motion(p, f_out, 0);
    wall_motion(p, g_out, 1);
    free(phi);
    free(dx);
    free(dy);
    free(lap);
    free(fs);
    free(gs);
    return 0;
}

/* nsteps steps in place: on return f, g hold the state after nsteps. */
int orc_run(const orc_params *p, double *f, double *g, long nsteps)
{
    if (orc_check(p) || nsteps < 0) return -1;
    const size_t N = (size_t)p->nx * p->ny;
    double *f2 = malloc(9 * N * sizeof(double)), *g2 = malloc(9 * N * sizeof(double));
    if (!f2 || !g2) {
        free(f2);
        free(g2);
        return -2;
    }
    for (long s = 0; s < nsteps; ++s) {
        int rc = orc_step(p, f, g, f2, g2);
        if (rc) {
            free(f2);
            free(g2);
            return rc;
        }
        memcpy(f, f2, 9 * N * sizeof(double));
        memcpy(g, g2, 9 * N * sizeof(double));
    }
    free(f2);
    free(g2);
    return 0;
}

/* Macroscopic fields (paragraph after Eq. (14)); v includes the half force as in the step;
   p0 is the bulk pressure of Eq. (13).  Any output may be NULL. */
int orc_fields(const orc_params *p, const double *f, const double *g, double *phi, double *rho,
               double *ux, double *uy, double *p0)
{
    if (orc_check(p) || !f || !g) return -1;
    const size_t N = (size_t)p->nx * p->ny;
#pragma omp parallel for num_threads(nthr(p))
    for (long long n = 0; n < (long long)N; ++n) {
        double r = 0, jx = 0, jy = 0, ph = 0;
        for (int i = 0; i < 9; ++i) {
            double v = f[(size_t)i * N + n];
            r += v;
            jx += v * CX[i];
            jy += v * CY[i];
            ph += g[(size_t)i * N + n];
        }
        if (phi) phi[n] = ph;
        if (rho) rho[n] = r;
        if (ux) ux[n] = (jx + 0.5 * p->force_x) / r;
        if (uy) uy[n] = (jy + 0.5 * p->force_y) / r;
        if (p0) p0[n] = orc_p0(p->a, r, ph);
    }
    return 0;
}
