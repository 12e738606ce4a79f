/*
 * smrt_oracle.c -- plain FP64 CPU oracle for the SRT and SmrtLBM D2Q9 lattice
 * Boltzmann updates (Zhou, arXiv:2409.01076).
 *
 * TEST INFRASTRUCTURE ONLY: written to check the GPU library and nothing else.
 * It is deliberately slow and literal: every node is treated the same way, the
 * populations are full f (not deviations), sums run in a fixed order, and the
 * build uses -ffp-contract=off so no fused multiply-add changes the rounding.
 *
 * Parity pins: every function here is pinned by the CPU tests against facts
 * the paper or the mathematics fixes (equilibrium moments, the MRT matrix form
 * of the paper's appendix, conservation, the viscosity relation through
 * shear-wave decay, Couette flow, symmetry).  The oracle_reduce residual
 * statistic is a reading of the steady-state test, not a paper formula.
 */
#include "smrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 velocity set in the paper's order (text below Eq. lb.srt). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Weights: 4/9 for the rest particle, 1/9 on the axes, 1/36 on the diagonals. */
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Index of the direction opposite to a: e_opp(a) = -e_a. */
static int opposite(int a)
{
    for (int b = 0; b < 9; ++b)
        if (EX[b] == -EX[a] && EY[b] == -EY[a]) return b;
    return -1;
}

void oracle_constants(int ex[9], int ey[9], double w[9], int opp[9])
{
    for (int a = 0; a < 9; ++a) {
        ex[a] = EX[a];
        ey[a] = EY[a];
        w[a] = W[a];
        opp[a] = opposite(a);
    }
}

/* Eq. (feq-full) with e = 1:
 * f^eq_a = w_a rho (1 + 3 e_a.u + 9/2 (e_a.u)^2 - 3/2 u.u). */
void oracle_equilibrium(double rho, double ux, double uy, double feq[9])
{
    double uu = ux * ux + uy * uy;
    for (int a = 0; a < 9; ++a) {
        double eu = EX[a] * ux + EY[a] * uy;
        feq[a] = W[a] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* Eq. (fea-0): rho = sum_a f_a, u = (1/rho) sum_a e_a f_a. */
void oracle_node_moments(const double f[9], double* rho, double* ux, double* uy)
{
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; ++a) {
        r += f[a];
        jx += EX[a] * f[a];
        jy += EY[a] * f[a];
    }
    *rho = r;
    *ux = jx / r;
    *uy = jy / r;
}

/* Indicator function of Eq. (indicator-fn): 1 when both m and n belong to the
 * set {lo, lo+1, lo+2, lo+3}, else 0. */
static double indicator(int lo, int m, int n)
{
    int m_in = (m >= lo && m <= lo + 3);
    int n_in = (n >= lo && n <= lo + 3);
    return (m_in && n_in) ? 1.0 : 0.0;
}

/* (-1)^k for k >= 0. */
static double sign_pow(int k) { return (k % 2 == 0) ? 1.0 : -1.0; }

/* The signed sum shared by Eq. (SmrtLBM-1) and Eq. (SmrtLBM-lb.1.5):
 * sum_{k=1..8} (-1)^k / 4 [1_{1234}(a,k) + 1_{5678}(a,k)] (f_k - f^eq_k). */
static double group_sum(int a, const double f[9], const double feq[9])
{
    double s = 0.0;
    for (int k = 1; k <= 8; ++k) {
        double ind = indicator(1, a, k) + indicator(5, a, k);
        s += sign_pow(k) / 4.0 * ind * (f[k] - feq[k]);
    }
    return s;
}

int oracle_node_collide(int scheme, double tau, double tau_s, const double f[9],
                        double fstar[9])
{
    if (!(tau > 0.5)) return -1;
    if (scheme == ORACLE_TRT && !(tau_s > 0.5)) return -1;
    double rho, ux, uy, feq[9];
    oracle_node_moments(f, &rho, &ux, &uy);
    oracle_equilibrium(rho, ux, uy, feq);
    switch (scheme) {
    case ORACLE_SRT: /* Eq. (lb.srt) */
        for (int a = 0; a < 9; ++a) fstar[a] = f[a] - (f[a] - feq[a]) / tau;
        return 0;
    case ORACLE_SMRT: /* Eq. (SmrtLBM-1) */
        for (int a = 0; a < 9; ++a)
            fstar[a] = feq[a] + sign_pow(a) * (1.0 - 1.0 / tau) * group_sum(a, f, feq);
        return 0;
    case ORACLE_TRT: /* Eq. (SmrtLBM-lb.1.5) */
        for (int a = 0; a < 9; ++a)
            fstar[a] = f[a] - (f[a] - feq[a]) / tau_s +
                       sign_pow(a) * (1.0 / tau_s - 1.0 / tau) * group_sum(a, f, feq);
        return 0;
    default:
        return -1;
    }
}

static int lattice_ok(const oracle_lattice* L)
{
    if (!L || L->nx < 1 || L->ny < 1) return 0;
    if (!(L->tau > 0.5)) return 0;
    if (L->scheme < ORACLE_SRT || L->scheme > ORACLE_TRT) return 0;
    if (L->scheme == ORACLE_TRT && !(L->tau_s > 0.5)) return 0;
    if (L->lid != 0 && (L->lid != 1 || L->periodic_y || L->ny < 2)) return 0;
    return 1;
}

int oracle_init_equilibrium(const oracle_lattice* L, const double* rho, const double* ux,
                            const double* uy, double* f)
{
    if (!lattice_ok(L) || !rho || !ux || !uy || !f) return -1;
    long n = (long)L->nx * L->ny;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) oracle_equilibrium(rho[i], ux[i], uy[i], f + 9 * i);
    return 0;
}

int oracle_collide_lattice(const oracle_lattice* L, const double* f, double* fstar)
{
    if (!lattice_ok(L) || !f || !fstar) return -1;
    long n = (long)L->nx * L->ny;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i)
        oracle_node_collide(L->scheme, L->tau, L->tau_s, f + 9 * i, fstar + 9 * i);
    return 0;
}

/* Second lid reading: the top row holds the lid.  Each of its nodes is set
 * to f^eq(rho, (u_lid, 0)) with rho from the populations that arrived from
 * inside the cavity: for a wall moving along itself (u_y = 0) the unknown
 * f_4, f_7, f_8 carry as much mass as the f_2, f_5, f_6 that left, so
 * rho = f_0 + f_1 + f_3 + 2 (f_2 + f_5 + f_6).  Applied after streaming; what
 * streaming wrote into f_4, f_7, f_8 of the top row is overwritten. */
static void apply_equilibrium_lid(const oracle_lattice* L, double* f)
{
    const int nx = L->nx, y = L->ny - 1;
    for (int x = 0; x < nx; ++x) {
        double* g = f + 9 * ((long)y * nx + x);
        double rho = g[0] + g[1] + g[3] + 2.0 * (g[2] + g[5] + g[6]);
        oracle_equilibrium(rho, L->u_lid, 0.0, g);
    }
}

/* Left-hand side of every update equation: the post-collision population
 * f*_a(x) moves to x + e_a.  If x + e_a lies beyond a wall, the population is
 * bounced back into the opposite direction at x (half-way bounce-back, the
 * wall sits half a link away).  A moving wall adds -2 w_a rho_w (e_a.u_w)/c_s^2
 * = -6 w_a (e_a.u_w) with rho_w = 1 (moving-wall bounce-back).  A link whose
 * far end lies in the row above the top fluid row (corners included) ends on
 * the lid; every other wall is at rest.  With the second lid reading the
 * top row is then set to the lid's equilibrium (apply_equilibrium_lid). */
int oracle_stream_lattice(const oracle_lattice* L, const double* fstar, double* fnext)
{
    if (!lattice_ok(L) || !fstar || !fnext || fstar == fnext) return -1;
    const int nx = L->nx, ny = L->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const double* src = fstar + 9 * ((long)y * nx + x);
            for (int a = 0; a < 9; ++a) {
                int tx = x + EX[a];
                int ty = y + EY[a];
                int inside = 1;
                if (tx < 0 || tx >= nx) {
                    if (L->periodic_x)
                        tx = (tx + nx) % nx;
                    else
                        inside = 0;
                }
                if (ty < 0 || ty >= ny) {
                    if (L->periodic_y)
                        ty = (ty + ny) % ny;
                    else
                        inside = 0;
                }
                if (inside) {
                    fnext[9 * ((long)ty * nx + tx) + a] = src[a];
                } else {
                    double uwx = (!L->periodic_y && ty == ny) ? L->u_lid : 0.0;
                    double uwy = 0.0;
                    double eu = EX[a] * uwx + EY[a] * uwy;
                    fnext[9 * ((long)y * nx + x) + opposite(a)] = src[a] - 6.0 * W[a] * 1.0 * eu;
                }
            }
        }
    }
    if (L->lid == 1) apply_equilibrium_lid(L, fnext);
    return 0;
}

int oracle_run(const oracle_lattice* L, double* f, long nsteps)
{
    if (!lattice_ok(L) || !f || nsteps < 0) return -1;
    size_t bytes = sizeof(double) * 9 * (size_t)L->nx * (size_t)L->ny;
    double* fstar = (double*)malloc(bytes);
    if (!fstar) return -1;
    for (long s = 0; s < nsteps; ++s) {
        oracle_collide_lattice(L, f, fstar);
        oracle_stream_lattice(L, fstar, f);
    }
    free(fstar);
    return 0;
}

int oracle_fields(const oracle_lattice* L, const double* f, double* rho, double* ux, double* uy)
{
    if (!lattice_ok(L) || !f || !rho || !ux || !uy) return -1;
    long n = (long)L->nx * L->ny;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) oracle_node_moments(f + 9 * i, rho + i, ux + i, uy + i);
    return 0;
}

int oracle_reduce(long n, const double* rho, const double* ux, const double* uy,
                  const double* ux_snap, const double* uy_snap, double out[4])
{
    if (n < 0 || !rho || !ux || !uy || !ux_snap || !uy_snap || !out) return -1;
    double du2 = 0.0, u2 = 0.0, mass = 0.0, bad = 0.0;
    for (long i = 0; i < n; ++i) {
        if (!isfinite(rho[i]) || !isfinite(ux[i]) || !isfinite(uy[i])) bad += 1.0;
        double dx = ux[i] - ux_snap[i], dy = uy[i] - uy_snap[i];
        du2 += dx * dx + dy * dy;
        u2 += ux[i] * ux[i] + uy[i] * uy[i];
        mass += rho[i];
    }
    out[0] = du2;
    out[1] = u2;
    out[2] = mass;
    out[3] = bad;
    return 0;
}

/* Eq. (relation-chapman-viscosity) with e = dx = 1: nu = (2 tau - 1)/6, and
 * Re = U N / nu, so tau = 3 U N / Re + 1/2. */
double oracle_tau_from_re(double re, double u_lid, int n)
{
    double nu = u_lid * (double)n / re;
    return 3.0 * nu + 0.5;
}

int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
