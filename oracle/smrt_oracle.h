/*
 * smrt_oracle.h -- plain FP64 CPU oracle for the D2Q9 lattice Boltzmann update
 * with the single-relaxation-time (SRT/BGK) collision and the single
 * MRT-featured (SmrtLBM) collision of Zhou, "Single MRT-featured Lattice
 * Boltzmann Method", arXiv:2409.01076.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no source, header, table or helper with the GPU
 * path, and it never reads anything the GPU path produced.
 *
 * Conventions (all arrays are plain C doubles, caller-owned):
 *   - velocity set and ordering as in the paper's D2Q9 definition below the
 *     SRT equation: e_0=(0,0), e_1=(1,0), e_2=(0,1), e_3=(-1,0), e_4=(0,-1),
 *     e_5=(1,1), e_6=(-1,1), e_7=(-1,-1), e_8=(1,-1); lattice units, so the
 *     particle speed e = dx/dt = 1.
 *   - lattice populations are stored node-major: f[(y*nx + x)*9 + a].
 *   - row y = 0 is the bottom; a non-periodic axis is closed by half-way
 *     bounce-back walls at -1/2 and n-1/2; the wall beyond the top row
 *     (y = ny) moves with velocity (u_lid, 0), every other wall is at rest.
 *   - second lid reading (lid = 1, non-periodic y only): the top row of
 *     nodes is the lid itself.  After each step its populations are set to
 *     the equilibrium at velocity (u_lid, 0) and the density that the
 *     populations it received from inside give for a wall moving along
 *     itself, rho = f_0 + f_1 + f_3 + 2 (f_2 + f_5 + f_6); nothing streams
 *     in from above.  The side and bottom walls stay half-way bounce-back.
 *
 * Error behaviour: functions returning int give 0 on success and -1 on an
 * invalid argument (NULL pointer, non-positive size, unknown scheme,
 * relaxation time <= 1/2).  Nothing is printed.
 */
#ifndef SMRT_ORACLE_H
#define SMRT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_SRT = 0, ORACLE_SMRT = 1, ORACLE_TRT = 2 };

typedef struct oracle_lattice {
    int nx, ny;
    int periodic_x, periodic_y; /* 1: wrap around; 0: bounce-back walls */
    int scheme;                 /* ORACLE_SRT, ORACLE_SMRT or ORACLE_TRT */
    double tau;                 /* relaxation time tied to viscosity      */
    double tau_s;               /* second relaxation time (TRT form only) */
    double u_lid;               /* x-velocity of the top wall             */
    int lid;                    /* 0: moving wall half a link above the
                                   top row; 1: equilibrium lid on the top
                                   row (see above)                          */
} oracle_lattice;

/* Copies the lattice constants (velocities, weights, opposite directions). */
void oracle_constants(int ex[9], int ey[9], double w[9], int opp[9]);

/* Equilibrium distribution, Eq. (feq-full). */
void oracle_equilibrium(double rho, double ux, double uy, double feq[9]);

/* Density and velocity of one node, Eq. (fea-0). */
void oracle_node_moments(const double f[9], double* rho, double* ux, double* uy);

/* Post-collision populations of one node:
 *   ORACLE_SRT : Eq. (lb.srt) right-hand side;
 *   ORACLE_SMRT: Eq. (SmrtLBM-1) right-hand side;
 *   ORACLE_TRT : Eq. (SmrtLBM-lb.1.5) right-hand side (uses tau_s). */
int oracle_node_collide(int scheme, double tau, double tau_s,
                        const double f[9], double fstar[9]);

/* f = f^eq(rho, u) at every node; rho/ux/uy are [ny][nx]. */
int oracle_init_equilibrium(const oracle_lattice* L, const double* rho,
                            const double* ux, const double* uy, double* f);

/* Collision at every node: fstar = collide(f). */
int oracle_collide_lattice(const oracle_lattice* L, const double* f, double* fstar);

/* Streaming with walls: fnext_a(x + e_a) = fstar_a(x), bounced back where
 * x + e_a lies beyond a wall; with lid = 1 the top row is then set to the
 * lid's equilibrium.  fstar and fnext must not overlap. */
int oracle_stream_lattice(const oracle_lattice* L, const double* fstar, double* fnext);

/* nsteps of collide-then-stream, in place on f (pre-collision populations). */
int oracle_run(const oracle_lattice* L, double* f, long nsteps);

/* Density and velocity at every node, [ny][nx] each. */
int oracle_fields(const oracle_lattice* L, const double* f,
                  double* rho, double* ux, double* uy);

/* Fixed-order FP64 sums over n nodes:
 *   out[0] = sum |u - u_snap|^2, out[1] = sum |u|^2, out[2] = sum rho,
 *   out[3] = number of nodes whose rho, ux or uy is not finite. */
int oracle_reduce(long n, const double* rho, const double* ux, const double* uy,
                  const double* ux_snap, const double* uy_snap, double out[4]);

/* Relaxation time for a target Reynolds number Re = U * N / nu, using the
 * viscosity relation nu = (2 tau - 1) / 6 in lattice units. */
double oracle_tau_from_re(double re, double u_lid, int n);

/* OpenMP threads used by the lattice functions; returns the value in force. */
int oracle_set_threads(int n);
int oracle_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
