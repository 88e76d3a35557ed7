/*
 * FP64 CPU oracle of the B-TriRT D2Q9 lattice Boltzmann time step
 * (Zhao, Wu, Chai & Shi, "A block triple-relaxation-time lattice Boltzmann
 * model for nonlinear anisotropic convection-diffusion equations",
 * arXiv:1902.09813).
 *
 * TEST INFRASTRUCTURE. This header and btrt_oracle.c are used only by the
 * tests, by the package's smoke check and by the benchmark's CPU-baseline leg.
 * The product library never includes, links or calls any of it, and this code
 * includes nothing from the product library.
 *
 * Units: lattice units throughout (dx = dt = 1, c = 1, c_s^2 = 1/3).
 * Layout of every population array: f[i*n + y*nx + x], n = nx*ny, i = 0..8 in
 * the velocity order of the moment matrix C of Eq. (85).
 */
#ifndef BTRT_ORACLE_H
#define BTRT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary side order: x-, x+, y-, y+. */
#define ORC_PERIODIC 0
#define ORC_DIRICHLET 1

typedef struct {
    int nx, ny;
    /* Convective flux B(phi) = a*phi + b*phi^2/2, per component (Eq. (1)). */
    double flux_a[2];
    double flux_b[2];
    /* Diffusion tensor A(phi) = A0*(1 + beta*phi^2), A0 = [[A0[0],A0[1]],[A0[1],A0[2]]]
     * (Eq. (1)); K1 follows from Eq. (30) at every node and step. */
    double A0[3];
    double beta;
    /* Relaxation: k0 (block S0) and the 2x2 block K2 (row major) of Eq. (6). */
    double k0;
    double K2[4];
    /* Boundary conditions per side: ORC_PERIODIC or ORC_DIRICHLET with value. */
    int bc_type[4];
    double bc_value[4];
    /* NULL, or a space-dependent A0(x) (Eq. (73), Eq. (74)): three values (a11, a12, a22)
     * per node at A0_field[3*(y*nx + x) + j], used in place of A0 by orc_run. */
    const double* A0_field;
    /* Power-law part of the flux: B(phi) gains flux_c * |phi|^flux_q per component (the
     * convection a phi^delta d_x phi of Eq. (67) is the divergence of a phi^(delta+1)/(delta+1)
     * along x). Ignored when both flux_c are 0. */
    double flux_c[2];
    double flux_q;
    /* Source depending on phi (Eq. (1), S(x, phi, t)): r phi (1 - |phi|^p) is added to the
     * given S, at phi(t) for S(t) and at phi(t-1) for S(t-1) (the reaction term of Eq. (67)
     * with r = b, p = delta). Ignored when src_r is 0. */
    double src_r;
    double src_p;
    /* D(phi) of Eq. (1) and Eq. (7): d_kind 0 is D = phi I; d_kind 1 is
     * D = (d_g phi + d_e |phi|^d_s) I. */
    int d_kind;
    double d_g, d_e, d_s;
} orc_problem_t;

/* D2Q9 equilibrium of Eq. (7) for a general D tensor (row major 2x2). */
void orc_equilibrium(double phi, const double B[2], const double D[4], double feq[9]);

/* One node collision of Eq. (6): f -> f+, with the correction G of Eq. (11)
 * (time derivative of B as a backward difference over one step), the source
 * of Eq. (8) and its time derivative by Scheme 2 (Remark III). S and S_prev are
 * the parts of the source that do not depend on phi; the phi-dependent part of
 * the problem is added at phi = sum f and at phi_prev. */
void orc_collide_node(const orc_problem_t* p, const double f[9], double phi_prev,
                      double S, double S_prev, double fpost[9]);

/* f := f^eq(phi0) at every node (initialisation of Section 4). */
void orc_init(const orc_problem_t* p, const double* phi0, double* f);

/* phi = sum_i f_i at every node (Eq. (9)). */
void orc_phi(const orc_problem_t* p, const double* f, double* phi);

/* Advance nsteps time steps: collide at every node, then stream (Eq. (38)),
 * with half-way bounce-back (Eqs. (54)-(56)) on Dirichlet sides.
 *   f        [9n]  post-streaming state at time t; on return, at t+nsteps
 *   work     [9n]  scratch
 *   phi_prev [n]   phi at t-1 (for dB/dt in G); on return, phi at t+nsteps-1
 *   S, S_prev [n]  source at t and t-1 (NULL: zero; S_prev NULL: equal to S)
 *   wall     [9n]  NULL, or the wall value phi_w for link i leaving node k through a
 *                  Dirichlet side, at wall[i*n + k] (time-dependent or varying walls);
 *                  NULL uses the per-side constants of the problem
 *   nthreads       OpenMP threads (<= 0: runtime default)
 * Returns 0, or -1 on bad arguments. */
int orc_run(const orc_problem_t* p, double* f, double* work, double* phi_prev,
            const double* S, const double* S_prev, const double* wall, long nsteps, int nthreads);

/* Number of OpenMP threads a parallel region would use with nthreads. */
int orc_threads(int nthreads);

#ifdef __cplusplus
}
#endif
#endif
