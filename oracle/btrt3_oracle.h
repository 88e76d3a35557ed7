/*
 * FP64 CPU oracle of the three-dimensional B-TriRT time step on the D3Q19 lattice
 * (Zhao, Wu, Chai & Shi, arXiv:1902.09813: Eq. (6) with the D3Q19 velocity set of
 * Eq. (86), K1 and K2 as 3x3 blocks, Eqs. (96), (100)).
 *
 * TEST INFRASTRUCTURE. Used only by the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg; the product library never includes, links or calls it,
 * and it includes nothing from the product library.
 *
 * Units: lattice units (dx = dt = 1, c = 1, c_s^2 = 1/3).
 * Layout of every population array: f[i*n + (z*ny + y)*nx + x], n = nx*ny*nz, i = 0..18
 * in the column order of C in Eq. (86).
 */
#ifndef BTRT3_ORACLE_H
#define BTRT3_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary face order: x-, x+, y-, y+, z-, z+; types as in btrt_oracle.h. */
typedef struct {
    int nx, ny, nz;
    /* B(phi) = a phi + b phi^2 / 2 per component (Eq. (1)). */
    double flux_a[3];
    double flux_b[3];
    /* A(phi) = A0 (1 + beta phi^2) with the symmetric A0 given as (a11, a12, a13, a22, a23, a33);
     * K1 from Eq. (30) at every node and step. */
    double A0[6];
    double beta;
    /* k0 on the S0 block, the 3x3 K2 block (row major) of Eq. (6). */
    double k0;
    double K2[9];
    int bc_type[6];
    double bc_value[6];
} orc3_problem_t;

/* D3Q19 equilibrium of Eq. (7) for a general D tensor (3x3 row major). */
void orc3_equilibrium(double phi, const double B[3], const double D[9], double feq[19]);

/* One node collision of Eq. (6) (f -> f+), with G of Eq. (11) (backward difference of B over
 * one step), the source of Eq. (8) and its Scheme 2 derivative (Remark III). */
void orc3_collide_node(const orc3_problem_t* p, const double f[19], double phi_prev, double S, double S_prev,
                       double fpost[19]);

/* f := f^eq(phi0) at every node. */
void orc3_init(const orc3_problem_t* p, const double* phi0, double* f);

/* phi = sum_i f_i at every node (Eq. (9)). */
void orc3_phi(const orc3_problem_t* p, const double* f, double* phi);

/* Advance nsteps steps: collide at every node, then push-stream (Eq. (38)) with half-way
 * bounce-back (Eqs. (54)-(56)) on Dirichlet faces; a link leaving through two faces (an edge)
 * takes the mean of their values.
 *   f [19n] post-streaming state at t (on return t + nsteps); work [19n] scratch;
 *   phi_prev [n] phi(t-1) (on return phi(t+nsteps-1)); S, S_prev [n] source at t and t-1
 *   (NULL: zero; S_prev NULL: equal to S). Returns 0, or -1 on bad arguments. */
int orc3_run(const orc3_problem_t* p, double* f, double* work, double* phi_prev, const double* S,
             const double* S_prev, long nsteps, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
