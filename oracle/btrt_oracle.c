/*
 * FP64 CPU oracle of one B-TriRT D2Q9 time step, written in the population
 * form of Eq. (6) with push streaming (Eq. (38)) and half-way bounce-back
 * (Eqs. (54)-(56)). Reference: Zhao, Wu, Chai & Shi, arXiv:1902.09813.
 *
 * TEST INFRASTRUCTURE: see btrt_oracle.h. Plain loops, no blocking, no fusion
 * beyond what the equations state; every node is independent, so the OpenMP
 * loop over rows gives the same bits for any thread count.
 *
 * Readings of points the paper leaves open (the same readings are listed with
 * the design notes of the project):
 *   - dB/dt in the correction G (Eq. (11)) is the backward difference
 *     B(phi(t)) - B(phi(t-1)); the caller seeds phi(t-1) with phi(0).
 *   - The Scheme 2 source derivative (Remark III) is (S(t) - S(t-1))/2 per
 *     population weight; the caller passes S(t-1) (NULL: time independent).
 *   - A diagonal link that leaves through a corner takes the mean of the two
 *     walls' values in the bounce-back rule.
 */
#include "btrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 velocities in the order of the columns of C, Eq. (85). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Weights, Section 3 (after Eq. (38)). */
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* Opposite directions (pairs used in Eqs. (54)-(56)). */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* c_s^2 = c^2/3 with c = 1. */
static const double CS2 = 1.0 / 3.0;

/* B(phi) = a*phi + b*phi^2/2 + c*|phi|^q (the flux families the library accepts). */
static void flux(const orc_problem_t* p, double phi, double B[2])
{
    for (int a = 0; a < 2; ++a) {
        B[a] = p->flux_a[a] * phi + p->flux_b[a] * phi * phi / 2.0;
        if (p->flux_c[a] != 0.0) B[a] += p->flux_c[a] * pow(fabs(phi), p->flux_q);
    }
}

/* The tensor D(phi) of Eq. (1), as it enters the equilibrium of Eq. (7). */
static void dterm(const orc_problem_t* p, double phi, double D[4])
{
    double d = phi;
    if (p->d_kind == 1) d = p->d_g * phi + p->d_e * pow(fabs(phi), p->d_s);
    D[0] = d;
    D[1] = 0.0;
    D[2] = 0.0;
    D[3] = d;
}

/* The phi-dependent part of S(x, phi, t) in Eq. (1): r phi (1 - |phi|^p). */
static double reaction(const orc_problem_t* p, double phi)
{
    if (p->src_r == 0.0) return 0.0;
    return p->src_r * phi * (1.0 - pow(fabs(phi), p->src_p));
}

void orc_equilibrium(double phi, const double B[2], const double D[4], double feq[9])
{
    /* Eq. (7): w_i [ phi + c_i.B / c_s^2 + (D - phi I):(c_i c_i - c_s^2 I) / (2 c_s^2) ]. */
    for (int i = 0; i < 9; ++i) {
        double c[2] = {(double)CX[i], (double)CY[i]};
        double cB = c[0] * B[0] + c[1] * B[1];
        double q = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double dm = D[2 * a + b] - (a == b ? phi : 0.0);
                double h = c[a] * c[b] - (a == b ? CS2 : 0.0);
                q += dm * h;
            }
        feq[i] = W[i] * (phi + cB / CS2 + q / (2.0 * CS2));
    }
}

/* K1 from Eq. (30): A = c_s^2 (K1^{-1} - I/2) dt, so K1 = (A / c_s^2 + I/2)^{-1}. */
static void k1_from_A(const double A[4], double K1[4])
{
    double m[4] = {A[0] / CS2 + 0.5, A[1] / CS2, A[2] / CS2, A[3] / CS2 + 0.5};
    double det = m[0] * m[3] - m[1] * m[2];
    K1[0] = m[3] / det;
    K1[1] = -m[1] / det;
    K1[2] = -m[2] / det;
    K1[3] = m[0] / det;
}

/* The collision of Eq. (6) with the diffusion tensor A0 (1 + beta phi^2) for the given A0. */
static void collide_with(const orc_problem_t* p, const double A0[3], const double f[9], double phi_prev,
                         double S, double S_prev, double fpost[9]);

void orc_collide_node(const orc_problem_t* p, const double f[9], double phi_prev,
                      double S, double S_prev, double fpost[9])
{
    collide_with(p, p->A0, f, phi_prev, S, S_prev, fpost);
}

static void collide_with(const orc_problem_t* p, const double A0[3], const double f[9], double phi_prev,
                         double S, double S_prev, double fpost[9])
{
    /* Eq. (9): phi is the zeroth moment. */
    double phi = 0.0;
    for (int i = 0; i < 9; ++i) phi += f[i];

    double B[2], Bp[2];
    flux(p, phi, B);
    flux(p, phi_prev, Bp);
    /* S(x, phi, t): the given part plus the phi-dependent one, at t and at t-1 (Scheme 2). */
    S += reaction(p, phi);
    S_prev += reaction(p, phi_prev);
    double D[4];
    dterm(p, phi, D);
    double g = 1.0 + p->beta * phi * phi;
    double A[4] = {A0[0] * g, A0[1] * g, A0[1] * g, A0[2] * g};
    double K1[4];
    k1_from_A(A, K1);

    double feq[9], fneq[9];
    orc_equilibrium(phi, B, D, feq);
    for (int i = 0; i < 9; ++i) fneq[i] = f[i] - feq[i];

    /* Non-equilibrium first and second moments (below Eq. (4) and Eq. (5)). */
    double M1[2] = {0.0, 0.0};
    double M2[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < 9; ++j) {
        double c[2] = {(double)CX[j], (double)CY[j]};
        for (int a = 0; a < 2; ++a) {
            M1[a] += c[a] * fneq[j];
            for (int b = 0; b < 2; ++b) M2[2 * a + b] += c[a] * c[b] * fneq[j];
        }
    }

    const double k0 = p->k0;
    /* (K1 - k0 I) M1 */
    double r[2];
    for (int a = 0; a < 2; ++a) {
        r[a] = 0.0;
        for (int b = 0; b < 2; ++b) r[a] += (K1[2 * a + b] - (a == b ? k0 : 0.0)) * M1[b];
    }
    /* (K2 - k0 Ihat) o M2, Ihat the all-ones matrix, o the Hadamard product. */
    double Pm[4];
    for (int ab = 0; ab < 4; ++ab) Pm[ab] = (p->K2[ab] - k0) * M2[ab];
    /* (I - K1/2) dB/dt with the backward difference over one step (Eq. (11)). */
    double dB[2] = {B[0] - Bp[0], B[1] - Bp[1]};
    double gv[2];
    for (int a = 0; a < 2; ++a) {
        gv[a] = 0.0;
        for (int b = 0; b < 2; ++b) gv[a] += ((a == b ? 1.0 : 0.0) - K1[2 * a + b] / 2.0) * dB[b];
    }

    for (int i = 0; i < 9; ++i) {
        double c[2] = {(double)CX[i], (double)CY[i]};
        double Ri = W[i] * (c[0] * r[0] + c[1] * r[1]) / CS2;
        double q = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) q += (c[a] * c[b] - (a == b ? CS2 : 0.0)) * Pm[2 * a + b];
        double Pi = W[i] * q / (2.0 * CS2 * CS2);
        double Gi = W[i] * (c[0] * gv[0] + c[1] * gv[1]) / CS2;
        double Si = W[i] * S;                          /* Eq. (8) */
        double dSi = 0.5 * (W[i] * S - W[i] * S_prev);  /* Scheme 2, Remark III */
        fpost[i] = f[i] - k0 * fneq[i] - Ri - Pi + Gi + Si + dSi;
    }
}

void orc_init(const orc_problem_t* p, const double* phi0, double* f)
{
    const long n = (long)p->nx * p->ny;
    for (long k = 0; k < n; ++k) {
        double B[2];
        flux(p, phi0[k], B);
        double D[4];
        dterm(p, phi0[k], D);
        double feq[9];
        orc_equilibrium(phi0[k], B, D, feq);
        for (int i = 0; i < 9; ++i) f[i * n + k] = feq[i];
    }
}

void orc_phi(const orc_problem_t* p, const double* f, double* phi)
{
    const long n = (long)p->nx * p->ny;
    for (long k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = 0; i < 9; ++i) s += f[i * n + k];
        phi[k] = s;
    }
}

int orc_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) return nthreads;
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* One collide + push-stream step from src into dst. */
static void one_step(const orc_problem_t* p, const double* src, double* dst, double* phi_prev,
                     const double* S, const double* S_prev, const double* wall, int nthreads)
{
    const int nx = p->nx, ny = p->ny;
    const long n = (long)nx * ny;
    const int perx = p->bc_type[0] == ORC_PERIODIC;
    const int pery = p->bc_type[2] == ORC_PERIODIC;
    (void)nthreads;

#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(orc_threads(nthreads))
#endif
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long k = (long)y * nx + x;
            double f[9], fp[9];
            for (int i = 0; i < 9; ++i) f[i] = src[i * n + k];
            double s = S ? S[k] : 0.0;
            double sp = S_prev ? S_prev[k] : s;
            collide_with(p, p->A0_field ? p->A0_field + 3 * k : p->A0, f, phi_prev[k], s, sp, fp);

            /* Eq. (38): f_i(x + c_i, t+1) = f_i^+(x, t); bounce-back at Dirichlet walls. */
            for (int i = 0; i < 9; ++i) {
                int xd = x + CX[i], yd = y + CY[i];
                int side_x = -1, side_y = -1;
                if (xd < 0) {
                    if (perx) xd += nx; else side_x = 0;
                } else if (xd >= nx) {
                    if (perx) xd -= nx; else side_x = 1;
                }
                if (yd < 0) {
                    if (pery) yd += ny; else side_y = 2;
                } else if (yd >= ny) {
                    if (pery) yd -= ny; else side_y = 3;
                }
                if (side_x < 0 && side_y < 0) {
                    dst[i * n + (long)yd * nx + xd] = fp[i];
                } else {
                    /* Eqs. (54)-(56): f_opp(x, t+1) = -f_i^+(x, t) + 2 w_i phi_w. */
                    double phiw;
                    if (wall)
                        phiw = wall[i * n + k];
                    else if (side_x >= 0 && side_y >= 0)
                        phiw = 0.5 * (p->bc_value[side_x] + p->bc_value[side_y]);
                    else
                        phiw = p->bc_value[side_x >= 0 ? side_x : side_y];
                    dst[OPP[i] * n + k] = -fp[i] + 2.0 * W[i] * phiw;
                }
            }
            /* phi at this step becomes phi(t-1) of the next one. */
            double phi = 0.0;
            for (int i = 0; i < 9; ++i) phi += f[i];
            phi_prev[k] = phi;
        }
    }
}

int orc_run(const orc_problem_t* p, double* f, double* work, double* phi_prev,
            const double* S, const double* S_prev, const double* wall, long nsteps, int nthreads)
{
    if (!p || !f || !work || !phi_prev || p->nx < 1 || p->ny < 1 || nsteps < 0) return -1;
    if ((p->bc_type[0] == ORC_PERIODIC) != (p->bc_type[1] == ORC_PERIODIC)) return -1;
    if ((p->bc_type[2] == ORC_PERIODIC) != (p->bc_type[3] == ORC_PERIODIC)) return -1;
    const long n = (long)p->nx * p->ny;
    double* a = f;
    double* b = work;
    for (long s = 0; s < nsteps; ++s) {
        one_step(p, a, b, phi_prev, S, S_prev, wall, nthreads);
        double* t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * 9 * (size_t)n);
    return 0;
}
