/*
 * FP64 CPU oracle of one B-TriRT time step on the D3Q19 lattice, in the population form of
 * Eq. (6) with push streaming (Eq. (38)) and half-way bounce-back (Eqs. (54)-(56)).
 * Reference: Zhao, Wu, Chai & Shi, arXiv:1902.09813.
 *
 * TEST INFRASTRUCTURE: see btrt3_oracle.h. Plain loops; each destination has one writer,
 * so the OpenMP loop over z-y rows gives the same bits for any thread count.
 *
 * The readings of the two-dimensional oracle carry over: dB/dt in G is the backward
 * difference over one step with phi(-1) := phi(0); the Scheme 2 source derivative uses
 * S(t-1) (S(-1) := S(0)); a link leaving through two walls takes the mean of their values.
 */
#include "btrt3_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D3Q19 velocities in the column order of C, Eq. (86). */
static const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
/* D3Q19 weights: 1/3 at rest, 1/18 along the axes, 1/36 along the face diagonals. */
static double weight(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
static const double CS2 = 1.0 / 3.0;

static int opposite(int i)
{
    for (int j = 0; j < 19; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) return j;
    return -1;
}

static void flux(const orc3_problem_t* p, double phi, double B[3])
{
    for (int a = 0; a < 3; ++a) B[a] = p->flux_a[a] * phi + p->flux_b[a] * phi * phi / 2.0;
}

void orc3_equilibrium(double phi, const double B[3], const double D[9], double feq[19])
{
    /* Eq. (7): w_i [ phi + c_i.B / c_s^2 + (D - phi I):(c_i c_i - c_s^2 I) / (2 c_s^2) ]. */
    for (int i = 0; i < 19; ++i) {
        const double c[3] = {CX[i], CY[i], CZ[i]};
        double cB = 0.0, q = 0.0;
        for (int a = 0; a < 3; ++a) cB += c[a] * B[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                q += (D[3 * a + b] - (a == b ? phi : 0.0)) * (c[a] * c[b] - (a == b ? CS2 : 0.0));
        feq[i] = weight(i) * (phi + cB / CS2 + q / (2.0 * CS2));
    }
}

/* K1 = (A / c_s^2 + I/2)^{-1} (Eq. (30)) for a 3x3 A, by the adjugate. */
static void k1_from_A(const double A[9], double K1[9])
{
    double m[9];
    for (int k = 0; k < 9; ++k) m[k] = A[k] / CS2 + ((k % 4) == 0 ? 0.5 : 0.0);
    const double c00 = m[4] * m[8] - m[5] * m[7];
    const double c01 = m[5] * m[6] - m[3] * m[8];
    const double c02 = m[3] * m[7] - m[4] * m[6];
    const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
    K1[0] = c00 / det;
    K1[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    K1[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    K1[3] = c01 / det;
    K1[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    K1[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    K1[6] = c02 / det;
    K1[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    K1[8] = (m[0] * m[4] - m[1] * m[3]) / det;
}

void orc3_collide_node(const orc3_problem_t* p, const double f[19], double phi_prev, double S, double S_prev,
                       double fpost[19])
{
    double phi = 0.0;
    for (int i = 0; i < 19; ++i) phi += f[i];
    double B[3], Bp[3];
    flux(p, phi, B);
    flux(p, phi_prev, Bp);
    const double D[9] = {phi, 0, 0, 0, phi, 0, 0, 0, phi};
    const double g = 1.0 + p->beta * phi * phi;
    const double* a = p->A0;
    const double A[9] = {a[0] * g, a[1] * g, a[2] * g, a[1] * g, a[3] * g, a[4] * g, a[2] * g, a[4] * g, a[5] * g};
    double K1[9];
    k1_from_A(A, K1);

    double feq[19], fneq[19];
    orc3_equilibrium(phi, B, D, feq);
    for (int i = 0; i < 19; ++i) fneq[i] = f[i] - feq[i];
    double M1[3] = {0, 0, 0}, M2[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j < 19; ++j) {
        const double c[3] = {CX[j], CY[j], CZ[j]};
        for (int x = 0; x < 3; ++x) {
            M1[x] += c[x] * fneq[j];
            for (int y = 0; y < 3; ++y) M2[3 * x + y] += c[x] * c[y] * fneq[j];
        }
    }
    const double k0 = p->k0;
    double r[3], gv[3], Pm[9];
    const double dB[3] = {B[0] - Bp[0], B[1] - Bp[1], B[2] - Bp[2]};
    for (int x = 0; x < 3; ++x) {
        r[x] = 0.0;
        gv[x] = 0.0;
        for (int y = 0; y < 3; ++y) {
            r[x] += (K1[3 * x + y] - (x == y ? k0 : 0.0)) * M1[y];           /* (K1 - k0 I) M1 */
            gv[x] += ((x == y ? 1.0 : 0.0) - K1[3 * x + y] / 2.0) * dB[y];  /* (I - K1/2) dB */
        }
    }
    for (int k = 0; k < 9; ++k) Pm[k] = (p->K2[k] - k0) * M2[k];            /* (K2 - k0 Ihat) o M2 */
    for (int i = 0; i < 19; ++i) {
        const double c[3] = {CX[i], CY[i], CZ[i]};
        const double w = weight(i);
        double cr = 0.0, cg = 0.0, q = 0.0;
        for (int x = 0; x < 3; ++x) {
            cr += c[x] * r[x];
            cg += c[x] * gv[x];
            for (int y = 0; y < 3; ++y) q += (c[x] * c[y] - (x == y ? CS2 : 0.0)) * Pm[3 * x + y];
        }
        const double Ri = w * cr / CS2;
        const double Pi = w * q / (2.0 * CS2 * CS2);
        const double Gi = w * cg / CS2;                 /* Eq. (11) */
        const double Si = w * S;                         /* Eq. (8) */
        const double dSi = 0.5 * (w * S - w * S_prev);   /* Scheme 2, Remark III */
        fpost[i] = f[i] - k0 * fneq[i] - Ri - Pi + Gi + Si + dSi;
    }
}

void orc3_init(const orc3_problem_t* p, const double* phi0, double* f)
{
    const long n = (long)p->nx * p->ny * p->nz;
    for (long k = 0; k < n; ++k) {
        double B[3], feq[19];
        flux(p, phi0[k], B);
        const double D[9] = {phi0[k], 0, 0, 0, phi0[k], 0, 0, 0, phi0[k]};
        orc3_equilibrium(phi0[k], B, D, feq);
        for (int i = 0; i < 19; ++i) f[i * n + k] = feq[i];
    }
}

void orc3_phi(const orc3_problem_t* p, const double* f, double* phi)
{
    const long n = (long)p->nx * p->ny * p->nz;
    for (long k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = 0; i < 19; ++i) s += f[i * n + k];
        phi[k] = s;
    }
}

static void one_step(const orc3_problem_t* p, const double* src, double* dst, double* phi_prev, const double* S,
                     const double* S_prev, int nthreads)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const long n = (long)nx * ny * nz;
    const int per[3] = {p->bc_type[0] == 0, p->bc_type[2] == 0, p->bc_type[4] == 0};
    const int dim[3] = {nx, ny, nz};
    int opp[19];
    for (int i = 0; i < 19; ++i) opp[i] = opposite(i);
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
    for (long row = 0; row < (long)ny * nz; ++row) {
        const int y = (int)(row % ny), z = (int)(row / ny);
        for (int x = 0; x < nx; ++x) {
            const long k = ((long)z * ny + y) * nx + x;
            double f[19], fp[19];
            for (int i = 0; i < 19; ++i) f[i] = src[i * n + k];
            const double s = S ? S[k] : 0.0;
            const double sp = S_prev ? S_prev[k] : s;
            orc3_collide_node(p, f, phi_prev[k], s, sp, fp);
            for (int i = 0; i < 19; ++i) {
                const int c[3] = {CX[i], CY[i], CZ[i]};
                int d[3] = {x + c[0], y + c[1], z + c[2]};
                int faces[2], nf = 0;
                for (int a = 0; a < 3; ++a) {
                    if (d[a] < 0 || d[a] >= dim[a]) {
                        if (per[a])
                            d[a] = (d[a] + dim[a]) % dim[a];
                        else
                            faces[nf++] = 2 * a + (d[a] < 0 ? 0 : 1);
                    }
                }
                if (nf == 0) {
                    dst[i * n + ((long)d[2] * ny + d[1]) * nx + d[0]] = fp[i];
                } else {
                    /* Eqs. (54)-(56): f_opp(x, t+1) = -f_i^+(x, t) + 2 w_i phi_w. */
                    double phiw = 0.0;
                    for (int q = 0; q < nf; ++q) phiw += p->bc_value[faces[q]];
                    phiw /= nf;
                    dst[opp[i] * n + k] = -fp[i] + 2.0 * weight(i) * phiw;
                }
            }
            double phi = 0.0;
            for (int i = 0; i < 19; ++i) phi += f[i];
            phi_prev[k] = phi;
        }
    }
}

int orc3_run(const orc3_problem_t* p, double* f, double* work, double* phi_prev, const double* S,
             const double* S_prev, long nsteps, int nthreads)
{
    if (!p || !f || !work || !phi_prev || p->nx < 1 || p->ny < 1 || p->nz < 1 || nsteps < 0) return -1;
    for (int a = 0; a < 3; ++a)
        if ((p->bc_type[2 * a] == 0) != (p->bc_type[2 * a + 1] == 0)) return -1;
    const long n = (long)p->nx * p->ny * p->nz;
    double* a = f;
    double* b = work;
    for (long s = 0; s < nsteps; ++s) {
        one_step(p, a, b, phi_prev, S, S_prev, nthreads);
        double* t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * 19 * (size_t)n);
    return 0;
}
