/*
 * Test driver that runs the CPU oracle (oracle/btrt_oracle.c, oracle/btrt3_oracle.c) on small
 * problems, built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitizers.py: walls, sources, per-link wall values, a space-dependent
 * tensor, the power-law flux, the phi-dependent source, a general D, and the D3Q19 step.
 * Exits 0 when every run returns 0 and keeps phi finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "btrt3_oracle.h"
#include "btrt_oracle.h"

static int finite_all(const double* v, long n)
{
    for (long k = 0; k < n; ++k)
        if (!isfinite(v[k])) return 0;
    return 1;
}

static int run2(int nx, int ny, int walls, int general)
{
    orc_problem_t p;
    memset(&p, 0, sizeof(p));
    p.nx = nx;
    p.ny = ny;
    p.flux_a[0] = 0.03;
    p.flux_a[1] = -0.02;
    p.flux_b[0] = 0.02;
    p.A0[0] = 0.04;
    p.A0[1] = 0.005;
    p.A0[2] = 0.03;
    p.beta = 0.5;
    p.k0 = 1.0;
    for (int q = 0; q < 4; ++q) p.K2[q] = 1.1;
    for (int s = 0; s < 4; ++s) {
        p.bc_type[s] = walls ? ORC_DIRICHLET : ORC_PERIODIC;
        p.bc_value[s] = 0.1 * (s + 1);
    }
    const long n = (long)nx * ny;
    double* field = NULL;
    if (general) {
        p.flux_c[0] = 0.05;
        p.flux_q = 2.5;
        p.src_r = 0.01;
        p.src_p = 1.5;
        p.d_kind = 1;
        p.d_g = 1.0;
        p.d_e = 0.1;
        p.d_s = 3.0;
        field = malloc(sizeof(double) * 3 * n);
        for (long k = 0; k < n; ++k) {
            field[3 * k] = 0.04 + 0.01 * (k % 3);
            field[3 * k + 1] = 0.002;
            field[3 * k + 2] = 0.03;
        }
        p.A0_field = field;
    }
    double* phi0 = malloc(sizeof(double) * n);
    double* f = malloc(sizeof(double) * 9 * n);
    double* work = malloc(sizeof(double) * 9 * n);
    double* phi_prev = malloc(sizeof(double) * n);
    double* S = malloc(sizeof(double) * n);
    double* wall = malloc(sizeof(double) * 9 * n);
    for (long k = 0; k < n; ++k) {
        phi0[k] = 0.3 + 0.4 * sin(0.7 * k);
        phi_prev[k] = phi0[k];
        S[k] = 1e-3 * cos(0.3 * k);
    }
    for (long k = 0; k < 9 * n; ++k) wall[k] = 0.2 + 0.01 * (k % 7);
    orc_init(&p, phi0, f);
    int rc = orc_run(&p, f, work, phi_prev, S, NULL, general ? wall : NULL, 7, 2);
    double* phi = malloc(sizeof(double) * n);
    orc_phi(&p, f, phi);
    const int ok = rc == 0 && finite_all(phi, n);
    free(phi0), free(f), free(work), free(phi_prev), free(S), free(wall), free(phi), free(field);
    return ok;
}

static int run3(int nx, int ny, int nz, int walls)
{
    orc3_problem_t p;
    memset(&p, 0, sizeof(p));
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.flux_a[0] = 0.02;
    p.flux_a[2] = -0.01;
    p.flux_b[1] = 0.03;
    p.A0[0] = 0.05;
    p.A0[1] = 0.01;
    p.A0[3] = 0.04;
    p.A0[5] = 0.03;
    p.beta = 0.5;
    p.k0 = 0.9;
    for (int q = 0; q < 9; ++q) p.K2[q] = 1.1;
    for (int s = 0; s < 6; ++s) {
        p.bc_type[s] = walls ? 1 : 0;
        p.bc_value[s] = 0.1 * (s + 1);
    }
    const long n = (long)nx * ny * nz;
    double* phi0 = malloc(sizeof(double) * n);
    double* f = malloc(sizeof(double) * 19 * n);
    double* work = malloc(sizeof(double) * 19 * n);
    double* phi_prev = malloc(sizeof(double) * n);
    double* S = malloc(sizeof(double) * n);
    for (long k = 0; k < n; ++k) {
        phi0[k] = 0.4 + 0.3 * cos(0.5 * k);
        phi_prev[k] = phi0[k];
        S[k] = 1e-3;
    }
    orc3_init(&p, phi0, f);
    const int rc = orc3_run(&p, f, work, phi_prev, S, NULL, 5, 2);
    double* phi = malloc(sizeof(double) * n);
    orc3_phi(&p, f, phi);
    const int ok = rc == 0 && finite_all(phi, n);
    free(phi0), free(f), free(work), free(phi_prev), free(S), free(phi);
    return ok;
}

int main(void)
{
    int ok = 1;
    const int sizes[][2] = {{1, 1}, {1, 7}, {9, 1}, {13, 11}, {64, 5}};
    for (int s = 0; s < 5; ++s)
        for (int walls = 0; walls < 2; ++walls)
            for (int general = 0; general < 2; ++general) ok &= run2(sizes[s][0], sizes[s][1], walls, general);
    const int sizes3[][3] = {{1, 1, 1}, {5, 4, 3}, {1, 6, 2}, {9, 1, 4}};
    for (int s = 0; s < 4; ++s)
        for (int walls = 0; walls < 2; ++walls) ok &= run3(sizes3[s][0], sizes3[s][1], sizes3[s][2], walls);
    printf(ok ? "oracle runs clean\n" : "oracle run failed\n");
    return ok ? 0 : 1;
}
