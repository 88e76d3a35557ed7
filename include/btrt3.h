/*
 * btrt3.h - C ABI of the three-dimensional B-TriRT lattice Boltzmann solver on the D3Q19
 * lattice (Zhao, Wu, Chai & Shi, arXiv:1902.09813, Appendix: Eqs. (80)-(81), (84), (86),
 * (89), (91), (93), (96), (100)) for MI355X (gfx950).
 *
 * The solver advances Eq. (1) in three dimensions,
 *     d_t phi + div B(phi) = div[ A(phi) grad phi ] + S(x),
 * in lattice units (dx = dt = 1, c_s^2 = 1/3) with the evolution equation Eq. (6) on D3Q19
 * (velocities in the column order of C in Eq. (86); weights 1/3, 1/18 on the axes, 1/36 on the
 * face diagonals), the equilibrium of Eq. (7) with D = phi I, the source of Eq. (8), the
 * correction G of Eq. (11), K1 = (A / c_s^2 + I/2)^-1 (Eq. (30), a 3x3 block) and a 3x3 K2
 * block whose off-diagonal rates enter as (k2_ab + k2_ba)/2 (Eq. (100)). Streaming is Eq. (38);
 * Dirichlet faces use half-way bounce-back (Eqs. (54)-(56)).
 *
 * The readings of the two-dimensional library (btrt.h) carry over: d_t B in G is the backward
 * difference over one step with phi(-1) = phi0; node (i, j, k) sits at the cell centre; a link
 * leaving through two faces (an edge of the box) bounces back with the mean of their values.
 * The slip of half-way bounce-back (Eq. (61)) holds on D3Q19 as on D2Q9, so the k2 rule of
 * Eq. (62) (BTRT_K2_HBB) applies unchanged.
 *
 * Conventions: return values are BTRT_OK or a BTRT_E_* code of btrt.h, with btrt_last_error()
 * holding a message; host arrays are x fastest: a[(k*ny + j)*nx + i] for node (i, j, k); host
 * inputs are read during the call only (copied where kept); a handle is not thread safe; work
 * is enqueued on the handle's HIP stream.
 */
#ifndef BTRT3_H
#define BTRT3_H

#include <stddef.h>
#include <stdint.h>

#include "btrt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct btrt3 btrt3_t; /* opaque; btrt3_create / btrt3_destroy */

typedef struct {
    int32_t nx, ny, nz; /* nodes per axis, each >= 1; 19 * pitch * ny * nz < 2^31 */
    int32_t precision;  /* BTRT_F64 or BTRT_F32 */
    int32_t device;     /* HIP device ordinal */
    void* stream;       /* hipStream_t to enqueue on; NULL: the library creates one */
} btrt3_grid_t;

/* B(phi) = a phi + b phi^2 / 2 per component. */
typedef struct {
    double a[3];
    double b[3];
} btrt3_flux_t;

/* A(phi) = A0 (1 + beta phi^2), A0 symmetric positive definite given as
 * (a11, a12, a13, a22, a23, a33); beta >= 0 (K1 per node when beta > 0). */
typedef struct {
    double a0[6];
    double beta;
} btrt3_diff_t;

/* S(x) of Eq. (8), time independent: none, or field[(k*ny + j)*nx + i] (copied at create). */
typedef struct {
    int32_t kind; /* BTRT_SRC_NONE or BTRT_SRC_FIELD */
    const double* field;
} btrt3_source_t;

/* Faces in the order x-, x+, y-, y+, z-, z+; a periodic face must be paired with its opposite. */
typedef struct {
    int32_t type[6];  /* BTRT_PERIODIC or BTRT_DIRICHLET */
    double value[6];  /* phi_w of a Dirichlet face */
} btrt3_bc_t;

/* k0 on the S0 block; K2 given (row major 3x3, diagonal and symmetrised off-diagonal rates in
 * (0, 2)) or from Eq. (62) (BTRT_K2_HBB: constant isotropic A, K2 = k2 Ihat). */
typedef struct {
    double k0;
    int32_t k2_rule;
    double k2[9];
    int32_t check_interval; /* steps between Eq. (64) checks in btrt3_solve (>= 1) */
} btrt3_relax_t;

typedef struct {
    int32_t nx, ny, nz, precision, pitch; /* pitch: padded row length of device planes */
    int32_t k1_per_node;
    double K1[9];                 /* Eq. (30) at phi = 0, row major */
    double K2[9];                 /* resolved K2 */
    double k0;
    size_t device_bytes;          /* device memory a handle holds */
    double bytes_per_node_launch; /* algorithmic HBM bytes per node and sweep: 19 populations and
                                     phi read and written once, plus a source field when given */
    int64_t step;                 /* steps taken (btrt3_get_info only) */
} btrt3_info_t;

/* Checks a problem and fills *info (optional) without touching a device. Errors:
 * BTRT_E_INVAL for sizes out of range, unpaired periodic faces, A0 not SPD, beta < 0, rates
 * outside (0, 2), BTRT_K2_HBB with a non-isotropic or phi-dependent A, an unknown source kind
 * or non-finite values. */
int btrt3_validate(const btrt3_grid_t* grid, const btrt3_flux_t* B, const btrt3_diff_t* K,
                   const btrt3_source_t* R, const btrt3_bc_t* bc, const btrt3_relax_t* relax, btrt3_info_t* info);

/* Creates a solver at t = 0 with f = f^eq(phi0) (phi0: nx*ny*nz host values, copied); the device
 * memory is allocated by the library. Errors: those of btrt3_validate, non-finite phi0 ->
 * BTRT_E_INVAL; BTRT_E_DEVICE; BTRT_E_NOMEM. Synchronises. */
int btrt3_create(const btrt3_grid_t* grid, const btrt3_flux_t* B, const btrt3_diff_t* K, const btrt3_source_t* R,
                 const btrt3_bc_t* bc, const btrt3_relax_t* relax, const double* phi0, btrt3_t** out);

/* Enqueues n >= 0 time steps and returns without waiting: one launch per step, or with two
 * steps per launch (btrt3_set_launch) n/2 launches of two steps and, for odd n, one of one. */
int btrt3_step(btrt3_t* h, int64_t n);

/* Launch shape of btrt3_step. Every shape gives bitwise identical results; only the speed differs.
 *   steps_per_launch  1 or 2 (0: automatic, 2 from 2^21 nodes up, else 1). With 2, a workgroup
 *                     owns an xy tile of columns plus a one-column halo ring and walks z over a
 *                     chunk of planes: step 1 of each plane goes to LDS, step 2 of the plane below
 *                     is computed from it, so the state is read and written once per two steps.
 *   z_chunk           two-step launches: output planes per workgroup (0: automatic, the chunk of
 *                     16 .. 64 planes that needs the fewest rounds of resident workgroups times
 *                     planes walked, so the launch's last round is nearly full)
 *   tile              two-step launches, threads per workgroup (output columns): 1 = 64 x 8
 *                     (62 x 6), 2 = 32 x 16 (30 x 14), 3 = 32 x 8 (30 x 6), 4 = 16 x 16 (14 x 14);
 *                     0: automatic (1) */
typedef struct {
    int32_t steps_per_launch;
    int32_t z_chunk;
    int32_t tile;
} btrt3_launch_t;

/* Sets the launch shape; fields as above. Errors: BTRT_E_INVAL (steps_per_launch outside
 * [0, 2], z_chunk < 0, tile outside [0, 4]); BTRT_E_STATE for a NULL handle. */
int btrt3_set_launch(btrt3_t* h, const btrt3_launch_t* cfg);

/* The launch shape in force, with the automatic fields resolved for this grid. */
int btrt3_get_launch(const btrt3_t* h, btrt3_launch_t* cfg);

/* phi(t) (nx*ny*nz values) into host memory; synchronises. */
int btrt3_field(btrt3_t* h, double* phi_out);

/* The post-streaming populations f_i(t), 19 * nx*ny*nz values, i slowest; synchronises. */
int btrt3_populations(btrt3_t* h, double* f_out);

/* Eq. (64) residual against the previous check (the first against phi0), FP64 reduction;
 * BTRT_E_UNSTABLE (out = NaN) when phi holds NaN/Inf. Synchronises. */
int btrt3_residual(btrt3_t* h, double* out);

/* Against a host reference (nx*ny*nz): out = (GRE of Eq. (63), max |phi - ref|, relative L2).
 * Synchronises. */
int btrt3_error(btrt3_t* h, const double* ref, double out[3]);

/* Steps in chunks of check_interval until the residual is <= tol or max_steps are taken. */
int btrt3_solve(btrt3_t* h, double tol, int64_t max_steps, int64_t* steps_taken, double* residual);

int btrt3_sync(btrt3_t* h);
int btrt3_get_info(const btrt3_t* h, btrt3_info_t* info);
int btrt3_destroy(btrt3_t* h);

#ifdef __cplusplus
}
#endif
#endif
