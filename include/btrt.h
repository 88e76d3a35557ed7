/*
 * btrt.h - C ABI of the MI355X (gfx950) library for the block triple-relaxation-time
 * (B-TriRT) lattice Boltzmann method on the D2Q9 lattice, for nonlinear anisotropic
 * convection-diffusion equations (Zhao, Wu, Chai & Shi, arXiv:1902.09813).
 *
 * The library solves Eq. (1),
 *     d_t phi + div B(phi) = div[ A(x, phi) grad . D(phi) ] + S(x, phi, t),
 * in lattice units (dx = dt = 1, c = 1, c_s^2 = 1/3), with the evolution equation
 * Eq. (6) (equivalently its moment form, Eq. (94) with the block relaxation matrix of
 * Eq. (99)), the equilibrium of Eq. (7), the source of Eq. (8), the correction G of
 * Eq. (11), streaming as in Eq. (38) and half-way bounce-back for Dirichlet sides
 * (Eqs. (54)-(56)). K1 follows from A through Eq. (30); k2 may follow the bounce-back
 * rule of Eq. (62).
 *
 * Discretisation choices where the paper leaves the detail open:
 *   - d_t B in G is the backward difference B(phi(t)) - B(phi(t-1)); at the first step
 *     phi(t-1) is phi0, so G starts at zero.
 *   - A source that changes in time or with phi enters through Scheme 2 (Remark III):
 *     S(t) + (S(t) - S(t-1))/2, with S(t-1) taken at phi(t-1) and S(-1) = S(0).
 *   - A diagonal link leaving through a corner point bounces back with the mean of the
 *     two walls' values.
 *   - Node x = (i, j) sits at the cell centre (i + 1/2, j + 1/2); walls lie at 0 and nx
 *     (resp. ny), as in y_n = (n - 1/2)/N below Eq. (49).
 *
 * Conventions for every call:
 *   - Return value: BTRT_OK (0) or one of the BTRT_E_* codes below; btrt_last_error()
 *     then holds a one-line message for the calling thread.
 *   - Host arrays are row major, x fastest: a[j*nx + i] for node (i, j).
 *   - All host pointers passed in are only read during the call (copied where kept);
 *     output buffers are owned by the caller.
 *   - A handle is not thread safe; distinct handles are independent. Work is enqueued on
 *     the handle's HIP stream; calls documented as synchronising wait for that stream.
 */
#ifndef BTRT_H
#define BTRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------------------ */
#define BTRT_OK 0
#define BTRT_E_INVAL 1    /* invalid argument; nothing was allocated or launched */
#define BTRT_E_NOMEM 2    /* device allocation failed or workspace too small */
#define BTRT_E_DEVICE 3   /* no usable HIP device, or a HIP call failed */
#define BTRT_E_UNSTABLE 4 /* a reduction saw NaN/Inf in phi; the handle stays usable */
#define BTRT_E_STATE 5    /* NULL handle */

/* ---- enumerations ------------------------------------------------------------------ */
#define BTRT_F64 0     /* populations stored and collided in FP64 */
#define BTRT_F32 1     /* populations stored and collided in FP32 (reductions stay FP64) */
#define BTRT_F16DEV 2  /* populations stored as FP16 scaled deviations from equilibrium,
                          h = q(s (f+ - f_eq(phi))) with phi in FP32 and a power-of-two s set
                          at create from max|phi0|; FP32 collision; single handles only */
#define BTRT_BF16DEV 3 /* the same with BF16 deviations */

#define BTRT_PERIODIC 0
#define BTRT_DIRICHLET 1 /* half-way bounce-back, Eqs. (54)-(56) */

#define BTRT_SRC_NONE 0
#define BTRT_SRC_FIELD 1 /* S(x) given per node */
#define BTRT_SRC_SIN 2   /* S = amp sin(kx pi x / nx) sin(ky pi y / ny) at cell centres */

#define BTRT_D_PHI_I 0   /* D(phi) = phi I */
#define BTRT_D_POLY 1    /* D(phi) = (g phi + e |phi|^s) I */

#define BTRT_K2_VALUE 0  /* K2 given explicitly (relax.k2) */
#define BTRT_K2_HBB 1    /* k2 = 8(k1-2)/(3(k1-4)), Eq. (62); needs A = alpha I constant */

/* ---- problem description ----------------------------------------------------------- */
typedef struct btrt btrt_t; /* opaque; created by btrt_create, released by btrt_destroy */

typedef struct {
    int32_t nx, ny;         /* nodes along x and y, each >= 1; nx*ny <= 2^31 - 1 */
    int32_t precision;      /* BTRT_F64, BTRT_F32, BTRT_F16DEV or BTRT_BF16DEV */
    int32_t device;         /* HIP device ordinal */
    void* stream;           /* hipStream_t to enqueue on; NULL: the library creates one */
    void* workspace;        /* device memory owned by the caller, >= btrt_workspace_size();
                               NULL: the library allocates and frees its own */
    size_t workspace_bytes; /* size of workspace in bytes (ignored when workspace is NULL) */
} btrt_grid_t;

/* B(phi) = a*phi + b*phi^2/2 + c*|phi|^q, per component (Eq. (1)). Linear convection with
 * velocity u is a = u, b = 0; the Burgers flux (phi^2/2)*c is a = 0, b = c; the convection
 * a phi^delta d_x phi of the Burgers-Fisher equation (Eq. (67)) is c = (a/(delta+1), 0),
 * q = delta + 1. q is read only when c != 0 and must then be >= 1. A nonzero c selects the
 * general node model (BTRT_F64 or BTRT_F32 storage, single handles only). */
typedef struct {
    double a[2];
    double b[2];
    double c[2];
    double q;
} btrt_flux_t;

/* A(x, phi) = A0 * (1 + beta*phi^2) (Eq. (1)) with A0 = [[k11, k12], [k12, k22]], or, when
 * field is not NULL, a space-dependent A0(x) (Eq. (73), Eq. (74)): field[3*(j*nx + i) + q] holds
 * (a11, a12, a22) of node (i, j), copied at create (k11, k12, k22 are then ignored). Every A0
 * symmetric positive definite, beta >= 0. K1 (Eq. (30)) is computed per node when beta > 0 or a
 * field is given. */
typedef struct {
    double k11, k12, k22;
    double beta;
    const double* field;
} btrt_diff_t;

/* D(phi) of Eq. (1), through the equilibrium of Eq. (7) (whose second moment is c_s^2 D, Eq. (9)):
 * phi I, or (g phi + e |phi|^s) I. s is read only when e != 0 and must then be >= 1. The
 * equilibrium rest population is w_0 (2 phi - d), so the scheme needs d(phi) < 2 phi where phi > 0.
 * BTRT_D_POLY selects the general node model (BTRT_F64 or BTRT_F32 storage, single handles only). */
typedef struct {
    int32_t kind; /* BTRT_D_PHI_I or BTRT_D_POLY */
    double g, e, s;
} btrt_dterm_t;

/* Source S of Eq. (8): S(x, phi, t) = exp(growth * t) * S0(x) + r*phi*(1 - |phi|^p) at step t
 * (t = 0, 1, ...), with S0 = 0 (NONE), field[j*nx + i] (FIELD, copied at create) or
 * amp*sin(kx pi (i+1/2)/nx)*sin(ky pi (j+1/2)/ny) (SIN). The phi-dependent part is the reaction
 * of the Burgers-Fisher equation (Eq. (67), r = b dt, p = delta) and is evaluated at the node's
 * phi(t). A source that changes in time or with phi enters with the Scheme 2 correction of
 * Remark III, S(t) + (S(t) - S(t-1))/2, with S(t-1) at phi(t-1) and S(-1) = S(0).
 * growth = 0: S0 time independent. p is read only when r != 0 and must then be > 0; a nonzero
 * r selects the general node model (BTRT_F64 or BTRT_F32 storage, single handles only). */
typedef struct {
    int32_t kind; /* BTRT_SRC_NONE, BTRT_SRC_FIELD or BTRT_SRC_SIN */
    double amp;
    int32_t kx, ky;
    const double* field;
    double growth;
    double r;
    double p;
} btrt_source_t;

/* Sides in the order x-, x+, y-, y+. A periodic side must be paired with its opposite. */
typedef struct {
    int32_t type[4];  /* BTRT_PERIODIC or BTRT_DIRICHLET */
    double value[4];  /* phi_w of a Dirichlet side */
} btrt_bc_t;

/* Relaxation blocks of Eq. (99): k0 on the S0 block; K2 (row major [[k2_11, k2_12],
 * [k2_21, k2_22]]) on the second-order block (pxy relaxes with (k2_12 + k2_21)/2);
 * K1 always from A through Eq. (30). */
typedef struct {
    double k0;              /* in (0, 2) */
    int32_t k2_rule;        /* BTRT_K2_VALUE or BTRT_K2_HBB */
    double k2[4];           /* used with BTRT_K2_VALUE; k2_11, k2_22, (k2_12+k2_21)/2 in (0, 2) */
    int32_t check_interval; /* steps between Eq. (64) checks in btrt_solve (>= 1) */
} btrt_relax_t;

/* Derived constants and sizes of a problem (host-side, no device work). */
typedef struct {
    int32_t nx, ny, precision, pitch; /* pitch: padded row length of device planes, elements */
    int32_t k1_per_node;              /* 1 when K1 depends on phi (beta != 0) */
    double K1[4];                     /* Eq. (30) at A(phi = 0), row major */
    double K2[4];                     /* resolved K2 */
    double k0;
    size_t workspace_bytes;           /* device bytes a handle needs */
    double bytes_per_node_launch;     /* algorithmic HBM bytes per node and sweep launch: the
                                         state read once and written once (9 populations +
                                         phi each way) plus a source field and an A0 field when
                                         given, however many steps the launch fuses */
    int64_t step;                     /* steps taken (btrt_get_info only) */
} btrt_info_t;

/* ---- calls --------------------------------------------------------------------------- */

/* Checks a problem and fills *info (optional) without touching any device.
 * Errors: BTRT_E_INVAL for sizes out of range, unpaired periodic sides, A (or any node of an
 * A0 field) not SPD or beta < 0, rates outside (0, 2), a power-law exponent q < 1 or a
 * reaction exponent p <= 0 where used, a D exponent s < 1 where used, the general node model
 * (a power-law flux, a phi-dependent source or BTRT_D_POLY) with BTRT_F16DEV or
 * BTRT_BF16DEV, BTRT_K2_HBB with a non-isotropic,
 * phi-dependent or space-dependent A, an unsupported D or source kind, or non-finite values. */
int btrt_validate(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K,
                  const btrt_dterm_t* D, const btrt_source_t* R, const btrt_bc_t* bc,
                  const btrt_relax_t* relax, btrt_info_t* info);

/* Device bytes btrt_create needs for this grid, diffusion tensor and source (K and R may be
 * NULL: constant tensor, no source); 0 when the grid is invalid. */
size_t btrt_workspace_size(const btrt_grid_t* grid, const btrt_diff_t* K, const btrt_source_t* R);

/* Creates a solver at t = 0 with f = f^eq(phi0) (Section 4: populations start at
 * equilibrium). phi0: nx*ny host values, copied. On success *out owns the device state.
 * Errors: those of btrt_validate; non-finite phi0 -> BTRT_E_INVAL; BTRT_E_DEVICE;
 * BTRT_E_NOMEM. Synchronises. */
int btrt_create(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K,
                const btrt_dterm_t* D, const btrt_source_t* R, const btrt_bc_t* bc,
                const btrt_relax_t* relax, const double* phi0, btrt_t** out);

/* Enqueues n >= 0 time steps (collide, stream, bounce back) on the handle's stream and
 * returns without waiting. With a wall schedule (btrt_set_walls) the steps must lie inside it:
 * BTRT_E_INVAL, with nothing enqueued, otherwise. */
int btrt_step(btrt_t* h, int64_t n);

/* Dirichlet values that change along the walls and in time (Eqs. (54)-(56) with phi_w(x, t),
 * as the Burgers-Fisher problem of Eqs. (67)-(69) needs) for the next `steps` >= 1 steps.
 * values[k*P + q], P = 4*(nx + ny) + 4: for the k-th step from now (k = 0 .. steps-1), the values
 * phi_w of the populations that the bounce-back returns into the grid at the end of that step
 * (time t + k + 1), sampled along each side every half lattice spacing from corner to corner:
 * x- at y = s/2 (q = s, s = 0 .. 2 ny), x+ at y = s/2 (q = 2 ny + 1 + s), y- at x = s/2
 * (q = 4 ny + 2 + s, s = 0 .. 2 nx) and y+ at x = s/2 (q = 4 ny + 2 nx + 3 + s), in lattice
 * units with the walls at 0 and nx (0 and ny); entries of periodic sides are ignored. Half-way
 * bounce-back puts the wall half a spacing beyond the last node, so the link from node (i, j)
 * along c meets it at (i + 1/2 + c_x/2, j + 1/2 + c_y/2): through an x side it takes sample
 * 2j + 1 + c_y, through a y side sample 2i + 1 + c_x, and a diagonal link through a corner point
 * the mean of the two sides' samples there. The values are copied (host memory, read during the
 * call); the handle allocates device memory for them ((P + 4) * (steps + 1) values, the corner
 * means included; freed by the next call or btrt_destroy).
 * Once set, btrt_step, btrt_solve and btrt_tune may advance at most `steps` steps past the
 * step count of this call; a new call continues from the current step. Selects the general
 * node model from the next step on. Errors: BTRT_E_INVAL for NULL values, steps < 1,
 * non-finite values, or a BTRT_F16DEV / BTRT_BF16DEV handle; BTRT_E_NOMEM; BTRT_E_DEVICE.
 * Synchronises. */
int btrt_set_walls(btrt_t* h, const double* values, int64_t steps);

/* Shape of the sweep launches btrt_step makes. Every shape gives bitwise identical results;
 * only the speed differs. Zero fields are chosen by the library for the grid.
 *   steps_per_launch  1 .. 7 time steps per launch (0: with FP64/FP32 storage and the standard
 *                     node model from 2^22 nodes up 7, or 6 for FP64 with a Dirichlet wall,
 *                     and for FP32 with a wall 7 from 2^24 nodes up; else 4 from 2^20 nodes
 *                     up, else 1). With
 *                     k >= 2 each wavefront walks a strip of 66 - 2k columns down the grid and
 *                     keeps the k - 1 intermediate time levels in registers, so the state is
 *                     read and written once per k steps. Step counts that are not a multiple of
 *                     k end with one shorter launch.
 *   strip_rows        rows per strip of the walkers (0: automatic, 8 .. 32 by grid size, up to
 *                     64 from six steps per launch on; FP64 walkers from six steps on, which
 *                     hold one wavefront per SIMD, take the height that fits every strip in
 *                     the resident slots at once when that is 64 rows or more);
 *                     with one step per launch, the tile height 1, 2, 4, 8 or 16 (0: 4)
 *   strips_per_group  1 or 4 strips per workgroup, walked side by side in lockstep (0: auto)
 *   tile              1 with steps_per_launch 2: the two-step LDS tile kernel instead of a
 *                     strip walker (tiles of 64 x 8 nodes in FP64, 64 x 16 otherwise) */
typedef struct {
    int32_t steps_per_launch;
    int32_t strip_rows;
    int32_t strips_per_group;
    int32_t tile;
} btrt_launch_t;

/* Sets the launch shape; fields as above. Errors: BTRT_E_INVAL (steps outside [0, 7],
 * strip_rows < 0 or, with one step per launch, not 0, 1, 2, 4, 8 or 16, strips_per_group not
 * 0, 1 or 4, tile without steps_per_launch 2). */
int btrt_set_launch(btrt_t* h, const btrt_launch_t* cfg);

/* The launch shape in force, with the automatic fields resolved for this grid. */
int btrt_get_launch(btrt_t* h, btrt_launch_t* cfg);

/* Shorthand for btrt_set_launch({steps_per_launch, 0, 0, 0}); steps_per_launch in [1, 7]
 * (BTRT_E_INVAL otherwise). */
int btrt_set_fusion(btrt_t* h, int32_t steps_per_launch);

/* Times candidate launch shapes on the handle's own state and keeps the fastest (per step):
 * the automatic shape, one step per launch (tiles of 4, 8, 16 rows), the LDS tile, strip walkers
 * over 2 .. 7 steps x 8, 16, 32, 64, 128 rows x 1, 4 strips per group, and the automatic strip
 * rows of six and seven steps, each for one untimed and one timed launch after a few warm-up
 * launches of the automatic shape (at most max_steps / 10 steps); then the four fastest and the
 * automatic shape again, in turn, twice over, one untimed and two timed launches each (the first
 * pass may run while the GPU clocks still rise); as far as max_steps allows. The state advances by *steps_used steps (the same
 * bits btrt_step would give); the Eq. (64) snapshot is not touched. Synchronises. best (may be
 * NULL) receives the shape kept, resolved. */
int btrt_tune(btrt_t* h, int64_t max_steps, btrt_launch_t* best, int64_t* steps_used);

/* phi(t) = sum_i f_i(x, t) (Eq. (9)) into phi_out[nx*ny]. Synchronises. */
int btrt_field(btrt_t* h, double* phi_out);

/* Post-streaming populations f_i(x, t) into f_out[9*nx*ny] as f_out[i*nx*ny + j*nx + x],
 * i in the velocity order of Eq. (85). Synchronises. */
int btrt_populations(btrt_t* h, double* f_out);

/* Eq. (64): sum|phi(t) - phi_snap| / sum|phi(t)| in FP64, where phi_snap is phi at the
 * previous btrt_residual call (phi0 for the first); then phi_snap := phi(t).
 * Synchronises. BTRT_E_UNSTABLE (with *out = NaN) if phi holds NaN/Inf. */
int btrt_residual(btrt_t* h, double* out);

/* Against a reference field ref[nx*ny]: out[0] = GRE of Eq. (63), out[1] = max |phi - ref|,
 * out[2] = sqrt(sum (phi - ref)^2 / sum ref^2). FP64. Synchronises. */
int btrt_error(btrt_t* h, const double* ref, double out[3]);

/* Runs check_interval steps at a time until the Eq. (64) residual is <= tol or max_steps
 * steps have been taken. Reports the steps taken and the last residual. Synchronises. */
int btrt_solve(btrt_t* h, double tol, int64_t max_steps, int64_t* steps_taken, double* residual);

/* Bytes of the fixed device array btrt_solve_static works in (16 MiB): a 256 x 256 grid fits in
 * any storage format, larger ones in the narrower formats (btrt_workspace_size() gives the need). */
#define BTRT_STATIC_BYTES (16u << 20)

/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): btrt_create + btrt_solve + btrt_field + btrt_destroy in one call, allocating
 * nothing. Every device buffer of the solve (the populations, phi planes, the Eq. (64) snapshot,
 * staging and reduction partials: a handle's workspace) lives in a fixed array of
 * BTRT_STATIC_BYTES bytes that the library holds on each device it runs on until the process
 * ends. Arguments are those of btrt_create (grid->workspace must be NULL; grid->stream NULL runs
 * on the device's null stream, none is created), then those of btrt_solve: tol and max_steps,
 * the steps taken and the last Eq. (64) residual (either may be NULL). phi_out receives phi at
 * the end (nx*ny, caller-owned host memory), also after BTRT_E_UNSTABLE. The results are those
 * of btrt_create, btrt_solve and btrt_field on the same arguments with the automatic launch
 * shape, bit for bit. Calls on one device share the array: within a process they run one at a
 * time (a lock per device); each call starts from its own inputs and leaves nothing running on
 * the array when it returns. Errors: those of btrt_create and btrt_solve; BTRT_E_INVAL also for a
 * workspace, a NULL phi_out, or a grid whose workspace would exceed BTRT_STATIC_BYTES (use
 * btrt_create). Synchronises. */
int btrt_solve_static(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K, const btrt_dterm_t* D,
                      const btrt_source_t* R, const btrt_bc_t* bc, const btrt_relax_t* relax, const double* phi0,
                      double tol, int64_t max_steps, double* phi_out, int64_t* steps_taken, double* residual);

/* Waits for all work enqueued on the handle's stream. */
int btrt_sync(btrt_t* h);

/* Derived constants plus the number of steps taken. */
int btrt_get_info(const btrt_t* h, btrt_info_t* info);

/* ---- checkpoint and resume -------------------------------------------------------------
 * A checkpoint holds the solver state between steps: the step count, the stored populations
 * f+(t-1) and phi(t-1) in the handle's storage format, the Eq. (64) residual snapshot, the
 * Dirichlet values the next pull reads, and a copy of the problem's derived constants. It is
 * plain host memory, laid out by the library (a header, then the arrays), valid on any handle
 * of the same library build. Per-node inputs (a source field, an A0 field) are not stored: the
 * handle a checkpoint is restored into must be created with the same problem. */

/* Bytes a checkpoint of h takes. */
int btrt_checkpoint_size(const btrt_t* h, size_t* bytes);

/* Writes the state of h into buf (host memory owned by the caller, at least
 * btrt_checkpoint_size bytes). Waits for the handle's stream. Errors: BTRT_E_INVAL for a NULL or
 * short buffer; BTRT_E_DEVICE. */
int btrt_checkpoint(btrt_t* h, void* buf, size_t bytes);

/* Loads a checkpoint into h, which must have been created with the same problem: grid,
 * precision and every derived constant (K1, K2, k0, flux, diffusion, source, walls, storage
 * scale) must match, else BTRT_E_INVAL with nothing changed. The handle continues from the
 * checkpoint's step with the bits the original handle would have produced (its own launch shape
 * is kept; every shape gives the same bits). A checkpoint taken under a wall schedule restores
 * the values in force; btrt_set_walls must then give the values of the following steps before
 * the handle steps again. Synchronises. */
int btrt_restore(btrt_t* h, const void* buf, size_t bytes);

/* Frees the handle and the device memory the library allocated. Synchronises. */
int btrt_destroy(btrt_t* h);

/* Static text for an error code. */
const char* btrt_strerror(int code);

/* Message of the calling thread's last failed call ("" if none). */
const char* btrt_last_error(void);

/* ---- many instances in one launch ----------------------------------------------------- */
/* A batch holds independent problems of different sizes, boundaries and coefficients and
 * advances all of them together: each sweep launch walks the tiles of every instance, so
 * one launch (not one per instance) serves the whole batch. Results are bitwise identical to
 * solving each instance alone with btrt_create/btrt_step. */

typedef struct btrt_batch btrt_batch_t; /* opaque; btrt_batch_create / btrt_batch_destroy */

/* One instance: the arguments of btrt_create, by value. grid.precision must be the same for
 * every instance of a batch; grid.device, grid.stream and grid.workspace are ignored (the
 * batch's own apply). phi0 (nx*ny) is copied at create. */
typedef struct {
    btrt_grid_t grid;
    btrt_flux_t B;
    btrt_diff_t K;
    btrt_dterm_t D;
    btrt_source_t R;
    btrt_bc_t bc;
    btrt_relax_t relax;
    const double* phi0;
} btrt_problem_t;

/* How a batch launches: time steps fused per launch (1: 64 x 4 tiles; 2: the two-step LDS
 * tiles; 4, 6 or 7 = k: strip walkers, one wavefront per strip of 66 - 2k columns by strip_rows
 * rows), resident blocks per compute unit of the persistent grid (0: one block per tile or
 * strip; with a walker four one-wavefront blocks per unit), launches captured per HIP graph replay (0: no graph;
 * otherwise even, >= 2), and the walkers' strip height (0: 16; at most 4096). Every
 * configuration gives the same bits. */
typedef struct {
    int32_t steps_per_launch;
    int32_t blocks_per_cu;
    int32_t graph_launches;
    int32_t strip_rows;
} btrt_batch_config_t;

/* Creates a batch of n >= 1 instances at t = 0 on `device`, enqueuing on `stream` (NULL: the
 * library creates one). Device memory is allocated by the library (the sum of the instances'
 * btrt_workspace_size plus small tables). Errors: any instance failing btrt_validate or
 * holding a non-finite phi0 -> BTRT_E_INVAL (btrt_last_error names the instance); mixed
 * precisions, an A0 field, a growing source or the general node model (a power-law flux or a
 * phi-dependent source) -> BTRT_E_INVAL; BTRT_E_DEVICE; BTRT_E_NOMEM.
 * Synchronises. */
int btrt_batch_create(int32_t n, const btrt_problem_t* problems, int32_t device, void* stream,
                      btrt_batch_t** out);

/* Enqueues n >= 0 time steps for every instance; returns without waiting. */
int btrt_batch_step(btrt_batch_t* b, int64_t n);

/* phi(t) of instance i into phi_out[nx_i*ny_i]. Synchronises. */
int btrt_batch_field(btrt_batch_t* b, int32_t i, double* phi_out);

/* Eq. (64) residual of every instance since its previous check into out[n] (phi0 for the
 * first). Synchronises. BTRT_E_UNSTABLE if any instance holds NaN/Inf (its entry is NaN). */
int btrt_batch_residual(btrt_batch_t* b, double* out);

/* Sets / reads the launch configuration (defaults: 2 steps per launch, one block per tile,
 * no graph). Errors: BTRT_E_INVAL for values outside the ranges above. */
int btrt_batch_set_config(btrt_batch_t* b, const btrt_batch_config_t* cfg);
int btrt_batch_get_config(const btrt_batch_t* b, btrt_batch_config_t* cfg);

/* Autotuner: times each candidate configuration on the batch itself by running steps of the
 * solve (every configuration computes the same bits, so these steps count as ordinary
 * steps), at most max_steps in total; keeps and reports the fastest per step. Candidates
 * (11): walkers of 4, 6 and 7 steps with 16- and 32-row strips and 16-launch graphs; 4-step
 * walkers with 32-row strips without graphs and with 4 blocks per CU; 2 steps with and without
 * graphs; 1 step with graphs. After a warm-up of the configuration in force (at most
 * max_steps / 10 steps), each candidate takes k or 2 k untimed steps (k steps per launch; the
 * timed run starts at the launch parity a graph replay starts from) and 16 k timed ones, as far
 * as three quarters of max_steps allow; then the three fastest run again in
 * turn, twice over, within the rest, and the lowest mean wins (the first pass may run while
 * the GPU clocks still rise). *steps_used = steps taken. Synchronises. */
int btrt_batch_tune(btrt_batch_t* b, int64_t max_steps, btrt_batch_config_t* best, int64_t* steps_used);

/* Steps taken so far. */
int btrt_batch_steps(const btrt_batch_t* b, int64_t* steps);

/* Waits for the batch's stream. */
int btrt_batch_sync(btrt_batch_t* b);

/* Frees the batch. Synchronises. */
int btrt_batch_destroy(btrt_batch_t* b);

/* ---- solve server (continuous batching) ------------------------------------------------ */
/* Requests (one problem each, solved to a residual tolerance or a step cap) arrive at any
 * time. Each btrt_server_pump call is one scheduling round: it admits queued requests in
 * arrival order while their device footprint fits in the server's memory and a slot is free
 * (a request that does not fit lets later, smaller ones pass), advances every resident request
 * by check_interval steps with batched launches (their work shares each launch), evaluates the
 * Eq. (64) residual of each, and retires those at tolerance, at their step cap, or unstable,
 * keeping their phi on the host until collected. A request takes whole rounds, so its result
 * is bitwise the same whether it runs alone or among others. Not thread safe. */

typedef struct btrt_server btrt_server_t; /* opaque; btrt_server_create / btrt_server_destroy */

#define BTRT_REQ_QUEUED 0
#define BTRT_REQ_RUNNING 1
#define BTRT_REQ_DONE 2   /* converged (residual <= tol) or reached its step cap */
#define BTRT_REQ_FAILED 3 /* NaN/Inf seen (error = BTRT_E_UNSTABLE) */

typedef struct {
    int32_t precision;          /* BTRT_F64 or BTRT_F32, for every request */
    int32_t device;
    void* stream;               /* hipStream_t; NULL: the server creates one */
    size_t memory_bytes;        /* device memory reserved for resident requests */
    int32_t max_active;         /* resident requests at most (>= 1) */
    int32_t check_interval;     /* steps per round; the residual is checked after each round */
    btrt_batch_config_t launch; /* launch configuration of the batched sweeps; steps_per_launch
                                   0: chosen per round (two-step tiles below 2^21 resident nodes,
                                   four-step walkers with 16-row strips from there on), and a
                                   request of 2^20 nodes or more, which fills the GPU alone, then
                                   advances by launches of its own in the automatic single-grid
                                   shape of btrt_step (the same bits) */
} btrt_server_opts_t;

typedef struct {
    int32_t status;  /* BTRT_REQ_* */
    int32_t error;   /* BTRT_OK, or the failure code */
    int32_t nx, ny;
    int64_t steps;   /* steps taken */
    double residual; /* last Eq. (64) residual (NaN before the first check) */
    double t_submit, t_admit, t_done; /* seconds on the server clock (-1: not yet) */
} btrt_request_info_t;

typedef struct {
    int64_t submitted, admitted, completed, failed;
    int32_t active, queued;
    int64_t node_updates;   /* node updates executed for all requests */
    double busy_seconds;    /* wall time spent inside btrt_server_pump */
    size_t memory_in_use, memory_high_water;
} btrt_server_stats_t;

/* Creates a server and reserves opts->memory_bytes of device memory. Errors: BTRT_E_INVAL
 * (bad options), BTRT_E_DEVICE, BTRT_E_NOMEM. */
int btrt_server_create(const btrt_server_opts_t* opts, btrt_server_t** out);

/* Queues one request: solve p until the residual is <= tol or max_steps steps (rounded up to
 * whole rounds). p's host arrays are copied. *id receives the request id. Errors: those of
 * btrt_validate, non-finite phi0, a precision other than the server's, an A0 field, a
 * growing source or the general node model -> BTRT_E_INVAL; a footprint larger than the server's memory -> BTRT_E_NOMEM. */
int btrt_server_submit(btrt_server_t* s, const btrt_problem_t* p, double tol, int64_t max_steps, int64_t* id);

/* One scheduling round (see above). Reports resident and queued counts. Synchronises. */
int btrt_server_pump(btrt_server_t* s, int32_t* active, int32_t* queued);

/* State of request id. Errors: BTRT_E_INVAL for an unknown or collected id. */
int btrt_server_info(const btrt_server_t* s, int64_t id, btrt_request_info_t* info);

/* phi of a DONE request into phi_out[nx*ny]; releases the request. A FAILED request is released
 * too and its error returned (BTRT_E_UNSTABLE, or the device error that ended it; phi_out is not
 * written). Errors: BTRT_E_INVAL for an unknown id or a request still queued or running. */
int btrt_server_result(btrt_server_t* s, int64_t id, double* phi_out);

int btrt_server_stats(const btrt_server_t* s, btrt_server_stats_t* stats);

/* Seconds since the server was created (the clock of btrt_request_info_t). */
double btrt_server_clock(const btrt_server_t* s);

/* Frees the server, its device memory and every request. Synchronises. */
int btrt_server_destroy(btrt_server_t* s);

#ifdef __cplusplus
}
#endif
#endif /* BTRT_H */
