// Internal interface between the host runtime (btrt_api.cpp) and the gfx950 kernels
// (btrt_kernels.hip). Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace btrtk {

// Source kinds as the kernels see them.
enum SrcKind : int { kSrcNone = 0, kSrcField = 1, kSrcSep = 2 };

// Reduction modes of the gather kernels.
enum ReduceMode : int { kResidual = 0, kError = 1 };

// How the kernels obtain K1 (Eq. (30)): the constant of the problem, or per node from
// A0 (1 + beta phi^2), or per node from a space-dependent A0(x) (1 + beta phi^2).
enum K1Mode : int { kK1Const = 0, kK1Phi = 1, kK1Field = 2 };
// Kernel mode = K1 mode | kGen. kGen selects the general node model: a power-law flux term
// c |phi|^q, a source part r phi (1 - |phi|^p) that depends on phi, and Dirichlet values read
// per boundary node and step from a wall table.
// kK0One marks k0 = 1 exactly (the paper's choice throughout): the (1 - k0) f_i term of the
// collision vanishes, so the populations need not stay live through it; every storage format
// with the standard node model has such kernels, and batches whose instances all have k0 = 1;
// the general node model ignores the bit.
constexpr int kK1Mask = 3;
constexpr int kGen = 4;
constexpr int kK0One = 8;
// kRcp1 (set by the 16-bit deviation formats' call sites, not a kernel variant): the FP32 1/det M
// of the per-node K1 from the hardware reciprocal and one Newton step instead of a division.
constexpr int kRcp1 = 16;

constexpr int kMaxFuse = 7;   // most time steps one sweep launch can fuse
constexpr int kAutoFuse = 4;  // steps per launch of the automatic shape on large grids

// Everything one sweep needs, by value in the kernel argument segment.
template <typename T>
struct SweepArgs {
    const T* fin;      // 9 planes of the post-collision populations f+(t-1)
    T* fout;           // 9 planes receiving f+(t)
    const T* phi_prev; // phi(t-1), one plane
    T* phi_out;        // phi(t), one plane
    const T* src;      // kSrcField: one plane; kSrcSep: sx[nx]
    const T* src_y;    // kSrcSep: sy[ny]
    int64_t plane;     // elements per plane (pitch * ny)
    int nx, ny, pitch;
    int perx, pery;    // 1 when the direction is periodic
    T wall[4];         // phi_w of sides x-, x+, y-, y+
    T ax, ay, bx, by;  // B(phi) = a phi + b phi^2 / 2
    T a11, a12, a22, beta; // A(phi) = A0 (1 + beta phi^2), used when K1 is per node
    T K11, K12, K22;   // K1 of Eq. (30) when A is constant
    T k0, k2xx, k2xy, k2yy;
    T cq[4];           // the collision's constants 3/2, -9/2, -9, 9 (read from the arguments, the
                       // kernels keep them in scalar registers instead of copying an accumulator
                       // for every multiply-add with an inline constant)
    T src_amp;
    T sfac[kMaxFuse];  // source factor of each step of the launch (1: time independent)
    T fcx, fcy, fq;    // kGen: B(phi) gains (fcx, fcy) |phi|^fq
    T rr, rp;          // kGen: the source gains rr phi (1 - |phi|^rp)
    T dg, de, ds;      // kGen with dpoly: D(phi) = (dg phi + de |phi|^ds) I
    int dpoly;
    const T* wtab;     // wall table (kGen, else null): entry e holds the Dirichlet values of the
                       // pull at step e of the launch at wtab + e * wstride: x- (ny, by row),
                       // x+ (ny), y- (nx, by column), y+ (nx)
    int wstride;       // elements between entries (0: one entry for every step)
    const T* afield;   // kK1Field: three planes a11, a12, a22 (plane stride `plane`)
    T dev_scale, dev_inv; // 16-bit deviation formats: h = q(dev_scale (f+ - f_eq)), f+ = f_eq + h dev_inv
    int tiles_x, tiles_y; // set by the launcher for the kernel it picks
    int rows;             // rows per strip of the strip walkers (set by the launcher)
    int nts;              // 1: the one-step and two-step tile kernels store non-temporally (grids
                          // much larger than the caches; the launcher picks the kernel by it)
};

// Storage formats of the post-collision populations (kernels' template selector).
enum Format : int { kFmtPlain = 0, kFmtF16Dev = 1, kFmtBF16Dev = 2 };

// Gather-reduce of phi(t) (for the residual, error norms, field and population reads): the
// sweep arguments of the current state (fin / phi_prev = the buffers holding f+(t-1) and
// phi(t-1)) plus the reduction buffers.
template <typename T>
struct GatherArgs {
    SweepArgs<T> s;
    double* snap;      // kResidual: phi snapshot (dense nx*ny, FP64), updated in place
    const double* ref; // kError: reference (dense nx*ny)
    double* out;       // dense nx*ny output for field / population reads
    double* partial;   // per-block partial sums (kReducePartials doubles per block)
    int population;    // population index for the population read, -1 for phi
};

// One instance of a batched launch: its arguments for both buffer parities and the kernel
// variant (source kind x per-node K1).
template <typename T>
struct BatchEntry {
    SweepArgs<T> a[2];
    int variant;  // 2 * source kind + (K1 per node)
    int pad;
};

constexpr int kReducePartials = 6; // sum a, sum b, sum c, sum d, max, non-finite count
constexpr int kReduceBlocks = 1024;
constexpr int kBlock = 256;

// Shape of one sweep launch; every shape gives bitwise identical results.
struct LaunchCfg {
    int steps = 0;  // time steps per launch, 1 .. kMaxFuse (0: automatic)
    int rows = 0;   // strip walkers (steps >= 2): rows per strip (0: automatic)
    int group = 0;  // strip walkers: strips per workgroup, 1 or kWalkGroup (0: automatic)
    int tile = 0;   // 1: steps == 2 through the LDS tile kernel instead of a strip walker
};
constexpr int kWalkGroup = 4;

// Launchers (defined in btrt_kernels.hip). They return the launch's hipError_t. fmt selects
// the storage format (kFmtPlain for double; any for float). cfg.steps (1 .. kMaxFuse) time
// steps advance in the launch: one node per thread for 1, strip walkers (intermediate time
// levels in registers) or the LDS tile kernel for more; automatic fields of cfg are resolved
// as resolve_launch does.
template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, int fmt, int src_kind, int kmode, const LaunchCfg& cfg,
                        hipStream_t s);
// cfg with its automatic fields filled in for this grid, format and device (the current one).
template <typename T>
LaunchCfg resolve_launch(const SweepArgs<T>& a, int fmt, int src_kind, int kmode, LaunchCfg cfg);
// f+(-1) and phi(-1) := phi0 into a.fin / a.phi_prev (see init_values); FP64 arithmetic.
// The flux of the init is B(phi) = a phi + b phi^2 / 2 + c |phi|^q (c = 0: no power-law term);
// D(phi) = phi I, or (g phi + e |phi|^s) I when dq = (1, g, e, s).
template <typename T>
hipError_t launch_init(const SweepArgs<T>& a, int fmt, const double* phi0, const double wall[4], const double ab[4],
                       const double cq[3], const double dq[4], hipStream_t s);
template <typename T>
hipError_t launch_gather_field(const GatherArgs<T>& a, int fmt, hipStream_t s);
template <typename T>
hipError_t launch_reduce(const GatherArgs<T>& a, int fmt, int mode, double* result, hipStream_t s);
template <typename T>
hipError_t launch_convert(const double* in, T* out, int nx, int ny, int pitch, hipStream_t s);
// All instances of a batch (plain storage) advance `steps` (1, 2, 4, 6 or 7) time steps in one
// launch of `grid` blocks (0: one block per tile) walking the concatenated tile list; from 4
// steps on the "tiles" are walker strips of batch_strip_columns(steps) columns by `rows` rows.
// k0one: every instance has k0 = 1 (the kK0One kernels, the bits of the single solves).
constexpr bool batch_walks(int steps) { return steps == 4 || steps == 6 || steps == 7; }
constexpr bool batch_steps_ok(int steps) { return steps == 1 || steps == 2 || batch_walks(steps); }
constexpr int kBatchMaxSteps = 7;
template <typename T>
hipError_t launch_batch_sweep(const BatchEntry<T>* ent, const int* begin, const int* par, int ninst, int total_tiles,
                              int flip, int steps, int grid, int rows, bool k0one, bool nts, hipStream_t s);
int batch_strip_columns(int steps);
// Tile height of the kernel that fuses `steps` steps (tile width is 64).
int tile_rows(int steps, int precision_bytes);
constexpr int kTileWidth = 64;

}  // namespace btrtk
