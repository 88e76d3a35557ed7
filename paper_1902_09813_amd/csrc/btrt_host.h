// Host-side pieces shared by the single-solver and batched C ABI (btrt_api.cpp,
// btrt_batch.cpp): validation, the constants of Eq. (30) and Eq. (62), the device memory
// layout of one problem instance, and the per-instance launch sequence.
#pragma once

#include "btrt.h"
#include "btrt_internal.h"

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace btrth {

using btrtk::GatherArgs;
using btrtk::SweepArgs;
using btrtk::kFmtPlain;
using btrtk::kFmtF16Dev;
using btrtk::kFmtBF16Dev;

// Error reporting: sets the calling thread's last-error message and returns code.
int fail(int code, const char* fmt, ...);
int ok();
int hip_fail(hipError_t e, const char* what);
const char* last_error();

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Row pitch (elements) of the device planes: rows start on 256-byte boundaries.
int pitch_for(int nx, int precision);
// Bytes of one stored population value; kernel storage format of a precision.
size_t pop_bytes(int precision);
int format_of(int precision);

// Byte offsets of every buffer of one instance inside its memory region.
struct Layout {
    size_t f[2], phi[2], snap, tmp, partial, result, src, src_y, afield, wall0, total;
};
// afield: three planes (a11, a12, a22) of a space-dependent A0(x). wall0: one wall-table entry
// (2 (nx + ny) values), the per-side constants of the general node model.
Layout layout_for(int nx, int ny, int precision, int src_kind, bool afield = false);
bool grid_ok(const btrt_grid_t* g);

// Constants derived from a validated problem.
struct Resolved {
    double K1[4];  // Eq. (30) at phi = 0
    double K2[4];  // given, or Eq. (62)
    double k0;
    bool k1_per_node;  // beta > 0 or a per-node A0(x)
    bool afield;       // A0(x) given per node
    double growth;     // source S(x, t) = exp(growth t) S0(x)
    bool gen;          // general node model: a power-law flux, a phi-dependent source or D != phi I
    double dq[4];      // D(phi): (0, ...) phi I; (1, g, e, s) (g phi + e |phi|^s) I
};

int validate(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K, const btrt_dterm_t* D,
             const btrt_source_t* R, const btrt_bc_t* bc, const btrt_relax_t* relax, Resolved* res);
// Also rejects a NULL or non-finite phi0.
int validate_phi0(const btrt_grid_t* grid, const double* phi0);
void fill_info(const btrt_grid_t* g, const Resolved& r, int src_kind, btrt_info_t* info);

// One problem placed in device memory. State between launches: f+(t-1) in f[cur] and
// phi(t-1) in phi[cur].
// K1 mode of the kernels: constant, A0 (1 + beta phi^2), or A0(x) (1 + beta phi^2).
struct Instance {
    int nx = 0, ny = 0, pitch = 0, precision = 0;
    int kind = 0;         // btrtk::SrcKind of the source
    bool k1_per_node = false;
    bool k0_one = false;  // k0 = 1 exactly: kernels without the (1 - k0) f_i term
    bool afield = false;  // per-node A0(x) planes in the workspace
    double growth = 0.0;  // source growth rate per step (Scheme 2 correction when nonzero)
    // General node model (kGen): wall table entries of wall_entry_slots() values in the phi type
    // (the wall_entry_values() samples a caller gives per step, see btrt_set_walls, then the four
    // corner means); the pull at step count t reads entry (t - wall_t0) at
    // wtab + (t - wall_t0) * wall_stride. Steps may advance the count up to wall_limit.
    bool gen = false;
    const char* wtab = nullptr;
    int64_t wall_t0 = 0;
    int64_t wall_limit = INT64_MAX;
    int wall_stride = 0;
    int perx = 1, pery = 1;
    int64_t plane = 0;
    double wall[4] = {0, 0, 0, 0};
    char* mem = nullptr;  // this instance's region; Layout offsets are relative to it
    Layout L{};
    int cur = 0;
    int64_t step = 0;
    double dev_scale = 1.0;   // 16-bit deviation formats: h = q(dev_scale (f+ - f_eq))
    SweepArgs<double> a64{};  // problem constants; buffer pointers are set per launch
    SweepArgs<float> a32{};
    btrt_info_t info{};
    int kmode() const
    {
        const int k1 = afield ? btrtk::kK1Field : (k1_per_node ? btrtk::kK1Phi : btrtk::kK1Const);
        if (gen) return k1 | btrtk::kGen;
        return k0_one ? (k1 | btrtk::kK0One) : k1;
    }
    // Samples per step of a wall schedule: each side every half spacing, corners included.
    int wall_entry_values() const { return 4 * (nx + ny) + 4; }
    // Device slots per wall-table entry: the samples and the means at the four corners.
    int wall_entry_slots() const { return wall_entry_values() + 4; }
};

// Places a validated problem into mem (at least layout_for(...).total bytes, 256-byte
// aligned): uploads the source and phi0, writes f+(-1) so that the first pull yields
// f^eq(phi0), phi(-1) := phi0 and the Eq. (64) snapshot := phi0. Synchronises s.
int instance_setup(Instance& I, const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K,
                   const btrt_source_t* R, const btrt_bc_t* bc, const Resolved& r, const double* phi0, char* mem,
                   hipStream_t s);

// Writes `rows` wall-table entries to device memory dst in I's phi type from rows of FP64
// samples (wall_entry_values() each): the samples, then the mean of the two sides' samples at
// each corner (x-y-, x+y-, x+y+, x-y+), rounded as the kernels round the mean of two per-side
// constants. Staged through a fixed host buffer (no allocation); synchronises s.
hipError_t upload_wall_values(const Instance& I, const double* v, size_t rows, char* dst, hipStream_t s);
// One wall-table entry of the per-side constants (the table of a general-model handle without a
// schedule).
hipError_t upload_wall_entry(const Instance& I, char* dst, hipStream_t s);

// Sweep arguments with the buffer pointers for the given parity (0: f[0] -> f[1]).
template <typename T>
SweepArgs<T> sweep_args(const Instance& I, int parity);
template <typename T>
GatherArgs<T> gather_args(const Instance& I);

// One sweep launch of shape cfg (cfg.steps >= 1 time steps; automatic fields allowed); flips
// the parity.
int instance_launch(Instance& I, const btrtk::LaunchCfg& cfg, hipStream_t s);
// n time steps as launches of shape `want` (automatic fields allowed); a count that is not a
// multiple of its steps per launch ends with one shorter launch. Refuses steps past a wall
// schedule's end (BTRT_E_INVAL, nothing enqueued).
int instance_steps(Instance& I, const btrtk::LaunchCfg& want, int64_t n, hipStream_t s);
// cfg with its automatic fields resolved for I's grid and format on the current device.
btrtk::LaunchCfg instance_resolve(const Instance& I, const btrtk::LaunchCfg& cfg);
// Enqueues the two-pass reduction (residual or error) into I's result slot (no sync).
int instance_reduce_async(Instance& I, int mode, hipStream_t s);
// Copies I's result slot to out (async).
int instance_result_async(const Instance& I, double out[btrtk::kReducePartials], hipStream_t s);
// phi(t) (population < 0) or f_i(t) into a host array; synchronises.
int instance_gather(Instance& I, int population, double* host_out, hipStream_t s);

// A set of resident instances advanced together by batched launches (used by the batch and
// the server). Device tables are sized for `capacity` instances; membership may change
// between calls (group_upload rebuilds the tables).
struct Group {
    int device = 0;
    hipStream_t stream = nullptr;
    int precision = BTRT_F64;
    int ncu = 256;
    int capacity = 0;
    std::vector<Instance*> inst;
    char* tables = nullptr;  // device: entries, tile offsets (1- and 2-step tiles, walker strips), parities
    void* d_ent = nullptr;
    int* d_begin[btrtk::kBatchMaxSteps + 1] = {};  // indexed by steps per launch (1, 2, 4, 6, 7)
    int* d_par = nullptr;
    int total[btrtk::kBatchMaxSteps + 1] = {};
    int walk_rows[btrtk::kBatchMaxSteps + 1] = {};  // strip height each walker table was built for (0: not built)
    int flip = 0;       // launches since group_upload, mod 2
    bool nts = false;   // the members' state exceeds the Infinity Cache: non-temporal stores in the
                        // one- and two-step batch kernels
    btrt_batch_config_t cfg{2, 0, 0, 0};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    btrt_batch_config_t gcfg{0, 0, 0, 0};
    double* h_res = nullptr;  // pinned, capacity * kReducePartials
};

int group_init(Group& g, int device, hipStream_t s, int precision, int capacity);
// Rebuilds the device tables from g.inst (synchronous); drops the captured graph.
int group_upload(Group& g);
// Enqueues n time steps of every member.
int group_enqueue(Group& g, int64_t n);
// Eq. (64) residual of every member into out[size]; *bad = members with NaN/Inf (out NaN).
int group_residuals(Group& g, double* out, int* bad);
// Times candidate configurations on the members' own steps; keeps the fastest.
int group_tune(Group& g, int64_t max_steps, btrt_batch_config_t* best, int64_t* used);
bool config_ok(const btrt_batch_config_t* c);
void group_free(Group& g);

// Runs the enclosed calls with a device current, restoring the caller's afterwards.
class DeviceGuard {
public:
    explicit DeviceGuard(int device);
    ~DeviceGuard();
    hipError_t status() const { return status_; }

private:
    int prev_ = -1;
    int device_ = 0;
    hipError_t status_ = hipSuccess;
};

}  // namespace btrth
