// Batched C ABI (include/btrt.h, btrt_batch_*): many independent problem instances of
// different sizes advanced together by one persistent launch per (fused) time step, with
// HIP-graph replay of the launch sequence and an autotuner over the launch configuration.

#include "btrt.h"
#include "btrt_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

using namespace btrth;
using btrtk::BatchEntry;
using btrtk::kReducePartials;
using btrtk::kResidual;

struct btrt_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int precision = BTRT_F64;
    int n = 0;
    char* arena = nullptr;
    std::vector<Instance> inst;
    // Device tables: instance entries, tile offsets for 1- and 2-step tiles, parities.
    void* d_ent = nullptr;
    int* d_begin[3] = {nullptr, nullptr, nullptr};
    int* d_par = nullptr;
    int total[3] = {0, 0, 0};
    int flip = 0;  // launches since the parity table was written, mod 2
    int64_t step = 0;
    int ncu = 256;
    btrt_batch_config_t cfg{2, 0, 0};
    // Captured launch sequence for cfg (rebuilt when cfg changes).
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    btrt_batch_config_t gcfg{0, 0, 0};
    double* h_res = nullptr;  // pinned, n * kReducePartials
};

namespace {

template <typename T>
void fill_entries(btrt_batch* b, std::vector<BatchEntry<T>>& ent, bool nts)
{
    ent.resize(b->n);
    for (int i = 0; i < b->n; ++i) {
        const Instance& I = b->inst[i];
        for (int p = 0; p < 2; ++p) {
            ent[i].a[p] = sweep_args<T>(I, p);
            ent[i].a[p].nts = nts ? 1 : 0;
        }
        ent[i].variant = 2 * I.kind + (I.k1_per_node ? 1 : 0);
        ent[i].pad = 0;
    }
}

void drop_graph(btrt_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

int grid_blocks(const btrt_batch* b) { return b->cfg.blocks_per_cu > 0 ? b->ncu * b->cfg.blocks_per_cu : 0; }

hipError_t raw_launch(btrt_batch* b, int steps, int flip)
{
    if (b->precision == BTRT_F64)
        return btrtk::launch_batch_sweep<double>(static_cast<const BatchEntry<double>*>(b->d_ent), b->d_begin[steps],
                                                 b->d_par, b->n, b->total[steps], flip, steps, grid_blocks(b), b->stream);
    return btrtk::launch_batch_sweep<float>(static_cast<const BatchEntry<float>*>(b->d_ent), b->d_begin[steps],
                                            b->d_par, b->n, b->total[steps], flip, steps, grid_blocks(b), b->stream);
}

void advance(btrt_batch* b, int steps, int launches)
{
    if (launches & 1) {
        b->flip ^= 1;
        for (Instance& I : b->inst) I.cur ^= 1;
    }
    for (Instance& I : b->inst) I.step += static_cast<int64_t>(steps) * launches;
    b->step += static_cast<int64_t>(steps) * launches;
}

int launch_once(btrt_batch* b, int steps)
{
    hipError_t e = raw_launch(b, steps, b->flip);
    if (e != hipSuccess) return hip_fail(e, "batch sweep launch");
    advance(b, steps, 1);
    return BTRT_OK;
}

// Captures cfg.graph_launches launches (flip 0, 1, 0, ...) into a graph.
int build_graph(btrt_batch* b)
{
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int j = 0; j < b->cfg.graph_launches && le == hipSuccess; ++j) le = raw_launch(b, b->cfg.steps_per_launch, j & 1);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (le != hipSuccess) return hip_fail(le, "batch sweep capture");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->gcfg = b->cfg;
    return BTRT_OK;
}

int enqueue(btrt_batch* b, int64_t n)
{
    const int k = b->cfg.steps_per_launch;
    const int L = b->cfg.graph_launches;
    int64_t left = n;
    if (L > 0) {
        const int64_t chunk = static_cast<int64_t>(L) * k;
        if (left >= chunk + (b->flip ? k : 0)) {
            if (b->flip) {  // the graph starts from flip 0
                int rc = launch_once(b, k);
                if (rc != BTRT_OK) return rc;
                left -= k;
            }
            if (!b->gexec || b->gcfg.steps_per_launch != b->cfg.steps_per_launch ||
                b->gcfg.blocks_per_cu != b->cfg.blocks_per_cu || b->gcfg.graph_launches != L) {
                int rc = build_graph(b);
                if (rc != BTRT_OK) return rc;
            }
            while (left >= chunk) {
                hipError_t e = hipGraphLaunch(b->gexec, b->stream);
                if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
                advance(b, k, L);
                left -= chunk;
            }
        }
    }
    while (left > 0) {
        const int s = (k == 2 && left >= 2) ? 2 : 1;
        int rc = launch_once(b, s);
        if (rc != BTRT_OK) return rc;
        left -= s;
    }
    return BTRT_OK;
}

void release(btrt_batch* b)
{
    if (!b) return;
    DeviceGuard g(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->arena) (void)hipFree(b->arena);
    if (b->h_res) (void)hipHostFree(b->h_res);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

bool config_ok(const btrt_batch_config_t* c)
{
    return c && (c->steps_per_launch == 1 || c->steps_per_launch == 2) && c->blocks_per_cu >= 0 &&
           c->blocks_per_cu <= 64 && c->graph_launches >= 0 && c->graph_launches <= 4096 &&
           (c->graph_launches == 0 || (c->graph_launches >= 2 && c->graph_launches % 2 == 0));
}

}  // namespace

extern "C" {

int btrt_batch_create(int32_t n, const btrt_problem_t* problems, int32_t device, void* stream, btrt_batch_t** out)
{
    if (!out) return fail(BTRT_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !problems) return fail(BTRT_E_INVAL, "need n >= 1 problems");
    std::vector<Resolved> res(n);
    const int precision = problems[0].grid.precision;
    std::vector<size_t> offs(n);
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        const btrt_problem_t& p = problems[i];
        int rc = validate(&p.grid, &p.B, &p.K, &p.D, &p.R, &p.bc, &p.relax, &res[i]);
        if (rc == BTRT_OK) rc = validate_phi0(&p.grid, p.phi0);
        if (rc != BTRT_OK) {
            const std::string msg = last_error();
            return fail(rc, "instance %d: %s", i, msg.c_str());
        }
        if (p.grid.precision != precision) return fail(BTRT_E_INVAL, "instance %d: precision differs from instance 0", i);
        offs[i] = total;
        total += align_up(layout_for(p.grid.nx, p.grid.ny, precision, p.R.kind).total);
    }
    const size_t ent_bytes = static_cast<size_t>(n) * (precision == BTRT_F64 ? sizeof(BatchEntry<double>)
                                                                             : sizeof(BatchEntry<float>));
    const size_t tables = align_up(ent_bytes) + 3 * align_up(static_cast<size_t>(n + 1) * sizeof(int));
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(BTRT_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(BTRT_E_DEVICE, "device %d not in [0, %d)", device, ndev);

    btrt_batch* b = new (std::nothrow) btrt_batch();
    if (!b) return fail(BTRT_E_NOMEM, "host allocation failed");
    b->device = device;
    b->precision = precision;
    b->n = n;
    b->inst.resize(n);
    int rc = BTRT_OK;
    {
        DeviceGuard g(device);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
            b->ncu = prop.multiProcessorCount;
        if (stream) {
            b->stream = static_cast<hipStream_t>(stream);
        } else if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) {
            rc = hip_fail(e, "hipStreamCreate");
        } else {
            b->own_stream = true;
        }
        if (rc == BTRT_OK && hipMalloc(reinterpret_cast<void**>(&b->arena), total + tables) != hipSuccess) {
            b->arena = nullptr;
            (void)hipGetLastError();
            rc = fail(BTRT_E_NOMEM, "hipMalloc of %zu bytes failed", total + tables);
        }
        if (rc == BTRT_OK && hipHostMalloc(reinterpret_cast<void**>(&b->h_res),
                                           static_cast<size_t>(n) * kReducePartials * sizeof(double)) != hipSuccess) {
            b->h_res = nullptr;
            rc = fail(BTRT_E_NOMEM, "pinned host allocation failed");
        }
        for (int i = 0; i < n && rc == BTRT_OK; ++i) {
            const btrt_problem_t& p = problems[i];
            rc = instance_setup(b->inst[i], &p.grid, &p.B, &p.K, &p.R, &p.bc, res[i], p.phi0, b->arena + offs[i],
                                b->stream);
        }
        if (rc == BTRT_OK) {
            // Tile lists for the one-step and the two-step kernels.
            char* tab = b->arena + total;
            b->d_ent = tab;
            tab += align_up(ent_bytes);
            std::vector<int> begin(n + 1), par(n, 0);
            for (int steps = 1; steps <= 2; ++steps) {
                b->d_begin[steps] = reinterpret_cast<int*>(tab);
                tab += align_up(static_cast<size_t>(n + 1) * sizeof(int));
                const int rows = btrtk::tile_rows(steps, precision == BTRT_F64 ? 8 : 4);
                int64_t acc = 0;
                for (int i = 0; i < n; ++i) {
                    begin[i] = static_cast<int>(acc);
                    const Instance& I = b->inst[i];
                    acc += static_cast<int64_t>((I.nx + btrtk::kTileWidth - 1) / btrtk::kTileWidth) *
                           ((I.ny + rows - 1) / rows);
                }
                if (acc > INT32_MAX) {
                    rc = fail(BTRT_E_INVAL, "batch has more than 2^31 - 1 tiles");
                    break;
                }
                begin[n] = static_cast<int>(acc);
                b->total[steps] = static_cast<int>(acc);
                e = hipMemcpy(b->d_begin[steps], begin.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice);
                if (e != hipSuccess) rc = hip_fail(e, "table upload");
            }
            b->d_par = reinterpret_cast<int*>(tab);
            if (rc == BTRT_OK) {
                e = hipMemcpy(b->d_par, par.data(), n * sizeof(int), hipMemcpyHostToDevice);
                if (e != hipSuccess) rc = hip_fail(e, "table upload");
            }
            if (rc == BTRT_OK) {
                double state = 0;
                for (const Instance& I : b->inst) state += 2.0 * 10.0 * I.plane * (precision == BTRT_F64 ? 8 : 4);
                const bool nts = state > 256.0 * 1024 * 1024;
                if (precision == BTRT_F64) {
                    std::vector<BatchEntry<double>> ent;
                    fill_entries(b, ent, nts);
                    e = hipMemcpy(b->d_ent, ent.data(), ent.size() * sizeof(ent[0]), hipMemcpyHostToDevice);
                } else {
                    std::vector<BatchEntry<float>> ent;
                    fill_entries(b, ent, nts);
                    e = hipMemcpy(b->d_ent, ent.data(), ent.size() * sizeof(ent[0]), hipMemcpyHostToDevice);
                }
                if (e != hipSuccess) rc = hip_fail(e, "table upload");
            }
        }
    }
    if (rc != BTRT_OK) {
        const std::string msg = last_error();
        release(b);
        return fail(rc, "%s", msg.c_str());
    }
    *out = b;
    return ok();
}

int btrt_batch_step(btrt_batch_t* b, int64_t n)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (n < 0) return fail(BTRT_E_INVAL, "n = %lld < 0", static_cast<long long>(n));
    DeviceGuard g(b->device);
    int rc = enqueue(b, n);
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_batch_field(btrt_batch_t* b, int32_t i, double* phi_out)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (i < 0 || i >= b->n || !phi_out) return fail(BTRT_E_INVAL, "bad instance index or NULL output");
    DeviceGuard g(b->device);
    int rc = instance_gather(b->inst[i], -1, phi_out, b->stream);
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_batch_residual(btrt_batch_t* b, double* out)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (!out) return fail(BTRT_E_INVAL, "out is NULL");
    DeviceGuard g(b->device);
    for (int i = 0; i < b->n; ++i) {
        int rc = instance_reduce_async(b->inst[i], kResidual, b->stream);
        if (rc == BTRT_OK) rc = instance_result_async(b->inst[i], b->h_res + i * kReducePartials, b->stream);
        if (rc != BTRT_OK) return rc;
    }
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int bad = 0;
    for (int i = 0; i < b->n; ++i) {
        const double* v = b->h_res + i * kReducePartials;
        if (v[5] > 0) {
            out[i] = NAN;
            ++bad;
        } else {
            out[i] = v[1] > 0 ? v[0] / v[1] : (v[0] > 0 ? INFINITY : 0.0);
        }
    }
    if (bad) return fail(BTRT_E_UNSTABLE, "%d instance(s) hold non-finite values", bad);
    return ok();
}

int btrt_batch_set_config(btrt_batch_t* b, const btrt_batch_config_t* cfg)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (!config_ok(cfg)) return fail(BTRT_E_INVAL, "invalid batch configuration");
    b->cfg = *cfg;
    return ok();
}

int btrt_batch_get_config(const btrt_batch_t* b, btrt_batch_config_t* cfg)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (!cfg) return fail(BTRT_E_INVAL, "cfg is NULL");
    *cfg = b->cfg;
    return ok();
}

int btrt_batch_tune(btrt_batch_t* b, int64_t max_steps, btrt_batch_config_t* best, int64_t* steps_used)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (max_steps < 0) return fail(BTRT_E_INVAL, "max_steps < 0");
    DeviceGuard g(b->device);
    std::vector<btrt_batch_config_t> cand;
    for (int steps : {2, 1})
        for (int bpc : {0, 2, 4, 8})
            for (int gl : {0, 16}) cand.push_back({steps, bpc, gl});
    // Each candidate: a warm-up launch pair, then a timed run of a multiple of 32 steps.
    const int64_t per = std::max<int64_t>(0, max_steps / static_cast<int64_t>(cand.size()) - 4) / 32 * 32;
    const btrt_batch_config_t keep = b->cfg;
    int64_t used = 0;
    double best_ms = INFINITY;
    btrt_batch_config_t best_cfg = keep;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (per > 0) {
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return fail(BTRT_E_DEVICE, "hipEventCreate");
        for (const btrt_batch_config_t& c : cand) {
            b->cfg = c;
            int rc = enqueue(b, 4);
            if (rc == BTRT_OK && c.graph_launches > 0) rc = build_graph(b);
            if (rc != BTRT_OK) {
                (void)hipEventDestroy(t0);
                (void)hipEventDestroy(t1);
                b->cfg = keep;
                return rc;
            }
            (void)hipEventRecord(t0, b->stream);
            rc = enqueue(b, per);
            (void)hipEventRecord(t1, b->stream);
            (void)hipEventSynchronize(t1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, t0, t1);
            used += 4 + per;
            if (rc != BTRT_OK) {
                (void)hipEventDestroy(t0);
                (void)hipEventDestroy(t1);
                b->cfg = keep;
                return rc;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best_cfg = c;
            }
        }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
    }
    b->cfg = best_cfg;
    if (best) *best = best_cfg;
    if (steps_used) *steps_used = used;
    return ok();
}

int btrt_batch_steps(const btrt_batch_t* b, int64_t* steps)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (!steps) return fail(BTRT_E_INVAL, "steps is NULL");
    *steps = b->step;
    return ok();
}

int btrt_batch_sync(btrt_batch_t* b)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    DeviceGuard g(b->device);
    hipError_t e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? ok() : hip_fail(e, "hipStreamSynchronize");
}

int btrt_batch_destroy(btrt_batch_t* b)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    release(b);
    return ok();
}

}  // extern "C"
