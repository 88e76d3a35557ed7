// A group of resident problem instances advanced together: one persistent launch per
// (fused) time step walks the tiles of every member. Shared by the batched C ABI and the
// solve server; membership can change between calls.

#include "btrt_host.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace btrth {

using btrtk::BatchEntry;
using btrtk::kReducePartials;
using btrtk::kResidual;

namespace {

size_t entry_bytes(int precision)
{
    return precision == BTRT_F64 ? sizeof(BatchEntry<double>) : sizeof(BatchEntry<float>);
}

void drop_graph(Group& g)
{
    if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.gexec = nullptr;
    g.graph = nullptr;
}

int grid_blocks(const Group& g) { return g.cfg.blocks_per_cu > 0 ? g.ncu * g.cfg.blocks_per_cu : 0; }

constexpr int kDefaultStripRows = 16;
int strip_rows(const btrt_batch_config_t& c) { return c.strip_rows > 0 ? c.strip_rows : kDefaultStripRows; }

hipError_t raw_launch(Group& g, int steps, int flip)
{
    const int n = static_cast<int>(g.inst.size());
    const int rows = strip_rows(g.cfg);
    bool k0one = true;
    for (const Instance* I : g.inst) k0one = k0one && I->k0_one;
    if (g.precision == BTRT_F64)
        return btrtk::launch_batch_sweep<double>(static_cast<const BatchEntry<double>*>(g.d_ent), g.d_begin[steps],
                                                 g.d_par, n, g.total[steps], flip, steps, grid_blocks(g), rows, k0one,
                                                 g.nts, g.stream);
    return btrtk::launch_batch_sweep<float>(static_cast<const BatchEntry<float>*>(g.d_ent), g.d_begin[steps], g.d_par,
                                            n, g.total[steps], flip, steps, grid_blocks(g), rows, k0one, g.nts,
                                            g.stream);
}

// Offsets of each member's units in the concatenated list for `steps` per launch: 64 x rows
// tiles (1 and 2 steps), or walker strips (batch_strip_columns(steps) x rows).
int upload_begin(Group& g, int steps, int rows)
{
    const int n = static_cast<int>(g.inst.size());
    std::vector<int> begin(n + 1);
    const int width = btrtk::batch_walks(steps) ? btrtk::batch_strip_columns(steps) : btrtk::kTileWidth;
    int64_t acc = 0;
    for (int i = 0; i < n; ++i) {
        begin[i] = static_cast<int>(acc);
        const Instance& I = *g.inst[i];
        acc += static_cast<int64_t>((I.nx + width - 1) / width) * ((I.ny + rows - 1) / rows);
    }
    if (acc > INT32_MAX) return fail(BTRT_E_INVAL, "more than 2^31 - 1 tiles in one group");
    begin[n] = static_cast<int>(acc);
    g.total[steps] = static_cast<int>(acc);
    hipError_t e = hipMemcpyAsync(g.d_begin[steps], begin.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice,
                                  g.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
    return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "group table upload");
}

// The strip table of the k-step walker for the configured strip height (built when first
// needed).
int ensure_walk_table(Group& g, int k)
{
    const int rows = strip_rows(g.cfg);
    if (g.walk_rows[k] == rows || g.inst.empty()) return BTRT_OK;
    int rc = upload_begin(g, k, rows);
    if (rc == BTRT_OK) g.walk_rows[k] = rows;
    return rc;
}

void advance(Group& g, int steps, int launches)
{
    if (launches & 1) {
        g.flip ^= 1;
        for (Instance* I : g.inst) I->cur ^= 1;
    }
    for (Instance* I : g.inst) I->step += static_cast<int64_t>(steps) * launches;
}

int launch_once(Group& g, int steps)
{
    hipError_t e = raw_launch(g, steps, g.flip);
    if (e != hipSuccess) return hip_fail(e, "batch sweep launch");
    advance(g, steps, 1);
    return BTRT_OK;
}

// Captures cfg.graph_launches launches (flip 0, 1, 0, ...) into a graph.
int build_graph(Group& g)
{
    drop_graph(g);
    hipError_t e = hipStreamBeginCapture(g.stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int j = 0; j < g.cfg.graph_launches && le == hipSuccess; ++j) le = raw_launch(g, g.cfg.steps_per_launch, j & 1);
    e = hipStreamEndCapture(g.stream, &g.graph);
    if (le != hipSuccess) return hip_fail(le, "batch sweep capture");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&g.gexec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    g.gcfg = g.cfg;
    return BTRT_OK;
}

template <typename T>
void fill_entries(const Group& g, std::vector<BatchEntry<T>>& ent, bool nts)
{
    ent.resize(g.inst.size());
    for (size_t i = 0; i < g.inst.size(); ++i) {
        const Instance& I = *g.inst[i];
        for (int p = 0; p < 2; ++p) {
            ent[i].a[p] = sweep_args<T>(I, p);
            ent[i].a[p].nts = nts ? 1 : 0;
        }
        ent[i].variant = 2 * I.kind + (I.k1_per_node ? 1 : 0);
        ent[i].pad = 0;
    }
}

}  // namespace

bool config_ok(const btrt_batch_config_t* c)
{
    return c && btrtk::batch_steps_ok(c->steps_per_launch) &&
           c->strip_rows >= 0 && c->strip_rows <= 4096 && c->blocks_per_cu >= 0 &&
           c->blocks_per_cu <= 64 && c->graph_launches >= 0 && c->graph_launches <= 4096 &&
           (c->graph_launches == 0 || (c->graph_launches >= 2 && c->graph_launches % 2 == 0));
}

int group_init(Group& g, int device, hipStream_t s, int precision, int capacity)
{
    g.device = device;
    g.stream = s;
    g.precision = precision;
    g.capacity = capacity;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        g.ncu = prop.multiProcessorCount;
    const size_t bytes = align_up(capacity * entry_bytes(precision)) +
                         6 * align_up(static_cast<size_t>(capacity + 1) * sizeof(int));
    if (hipMalloc(reinterpret_cast<void**>(&g.tables), bytes) != hipSuccess) {
        g.tables = nullptr;
        (void)hipGetLastError();
        return fail(BTRT_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    char* t = g.tables;
    g.d_ent = t;
    t += align_up(capacity * entry_bytes(precision));
    for (int k : {1, 2, 4, 6, 7}) {
        g.d_begin[k] = reinterpret_cast<int*>(t);
        t += align_up(static_cast<size_t>(capacity + 1) * sizeof(int));
    }
    g.d_par = reinterpret_cast<int*>(t);
    if (hipHostMalloc(reinterpret_cast<void**>(&g.h_res),
                      static_cast<size_t>(capacity) * kReducePartials * sizeof(double)) != hipSuccess) {
        g.h_res = nullptr;
        return fail(BTRT_E_NOMEM, "pinned host allocation failed");
    }
    return BTRT_OK;
}

int group_upload(Group& g)
{
    drop_graph(g);
    const int n = static_cast<int>(g.inst.size());
    if (n > g.capacity) return fail(BTRT_E_INVAL, "group of %d exceeds its capacity %d", n, g.capacity);
    g.flip = 0;
    for (int k = 0; k <= btrtk::kBatchMaxSteps; ++k) {
        g.walk_rows[k] = 0;
        if (n == 0) g.total[k] = 0;
    }
    if (n == 0) return BTRT_OK;
    std::vector<int> par(n);
    hipError_t e = hipSuccess;
    for (int steps = 1; steps <= 2; ++steps) {
        int rc = upload_begin(g, steps, btrtk::tile_rows(steps, g.precision == BTRT_F64 ? 8 : 4));
        if (rc != BTRT_OK) return rc;
    }
    for (int i = 0; i < n; ++i) par[i] = g.inst[i]->cur;
    if (e == hipSuccess)
        e = hipMemcpyAsync(g.d_par, par.data(), n * sizeof(int), hipMemcpyHostToDevice, g.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
    double state = 0;
    for (const Instance* I : g.inst) state += 2.0 * 10.0 * I->plane * (g.precision == BTRT_F64 ? 8 : 4);
    const bool nts = state > 256.0 * 1024 * 1024;  // the members' state exceeds the Infinity Cache
    g.nts = nts;
    if (e == hipSuccess) {
        if (g.precision == BTRT_F64) {
            std::vector<BatchEntry<double>> ent;
            fill_entries(g, ent, nts);
            e = hipMemcpyAsync(g.d_ent, ent.data(), ent.size() * sizeof(ent[0]), hipMemcpyHostToDevice, g.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
        } else {
            std::vector<BatchEntry<float>> ent;
            fill_entries(g, ent, nts);
            e = hipMemcpyAsync(g.d_ent, ent.data(), ent.size() * sizeof(ent[0]), hipMemcpyHostToDevice, g.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
        }
    }
    return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "group table upload");
}

int group_enqueue(Group& g, int64_t n)
{
    if (g.inst.empty()) return BTRT_OK;
    if (btrtk::batch_walks(g.cfg.steps_per_launch)) {
        int rc = ensure_walk_table(g, g.cfg.steps_per_launch);
        if (rc != BTRT_OK) return rc;
    }
    const int k = g.cfg.steps_per_launch;
    const int L = g.cfg.graph_launches;
    int64_t left = n;
    if (L > 0) {
        const int64_t chunk = static_cast<int64_t>(L) * k;
        if (left >= chunk + (g.flip ? k : 0)) {
            if (g.flip) {  // the graph starts from flip 0
                int rc = launch_once(g, k);
                if (rc != BTRT_OK) return rc;
                left -= k;
            }
            if (!g.gexec || g.gcfg.steps_per_launch != g.cfg.steps_per_launch ||
                g.gcfg.blocks_per_cu != g.cfg.blocks_per_cu || g.gcfg.graph_launches != L ||
                strip_rows(g.gcfg) != strip_rows(g.cfg)) {
                int rc = build_graph(g);
                if (rc != BTRT_OK) return rc;
            }
            while (left >= chunk) {
                hipError_t e = hipGraphLaunch(g.gexec, g.stream);
                if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
                advance(g, k, L);
                left -= chunk;
            }
        }
    }
    while (left > 0) {
        // Whole launches of k steps, then 2 and 1 for the remainder.
        const int s = left >= k ? k : (left >= 2 ? 2 : 1);
        int rc = launch_once(g, s);
        if (rc != BTRT_OK) return rc;
        left -= s;
    }
    return BTRT_OK;
}

int group_residuals(Group& g, double* out, int* bad)
{
    const int n = static_cast<int>(g.inst.size());
    for (int i = 0; i < n; ++i) {
        int rc = instance_reduce_async(*g.inst[i], kResidual, g.stream);
        if (rc == BTRT_OK) rc = instance_result_async(*g.inst[i], g.h_res + i * kReducePartials, g.stream);
        if (rc != BTRT_OK) return rc;
    }
    hipError_t e = hipStreamSynchronize(g.stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int nb = 0;
    for (int i = 0; i < n; ++i) {
        const double* v = g.h_res + i * kReducePartials;
        if (v[5] > 0) {
            out[i] = NAN;
            ++nb;
        } else {
            out[i] = v[1] > 0 ? v[0] / v[1] : (v[0] > 0 ? INFINITY : 0.0);
        }
    }
    if (bad) *bad = nb;
    return BTRT_OK;
}

int group_tune(Group& g, int64_t max_steps, btrt_batch_config_t* best, int64_t* used_out)
{
    std::vector<btrt_batch_config_t> cand;
    for (int k : {4, 6, 7})
        for (int rows : {16, 32}) cand.push_back({k, 0, 16, rows});
    cand.push_back({4, 0, 0, 32});
    cand.push_back({4, 4, 16, 32});
    for (int gl : {0, 16}) cand.push_back({2, 0, gl, 0});
    cand.push_back({1, 0, 16, 0});
    // A few warm-up steps of the configuration in force, then pass 1: each candidate runs k untimed
    // steps and one timed graph-replay's worth (16 launches of k steps), as far as three quarters
    // of max_steps allow. Pass 1 may run while the GPU clocks still rise, which favours candidates
    // timed late, so pass 2 re-times the kFinal fastest in turn, twice over, within the rest of
    // max_steps, and the lowest mean time per step wins.
    constexpr int kFinal = 3;
    const btrt_batch_config_t keep = g.cfg;
    int64_t used = 0;
    btrt_batch_config_t best_cfg = keep;
    if (!g.inst.empty()) {
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
            if (t0) (void)hipEventDestroy(t0);
            return fail(BTRT_E_DEVICE, "hipEventCreate");
        }
        int rc = BTRT_OK;
        std::vector<double> ms_sum(cand.size(), 0.0);
        std::vector<int> n(cand.size(), 0);
        // Times candidate c (k untimed steps, or 2 k so that the timed run starts at launch
        // parity 0 where a graph replay starts, then 16 k timed) if it fits within `limit` steps.
        auto time_one = [&](size_t c, int64_t limit) -> int {
            const int k = cand[c].steps_per_launch;
            const int64_t per = 16LL * k;
            const int64_t warm_k = g.flip ? k : 2LL * k;  // each launch flips the parity
            if (used + warm_k + per > limit) return BTRT_OK;
            g.cfg = cand[c];
            int r = group_enqueue(g, warm_k);
            used += warm_k;
            if (r == BTRT_OK && cand[c].graph_launches > 0) r = build_graph(g);
            if (r != BTRT_OK) return r;
            (void)hipEventRecord(t0, g.stream);
            r = group_enqueue(g, per);
            (void)hipEventRecord(t1, g.stream);
            (void)hipEventSynchronize(t1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, t0, t1);
            used += per;
            if (r == BTRT_OK) {
                ms_sum[c] += ms / per;
                ++n[c];
            }
            return r;
        };
        const int64_t warm = std::min<int64_t>(max_steps / 10, 64) / keep.steps_per_launch * keep.steps_per_launch;
        if (warm > 0) {
            rc = group_enqueue(g, warm);
            used += warm;
        }
        for (size_t c = 0; c < cand.size() && rc == BTRT_OK; ++c) rc = time_one(c, max_steps * 3 / 4);
        std::vector<size_t> ranked;
        for (size_t c = 0; c < cand.size(); ++c)
            if (n[c] > 0) ranked.push_back(c);
        std::sort(ranked.begin(), ranked.end(), [&](size_t x, size_t y) { return ms_sum[x] < ms_sum[y]; });
        if (ranked.size() > static_cast<size_t>(kFinal)) ranked.resize(kFinal);
        std::vector<double> first(ms_sum);
        std::vector<int> n1(n);
        for (size_t c : ranked) {
            ms_sum[c] = 0.0;
            n[c] = 0;
        }
        for (int round = 0; round < 2 && rc == BTRT_OK; ++round)
            for (size_t j = 0; j < ranked.size() && rc == BTRT_OK; ++j) rc = time_one(ranked[j], max_steps);
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        if (rc != BTRT_OK) {
            g.cfg = keep;
            return rc;
        }
        double best_ms = INFINITY;
        for (size_t c : ranked) {
            const double ms = n[c] > 0 ? ms_sum[c] / n[c] : first[c] / n1[c];  // pass 1 only if the steps ran out
            if (ms < best_ms) {
                best_ms = ms;
                best_cfg = cand[c];
            }
        }
    }
    g.cfg = best_cfg;
    if (best) *best = best_cfg;
    if (used_out) *used_out = used;
    return BTRT_OK;
}

void group_free(Group& g)
{
    drop_graph(g);
    if (g.tables) (void)hipFree(g.tables);
    if (g.h_res) (void)hipHostFree(g.h_res);
    g.tables = nullptr;
    g.h_res = nullptr;
    g.inst.clear();
}

}  // namespace btrth
