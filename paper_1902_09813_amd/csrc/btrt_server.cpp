// Solve server (include/btrt.h, btrt_server_*): continuous batching of independent requests.
// Requests are admitted by device footprint into a first-fit arena, stay resident until they
// finish, and share every batched launch with the other resident requests (btrt_group.cpp).

#include "btrt.h"
#include "btrt_host.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

using namespace btrth;

namespace {

// First-fit allocator over [0, size) with coalescing of freed blocks.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        free_[0] = size;
        used_ = 0;
        high_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                high_ = used_ > high_ ? used_ : high_;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t high() const { return high_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, high_ = 0;
};

struct Request {
    int64_t id = 0;
    // Host copy of the problem.
    btrt_grid_t grid{};
    btrt_flux_t B{};
    btrt_diff_t K{};
    btrt_source_t R{};
    btrt_bc_t bc{};
    Resolved res{};
    std::vector<double> phi0, field;
    double tol = 0;
    int64_t max_steps = 0;
    size_t bytes = 0;
    // Device state while resident.
    Instance inst;
    size_t off = 0;
    // Outcome.
    btrt_request_info_t info{};
    std::vector<double> result;
};

}  // namespace

// Resident nodes from which an automatic launch configuration uses the strip walkers (measured
// on gfx950 with the served workload: below it the rounds are latency-bound).
constexpr int64_t kAutoWalkNodes = int64_t(1) << 21;
// With the automatic launch configuration, a request of at least this many nodes fills the GPU by
// itself: it advances by its own launches in the automatic single-grid shape (the seven-step
// walker on large periodic grids) instead of sharing the batched launch of the smaller requests,
// whose strips are shorter and whose launch shape suits small grids. Every shape gives the same
// bits, so a result is the same either way.
constexpr int64_t kSoloNodes = int64_t(1) << 20;

struct btrt_server {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int precision = BTRT_F64;
    int max_active = 1;
    int check_interval = 1000;
    char* mem = nullptr;
    size_t mem_bytes = 0;
    Arena arena;
    Group group;
    int64_t next_id = 1;
    std::unordered_map<int64_t, std::unique_ptr<Request>> req;
    std::deque<int64_t> queue;
    std::vector<int64_t> active;
    bool dirty = false;  // membership changed since the group tables were written
    bool auto_launch = false;  // choose the launch configuration per round from the resident work
    btrt_server_stats_t st{};
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

bool solo(const btrt_server* s, const Instance& I)
{
    return s->auto_launch && static_cast<int64_t>(I.nx) * I.ny >= kSoloNodes;
}

// Eq. (64) residual of every active request into out (NaN for a non-finite phi): one reduction per
// request, then one synchronisation.
int residuals(btrt_server* s, double* out)
{
    double* h = s->group.h_res;  // pinned, max_active slots
    for (size_t k = 0; k < s->active.size(); ++k) {
        Instance& I = s->req[s->active[k]]->inst;
        int rc = instance_reduce_async(I, btrtk::kResidual, s->stream);
        if (rc == BTRT_OK) rc = instance_result_async(I, h + k * btrtk::kReducePartials, s->stream);
        if (rc != BTRT_OK) return rc;
    }
    const hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (size_t k = 0; k < s->active.size(); ++k) {
        const double* v = h + k * btrtk::kReducePartials;
        out[k] = v[5] > 0 ? NAN : (v[1] > 0 ? v[0] / v[1] : (v[0] > 0 ? INFINITY : 0.0));
    }
    return BTRT_OK;
}

void release(btrt_server* s)
{
    if (!s) return;
    DeviceGuard g(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    group_free(s->group);
    if (s->mem) (void)hipFree(s->mem);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// Moves queued requests into free slots and memory, in arrival order.
int admit(btrt_server* s)
{
    for (auto it = s->queue.begin(); it != s->queue.end() && static_cast<int>(s->active.size()) < s->max_active;) {
        Request& r = *s->req[*it];
        size_t off = 0;
        if (!s->arena.alloc(r.bytes, &off)) {
            ++it;  // does not fit now; later, smaller requests may
            continue;
        }
        r.off = off;
        btrt_source_t R = r.R;
        if (R.kind == BTRT_SRC_FIELD) R.field = r.field.data();
        int rc = instance_setup(r.inst, &r.grid, &r.B, &r.K, &R, &r.bc, r.res, r.phi0.data(), s->mem + off, s->stream);
        if (rc != BTRT_OK) {
            s->arena.release(off, r.bytes);
            return rc;
        }
        r.phi0.clear();
        r.phi0.shrink_to_fit();
        r.info.status = BTRT_REQ_RUNNING;
        r.info.t_admit = s->now();
        s->active.push_back(r.id);
        s->st.admitted++;
        s->dirty = true;
        it = s->queue.erase(it);
    }
    return BTRT_OK;
}

void retire(btrt_server* s, Request& r, int status, int error)
{
    s->arena.release(r.off, r.bytes);
    r.info.status = status;
    r.info.error = error;
    r.info.t_done = s->now();
    if (status == BTRT_REQ_DONE)
        s->st.completed++;
    else
        s->st.failed++;
    s->dirty = true;
}

}  // namespace

extern "C" {

int btrt_server_create(const btrt_server_opts_t* o, btrt_server_t** out)
{
    if (!out) return fail(BTRT_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!o || (o->precision != BTRT_F64 && o->precision != BTRT_F32) || o->max_active < 1 || o->check_interval < 1 ||
        o->memory_bytes < kAlign || (o->launch.steps_per_launch != 0 && !config_ok(&o->launch)))
        return fail(BTRT_E_INVAL, "invalid server options");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(BTRT_E_DEVICE, "no HIP device available");
    if (o->device < 0 || o->device >= ndev) return fail(BTRT_E_DEVICE, "device %d not in [0, %d)", o->device, ndev);
    btrt_server* s = new (std::nothrow) btrt_server();
    if (!s) return fail(BTRT_E_NOMEM, "host allocation failed");
    s->device = o->device;
    s->precision = o->precision;
    s->max_active = o->max_active;
    s->check_interval = o->check_interval;
    s->mem_bytes = o->memory_bytes / kAlign * kAlign;
    int rc = BTRT_OK;
    {
        DeviceGuard g(s->device);
        if (o->stream) {
            s->stream = static_cast<hipStream_t>(o->stream);
        } else if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess) {
            rc = hip_fail(e, "hipStreamCreate");
        } else {
            s->own_stream = true;
        }
        if (rc == BTRT_OK && hipMalloc(reinterpret_cast<void**>(&s->mem), s->mem_bytes) != hipSuccess) {
            s->mem = nullptr;
            (void)hipGetLastError();
            rc = fail(BTRT_E_NOMEM, "hipMalloc of %zu bytes failed", s->mem_bytes);
        }
        if (rc == BTRT_OK) rc = group_init(s->group, s->device, s->stream, s->precision, s->max_active);
    }
    if (rc != BTRT_OK) {
        const std::string msg = last_error();
        release(s);
        return fail(rc, "%s", msg.c_str());
    }
    s->auto_launch = o->launch.steps_per_launch == 0;
    if (!s->auto_launch) s->group.cfg = o->launch;
    s->arena.reset(s->mem_bytes);
    *out = s;
    return ok();
}

int btrt_server_submit(btrt_server_t* s, const btrt_problem_t* p, double tol, int64_t max_steps, int64_t* id)
{
    if (!s) return fail(BTRT_E_STATE, "NULL server");
    if (!p || !id) return fail(BTRT_E_INVAL, "NULL argument");
    if (!(tol >= 0.0) || max_steps < 1) return fail(BTRT_E_INVAL, "need tol >= 0 and max_steps >= 1");
    auto r = std::make_unique<Request>();
    int rc = validate(&p->grid, &p->B, &p->K, &p->D, &p->R, &p->bc, &p->relax, &r->res);
    if (rc == BTRT_OK) rc = validate_phi0(&p->grid, p->phi0);
    if (rc != BTRT_OK) return rc;
    if (p->grid.precision != s->precision) return fail(BTRT_E_INVAL, "request precision differs from the server's");
    if (r->res.afield || r->res.growth != 0.0 || r->res.gen)
        return fail(BTRT_E_INVAL,
                    "served requests take no A0 field, growing source, power-law flux or phi-dependent source");
    r->bytes = layout_for(p->grid.nx, p->grid.ny, s->precision, p->R.kind).total;
    if (align_up(r->bytes) > s->mem_bytes)
        return fail(BTRT_E_NOMEM, "request needs %zu bytes, server has %zu", r->bytes, s->mem_bytes);
    r->id = s->next_id++;
    r->grid = p->grid;
    r->grid.stream = nullptr;
    r->grid.workspace = nullptr;
    r->B = p->B;
    r->K = p->K;
    r->R = p->R;
    r->bc = p->bc;
    const size_t nn = static_cast<size_t>(p->grid.nx) * p->grid.ny;
    r->phi0.assign(p->phi0, p->phi0 + nn);
    if (p->R.kind == BTRT_SRC_FIELD) r->field.assign(p->R.field, p->R.field + nn);
    r->R.field = nullptr;
    r->tol = tol;
    r->max_steps = max_steps;
    r->info.status = BTRT_REQ_QUEUED;
    r->info.error = BTRT_OK;
    r->info.nx = p->grid.nx;
    r->info.ny = p->grid.ny;
    r->info.steps = 0;
    r->info.residual = NAN;
    r->info.t_submit = s->now();
    r->info.t_admit = r->info.t_done = -1.0;
    *id = r->id;
    s->queue.push_back(r->id);
    s->req.emplace(r->id, std::move(r));
    s->st.submitted++;
    return ok();
}

int btrt_server_pump(btrt_server_t* s, int32_t* active, int32_t* queued)
{
    if (!s) return fail(BTRT_E_STATE, "NULL server");
    const double t_in = s->now();
    DeviceGuard g(s->device);
    int rc = admit(s);
    if (rc == BTRT_OK && s->dirty) {
        s->group.inst.clear();
        for (int64_t id : s->active) {
            Instance& I = s->req[id]->inst;
            if (!solo(s, I)) s->group.inst.push_back(&I);
        }
        rc = group_upload(s->group);
        s->dirty = false;
    }
    if (rc == BTRT_OK && !s->active.empty()) {
        if (s->auto_launch) {
            // Few resident nodes: the rounds are latency-bound and the fully parallel two-step
            // tiles finish them sooner; from kAutoWalkNodes on, four-step strip walkers (16-row
            // strips) move the state once per four steps. Every configuration gives the same bits.
            int64_t nodes = 0;
            for (const Instance* I : s->group.inst) nodes += static_cast<int64_t>(I->nx) * I->ny;
            s->group.cfg = nodes >= kAutoWalkNodes ? btrt_batch_config_t{4, 0, 0, 16} : btrt_batch_config_t{2, 0, 0, 0};
        }
        rc = group_enqueue(s->group, s->check_interval);
        for (int64_t id : s->active) {
            Instance& I = s->req[id]->inst;
            if (rc == BTRT_OK && solo(s, I)) rc = instance_steps(I, btrtk::LaunchCfg{}, s->check_interval, s->stream);
        }
        std::vector<double> res(s->active.size());
        if (rc == BTRT_OK) rc = residuals(s, res.data());
        if (rc == BTRT_OK) {
            // Every member is either kept or retired (its arena block released) in this pass, and
            // the kept list replaces the active one whatever happens: a retired request never
            // stays in the group. A request whose result cannot be read back fails alone; the
            // round reports the first such error after finishing the pass.
            std::vector<int64_t> keep;
            for (size_t k = 0; k < s->active.size(); ++k) {
                Request& r = *s->req[s->active[k]];
                r.info.steps = r.inst.step;
                r.info.residual = res[k];
                s->st.node_updates += static_cast<int64_t>(r.inst.nx) * r.inst.ny * s->check_interval;
                if (std::isnan(res[k])) {
                    retire(s, r, BTRT_REQ_FAILED, BTRT_E_UNSTABLE);
                } else if (res[k] <= r.tol || r.inst.step >= r.max_steps) {
                    r.result.resize(static_cast<size_t>(r.inst.nx) * r.inst.ny);
                    const int grc = instance_gather(r.inst, -1, r.result.data(), s->stream);
                    if (grc != BTRT_OK) {
                        r.result.clear();
                        retire(s, r, BTRT_REQ_FAILED, grc);
                        if (rc == BTRT_OK) rc = grc;
                    } else {
                        retire(s, r, BTRT_REQ_DONE, BTRT_OK);
                    }
                } else {
                    keep.push_back(r.id);
                }
            }
            s->active.swap(keep);
        }
    }
    s->st.busy_seconds += s->now() - t_in;
    if (active) *active = static_cast<int32_t>(s->active.size());
    if (queued) *queued = static_cast<int32_t>(s->queue.size());
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_server_info(const btrt_server_t* s, int64_t id, btrt_request_info_t* info)
{
    if (!s) return fail(BTRT_E_STATE, "NULL server");
    auto it = s->req.find(id);
    if (it == s->req.end() || !info) return fail(BTRT_E_INVAL, "unknown request %lld", static_cast<long long>(id));
    *info = it->second->info;
    return ok();
}

int btrt_server_result(btrt_server_t* s, int64_t id, double* phi_out)
{
    if (!s) return fail(BTRT_E_STATE, "NULL server");
    auto it = s->req.find(id);
    if (it == s->req.end() || !phi_out) return fail(BTRT_E_INVAL, "unknown request %lld", static_cast<long long>(id));
    Request& r = *it->second;
    if (r.info.status == BTRT_REQ_FAILED) {
        // A failed request has no result; collecting it releases it and reports its error.
        const int err = r.info.error != BTRT_OK ? r.info.error : BTRT_E_DEVICE;
        s->req.erase(it);
        return fail(err, "request %lld failed", static_cast<long long>(id));
    }
    if (r.info.status != BTRT_REQ_DONE) return fail(BTRT_E_INVAL, "request %lld is not done", static_cast<long long>(id));
    std::copy(r.result.begin(), r.result.end(), phi_out);
    s->req.erase(it);
    return ok();
}

int btrt_server_stats(const btrt_server_t* s, btrt_server_stats_t* st)
{
    if (!s) return fail(BTRT_E_STATE, "NULL server");
    if (!st) return fail(BTRT_E_INVAL, "stats is NULL");
    *st = s->st;
    st->active = static_cast<int32_t>(s->active.size());
    st->queued = static_cast<int32_t>(s->queue.size());
    st->memory_in_use = s->arena.used();
    st->memory_high_water = s->arena.high();
    return ok();
}

double btrt_server_clock(const btrt_server_t* s) { return s ? s->now() : NAN; }

int btrt_server_destroy(btrt_server_t* s)
{
    if (!s) return fail(BTRT_E_STATE, "NULL server");
    release(s);
    return ok();
}

}  // extern "C"
