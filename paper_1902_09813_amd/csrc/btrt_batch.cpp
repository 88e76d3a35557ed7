// Batched C ABI (include/btrt.h, btrt_batch_*): a fixed set of independent problem instances
// of different sizes in one arena, advanced together (btrt_group.cpp).

#include "btrt.h"
#include "btrt_host.h"

#include <hip/hip_runtime.h>

#include <new>
#include <string>
#include <vector>

using namespace btrth;

struct btrt_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* arena = nullptr;
    std::vector<Instance> inst;
    Group group;
};

namespace {

void release(btrt_batch* b)
{
    if (!b) return;
    DeviceGuard g(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    group_free(b->group);
    if (b->arena) (void)hipFree(b->arena);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
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
        if (precision != BTRT_F64 && precision != BTRT_F32)
            return fail(BTRT_E_INVAL, "batches take BTRT_F64 or BTRT_F32 storage");
        if (res[i].afield || res[i].growth != 0.0 || res[i].gen)
            return fail(BTRT_E_INVAL,
                        "instance %d: batches take no A0 field, growing source, power-law flux or phi-dependent source",
                        i);
        offs[i] = total;
        total += align_up(layout_for(p.grid.nx, p.grid.ny, precision, p.R.kind).total);
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(BTRT_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(BTRT_E_DEVICE, "device %d not in [0, %d)", device, ndev);

    btrt_batch* b = new (std::nothrow) btrt_batch();
    if (!b) return fail(BTRT_E_NOMEM, "host allocation failed");
    b->device = device;
    b->inst.resize(n);
    int rc = BTRT_OK;
    {
        DeviceGuard g(device);
        if (stream) {
            b->stream = static_cast<hipStream_t>(stream);
        } else if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) {
            rc = hip_fail(e, "hipStreamCreate");
        } else {
            b->own_stream = true;
        }
        if (rc == BTRT_OK && hipMalloc(reinterpret_cast<void**>(&b->arena), total) != hipSuccess) {
            b->arena = nullptr;
            (void)hipGetLastError();
            rc = fail(BTRT_E_NOMEM, "hipMalloc of %zu bytes failed", total);
        }
        if (rc == BTRT_OK) rc = group_init(b->group, device, b->stream, precision, n);
        for (int i = 0; i < n && rc == BTRT_OK; ++i) {
            const btrt_problem_t& p = problems[i];
            rc = instance_setup(b->inst[i], &p.grid, &p.B, &p.K, &p.R, &p.bc, res[i], p.phi0, b->arena + offs[i],
                                b->stream);
            b->group.inst.push_back(&b->inst[i]);
        }
        if (rc == BTRT_OK) rc = group_upload(b->group);
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
    int rc = group_enqueue(b->group, n);
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_batch_field(btrt_batch_t* b, int32_t i, double* phi_out)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (i < 0 || i >= static_cast<int>(b->inst.size()) || !phi_out)
        return fail(BTRT_E_INVAL, "bad instance index or NULL output");
    DeviceGuard g(b->device);
    int rc = instance_gather(b->inst[i], -1, phi_out, b->stream);
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_batch_residual(btrt_batch_t* b, double* out)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (!out) return fail(BTRT_E_INVAL, "out is NULL");
    DeviceGuard g(b->device);
    int bad = 0;
    int rc = group_residuals(b->group, out, &bad);
    if (rc != BTRT_OK) return rc;
    if (bad) return fail(BTRT_E_UNSTABLE, "%d instance(s) hold non-finite values", bad);
    return ok();
}

int btrt_batch_set_config(btrt_batch_t* b, const btrt_batch_config_t* cfg)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (!config_ok(cfg)) return fail(BTRT_E_INVAL, "invalid batch configuration");
    b->group.cfg = *cfg;
    return ok();
}

int btrt_batch_get_config(const btrt_batch_t* b, btrt_batch_config_t* cfg)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (!cfg) return fail(BTRT_E_INVAL, "cfg is NULL");
    *cfg = b->group.cfg;
    return ok();
}

int btrt_batch_tune(btrt_batch_t* b, int64_t max_steps, btrt_batch_config_t* best, int64_t* steps_used)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (max_steps < 0) return fail(BTRT_E_INVAL, "max_steps < 0");
    DeviceGuard g(b->device);
    int rc = group_tune(b->group, max_steps, best, steps_used);
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_batch_steps(const btrt_batch_t* b, int64_t* steps)
{
    if (!b) return fail(BTRT_E_STATE, "NULL batch");
    if (!steps) return fail(BTRT_E_INVAL, "steps is NULL");
    *steps = b->inst.empty() ? 0 : b->inst[0].step;
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
