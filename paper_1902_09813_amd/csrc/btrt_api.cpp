// C ABI of one solver handle (include/btrt.h): a single problem instance on one stream.

#include "btrt.h"
#include "btrt_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

using namespace btrth;
using btrtk::kError;
using btrtk::kReducePartials;
using btrtk::kResidual;

struct btrt {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* mem = nullptr;
    bool own_mem = false;
    int check_interval = 1000;
    int fuse = 2;  // time steps fused per sweep launch (1 or 2)
    Instance inst;
};

namespace {

int enqueue_steps(btrt* h, int64_t n)
{
    for (int64_t i = 0; i < n;) {
        const int k = (h->fuse >= 2 && n - i >= 2) ? 2 : 1;
        int rc = instance_launch(h->inst, k, h->stream);
        if (rc != BTRT_OK) return rc;
        i += k;
    }
    return BTRT_OK;
}

int reduce_sync(btrt* h, int mode, double out[kReducePartials])
{
    int rc = instance_reduce_async(h->inst, mode, h->stream);
    if (rc == BTRT_OK) rc = instance_result_async(h->inst, out, h->stream);
    if (rc != BTRT_OK) return rc;
    hipError_t e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "hipStreamSynchronize");
}

// Waits for the handle's stream, frees what the library allocated and deletes the handle.
void release(btrt* h)
{
    if (!h) return;
    DeviceGuard g(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->own_mem && h->mem) (void)hipFree(h->mem);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

}  // namespace

extern "C" {

int btrt_validate(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K, const btrt_dterm_t* D,
                  const btrt_source_t* R, const btrt_bc_t* bc, const btrt_relax_t* relax, btrt_info_t* info)
{
    Resolved r{};
    int rc = validate(grid, B, K, D, R, bc, relax, &r);
    if (rc != BTRT_OK) return rc;
    if (info) fill_info(grid, r, R ? R->kind : BTRT_SRC_NONE, info);
    return ok();
}

size_t btrt_workspace_size(const btrt_grid_t* grid, const btrt_source_t* R)
{
    if (!grid_ok(grid)) return 0;
    return layout_for(grid->nx, grid->ny, grid->precision, R ? R->kind : BTRT_SRC_NONE).total;
}

int btrt_create(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K, const btrt_dterm_t* D,
                const btrt_source_t* R, const btrt_bc_t* bc, const btrt_relax_t* relax, const double* phi0,
                btrt_t** out)
{
    if (!out) return fail(BTRT_E_INVAL, "out is NULL");
    *out = nullptr;
    Resolved r{};
    int rc = validate(grid, B, K, D, R, bc, relax, &r);
    if (rc != BTRT_OK) return rc;
    rc = validate_phi0(grid, phi0);
    if (rc != BTRT_OK) return rc;
    const size_t need = layout_for(grid->nx, grid->ny, grid->precision, R ? R->kind : BTRT_SRC_NONE).total;
    if (grid->workspace && grid->workspace_bytes < need)
        return fail(BTRT_E_NOMEM, "workspace of %zu bytes < %zu needed", grid->workspace_bytes, need);

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(BTRT_E_DEVICE, "no HIP device available");
    if (grid->device < 0 || grid->device >= ndev)
        return fail(BTRT_E_DEVICE, "device %d not in [0, %d)", grid->device, ndev);

    btrt* h = new (std::nothrow) btrt();
    if (!h) return fail(BTRT_E_NOMEM, "host allocation failed");
    h->device = grid->device;
    h->check_interval = relax->check_interval;
    {
        DeviceGuard g(h->device);
        if (g.status() != hipSuccess) {
            rc = hip_fail(g.status(), "hipSetDevice");
        } else {
            if (grid->stream) {
                h->stream = static_cast<hipStream_t>(grid->stream);
            } else {
                e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
                if (e != hipSuccess)
                    rc = hip_fail(e, "hipStreamCreate");
                else
                    h->own_stream = true;
            }
            if (rc == BTRT_OK) {
                if (grid->workspace) {
                    h->mem = static_cast<char*>(grid->workspace);
                } else if (hipMalloc(reinterpret_cast<void**>(&h->mem), need) != hipSuccess) {
                    h->mem = nullptr;
                    (void)hipGetLastError();
                    rc = fail(BTRT_E_NOMEM, "hipMalloc of %zu bytes failed", need);
                } else {
                    h->own_mem = true;
                }
            }
            if (rc == BTRT_OK) rc = instance_setup(h->inst, grid, B, K, R, bc, r, phi0, h->mem, h->stream);
        }
    }
    if (rc != BTRT_OK) {
        const std::string msg = last_error();
        release(h);
        return fail(rc, "%s", msg.c_str());
    }
    *out = h;
    return ok();
}

int btrt_step(btrt_t* h, int64_t n)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (n < 0) return fail(BTRT_E_INVAL, "n = %lld < 0", static_cast<long long>(n));
    DeviceGuard g(h->device);
    if (g.status() != hipSuccess) return hip_fail(g.status(), "hipSetDevice");
    int rc = enqueue_steps(h, n);
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_set_fusion(btrt_t* h, int32_t steps_per_launch)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (steps_per_launch != 1 && steps_per_launch != 2)
        return fail(BTRT_E_INVAL, "steps_per_launch = %d: must be 1 or 2", steps_per_launch);
    h->fuse = steps_per_launch;
    return ok();
}

int btrt_field(btrt_t* h, double* phi_out)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!phi_out) return fail(BTRT_E_INVAL, "phi_out is NULL");
    DeviceGuard g(h->device);
    int rc = instance_gather(h->inst, -1, phi_out, h->stream);
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_populations(btrt_t* h, double* f_out)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!f_out) return fail(BTRT_E_INVAL, "f_out is NULL");
    DeviceGuard g(h->device);
    const size_t nn = static_cast<size_t>(h->inst.nx) * h->inst.ny;
    for (int i = 0; i < 9; ++i) {
        int rc = instance_gather(h->inst, i, f_out + i * nn, h->stream);
        if (rc != BTRT_OK) return rc;
    }
    return ok();
}

int btrt_residual(btrt_t* h, double* out)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!out) return fail(BTRT_E_INVAL, "out is NULL");
    double v[kReducePartials];
    DeviceGuard g(h->device);
    int rc = reduce_sync(h, kResidual, v);
    if (rc != BTRT_OK) return rc;
    if (v[5] > 0) {
        *out = NAN;
        return fail(BTRT_E_UNSTABLE, "phi holds %.0f non-finite values at step %lld", v[5],
                    static_cast<long long>(h->inst.step));
    }
    *out = v[1] > 0 ? v[0] / v[1] : (v[0] > 0 ? INFINITY : 0.0);
    return ok();
}

int btrt_error(btrt_t* h, const double* ref, double out[3])
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!ref || !out) return fail(BTRT_E_INVAL, "NULL argument");
    const size_t nn = static_cast<size_t>(h->inst.nx) * h->inst.ny;
    double v[kReducePartials];
    DeviceGuard g(h->device);
    hipError_t e = hipMemcpyAsync(h->inst.mem + h->inst.L.tmp, ref, nn * sizeof(double), hipMemcpyHostToDevice,
                                  h->stream);
    if (e != hipSuccess) return hip_fail(e, "reference upload");
    int rc = reduce_sync(h, kError, v);
    if (rc != BTRT_OK) return rc;
    if (v[5] > 0) {
        out[0] = out[1] = out[2] = NAN;
        return fail(BTRT_E_UNSTABLE, "phi holds %.0f non-finite values", v[5]);
    }
    out[0] = v[0] / v[1];
    out[1] = v[4];
    out[2] = std::sqrt(v[2] / v[3]);
    return ok();
}

int btrt_solve(btrt_t* h, double tol, int64_t max_steps, int64_t* steps_taken, double* residual)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (max_steps < 0 || !(tol >= 0.0)) return fail(BTRT_E_INVAL, "bad tol or max_steps");
    int64_t done = 0;
    double res = INFINITY;
    int rc = BTRT_OK;
    while (done < max_steps) {
        const int64_t k = std::min<int64_t>(h->check_interval, max_steps - done);
        rc = btrt_step(h, k);
        if (rc != BTRT_OK) break;
        done += k;
        rc = btrt_residual(h, &res);
        if (rc != BTRT_OK || res <= tol) break;
    }
    if (steps_taken) *steps_taken = done;
    if (residual) *residual = res;
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_sync(btrt_t* h)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    DeviceGuard g(h->device);
    hipError_t e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? ok() : hip_fail(e, "hipStreamSynchronize");
}

int btrt_get_info(const btrt_t* h, btrt_info_t* info)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!info) return fail(BTRT_E_INVAL, "info is NULL");
    *info = h->inst.info;
    info->step = h->inst.step;
    return ok();
}

int btrt_destroy(btrt_t* h)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    release(h);
    return ok();
}

const char* btrt_strerror(int code)
{
    switch (code) {
        case BTRT_OK: return "ok";
        case BTRT_E_INVAL: return "invalid argument";
        case BTRT_E_NOMEM: return "out of device memory";
        case BTRT_E_DEVICE: return "HIP device error";
        case BTRT_E_UNSTABLE: return "non-finite values in phi (unstable run)";
        case BTRT_E_STATE: return "invalid handle";
        default: return "unknown error code";
    }
}

const char* btrt_last_error(void) { return last_error(); }

}  // extern "C"
