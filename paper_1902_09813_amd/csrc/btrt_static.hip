// btrt_solve_static (include/btrt.h): one solve of a small problem without any device
// allocation, for callers that cannot allocate (tight serving loops, harnesses that forbid
// hipMalloc). It is btrt_create + btrt_solve + btrt_field + btrt_destroy in one call, with the
// handle's whole workspace (populations, phi planes, the Eq. (64) snapshot, staging and the
// reduction partials) in a fixed device array instead of memory the library allocates.

#include "btrt.h"
#include "btrt_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

using namespace btrth;

// The workspace of btrt_solve_static calls, laid out as a handle's (layout_for). Every device the
// library runs on holds its own copy until the process ends; each call overwrites it.
static __device__ __align__(256) char scratch[BTRT_STATIC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_lock[kMaxDevices];         // one call at a time per device (the array is shared)
char* g_addr[kMaxDevices] = {};         // device address of `scratch` per device, once known
std::mutex g_addr_lock;

// Device address of `scratch` on `device`, which must be current: host code must never use the
// array's name as an address (it names a host-side stand-in), so the address is looked up once
// per device and kept.
int scratch_on(int device, char** out)
{
    std::lock_guard<std::mutex> guard(g_addr_lock);
    if (!g_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_addr[device] = static_cast<char*>(p);
    }
    *out = g_addr[device];
    return BTRT_OK;
}

// The solve on a workspace at mem (btrt_solve's loop: check_interval steps, then the Eq. (64)
// residual, until it is <= tol or max_steps are done), then phi into phi_out.
int solve_in(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K, const btrt_source_t* R,
             const btrt_bc_t* bc, const btrt_relax_t* relax, const Resolved& r, const double* phi0, double tol,
             int64_t max_steps, char* mem, hipStream_t s, double* phi_out, int64_t* steps_taken, double* residual)
{
    Instance I;
    int rc = instance_setup(I, grid, B, K, R, bc, r, phi0, mem, s);
    if (rc != BTRT_OK) return rc;
    int64_t done = 0;
    double res = INFINITY;
    while (done < max_steps && rc == BTRT_OK) {
        const int64_t k = std::min<int64_t>(relax->check_interval, max_steps - done);
        rc = instance_steps(I, btrtk::LaunchCfg{}, k, s);
        if (rc != BTRT_OK) break;
        done += k;
        double v[btrtk::kReducePartials];
        rc = instance_reduce_async(I, btrtk::kResidual, s);
        if (rc == BTRT_OK) rc = instance_result_async(I, v, s);
        if (rc != BTRT_OK) break;
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "hipStreamSynchronize");
            break;
        }
        if (v[5] > 0) {
            res = NAN;
            rc = fail(BTRT_E_UNSTABLE, "phi holds %.0f non-finite values at step %lld", v[5],
                      static_cast<long long>(I.step));
            break;
        }
        res = v[1] > 0 ? v[0] / v[1] : (v[0] > 0 ? INFINITY : 0.0);
        if (res <= tol) break;
    }
    if (steps_taken) *steps_taken = done;
    if (residual) *residual = res;
    if (rc != BTRT_OK && rc != BTRT_E_UNSTABLE) return rc;
    // The field, also after a non-finite residual (for inspection, as btrt_field would give it).
    const int grc = instance_gather(I, -1, phi_out, s);
    return rc != BTRT_OK ? rc : grc;
}

}  // namespace

extern "C" int btrt_solve_static(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K,
                                 const btrt_dterm_t* D, const btrt_source_t* R, const btrt_bc_t* bc,
                                 const btrt_relax_t* relax, const double* phi0, double tol, int64_t max_steps,
                                 double* phi_out, int64_t* steps_taken, double* residual)
{
    Resolved r{};
    int rc = validate(grid, B, K, D, R, bc, relax, &r);
    if (rc != BTRT_OK) return rc;
    rc = validate_phi0(grid, phi0);
    if (rc != BTRT_OK) return rc;
    if (!phi_out) return fail(BTRT_E_INVAL, "phi_out is NULL");
    if (max_steps < 0 || !(tol >= 0.0)) return fail(BTRT_E_INVAL, "bad tol or max_steps");
    if (grid->workspace)
        return fail(BTRT_E_INVAL, "btrt_solve_static keeps its buffers in the library's fixed array: workspace must be NULL");
    const size_t need = layout_for(grid->nx, grid->ny, grid->precision, R ? R->kind : BTRT_SRC_NONE, r.afield).total;
    if (need > static_cast<size_t>(BTRT_STATIC_BYTES))
        return fail(BTRT_E_INVAL,
                    "a %d x %d grid (precision %d) needs %zu bytes of device memory, more than the %zu bytes "
                    "btrt_solve_static holds; use btrt_create",
                    grid->nx, grid->ny, grid->precision, need, static_cast<size_t>(BTRT_STATIC_BYTES));
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(BTRT_E_DEVICE, "no HIP device available");
    if (grid->device < 0 || grid->device >= ndev || grid->device >= kMaxDevices)
        return fail(BTRT_E_DEVICE, "device %d not in [0, %d)", grid->device, std::min(ndev, kMaxDevices));

    std::lock_guard<std::mutex> one_at_a_time(g_lock[grid->device]);
    DeviceGuard g(grid->device);
    if (g.status() != hipSuccess) return hip_fail(g.status(), "hipSetDevice");
    char* mem = nullptr;
    rc = scratch_on(grid->device, &mem);
    if (rc != BTRT_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(grid->stream);  // NULL: the device's null stream
    rc = solve_in(grid, B, K, R, bc, relax, r, phi0, tol, max_steps, mem, s, phi_out, steps_taken, residual);
    // Nothing of this call may still run on the array when the next call takes it.
    (void)hipStreamSynchronize(s);
    return rc == BTRT_OK ? ok() : rc;
}
