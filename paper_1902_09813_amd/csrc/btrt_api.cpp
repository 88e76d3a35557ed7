// Host runtime and C ABI of libbtrt (see include/btrt.h): problem validation, the
// constants of Eq. (30) and Eq. (62), device memory layout, and the launch sequence of
// one time step on the handle's HIP stream.

#include "btrt.h"
#include "btrt_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace btrtk;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok()
{
    g_last_error.clear();
    return BTRT_OK;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Row pitch of the device planes: rows start on 256-byte boundaries.
inline int pitch_for(int nx, int precision)
{
    const int per = static_cast<int>(kAlign / (precision == BTRT_F64 ? 8 : 4));
    return (nx + per - 1) / per * per;
}

inline bool is_finite(double v) { return std::isfinite(v); }

// Byte offsets of every buffer inside one workspace allocation.
struct Layout {
    size_t f[2], phi[2], snap, tmp, partial, result, src, src_y, total;
};

Layout layout_for(int nx, int ny, int precision, int src_kind)
{
    const size_t es = precision == BTRT_F64 ? 8 : 4;
    const size_t pitch = static_cast<size_t>(pitch_for(nx, precision));
    const size_t plane = pitch * static_cast<size_t>(ny);
    const size_t nn = static_cast<size_t>(nx) * static_cast<size_t>(ny);
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.f[0] = take(9 * plane * es);
    L.f[1] = take(9 * plane * es);
    L.phi[0] = take(plane * es);
    L.phi[1] = take(plane * es);
    // The FP64 phi snapshot of Eq. (64), dense nx*ny.
    L.snap = take(nn * 8);
    L.tmp = take(nn * 8);
    L.partial = take(static_cast<size_t>(kReduceBlocks) * kReducePartials * 8);
    L.result = take(kReducePartials * 8);
    L.src = L.src_y = 0;
    if (src_kind == BTRT_SRC_FIELD) L.src = take(plane * es);
    if (src_kind == BTRT_SRC_SIN) {
        L.src = take(static_cast<size_t>(nx) * es);
        L.src_y = take(static_cast<size_t>(ny) * es);
    }
    L.total = off;
    return L;
}

bool grid_ok(const btrt_grid_t* g)
{
    if (!g) return false;
    if (g->nx < 1 || g->ny < 1) return false;
    if (g->precision != BTRT_F64 && g->precision != BTRT_F32) return false;
    const int64_t pitch = pitch_for(g->nx, g->precision);
    // Node and in-plane indices are 32-bit in the kernels.
    if (static_cast<int64_t>(g->nx) * g->ny > INT32_MAX) return false;
    if (pitch * (static_cast<int64_t>(g->ny) + 1) > INT32_MAX) return false;
    return true;
}

struct Resolved {
    double K1[4];
    double K2[4];
    double k0;
    bool k1_per_node;
};

int validate(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K, const btrt_dterm_t* D,
             const btrt_source_t* R, const btrt_bc_t* bc, const btrt_relax_t* relax, Resolved* res)
{
    if (!grid || !B || !K || !D || !bc || !relax) return fail(BTRT_E_INVAL, "NULL argument");
    if (grid->nx < 1 || grid->ny < 1) return fail(BTRT_E_INVAL, "grid %d x %d: both sides must be >= 1", grid->nx, grid->ny);
    if (grid->precision != BTRT_F64 && grid->precision != BTRT_F32)
        return fail(BTRT_E_INVAL, "precision %d is not BTRT_F64 or BTRT_F32", grid->precision);
    if (!grid_ok(grid)) return fail(BTRT_E_INVAL, "grid %d x %d exceeds 2^31 - 1 nodes", grid->nx, grid->ny);
    for (int a = 0; a < 2; ++a)
        if (!is_finite(B->a[a]) || !is_finite(B->b[a])) return fail(BTRT_E_INVAL, "non-finite flux coefficient");
    if (!is_finite(K->k11) || !is_finite(K->k12) || !is_finite(K->k22) || !is_finite(K->beta))
        return fail(BTRT_E_INVAL, "non-finite diffusion tensor");
    if (!(K->k11 > 0.0) || !(K->k22 > 0.0) || !(K->k11 * K->k22 - K->k12 * K->k12 > 0.0))
        return fail(BTRT_E_INVAL, "diffusion tensor [[%g,%g],[%g,%g]] is not positive definite", K->k11, K->k12,
                    K->k12, K->k22);
    if (K->beta < 0.0) return fail(BTRT_E_INVAL, "beta = %g < 0", K->beta);
    if (D->kind != BTRT_D_PHI_I) return fail(BTRT_E_INVAL, "D kind %d: only D = phi I is supported", D->kind);
    for (int s = 0; s < 4; ++s) {
        if (bc->type[s] != BTRT_PERIODIC && bc->type[s] != BTRT_DIRICHLET)
            return fail(BTRT_E_INVAL, "side %d: boundary type %d", s, bc->type[s]);
        if (bc->type[s] == BTRT_DIRICHLET && !is_finite(bc->value[s]))
            return fail(BTRT_E_INVAL, "side %d: non-finite wall value", s);
    }
    if ((bc->type[0] == BTRT_PERIODIC) != (bc->type[1] == BTRT_PERIODIC) ||
        (bc->type[2] == BTRT_PERIODIC) != (bc->type[3] == BTRT_PERIODIC))
        return fail(BTRT_E_INVAL, "a periodic side must be paired with the opposite side");
    if (R) {
        if (R->kind == BTRT_SRC_FIELD) {
            if (!R->field) return fail(BTRT_E_INVAL, "source field is NULL");
            const int64_t nn = static_cast<int64_t>(grid->nx) * grid->ny;
            for (int64_t k = 0; k < nn; ++k)
                if (!is_finite(R->field[k])) return fail(BTRT_E_INVAL, "non-finite source at node %lld", (long long)k);
        } else if (R->kind == BTRT_SRC_SIN) {
            if (!is_finite(R->amp)) return fail(BTRT_E_INVAL, "non-finite source amplitude");
        } else if (R->kind != BTRT_SRC_NONE) {
            return fail(BTRT_E_INVAL, "source kind %d", R->kind);
        }
    }
    if (!(relax->k0 > 0.0 && relax->k0 < 2.0)) return fail(BTRT_E_INVAL, "k0 = %g outside (0, 2)", relax->k0);
    if (relax->check_interval < 1) return fail(BTRT_E_INVAL, "check_interval = %d < 1", relax->check_interval);

    // K1 from Eq. (30): K1 = (A / c_s^2 + I/2)^-1 with A at phi = 0. For an SPD A its
    // eigenvalues 1/(3 lambda + 1/2) lie in (0, 2).
    const double m11 = 3.0 * K->k11 + 0.5, m12 = 3.0 * K->k12, m22 = 3.0 * K->k22 + 0.5;
    const double det = m11 * m22 - m12 * m12;
    res->K1[0] = m22 / det;
    res->K1[1] = -m12 / det;
    res->K1[2] = -m12 / det;
    res->K1[3] = m11 / det;
    res->k0 = relax->k0;
    res->k1_per_node = K->beta != 0.0;

    if (relax->k2_rule == BTRT_K2_HBB) {
        // Eq. (62) removes the bounce-back slip for K1 = k1 I (Section 3).
        if (K->k12 != 0.0 || K->k11 != K->k22 || K->beta != 0.0)
            return fail(BTRT_E_INVAL, "BTRT_K2_HBB needs a constant isotropic A (k11 == k22, k12 == 0, beta == 0)");
        const double k1 = res->K1[0];
        const double k2 = 8.0 * (k1 - 2.0) / (3.0 * (k1 - 4.0));
        for (int q = 0; q < 4; ++q) res->K2[q] = k2;
    } else if (relax->k2_rule == BTRT_K2_VALUE) {
        for (int q = 0; q < 4; ++q) {
            if (!is_finite(relax->k2[q])) return fail(BTRT_E_INVAL, "non-finite k2");
            res->K2[q] = relax->k2[q];
        }
    } else {
        return fail(BTRT_E_INVAL, "k2 rule %d", relax->k2_rule);
    }
    const double kxy = 0.5 * (res->K2[1] + res->K2[2]);
    if (!(res->K2[0] > 0 && res->K2[0] < 2) || !(res->K2[3] > 0 && res->K2[3] < 2) || !(kxy > 0 && kxy < 2))
        return fail(BTRT_E_INVAL, "K2 rates (%g, %g, %g) must lie in (0, 2)", res->K2[0], kxy, res->K2[3]);
    return ok();
}

void fill_info(const btrt_grid_t* g, const Resolved& r, int src_kind, btrt_info_t* info)
{
    info->nx = g->nx;
    info->ny = g->ny;
    info->precision = g->precision;
    info->pitch = pitch_for(g->nx, g->precision);
    info->k1_per_node = r.k1_per_node ? 1 : 0;
    for (int q = 0; q < 4; ++q) {
        info->K1[q] = r.K1[q];
        info->K2[q] = r.K2[q];
    }
    info->k0 = r.k0;
    info->workspace_bytes = layout_for(g->nx, g->ny, g->precision, src_kind).total;
    // 9 population reads + 9 writes + phi(t-1) read + phi(t) write, plus a per-node source.
    const double es = g->precision == BTRT_F64 ? 8.0 : 4.0;
    info->bytes_per_node_launch = (20.0 + (src_kind == BTRT_SRC_FIELD ? 1.0 : 0.0)) * es;
    info->step = 0;
}

}  // namespace

struct btrt {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* mem = nullptr;
    bool own_mem = false;
    Layout L{};
    int nx = 0, ny = 0, pitch = 0, precision = 0, src_kind = 0;
    int64_t plane = 0;
    int cur = 0;        // buffer index holding f+(t-1) and phi(t-1)
    int64_t step = 0;
    int check_interval = 1000;
    bool k1_per_node = false;
    int fuse = 2;       // time steps fused per launch (1 or 2)
    btrt_info_t info{};
    SweepArgs<double> a64{};
    SweepArgs<float> a32{};
    double wall[4] = {0, 0, 0, 0};
    int perx = 1, pery = 1;
};

namespace {

template <typename T>
void fill_sweep(btrt* h, SweepArgs<T>& a, const btrt_flux_t* B, const btrt_diff_t* K, const btrt_source_t* R,
                const Resolved& r)
{
    a.plane = h->plane;
    a.nx = h->nx;
    a.ny = h->ny;
    a.pitch = h->pitch;
    a.perx = h->perx;
    a.pery = h->pery;
    for (int s = 0; s < 4; ++s) a.wall[s] = static_cast<T>(h->wall[s]);
    a.ax = static_cast<T>(B->a[0]);
    a.ay = static_cast<T>(B->a[1]);
    a.bx = static_cast<T>(B->b[0]);
    a.by = static_cast<T>(B->b[1]);
    a.a11 = static_cast<T>(K->k11);
    a.a12 = static_cast<T>(K->k12);
    a.a22 = static_cast<T>(K->k22);
    a.beta = static_cast<T>(K->beta);
    a.K11 = static_cast<T>(r.K1[0]);
    a.K12 = static_cast<T>(r.K1[1]);
    a.K22 = static_cast<T>(r.K1[3]);
    a.k0 = static_cast<T>(r.k0);
    a.k2xx = static_cast<T>(r.K2[0]);
    a.k2xy = static_cast<T>(0.5 * (r.K2[1] + r.K2[2]));
    a.k2yy = static_cast<T>(r.K2[3]);
    a.src_amp = static_cast<T>(R && R->kind == BTRT_SRC_SIN ? R->amp : 0.0);
    a.src = h->src_kind == kSrcNone ? nullptr : reinterpret_cast<const T*>(h->mem + h->L.src);
    a.src_y = h->src_kind == kSrcSep ? reinterpret_cast<const T*>(h->mem + h->L.src_y) : nullptr;
    // Non-temporal stores once the two population buffers exceed the 256 MB Infinity Cache.
    const double state_bytes = 2.0 * 10.0 * static_cast<double>(h->plane) * sizeof(T);
    a.nts = state_bytes > 256.0 * 1024 * 1024 ? 1 : 0;
}

template <typename T>
GatherArgs<T> gather_args(const btrt* h)
{
    GatherArgs<T> g{};
    g.fin = reinterpret_cast<const T*>(h->mem + h->L.f[h->cur]);
    g.plane = h->plane;
    g.nx = h->nx;
    g.ny = h->ny;
    g.pitch = h->pitch;
    g.perx = h->perx;
    g.pery = h->pery;
    for (int s = 0; s < 4; ++s) g.wall[s] = static_cast<T>(h->wall[s]);
    g.snap = reinterpret_cast<double*>(h->mem + h->L.snap);
    g.ref = reinterpret_cast<const double*>(h->mem + h->L.tmp);
    g.out = reinterpret_cast<double*>(h->mem + h->L.tmp);
    g.partial = reinterpret_cast<double*>(h->mem + h->L.partial);
    g.population = -1;
    return g;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(BTRT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Runs fn with the handle's device current, restoring the caller's device afterwards.
template <typename Fn>
int on_device(const btrt* h, Fn fn)
{
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != h->device) {
        hipError_t e = hipSetDevice(h->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    }
    int rc = fn();
    if (prev >= 0 && prev != h->device) (void)hipSetDevice(prev);
    return rc;
}

int reduce(btrt* h, int mode, double out[kReducePartials])
{
    hipError_t e;
    double* result = reinterpret_cast<double*>(h->mem + h->L.result);
    if (h->precision == BTRT_F64)
        e = launch_reduce<double>(gather_args<double>(h), mode, result, h->stream);
    else
        e = launch_reduce<float>(gather_args<float>(h), mode, result, h->stream);
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
    e = hipMemcpyAsync(out, result, kReducePartials * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return BTRT_OK;
}

int gather_dense(btrt* h, int population, double* host_out)
{
    hipError_t e;
    const size_t nn = static_cast<size_t>(h->nx) * h->ny;
    if (h->precision == BTRT_F64) {
        GatherArgs<double> g = gather_args<double>(h);
        g.population = population;
        e = launch_gather_field<double>(g, h->stream);
    } else {
        GatherArgs<float> g = gather_args<float>(h);
        g.population = population;
        e = launch_gather_field<float>(g, h->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "gather launch");
    e = hipMemcpyAsync(host_out, h->mem + h->L.tmp, nn * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return BTRT_OK;
}

int enqueue_steps(btrt* h, int64_t n)
{
    for (int64_t i = 0; i < n;) {
        const int k = (h->fuse >= 2 && n - i >= 2) ? 2 : 1;  // time steps in this launch
        const int nxt = h->cur ^ 1;
        hipError_t e;
        if (h->precision == BTRT_F64) {
            SweepArgs<double>& a = h->a64;
            a.fin = reinterpret_cast<const double*>(h->mem + h->L.f[h->cur]);
            a.fout = reinterpret_cast<double*>(h->mem + h->L.f[nxt]);
            a.phi_prev = reinterpret_cast<const double*>(h->mem + h->L.phi[h->cur]);
            a.phi_out = reinterpret_cast<double*>(h->mem + h->L.phi[nxt]);
            e = launch_sweep<double>(a, h->src_kind, h->k1_per_node, k, h->stream);
        } else {
            SweepArgs<float>& a = h->a32;
            a.fin = reinterpret_cast<const float*>(h->mem + h->L.f[h->cur]);
            a.fout = reinterpret_cast<float*>(h->mem + h->L.f[nxt]);
            a.phi_prev = reinterpret_cast<const float*>(h->mem + h->L.phi[h->cur]);
            a.phi_out = reinterpret_cast<float*>(h->mem + h->L.phi[nxt]);
            e = launch_sweep<float>(a, h->src_kind, h->k1_per_node, k, h->stream);
        }
        if (e != hipSuccess) return hip_fail(e, "sweep launch");
        h->cur = nxt;
        h->step += k;
        i += k;
    }
    return BTRT_OK;
}

// Waits for the handle's stream, frees what the library allocated and deletes the handle,
// with the handle's device current during the calls.
void release_on_device(btrt* h)
{
    if (!h) return;
    const int dev = h->device;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->own_mem && h->mem) (void)hipFree(h->mem);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
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
    if (!phi0) return fail(BTRT_E_INVAL, "phi0 is NULL");
    const size_t nn = static_cast<size_t>(grid->nx) * grid->ny;
    for (size_t k = 0; k < nn; ++k)
        if (!is_finite(phi0[k])) return fail(BTRT_E_INVAL, "non-finite phi0 at node %zu", k);
    const int src_kind = R ? R->kind : BTRT_SRC_NONE;
    const Layout L = layout_for(grid->nx, grid->ny, grid->precision, src_kind);
    if (grid->workspace && grid->workspace_bytes < L.total)
        return fail(BTRT_E_NOMEM, "workspace of %zu bytes < %zu needed", grid->workspace_bytes, L.total);

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(BTRT_E_DEVICE, "no HIP device available");
    if (grid->device < 0 || grid->device >= ndev)
        return fail(BTRT_E_DEVICE, "device %d not in [0, %d)", grid->device, ndev);

    btrt* h = new (std::nothrow) btrt();
    if (!h) return fail(BTRT_E_NOMEM, "host allocation failed");
    h->device = grid->device;
    h->L = L;
    h->nx = grid->nx;
    h->ny = grid->ny;
    h->precision = grid->precision;
    h->pitch = pitch_for(grid->nx, grid->precision);
    h->plane = static_cast<int64_t>(h->pitch) * grid->ny;
    h->check_interval = relax->check_interval;
    h->k1_per_node = r.k1_per_node;
    h->src_kind = src_kind == BTRT_SRC_FIELD ? kSrcField : (src_kind == BTRT_SRC_SIN ? kSrcSep : kSrcNone);
    h->perx = bc->type[0] == BTRT_PERIODIC;
    h->pery = bc->type[2] == BTRT_PERIODIC;
    for (int s = 0; s < 4; ++s) h->wall[s] = bc->type[s] == BTRT_DIRICHLET ? bc->value[s] : 0.0;
    fill_info(grid, r, src_kind, &h->info);

    rc = on_device(h, [&]() -> int {
        hipError_t err;
        if (grid->stream) {
            h->stream = static_cast<hipStream_t>(grid->stream);
        } else {
            err = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
            if (err != hipSuccess) return hip_fail(err, "hipStreamCreate");
            h->own_stream = true;
        }
        if (grid->workspace) {
            h->mem = static_cast<char*>(grid->workspace);
        } else {
            err = hipMalloc(reinterpret_cast<void**>(&h->mem), L.total);
            if (err != hipSuccess) {
                h->mem = nullptr;
                (void)hipGetLastError();
                return fail(BTRT_E_NOMEM, "hipMalloc of %zu bytes failed", L.total);
            }
            h->own_mem = true;
        }
        if (reinterpret_cast<uintptr_t>(h->mem) % kAlign != 0)
            return fail(BTRT_E_INVAL, "workspace must be %zu-byte aligned", kAlign);

        const size_t es = h->precision == BTRT_F64 ? 8 : 4;
        double* tmp = reinterpret_cast<double*>(h->mem + L.tmp);
        // Source of Eq. (8): a per-node field, or separable sin tables at cell centres.
        if (src_kind == BTRT_SRC_FIELD) {
            err = hipMemcpyAsync(tmp, R->field, nn * sizeof(double), hipMemcpyHostToDevice, h->stream);
            if (err != hipSuccess) return hip_fail(err, "source upload");
            err = h->precision == BTRT_F64
                      ? launch_convert<double>(tmp, reinterpret_cast<double*>(h->mem + L.src), h->nx, h->ny, h->pitch,
                                               h->stream)
                      : launch_convert<float>(tmp, reinterpret_cast<float*>(h->mem + L.src), h->nx, h->ny, h->pitch,
                                              h->stream);
            if (err != hipSuccess) return hip_fail(err, "source convert");
            err = hipStreamSynchronize(h->stream);
            if (err != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
        } else if (src_kind == BTRT_SRC_SIN) {
            const double pi = 3.14159265358979323846;
            std::vector<double> sx(h->nx), sy(h->ny);
            for (int i = 0; i < h->nx; ++i) sx[i] = std::sin(R->kx * pi * (i + 0.5) / h->nx);
            for (int j = 0; j < h->ny; ++j) sy[j] = std::sin(R->ky * pi * (j + 0.5) / h->ny);
            std::vector<float> fx, fy;
            const void* px = sx.data();
            const void* py = sy.data();
            if (h->precision == BTRT_F32) {
                fx.assign(sx.begin(), sx.end());
                fy.assign(sy.begin(), sy.end());
                px = fx.data();
                py = fy.data();
            }
            err = hipMemcpy(h->mem + L.src, px, h->nx * es, hipMemcpyHostToDevice);
            if (err == hipSuccess) err = hipMemcpy(h->mem + L.src_y, py, h->ny * es, hipMemcpyHostToDevice);
            if (err != hipSuccess) return hip_fail(err, "source table upload");
        }

        if (h->precision == BTRT_F64)
            fill_sweep<double>(h, h->a64, B, K, R, r);
        else
            fill_sweep<float>(h, h->a32, B, K, R, r);

        // phi0 -> device, f+(-1) so that the first pull gives f^eq(phi0), phi(-1) := phi0,
        // and the Eq. (64) snapshot := phi0.
        err = hipMemcpyAsync(tmp, phi0, nn * sizeof(double), hipMemcpyHostToDevice, h->stream);
        if (err != hipSuccess) return hip_fail(err, "phi0 upload");
        if (h->precision == BTRT_F64)
            err = launch_init<double>(nullptr, reinterpret_cast<double*>(h->mem + L.f[0]),
                                      reinterpret_cast<double*>(h->mem + L.phi[0]), tmp, h->plane, h->nx, h->ny,
                                      h->pitch, h->perx, h->pery, h->wall, B->a[0], B->a[1], B->b[0], B->b[1],
                                      h->stream);
        else
            err = launch_init<float>(nullptr, reinterpret_cast<float*>(h->mem + L.f[0]),
                                     reinterpret_cast<float*>(h->mem + L.phi[0]), tmp, h->plane, h->nx, h->ny,
                                     h->pitch, h->perx, h->pery, h->wall, B->a[0], B->a[1], B->b[0], B->b[1],
                                     h->stream);
        if (err != hipSuccess) return hip_fail(err, "init launch");
        err = hipMemcpyAsync(h->mem + L.snap, tmp, nn * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
        if (err != hipSuccess) return hip_fail(err, "snapshot copy");
        err = hipStreamSynchronize(h->stream);
        if (err != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
        h->cur = 0;
        h->step = 0;
        return BTRT_OK;
    });
    if (rc != BTRT_OK) {
        release_on_device(h);
        return rc;
    }
    *out = h;
    return ok();
}

int btrt_step(btrt_t* h, int64_t n)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (n < 0) return fail(BTRT_E_INVAL, "n = %lld < 0", static_cast<long long>(n));
    int rc = on_device(h, [&]() { return enqueue_steps(h, n); });
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
    int rc = on_device(h, [&]() { return gather_dense(h, -1, phi_out); });
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_populations(btrt_t* h, double* f_out)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!f_out) return fail(BTRT_E_INVAL, "f_out is NULL");
    const size_t nn = static_cast<size_t>(h->nx) * h->ny;
    int rc = on_device(h, [&]() {
        for (int i = 0; i < 9; ++i) {
            int r = gather_dense(h, i, f_out + i * nn);
            if (r != BTRT_OK) return r;
        }
        return static_cast<int>(BTRT_OK);
    });
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_residual(btrt_t* h, double* out)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!out) return fail(BTRT_E_INVAL, "out is NULL");
    double v[kReducePartials];
    int rc = on_device(h, [&]() { return reduce(h, kResidual, v); });
    if (rc != BTRT_OK) return rc;
    if (v[5] > 0) {
        *out = NAN;
        return fail(BTRT_E_UNSTABLE, "phi holds %.0f non-finite values at step %lld", v[5],
                    static_cast<long long>(h->step));
    }
    *out = v[1] > 0 ? v[0] / v[1] : (v[0] > 0 ? INFINITY : 0.0);
    return ok();
}

int btrt_error(btrt_t* h, const double* ref, double out[3])
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!ref || !out) return fail(BTRT_E_INVAL, "NULL argument");
    const size_t nn = static_cast<size_t>(h->nx) * h->ny;
    double v[kReducePartials];
    int rc = on_device(h, [&]() -> int {
        hipError_t e = hipMemcpyAsync(h->mem + h->L.tmp, ref, nn * sizeof(double), hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) return hip_fail(e, "reference upload");
        return reduce(h, kError, v);
    });
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
    int rc = on_device(h, [&]() -> int {
        hipError_t e = hipStreamSynchronize(h->stream);
        return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "hipStreamSynchronize");
    });
    return rc == BTRT_OK ? ok() : rc;
}

int btrt_get_info(const btrt_t* h, btrt_info_t* info)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!info) return fail(BTRT_E_INVAL, "info is NULL");
    *info = h->info;
    info->step = h->step;
    return ok();
}

int btrt_destroy(btrt_t* h)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    release_on_device(h);
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

const char* btrt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
