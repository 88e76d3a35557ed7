// C ABI of the D3Q19 solver (include/btrt3.h): validation, constants of Eq. (30) and Eq. (62)
// for 3x3 blocks, device memory of one problem, and the launch sequence.

#include "btrt3.h"
#include "btrt3_internal.h"
#include "btrt_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

using namespace btrth;
using namespace btrt3k;

namespace {

inline bool is_fin(double v) { return std::isfinite(v); }

struct Layout3 {
    size_t f[2], phi[2], snap, tmp, partial, result, src, total;
};

Layout3 layout3(int nx, int ny, int nz, int precision, bool src)
{
    const size_t es = precision == BTRT_F64 ? 8 : 4;
    const size_t plane = static_cast<size_t>(pitch_for(nx, precision)) * ny * nz;
    const size_t nn = static_cast<size_t>(nx) * ny * nz;
    Layout3 L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.f[0] = take(kQ * plane * es);
    L.f[1] = take(kQ * plane * es);
    L.phi[0] = take(plane * es);
    L.phi[1] = take(plane * es);
    L.snap = take(nn * 8);
    L.tmp = take(nn * 8);
    L.partial = take(static_cast<size_t>(kReduceBlocks3) * kPartials * 8);
    L.result = take(kPartials * 8);
    L.src = src ? take(plane * es) : 0;
    L.total = off;
    return L;
}

// Symmetric 3x3 inverse of (3 A + I/2) for A given as (a11, a12, a13, a22, a23, a33): Eq. (30).
void k1_of(const double A[6], double K[9])
{
    const double m11 = 3 * A[0] + 0.5, m12 = 3 * A[1], m13 = 3 * A[2], m22 = 3 * A[3] + 0.5, m23 = 3 * A[4],
                 m33 = 3 * A[5] + 0.5;
    const double c11 = m22 * m33 - m23 * m23, c12 = m13 * m23 - m12 * m33, c13 = m12 * m23 - m13 * m22;
    const double det = m11 * c11 + m12 * c12 + m13 * c13;
    K[0] = c11 / det;
    K[1] = K[3] = c12 / det;
    K[2] = K[6] = c13 / det;
    K[4] = (m11 * m33 - m13 * m13) / det;
    K[5] = K[7] = (m12 * m13 - m11 * m23) / det;
    K[8] = (m11 * m22 - m12 * m12) / det;
}

struct Resolved3 {
    double K1[9], K2[9], k0;
    bool k1_per_node;
};

bool grid3_ok(const btrt3_grid_t* g)
{
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return false;
    if (g->precision != BTRT_F64 && g->precision != BTRT_F32) return false;
    const int64_t plane = static_cast<int64_t>(pitch_for(g->nx, g->precision)) * g->ny * g->nz;
    return plane * kQ <= INT32_MAX && static_cast<int64_t>(g->nx) * g->ny * g->nz <= INT32_MAX;
}

int validate3(const btrt3_grid_t* grid, const btrt3_flux_t* B, const btrt3_diff_t* K, const btrt3_source_t* R,
              const btrt3_bc_t* bc, const btrt3_relax_t* relax, Resolved3* res)
{
    if (!grid || !B || !K || !bc || !relax) return fail(BTRT_E_INVAL, "NULL argument");
    if (grid->precision != BTRT_F64 && grid->precision != BTRT_F32)
        return fail(BTRT_E_INVAL, "precision %d: the D3Q19 solver takes BTRT_F64 or BTRT_F32", grid->precision);
    if (!grid3_ok(grid))
        return fail(BTRT_E_INVAL, "grid %d x %d x %d: sides must be >= 1 and 19 padded planes < 2^31 elements",
                    grid->nx, grid->ny, grid->nz);
    for (int c = 0; c < 3; ++c)
        if (!is_fin(B->a[c]) || !is_fin(B->b[c])) return fail(BTRT_E_INVAL, "non-finite flux coefficient");
    for (int c = 0; c < 6; ++c)
        if (!is_fin(K->a0[c])) return fail(BTRT_E_INVAL, "non-finite diffusion tensor");
    if (!is_fin(K->beta) || K->beta < 0.0) return fail(BTRT_E_INVAL, "beta = %g: must be finite and >= 0", K->beta);
    // Positive definite: leading principal minors > 0.
    const double* a = K->a0;
    const double m2 = a[0] * a[3] - a[1] * a[1];
    const double m3 = a[0] * (a[3] * a[5] - a[4] * a[4]) - a[1] * (a[1] * a[5] - a[4] * a[2]) +
                      a[2] * (a[1] * a[4] - a[3] * a[2]);
    if (!(a[0] > 0.0) || !(m2 > 0.0) || !(m3 > 0.0))
        return fail(BTRT_E_INVAL, "diffusion tensor is not positive definite");
    for (int s = 0; s < 6; ++s) {
        if (bc->type[s] != BTRT_PERIODIC && bc->type[s] != BTRT_DIRICHLET)
            return fail(BTRT_E_INVAL, "face %d: boundary type %d", s, bc->type[s]);
        if (bc->type[s] == BTRT_DIRICHLET && !is_fin(bc->value[s]))
            return fail(BTRT_E_INVAL, "face %d: non-finite wall value", s);
    }
    for (int c = 0; c < 3; ++c)
        if ((bc->type[2 * c] == BTRT_PERIODIC) != (bc->type[2 * c + 1] == BTRT_PERIODIC))
            return fail(BTRT_E_INVAL, "a periodic face must be paired with the opposite face");
    if (R) {
        if (R->kind == BTRT_SRC_FIELD) {
            if (!R->field) return fail(BTRT_E_INVAL, "source field is NULL");
            const int64_t nn = static_cast<int64_t>(grid->nx) * grid->ny * grid->nz;
            for (int64_t k = 0; k < nn; ++k)
                if (!is_fin(R->field[k])) return fail(BTRT_E_INVAL, "non-finite source at node %lld", (long long)k);
        } else if (R->kind != BTRT_SRC_NONE) {
            return fail(BTRT_E_INVAL, "source kind %d: the D3Q19 solver takes BTRT_SRC_NONE or BTRT_SRC_FIELD",
                        R->kind);
        }
    }
    if (!(relax->k0 > 0.0 && relax->k0 < 2.0)) return fail(BTRT_E_INVAL, "k0 = %g outside (0, 2)", relax->k0);
    if (relax->check_interval < 1) return fail(BTRT_E_INVAL, "check_interval = %d < 1", relax->check_interval);
    k1_of(K->a0, res->K1);
    res->k0 = relax->k0;
    res->k1_per_node = K->beta != 0.0;
    if (relax->k2_rule == BTRT_K2_HBB) {
        // Eq. (62); the slip of Eq. (61) holds on D3Q19 as on D2Q9.
        if (a[1] != 0.0 || a[2] != 0.0 || a[4] != 0.0 || a[0] != a[3] || a[0] != a[5] || K->beta != 0.0)
            return fail(BTRT_E_INVAL, "BTRT_K2_HBB needs a constant isotropic A");
        const double k1 = res->K1[0];
        for (int q = 0; q < 9; ++q) res->K2[q] = 8.0 * (k1 - 2.0) / (3.0 * (k1 - 4.0));
    } else if (relax->k2_rule == BTRT_K2_VALUE) {
        for (int q = 0; q < 9; ++q) {
            if (!is_fin(relax->k2[q])) return fail(BTRT_E_INVAL, "non-finite k2");
            res->K2[q] = relax->k2[q];
        }
    } else {
        return fail(BTRT_E_INVAL, "k2 rule %d", relax->k2_rule);
    }
    const double* k2 = res->K2;
    const double rates[6] = {k2[0], k2[4], k2[8], 0.5 * (k2[1] + k2[3]), 0.5 * (k2[2] + k2[6]), 0.5 * (k2[5] + k2[7])};
    for (double r : rates)
        if (!(r > 0.0 && r < 2.0)) return fail(BTRT_E_INVAL, "K2 rate %g outside (0, 2)", r);
    return ok();
}

void fill_info3(const btrt3_grid_t* g, const Resolved3& r, bool src, btrt3_info_t* info)
{
    info->nx = g->nx;
    info->ny = g->ny;
    info->nz = g->nz;
    info->precision = g->precision;
    info->pitch = pitch_for(g->nx, g->precision);
    info->k1_per_node = r.k1_per_node ? 1 : 0;
    for (int q = 0; q < 9; ++q) {
        info->K1[q] = r.K1[q];
        info->K2[q] = r.K2[q];
    }
    info->k0 = r.k0;
    info->device_bytes = layout3(g->nx, g->ny, g->nz, g->precision, src).total;
    const double es = g->precision == BTRT_F64 ? 8.0 : 4.0;
    info->bytes_per_node_launch = (2.0 * kQ + 2.0 + (src ? 1.0 : 0.0)) * es;
    info->step = 0;
}

}  // namespace

struct btrt3 {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* mem = nullptr;
    Layout3 L{};
    int precision = BTRT_F64;
    int nx = 0, ny = 0, nz = 0, pitch = 0;
    bool src = false, k1_per_node = false;
    int cur = 0;
    int64_t step = 0;
    int check_interval = 1000;
    int cus = 256;                          // compute units of the device
    btrt3_launch_t launch{0, 0, 0};         // as set (0: automatic)
    Sweep3<double> a64{};
    Sweep3<float> a32{};
    btrt3_info_t info{};
};

namespace {

template <typename T>
Sweep3<T> args(const btrt3* h, int parity)
{
    Sweep3<T> a;
    if constexpr (sizeof(T) == 8)
        a = h->a64;
    else
        a = h->a32;
    a.fin = reinterpret_cast<const T*>(h->mem + h->L.f[parity]);
    a.fout = reinterpret_cast<T*>(h->mem + h->L.f[parity ^ 1]);
    a.phi_prev = reinterpret_cast<const T*>(h->mem + h->L.phi[parity]);
    a.phi_out = reinterpret_cast<T*>(h->mem + h->L.phi[parity ^ 1]);
    return a;
}

template <typename T>
void fill3(btrt3* h, Sweep3<T>& a, const btrt3_flux_t* B, const btrt3_diff_t* K, const btrt3_bc_t* bc,
           const Resolved3& r)
{
    a.plane = static_cast<int64_t>(h->pitch) * h->ny * h->nz;
    a.nx = h->nx;
    a.ny = h->ny;
    a.nz = h->nz;
    a.pitch = h->pitch;
    a.slab = h->pitch * h->ny;
    for (int c = 0; c < 3; ++c) {
        a.per[c] = bc->type[2 * c] == BTRT_PERIODIC ? 1 : 0;
        a.a[c] = static_cast<T>(B->a[c]);
        a.b[c] = static_cast<T>(B->b[c]);
    }
    for (int s = 0; s < 6; ++s) a.wall[s] = static_cast<T>(bc->type[s] == BTRT_DIRICHLET ? bc->value[s] : 0.0);
    for (int c = 0; c < 6; ++c) a.A0[c] = static_cast<T>(K->a0[c]);
    a.beta = static_cast<T>(K->beta);
    const double k1s[6] = {r.K1[0], r.K1[1], r.K1[2], r.K1[4], r.K1[5], r.K1[8]};
    for (int c = 0; c < 6; ++c) a.K1[c] = static_cast<T>(k1s[c]);
    a.k0 = static_cast<T>(r.k0);
    const double cq[6] = {1.5, -4.5, 3.0, -3.0, 9.0, -9.0};
    for (int c = 0; c < 6; ++c) a.cq[c] = static_cast<T>(cq[c]);
    const double* k2 = r.K2;
    const double q2[6] = {k2[0], 0.5 * (k2[1] + k2[3]), 0.5 * (k2[2] + k2[6]), k2[4], 0.5 * (k2[5] + k2[7]), k2[8]};
    for (int c = 0; c < 6; ++c) a.q2[c] = static_cast<T>(q2[c]);
    a.src = h->src ? reinterpret_cast<const T*>(h->mem + h->L.src) : nullptr;
    // Non-temporal stores once the two copies of the state exceed the 256 MB Infinity Cache.
    const double state = 2.0 * static_cast<double>(a.plane) * (kQ + 1) * sizeof(T);
    a.nts = state > 256.0 * 1024 * 1024 ? 1 : 0;
}

template <typename T>
Gather3<T> gather_args(const btrt3* h)
{
    Gather3<T> g{};
    g.s = args<T>(h, h->cur);
    g.snap = reinterpret_cast<double*>(h->mem + h->L.snap);
    g.ref = reinterpret_cast<const double*>(h->mem + h->L.tmp);
    g.out = reinterpret_cast<double*>(h->mem + h->L.tmp);
    g.partial = reinterpret_cast<double*>(h->mem + h->L.partial);
    g.population = -1;
    return g;
}

void release(btrt3* h)
{
    if (!h) return;
    DeviceGuard g(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->mem) (void)hipFree(h->mem);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int setup(btrt3* h, const btrt3_flux_t* B, const btrt3_diff_t* K, const btrt3_source_t* R, const btrt3_bc_t* bc,
          const Resolved3& r, const double* phi0)
{
    const size_t nn = static_cast<size_t>(h->nx) * h->ny * h->nz;
    double* tmp = reinterpret_cast<double*>(h->mem + h->L.tmp);
    hipError_t e = hipSuccess;
    if (h->precision == BTRT_F64)
        fill3<double>(h, h->a64, B, K, bc, r);
    else
        fill3<float>(h, h->a32, B, K, bc, r);
    if (h->src) {
        e = hipMemcpyAsync(tmp, R->field, nn * sizeof(double), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = h->precision == BTRT_F64
                    ? launch3_convert<double>(tmp, reinterpret_cast<double*>(h->mem + h->L.src), h->nx, h->ny, h->nz,
                                              h->pitch, h->stream)
                    : launch3_convert<float>(tmp, reinterpret_cast<float*>(h->mem + h->L.src), h->nx, h->ny, h->nz,
                                             h->pitch, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "source upload");
    }
    e = hipMemcpyAsync(tmp, phi0, nn * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "phi0 upload");
    // The init writes through the outputs of parity 1: f[0] and phi[0].
    e = h->precision == BTRT_F64 ? launch3_init<double>(args<double>(h, 1), tmp, h->stream)
                                 : launch3_init<float>(args<float>(h, 1), tmp, h->stream);
    if (e != hipSuccess) return hip_fail(e, "init launch");
    e = hipMemcpyAsync(h->mem + h->L.snap, tmp, nn * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "init");
}

// Launch shape with the automatic fields resolved for the handle's grid.
btrt3_launch_t resolve_launch(const btrt3* h)
{
    btrt3_launch_t c = h->launch;
    const int64_t nodes = static_cast<int64_t>(h->nx) * h->ny * h->nz;
    if (c.steps_per_launch == 0) c.steps_per_launch = nodes >= (int64_t(1) << 21) ? 2 : 1;
    if (c.tile == 0) c.tile = 1;
    if (c.z_chunk == 0) {
        // Workgroups run in rounds of (compute units x workgroups each holds); a workgroup walks its
        // chunk plus one plane on each side. Among chunks of 16 .. 64 planes take the one with the
        // fewest rounds x (chunk + 2) planes walked: the last round of a launch is then nearly
        // full (256^3: 32 planes in FP64, one workgroup per CU, 16 in FP32, two per CU; 27, the
        // earlier rule of about eight workgroups per CU, left 0.4 of a round and ran 2-4 % slower).
        const int* per = h->precision == BTRT_F64 ? h->a64.per : h->a32.per;
        const bool walls = !(per[0] && per[1] && per[2]);
        const int per_cu = h->precision == BTRT_F64 ? sweep2_blocks_per_cu<double>(walls, h->src, h->k1_per_node, c.tile)
                                                    : sweep2_blocks_per_cu<float>(walls, h->src, h->k1_per_node, c.tile);
        const int64_t slots = static_cast<int64_t>(h->cus) * per_cu;
        int64_t best = -1;
        c.z_chunk = h->nz;
        for (int zc = 16; zc <= 64; ++zc) {
            const int use = std::min(zc, h->nz);
            const int64_t rounds = (sweep2_workgroups(h->nx, h->ny, h->nz, c.tile, use) + slots - 1) / slots;
            const int64_t cost = rounds * (use + 2);
            if (best < 0 || cost < best) {
                best = cost;
                c.z_chunk = use;
            }
            if (use == h->nz) break;
        }
    }
    return c;
}

int reduce_sync(btrt3* h, int mode, double out[kPartials])
{
    double* result = reinterpret_cast<double*>(h->mem + h->L.result);
    hipError_t e = h->precision == BTRT_F64 ? launch3_reduce<double>(gather_args<double>(h), mode, result, h->stream)
                                            : launch3_reduce<float>(gather_args<float>(h), mode, result, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, result, kPartials * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "reduction");
}

int gather_sync(btrt3* h, int population, double* host_out)
{
    const size_t nn = static_cast<size_t>(h->nx) * h->ny * h->nz;
    hipError_t e;
    if (h->precision == BTRT_F64) {
        Gather3<double> g = gather_args<double>(h);
        g.population = population;
        e = launch3_gather<double>(g, h->stream);
    } else {
        Gather3<float> g = gather_args<float>(h);
        g.population = population;
        e = launch3_gather<float>(g, h->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(host_out, h->mem + h->L.tmp, nn * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "field read");
}

}  // namespace

extern "C" {

int btrt3_validate(const btrt3_grid_t* grid, const btrt3_flux_t* B, const btrt3_diff_t* K, const btrt3_source_t* R,
                   const btrt3_bc_t* bc, const btrt3_relax_t* relax, btrt3_info_t* info)
{
    Resolved3 r{};
    int rc = validate3(grid, B, K, R, bc, relax, &r);
    if (rc != BTRT_OK) return rc;
    if (info) fill_info3(grid, r, R && R->kind == BTRT_SRC_FIELD, info);
    return ok();
}

int btrt3_create(const btrt3_grid_t* grid, const btrt3_flux_t* B, const btrt3_diff_t* K, const btrt3_source_t* R,
                 const btrt3_bc_t* bc, const btrt3_relax_t* relax, const double* phi0, btrt3_t** out)
{
    if (!out) return fail(BTRT_E_INVAL, "out is NULL");
    *out = nullptr;
    Resolved3 r{};
    int rc = validate3(grid, B, K, R, bc, relax, &r);
    if (rc != BTRT_OK) return rc;
    if (!phi0) return fail(BTRT_E_INVAL, "phi0 is NULL");
    const size_t nn = static_cast<size_t>(grid->nx) * grid->ny * grid->nz;
    for (size_t k = 0; k < nn; ++k)
        if (!is_fin(phi0[k])) return fail(BTRT_E_INVAL, "non-finite phi0 at node %zu", k);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(BTRT_E_DEVICE, "no HIP device available");
    if (grid->device < 0 || grid->device >= ndev)
        return fail(BTRT_E_DEVICE, "device %d not in [0, %d)", grid->device, ndev);

    btrt3* h = new (std::nothrow) btrt3();
    if (!h) return fail(BTRT_E_NOMEM, "host allocation failed");
    h->device = grid->device;
    h->precision = grid->precision;
    h->nx = grid->nx;
    h->ny = grid->ny;
    h->nz = grid->nz;
    h->pitch = pitch_for(grid->nx, grid->precision);
    h->src = R && R->kind == BTRT_SRC_FIELD;
    h->k1_per_node = r.k1_per_node;
    h->check_interval = relax->check_interval;
    h->L = layout3(h->nx, h->ny, h->nz, h->precision, h->src);
    fill_info3(grid, r, h->src, &h->info);
    {
        DeviceGuard g(h->device);
        if (g.status() != hipSuccess) {
            rc = hip_fail(g.status(), "hipSetDevice");
        } else {
            int cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cus > 0)
                h->cus = cus;
            if (grid->stream) {
                h->stream = static_cast<hipStream_t>(grid->stream);
            } else if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
                h->stream = nullptr;
                rc = fail(BTRT_E_DEVICE, "hipStreamCreate failed");
            } else {
                h->own_stream = true;
            }
            if (rc == BTRT_OK && hipMalloc(reinterpret_cast<void**>(&h->mem), h->L.total) != hipSuccess) {
                h->mem = nullptr;
                (void)hipGetLastError();
                rc = fail(BTRT_E_NOMEM, "hipMalloc of %zu bytes failed", h->L.total);
            }
            if (rc == BTRT_OK) rc = setup(h, B, K, R, bc, r, phi0);
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

int btrt3_step(btrt3_t* h, int64_t n)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (n < 0) return fail(BTRT_E_INVAL, "n = %lld < 0", static_cast<long long>(n));
    DeviceGuard g(h->device);
    if (g.status() != hipSuccess) return hip_fail(g.status(), "hipSetDevice");
    const btrt3_launch_t c = resolve_launch(h);
    for (int64_t s = 0; s < n;) {
        const bool two = c.steps_per_launch == 2 && n - s >= 2;
        const bool f64 = h->precision == BTRT_F64;
        hipError_t e;
        if (two)
            e = f64 ? launch3_sweep2<double>(args<double>(h, h->cur), h->src, h->k1_per_node, c.tile, c.z_chunk,
                                             h->stream)
                    : launch3_sweep2<float>(args<float>(h, h->cur), h->src, h->k1_per_node, c.tile, c.z_chunk,
                                            h->stream);
        else
            e = f64 ? launch3_sweep<double>(args<double>(h, h->cur), h->src, h->k1_per_node, h->stream)
                    : launch3_sweep<float>(args<float>(h, h->cur), h->src, h->k1_per_node, h->stream);
        if (e != hipSuccess) return hip_fail(e, "sweep launch");
        h->cur ^= 1;
        const int k = two ? 2 : 1;
        s += k;
        h->step += k;
    }
    return ok();
}

int btrt3_set_launch(btrt3_t* h, const btrt3_launch_t* cfg)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!cfg) return fail(BTRT_E_INVAL, "cfg is NULL");
    if (cfg->steps_per_launch < 0 || cfg->steps_per_launch > 2)
        return fail(BTRT_E_INVAL, "steps_per_launch = %d: must be 0, 1 or 2", cfg->steps_per_launch);
    if (cfg->z_chunk < 0) return fail(BTRT_E_INVAL, "z_chunk = %d < 0", cfg->z_chunk);
    if (cfg->tile < 0 || cfg->tile >= kTiles2)
        return fail(BTRT_E_INVAL, "tile = %d: must be in [0, %d]", cfg->tile, kTiles2 - 1);
    h->launch = *cfg;
    return ok();
}

int btrt3_get_launch(const btrt3_t* h, btrt3_launch_t* cfg)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!cfg) return fail(BTRT_E_INVAL, "cfg is NULL");
    *cfg = resolve_launch(h);
    return ok();
}

int btrt3_field(btrt3_t* h, double* phi_out)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!phi_out) return fail(BTRT_E_INVAL, "phi_out is NULL");
    DeviceGuard g(h->device);
    int rc = gather_sync(h, -1, phi_out);
    return rc == BTRT_OK ? ok() : rc;
}

int btrt3_populations(btrt3_t* h, double* f_out)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!f_out) return fail(BTRT_E_INVAL, "f_out is NULL");
    DeviceGuard g(h->device);
    const size_t nn = static_cast<size_t>(h->nx) * h->ny * h->nz;
    for (int i = 0; i < kQ; ++i) {
        int rc = gather_sync(h, i, f_out + i * nn);
        if (rc != BTRT_OK) return rc;
    }
    return ok();
}

int btrt3_residual(btrt3_t* h, double* out)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!out) return fail(BTRT_E_INVAL, "out is NULL");
    DeviceGuard g(h->device);
    double v[kPartials];
    int rc = reduce_sync(h, 0, v);
    if (rc != BTRT_OK) return rc;
    if (v[5] > 0) {
        *out = NAN;
        return fail(BTRT_E_UNSTABLE, "phi holds %.0f non-finite values at step %lld", v[5],
                    static_cast<long long>(h->step));
    }
    *out = v[1] > 0 ? v[0] / v[1] : (v[0] > 0 ? INFINITY : 0.0);
    return ok();
}

int btrt3_error(btrt3_t* h, const double* ref, double out[3])
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!ref || !out) return fail(BTRT_E_INVAL, "NULL argument");
    DeviceGuard g(h->device);
    const size_t nn = static_cast<size_t>(h->nx) * h->ny * h->nz;
    hipError_t e = hipMemcpyAsync(h->mem + h->L.tmp, ref, nn * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "reference upload");
    double v[kPartials];
    int rc = reduce_sync(h, 1, v);
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

int btrt3_solve(btrt3_t* h, double tol, int64_t max_steps, int64_t* steps_taken, double* residual)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (max_steps < 0 || !(tol >= 0.0)) return fail(BTRT_E_INVAL, "bad tol or max_steps");
    int64_t done = 0;
    double res = INFINITY;
    int rc = BTRT_OK;
    while (done < max_steps) {
        const int64_t k = std::min<int64_t>(h->check_interval, max_steps - done);
        rc = btrt3_step(h, k);
        if (rc != BTRT_OK) break;
        done += k;
        rc = btrt3_residual(h, &res);
        if (rc != BTRT_OK || res <= tol) break;
    }
    if (steps_taken) *steps_taken = done;
    if (residual) *residual = res;
    return rc == BTRT_OK ? ok() : rc;
}

int btrt3_sync(btrt3_t* h)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    DeviceGuard g(h->device);
    hipError_t e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? ok() : hip_fail(e, "hipStreamSynchronize");
}

int btrt3_get_info(const btrt3_t* h, btrt3_info_t* info)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    if (!info) return fail(BTRT_E_INVAL, "info is NULL");
    *info = h->info;
    info->step = h->step;
    return ok();
}

int btrt3_destroy(btrt3_t* h)
{
    if (!h) return fail(BTRT_E_STATE, "NULL handle");
    release(h);
    return ok();
}

}  // extern "C"
