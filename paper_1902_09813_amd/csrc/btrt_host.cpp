// Host-side validation, constants, memory layout and per-instance launch sequence shared by
// the single-solver and batched C ABI.
#include "btrt_host.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

namespace btrth {

using namespace btrtk;


namespace {
// The calling thread's last error message (a fixed buffer: reporting an error allocates nothing).
thread_local char g_last_error[512];
inline bool is_finite(double v) { return std::isfinite(v); }
}  // namespace

const char* last_error() { return g_last_error; }

int hip_fail(hipError_t e, const char* what)
{
    return fail(BTRT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);  // the arguments may point into g_last_error
    va_end(ap);
    std::memcpy(g_last_error, buf, sizeof(buf));
    return code;
}

int ok()
{
    g_last_error[0] = '\0';
    return BTRT_OK;
}

namespace {
// Copies count values value(0 .. count-1), converted to T, to device memory dst, staged through a
// fixed buffer on the stack (no host allocation); synchronises s after each chunk.
template <typename T, typename V>
hipError_t upload_values(char* dst, size_t count, V value, hipStream_t s)
{
    constexpr size_t kChunk = 4096;
    T buf[kChunk];
    for (size_t at = 0; at < count; at += kChunk) {
        const size_t m = std::min(kChunk, count - at);
        for (size_t k = 0; k < m; ++k) buf[k] = static_cast<T>(value(at + k));
        hipError_t e = hipMemcpyAsync(dst + at * sizeof(T), buf, m * sizeof(T), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // buf is reused by the next chunk
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

size_t pop_bytes(int precision)
{
    return precision == BTRT_F64 ? 8 : (precision == BTRT_F32 ? 4 : 2);
}

int format_of(int precision)
{
    return precision == BTRT_F16DEV ? kFmtF16Dev : (precision == BTRT_BF16DEV ? kFmtBF16Dev : kFmtPlain);
}

int pitch_for(int nx, int precision)
{
    // 16-bit deviation formats share the pitch of their FP32 phi plane: 128 elements.
    const int per = static_cast<int>(kAlign / (precision == BTRT_F64 ? 8 : (precision == BTRT_F32 ? 4 : 2)));
    return (nx + per - 1) / per * per;
}

Layout layout_for(int nx, int ny, int precision, int src_kind, bool afield)
{
    const size_t es = pop_bytes(precision);     // one population value
    const size_t ps = precision == BTRT_F64 ? 8 : 4;  // phi and source values
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
    L.phi[0] = take(plane * ps);
    L.phi[1] = take(plane * ps);
    // The FP64 phi snapshot of Eq. (64), dense nx*ny.
    L.snap = take(nn * 8);
    L.tmp = take(nn * 8);
    L.partial = take(static_cast<size_t>(kReduceBlocks) * kReducePartials * 8);
    L.result = take(kReducePartials * 8);
    L.src = L.src_y = 0;
    if (src_kind == BTRT_SRC_FIELD) L.src = take(plane * ps);
    if (src_kind == BTRT_SRC_SIN) {
        L.src = take(static_cast<size_t>(nx) * ps);
        L.src_y = take(static_cast<size_t>(ny) * ps);
    }
    L.afield = afield ? take(3 * plane * ps) : 0;
    L.wall0 = take((4 * (static_cast<size_t>(nx) + static_cast<size_t>(ny)) + 8) * ps);  // one wall-table entry
    L.total = off;
    return L;
}

bool grid_ok(const btrt_grid_t* g)
{
    if (!g) return false;
    if (g->nx < 1 || g->ny < 1) return false;
    if (g->precision < BTRT_F64 || g->precision > BTRT_BF16DEV) return false;
    const int64_t pitch = pitch_for(g->nx, g->precision);
    // Node and in-plane indices are 32-bit in the kernels.
    if (static_cast<int64_t>(g->nx) * g->ny > INT32_MAX) return false;
    if (pitch * (static_cast<int64_t>(g->ny) + 1) > INT32_MAX) return false;
    return true;
}

int validate(const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K, const btrt_dterm_t* D,
             const btrt_source_t* R, const btrt_bc_t* bc, const btrt_relax_t* relax, Resolved* res)
{
    if (!grid || !B || !K || !D || !bc || !relax) return fail(BTRT_E_INVAL, "NULL argument");
    if (grid->nx < 1 || grid->ny < 1) return fail(BTRT_E_INVAL, "grid %d x %d: both sides must be >= 1", grid->nx, grid->ny);
    if (grid->precision < BTRT_F64 || grid->precision > BTRT_BF16DEV)
        return fail(BTRT_E_INVAL, "precision %d is not one of BTRT_F64, BTRT_F32, BTRT_F16DEV, BTRT_BF16DEV",
                    grid->precision);
    if (!grid_ok(grid)) return fail(BTRT_E_INVAL, "grid %d x %d exceeds 2^31 - 1 nodes", grid->nx, grid->ny);
    for (int a = 0; a < 2; ++a)
        if (!is_finite(B->a[a]) || !is_finite(B->b[a]) || !is_finite(B->c[a]))
            return fail(BTRT_E_INVAL, "non-finite flux coefficient");
    const bool power = B->c[0] != 0.0 || B->c[1] != 0.0;
    if (power && !(is_finite(B->q) && B->q >= 1.0))
        return fail(BTRT_E_INVAL, "power-law flux exponent q = %g: must be finite and >= 1", B->q);
    bool reaction = false;
    if (R) {
        if (!is_finite(R->r)) return fail(BTRT_E_INVAL, "non-finite reaction rate r");
        reaction = R->r != 0.0;
        if (reaction && !(is_finite(R->p) && R->p > 0.0))
            return fail(BTRT_E_INVAL, "reaction exponent p = %g: must be finite and > 0", R->p);
    }
    if ((power || reaction) && grid->precision != BTRT_F64 && grid->precision != BTRT_F32)
        return fail(BTRT_E_INVAL, "a power-law flux or a phi-dependent source needs BTRT_F64 or BTRT_F32 storage");
    if (!is_finite(K->beta)) return fail(BTRT_E_INVAL, "non-finite beta");
    if (K->field) {
        // Eq. (73)/(74): every node's A0 must be a finite symmetric positive definite tensor.
        const int64_t nn = static_cast<int64_t>(grid->nx) * grid->ny;
        for (int64_t k = 0; k < nn; ++k) {
            const double a11 = K->field[3 * k], a12 = K->field[3 * k + 1], a22 = K->field[3 * k + 2];
            if (!is_finite(a11) || !is_finite(a12) || !is_finite(a22) || !(a11 > 0.0) || !(a22 > 0.0) ||
                !(a11 * a22 - a12 * a12 > 0.0))
                return fail(BTRT_E_INVAL, "A0 field at node %lld is not a finite SPD tensor", (long long)k);
        }
    } else {
        if (!is_finite(K->k11) || !is_finite(K->k12) || !is_finite(K->k22))
            return fail(BTRT_E_INVAL, "non-finite diffusion tensor");
        if (!(K->k11 > 0.0) || !(K->k22 > 0.0) || !(K->k11 * K->k22 - K->k12 * K->k12 > 0.0))
            return fail(BTRT_E_INVAL, "diffusion tensor [[%g,%g],[%g,%g]] is not positive definite", K->k11, K->k12,
                        K->k12, K->k22);
    }
    if (K->beta < 0.0) return fail(BTRT_E_INVAL, "beta = %g < 0", K->beta);
    if (D->kind != BTRT_D_PHI_I && D->kind != BTRT_D_POLY)
        return fail(BTRT_E_INVAL, "D kind %d: not BTRT_D_PHI_I or BTRT_D_POLY", D->kind);
    const bool dpoly = D->kind == BTRT_D_POLY;
    if (dpoly) {
        if (!is_finite(D->g) || !is_finite(D->e)) return fail(BTRT_E_INVAL, "non-finite D coefficient");
        if (D->e != 0.0 && !(is_finite(D->s) && D->s >= 1.0))
            return fail(BTRT_E_INVAL, "D exponent s = %g: must be finite and >= 1", D->s);
        if (grid->precision != BTRT_F64 && grid->precision != BTRT_F32)
            return fail(BTRT_E_INVAL, "D other than phi I needs BTRT_F64 or BTRT_F32 storage");
    }
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
        if (R->kind != BTRT_SRC_NONE && !is_finite(R->growth)) return fail(BTRT_E_INVAL, "non-finite source growth");
    }
    if (!(relax->k0 > 0.0 && relax->k0 < 2.0)) return fail(BTRT_E_INVAL, "k0 = %g outside (0, 2)", relax->k0);
    if (relax->check_interval < 1) return fail(BTRT_E_INVAL, "check_interval = %d < 1", relax->check_interval);

    // K1 from Eq. (30): K1 = (A / c_s^2 + I/2)^-1 with A at phi = 0. For an SPD A its
    // eigenvalues 1/(3 lambda + 1/2) lie in (0, 2). (With an A0 field K1 is per node; these
    // constants are then unused.)
    const double m11 = 3.0 * K->k11 + 0.5, m12 = 3.0 * K->k12, m22 = 3.0 * K->k22 + 0.5;
    const double det = m11 * m22 - m12 * m12;
    res->K1[0] = m22 / det;
    res->K1[1] = -m12 / det;
    res->K1[2] = -m12 / det;
    res->K1[3] = m11 / det;
    res->k0 = relax->k0;
    res->afield = K->field != nullptr;
    res->k1_per_node = K->beta != 0.0 || res->afield;
    res->growth = R && R->kind != BTRT_SRC_NONE ? R->growth : 0.0;
    res->gen = power || reaction || dpoly;
    res->dq[0] = dpoly ? 1.0 : 0.0;
    res->dq[1] = dpoly ? D->g : 1.0;
    res->dq[2] = dpoly ? D->e : 0.0;
    res->dq[3] = dpoly && D->e != 0.0 ? D->s : 1.0;

    if (relax->k2_rule == BTRT_K2_HBB) {
        // Eq. (62) removes the bounce-back slip for K1 = k1 I (Section 3).
        if (K->field || K->k12 != 0.0 || K->k11 != K->k22 || K->beta != 0.0)
            return fail(BTRT_E_INVAL,
                        "BTRT_K2_HBB needs a constant isotropic A (no field, k11 == k22, k12 == 0, beta == 0)");
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
    info->workspace_bytes = layout_for(g->nx, g->ny, g->precision, src_kind, r.afield).total;
    // 9 population reads + 9 writes + phi(t-1) read + phi(t) write, plus a per-node source and
    // the three planes of a per-node A0.
    const double es = static_cast<double>(pop_bytes(g->precision));
    const double ps = g->precision == BTRT_F64 ? 8.0 : 4.0;
    info->bytes_per_node_launch =
        18.0 * es + (2.0 + (src_kind == BTRT_SRC_FIELD ? 1.0 : 0.0) + (r.afield ? 3.0 : 0.0)) * ps;
    info->step = 0;
}


int validate_phi0(const btrt_grid_t* grid, const double* phi0)
{
    if (!phi0) return fail(BTRT_E_INVAL, "phi0 is NULL");
    const size_t nn = static_cast<size_t>(grid->nx) * grid->ny;
    for (size_t k = 0; k < nn; ++k)
        if (!is_finite(phi0[k])) return fail(BTRT_E_INVAL, "non-finite phi0 at node %zu", k);
    return BTRT_OK;
}

DeviceGuard::DeviceGuard(int device) : device_(device)
{
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != device_) status_ = hipSetDevice(device_);
}

DeviceGuard::~DeviceGuard()
{
    if (prev_ >= 0 && prev_ != device_) (void)hipSetDevice(prev_);
}

namespace {

template <typename T>
void fill_constants(Instance& I, SweepArgs<T>& a, const btrt_flux_t* B, const btrt_diff_t* K,
                    const btrt_source_t* R, const Resolved& r)
{
    a.plane = I.plane;
    a.nx = I.nx;
    a.ny = I.ny;
    a.pitch = I.pitch;
    a.perx = I.perx;
    a.pery = I.pery;
    for (int s = 0; s < 4; ++s) a.wall[s] = static_cast<T>(I.wall[s]);
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
    a.cq[0] = T(1.5);
    a.cq[1] = T(-4.5);
    a.cq[2] = T(-9);
    a.cq[3] = T(9);
    a.src_amp = static_cast<T>(R && R->kind == BTRT_SRC_SIN ? R->amp : 0.0);
    a.src = I.kind == kSrcNone ? nullptr : reinterpret_cast<const T*>(I.mem + I.L.src);
    a.src_y = I.kind == kSrcSep ? reinterpret_cast<const T*>(I.mem + I.L.src_y) : nullptr;
    a.afield = I.afield ? reinterpret_cast<const T*>(I.mem + I.L.afield) : nullptr;
    for (int l = 0; l < btrtk::kMaxFuse; ++l) a.sfac[l] = T(1);
    a.fcx = static_cast<T>(B->c[0]);
    a.fcy = static_cast<T>(B->c[1]);
    a.fq = static_cast<T>(B->c[0] != 0.0 || B->c[1] != 0.0 ? B->q : 1.0);
    a.rr = static_cast<T>(R ? R->r : 0.0);
    a.rp = static_cast<T>(R && R->r != 0.0 ? R->p : 1.0);
    a.dpoly = r.dq[0] != 0.0 ? 1 : 0;
    a.dg = static_cast<T>(r.dq[1]);
    a.de = static_cast<T>(r.dq[2]);
    a.ds = static_cast<T>(r.dq[3]);
    a.wtab = nullptr;  // set per launch (sweep_args) for the general node model
    a.wstride = 0;
    // Non-temporal stores once the two buffers of populations and phi exceed the 256 MB
    // Infinity Cache.
    const double state_bytes = 2.0 * static_cast<double>(I.plane) * (9.0 * pop_bytes(I.precision) + sizeof(T));
    a.nts = state_bytes > 256.0 * 1024 * 1024 ? 1 : 0;
    a.dev_scale = static_cast<T>(I.dev_scale);
    a.dev_inv = static_cast<T>(1.0 / I.dev_scale);
}

}  // namespace

int instance_setup(Instance& I, const btrt_grid_t* grid, const btrt_flux_t* B, const btrt_diff_t* K,
                   const btrt_source_t* R, const btrt_bc_t* bc, const Resolved& r, const double* phi0, char* mem,
                   hipStream_t s)
{
    const int src_kind = R ? R->kind : BTRT_SRC_NONE;
    I.nx = grid->nx;
    I.ny = grid->ny;
    I.precision = grid->precision;
    I.pitch = pitch_for(grid->nx, grid->precision);
    I.plane = static_cast<int64_t>(I.pitch) * grid->ny;
    I.kind = src_kind == BTRT_SRC_FIELD ? kSrcField : (src_kind == BTRT_SRC_SIN ? kSrcSep : kSrcNone);
    I.k1_per_node = r.k1_per_node;
    I.k0_one = r.k0 == 1.0;
    I.afield = r.afield;
    I.growth = r.growth;
    I.gen = r.gen;
    I.wtab = nullptr;
    I.wall_t0 = 0;
    I.wall_limit = INT64_MAX;
    I.wall_stride = 0;
    I.perx = bc->type[0] == BTRT_PERIODIC;
    I.pery = bc->type[2] == BTRT_PERIODIC;
    for (int q = 0; q < 4; ++q) I.wall[q] = bc->type[q] == BTRT_DIRICHLET ? bc->value[q] : 0.0;
    I.mem = mem;
    I.L = layout_for(I.nx, I.ny, I.precision, src_kind, I.afield);
    I.cur = 0;
    I.step = 0;
    fill_info(grid, r, src_kind, &I.info);
    if (reinterpret_cast<uintptr_t>(mem) % kAlign != 0)
        return fail(BTRT_E_INVAL, "workspace must be %zu-byte aligned", kAlign);

    const size_t nn = static_cast<size_t>(I.nx) * I.ny;
    const size_t es = I.precision == BTRT_F64 ? 8 : 4;  // source values
    double* tmp = reinterpret_cast<double*>(mem + I.L.tmp);
    hipError_t err = hipSuccess;
    // Source of Eq. (8): a per-node field, or separable sin tables at cell centres.
    if (src_kind == BTRT_SRC_FIELD) {
        err = hipMemcpyAsync(tmp, R->field, nn * sizeof(double), hipMemcpyHostToDevice, s);
        if (err != hipSuccess) return hip_fail(err, "source upload");
        err = I.precision == BTRT_F64
                  ? launch_convert<double>(tmp, reinterpret_cast<double*>(mem + I.L.src), I.nx, I.ny, I.pitch, s)
                  : launch_convert<float>(tmp, reinterpret_cast<float*>(mem + I.L.src), I.nx, I.ny, I.pitch, s);
        if (err != hipSuccess) return hip_fail(err, "source convert");
        err = hipStreamSynchronize(s);
        if (err != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
    } else if (src_kind == BTRT_SRC_SIN) {
        const double pi = 3.14159265358979323846;
        auto sx = [&](size_t i) { return std::sin(R->kx * pi * (static_cast<double>(i) + 0.5) / I.nx); };
        auto sy = [&](size_t j) { return std::sin(R->ky * pi * (static_cast<double>(j) + 0.5) / I.ny); };
        if (I.precision == BTRT_F64) {
            err = upload_values<double>(mem + I.L.src, static_cast<size_t>(I.nx), sx, s);
            if (err == hipSuccess) err = upload_values<double>(mem + I.L.src_y, static_cast<size_t>(I.ny), sy, s);
        } else {
            err = upload_values<float>(mem + I.L.src, static_cast<size_t>(I.nx), sx, s);
            if (err == hipSuccess) err = upload_values<float>(mem + I.L.src_y, static_cast<size_t>(I.ny), sy, s);
        }
        if (err != hipSuccess) return hip_fail(err, "source table upload");
    }
    // Per-node A0(x): three planes (a11, a12, a22) in the phi type.
    if (I.afield) {
        for (int q = 0; q < 3 && err == hipSuccess; ++q) {
            char* dst = mem + I.L.afield + q * static_cast<size_t>(I.plane) * es;
            err = upload_values<double>(reinterpret_cast<char*>(tmp), nn, [&](size_t k) { return K->field[3 * k + q]; },
                                        s);
            if (err == hipSuccess)
                err = I.precision == BTRT_F64
                          ? launch_convert<double>(tmp, reinterpret_cast<double*>(dst), I.nx, I.ny, I.pitch, s)
                          : launch_convert<float>(tmp, reinterpret_cast<float*>(dst), I.nx, I.ny, I.pitch, s);
            if (err == hipSuccess) err = hipStreamSynchronize(s);  // tmp is reused
        }
        if (err != hipSuccess) return hip_fail(err, "A0 field upload");
    }
    // 16-bit deviation formats: a power-of-two scale that maps the initial magnitude of phi
    // (and of the wall values) to 2^14, far inside the FP16 range; deviations from
    // equilibrium are much smaller than phi.
    I.dev_scale = 1.0;
    if (I.precision == BTRT_F16DEV || I.precision == BTRT_BF16DEV) {
        double m = 0.0;
        for (size_t k = 0; k < nn; ++k) m = std::max(m, std::fabs(phi0[k]));
        for (int q = 0; q < 4; ++q) m = std::max(m, std::fabs(I.wall[q]));
        int ex = 0;
        std::frexp(m > 0.0 ? m : 1.0, &ex);
        I.dev_scale = std::ldexp(1.0, 14 - ex);
    }
    if (I.precision == BTRT_F64)
        fill_constants<double>(I, I.a64, B, K, R, r);
    else
        fill_constants<float>(I, I.a32, B, K, R, r);
    // The general node model reads its Dirichlet values from a wall table: one entry holding
    // the per-side constants, used by every step until a schedule replaces it.
    if (I.gen) {
        err = upload_wall_entry(I, I.mem + I.L.wall0, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        if (err != hipSuccess) return hip_fail(err, "wall table upload");
        I.wtab = I.mem + I.L.wall0;
    }

    err = hipMemcpyAsync(tmp, phi0, nn * sizeof(double), hipMemcpyHostToDevice, s);
    if (err != hipSuccess) return hip_fail(err, "phi0 upload");
    // The init kernel writes through a sweep's outputs: parity 1 outputs are f[0] and phi[0].
    const double ab[4] = {B->a[0], B->a[1], B->b[0], B->b[1]};
    const double cq[3] = {B->c[0], B->c[1], B->c[0] != 0.0 || B->c[1] != 0.0 ? B->q : 1.0};
    if (I.precision == BTRT_F64)
        err = launch_init<double>(sweep_args<double>(I, 1), kFmtPlain, tmp, I.wall, ab, cq, r.dq, s);
    else
        err = launch_init<float>(sweep_args<float>(I, 1), format_of(I.precision), tmp, I.wall, ab, cq, r.dq, s);
    if (err != hipSuccess) return hip_fail(err, "init launch");
    err = hipMemcpyAsync(mem + I.L.snap, tmp, nn * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (err != hipSuccess) return hip_fail(err, "snapshot copy");
    err = hipStreamSynchronize(s);
    if (err != hipSuccess) return hip_fail(err, "hipStreamSynchronize");
    return BTRT_OK;
}

template <typename T>
SweepArgs<T> sweep_args(const Instance& I, int parity)
{
    SweepArgs<T> a;
    if constexpr (sizeof(T) == 8)
        a = I.a64;
    else
        a = I.a32;
    const int nxt = parity ^ 1;
    a.fin = reinterpret_cast<const T*>(I.mem + I.L.f[parity]);
    a.fout = reinterpret_cast<T*>(I.mem + I.L.f[nxt]);
    a.phi_prev = reinterpret_cast<const T*>(I.mem + I.L.phi[parity]);
    a.phi_out = reinterpret_cast<T*>(I.mem + I.L.phi[nxt]);
    if (I.gen && I.wtab) {
        a.wtab = reinterpret_cast<const T*>(I.wtab) + (I.step - I.wall_t0) * I.wall_stride;
        a.wstride = I.wall_stride;
    }
    return a;
}

namespace {
// Slot q of a wall-table entry built from the samples r of one step (wall_entry_values() of them):
// the samples, then the corner means. Corner samples: x- and x+ at their first (y = 0) and last
// (y = ny) sample, y- and y+ likewise at x = 0 and x = nx. A link through a corner takes the mean
// of the two sides that meet there, computed in the storage type as the kernels compute it for
// per-side constants.
template <typename T, typename R>
T wall_slot(const Instance& I, R r, size_t q)
{
    const size_t P = static_cast<size_t>(I.wall_entry_values());
    if (q < P) return static_cast<T>(r(q));
    const size_t sx = 2 * static_cast<size_t>(I.ny) + 1, sy = 2 * static_cast<size_t>(I.nx) + 1;
    const size_t xside[4] = {0, sx, 2 * sx - 1, sx - 1};                    // x- at y = 0, x+ at y = 0, x+ at ny, x- at ny
    const size_t yside[4] = {2 * sx, 2 * sx + sy - 1, 2 * sx + 2 * sy - 1, 2 * sx + sy};  // y- at 0, y- at nx, y+ at nx, y+ at 0
    const size_t c = q - P;
    return T(0.5) * (static_cast<T>(r(xside[c])) + static_cast<T>(r(yside[c])));
}

template <typename T, typename R>
hipError_t upload_entries(const Instance& I, R r, size_t rows, char* dst, hipStream_t s)
{
    const size_t P = static_cast<size_t>(I.wall_entry_values()), S = static_cast<size_t>(I.wall_entry_slots());
    return upload_values<T>(dst, rows * S, [&](size_t k) {
        const size_t row = k / S;
        return wall_slot<T>(I, [&](size_t q) { return r(row * P + q); }, k - row * S);
    }, s);
}

// Sample q of the per-side constants (the same value along each side).
double constant_sample(const Instance& I, size_t q)
{
    const size_t sx = 2 * static_cast<size_t>(I.ny) + 1, sy = 2 * static_cast<size_t>(I.nx) + 1;
    return q < sx ? I.wall[0] : (q < 2 * sx ? I.wall[1] : (q < 2 * sx + sy ? I.wall[2] : I.wall[3]));
}
}  // namespace

hipError_t upload_wall_values(const Instance& I, const double* v, size_t rows, char* dst, hipStream_t s)
{
    auto r = [v](size_t k) { return v[k]; };
    return I.precision == BTRT_F64 ? upload_entries<double>(I, r, rows, dst, s) : upload_entries<float>(I, r, rows, dst, s);
}

hipError_t upload_wall_entry(const Instance& I, char* dst, hipStream_t s)
{
    const size_t P = static_cast<size_t>(I.wall_entry_values());
    auto r = [&I, P](size_t k) { return constant_sample(I, k % P); };
    return I.precision == BTRT_F64 ? upload_entries<double>(I, r, 1, dst, s) : upload_entries<float>(I, r, 1, dst, s);
}

template <typename T>
GatherArgs<T> gather_args(const Instance& I)
{
    GatherArgs<T> g{};
    g.s = sweep_args<T>(I, I.cur);
    g.snap = reinterpret_cast<double*>(I.mem + I.L.snap);
    g.ref = reinterpret_cast<const double*>(I.mem + I.L.tmp);
    g.out = reinterpret_cast<double*>(I.mem + I.L.tmp);
    g.partial = reinterpret_cast<double*>(I.mem + I.L.partial);
    g.population = -1;
    return g;
}

template SweepArgs<double> sweep_args<double>(const Instance&, int);
template SweepArgs<float> sweep_args<float>(const Instance&, int);
template GatherArgs<double> gather_args<double>(const Instance&);
template GatherArgs<float> gather_args<float>(const Instance&);

namespace {

// Source factors of the steps a launch advances: S(t) + (S(t) - S(t-1))/2 = S0 (1.5 e(t) -
// 0.5 e(t-1)) with e(t) = exp(g t) and S(-1) = S(0) (Scheme 2, Remark III); 1 when the source
// does not change in time. Computed in FP64 on the host, so every launch shape gets the same
// factors.
template <typename T>
SweepArgs<T> with_source_factors(const Instance& I, SweepArgs<T> a, int steps)
{
    if (I.growth != 0.0) {
        for (int l = 0; l < steps && l < btrtk::kMaxFuse; ++l) {
            const double t = static_cast<double>(I.step + l);
            const double e = std::exp(I.growth * t);
            const double ep = t > 0 ? std::exp(I.growth * (t - 1.0)) : e;
            a.sfac[l] = static_cast<T>(1.5 * e - 0.5 * ep);
        }
    }
    return a;
}

}  // namespace

int instance_launch(Instance& I, const LaunchCfg& cfg, hipStream_t s)
{
    hipError_t e;
    if (I.precision == BTRT_F64)
        e = launch_sweep<double>(with_source_factors(I, sweep_args<double>(I, I.cur), cfg.steps), kFmtPlain, I.kind,
                                 I.kmode(), cfg, s);
    else
        e = launch_sweep<float>(with_source_factors(I, sweep_args<float>(I, I.cur), cfg.steps),
                                format_of(I.precision), I.kind, I.kmode(), cfg, s);
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    I.cur ^= 1;
    I.step += cfg.steps;
    return BTRT_OK;
}

int instance_steps(Instance& I, const LaunchCfg& want, int64_t n, hipStream_t s)
{
    if (n <= 0) return BTRT_OK;
    if (n > I.wall_limit - I.step)
        return fail(BTRT_E_INVAL, "%lld steps from step %lld go past the wall schedule (it ends at step %lld)",
                    static_cast<long long>(n), static_cast<long long>(I.step), static_cast<long long>(I.wall_limit));
    const LaunchCfg c = instance_resolve(I, want);
    for (int64_t i = 0; i < n;) {
        LaunchCfg k = c;
        k.steps = static_cast<int>(std::min<int64_t>(c.steps, n - i));
        if (k.steps != 2) k.tile = 0;
        if (k.steps == 1 && c.steps != 1) k.rows = k.group = 0;  // the one-step kernel's own tiles
        int rc = instance_launch(I, k, s);
        if (rc != BTRT_OK) return rc;
        i += k.steps;
    }
    return BTRT_OK;
}

LaunchCfg instance_resolve(const Instance& I, const LaunchCfg& cfg)
{
    if (I.precision == BTRT_F64)
        return resolve_launch<double>(sweep_args<double>(I, I.cur), kFmtPlain, I.kind, I.kmode(), cfg);
    return resolve_launch<float>(sweep_args<float>(I, I.cur), format_of(I.precision), I.kind, I.kmode(), cfg);
}

int instance_reduce_async(Instance& I, int mode, hipStream_t s)
{
    double* result = reinterpret_cast<double*>(I.mem + I.L.result);
    hipError_t e = I.precision == BTRT_F64
                       ? launch_reduce<double>(gather_args<double>(I), kFmtPlain, mode, result, s)
                       : launch_reduce<float>(gather_args<float>(I), format_of(I.precision), mode, result, s);
    return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "reduce launch");
}

int instance_result_async(const Instance& I, double out[kReducePartials], hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(out, I.mem + I.L.result, kReducePartials * sizeof(double), hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "hipMemcpyAsync");
}

int instance_gather(Instance& I, int population, double* host_out, hipStream_t s)
{
    hipError_t e;
    const size_t nn = static_cast<size_t>(I.nx) * I.ny;
    if (I.precision == BTRT_F64) {
        GatherArgs<double> g = gather_args<double>(I);
        g.population = population;
        e = launch_gather_field<double>(g, kFmtPlain, s);
    } else {
        GatherArgs<float> g = gather_args<float>(I);
        g.population = population;
        e = launch_gather_field<float>(g, format_of(I.precision), s);
    }
    if (e != hipSuccess) return hip_fail(e, "gather launch");
    e = hipMemcpyAsync(host_out, I.mem + I.L.tmp, nn * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    return e == hipSuccess ? static_cast<int>(BTRT_OK) : hip_fail(e, "hipStreamSynchronize");
}

}  // namespace btrth
