// Set-up, field read and reduction kernels of the B-TriRT library, and the storage-format
// dispatch of the sweep launchers (the sweeps themselves live in btrt_sweep_<format>.hip and
// the batched launchers in btrt_batch_kernels.hip; the device code in btrt_device.h).

#include "btrt_device.h"

namespace btrtk {
namespace {

// ---- set-up, field reads and reductions -------------------------------------------------

// f+(-1) such that the first pull yields f(0) = f^eq(phi0) (Section 4 initialisation), and
// phi(-1) := phi0; written through the format's put into a.fout / a.phi_out.
struct InitConsts {
    double wall[4];
    double ab[4];  // ax, ay, bx, by
    double cq[3];  // cx, cy, q
    double dq[4];  // D kind, g, e, s
};

template <typename F>
__global__ __launch_bounds__(kBlock) void init_kernel(SweepArgs<typename F::T> a, const double* __restrict__ phi0,
                                                      InitConsts c)
{
    using T = typename F::T;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= static_cast<int64_t>(a.nx) * a.ny) return;
    const int y = static_cast<int>(k / a.nx);
    const int x = static_cast<int>(k - static_cast<int64_t>(y) * a.nx);
    T f[9];
    init_values(phi0, x, y, a.nx, a.ny, a.perx, a.pery, c.wall, c.ab, c.cq, c.dq,
                [&](int i, double v) { f[i] = static_cast<T>(v); });
    F::template put<false>(a, y * a.pitch + x, f, static_cast<T>(phi0[k]));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void convert_kernel(const double* __restrict__ in, T* __restrict__ out,
                                                         int nx, int ny, int pitch)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= static_cast<int64_t>(nx) * ny) return;
    const int y = static_cast<int>(k / nx);
    const int x = static_cast<int>(k - static_cast<int64_t>(y) * nx);
    out[y * pitch + x] = static_cast<T>(in[k]);
}

// The pull of a sweep's first step, for a handle with or without a wall table (the gathers
// serve every node model).
template <typename F>
__device__ __forceinline__ void pull_any(const SweepArgs<typename F::T>& a, int x, int y, typename F::T f[9])
{
    if (a.wtab != nullptr)
        F::template pull<true>(a, x, y, f);
    else
        F::template pull<false>(a, x, y, f);
}

// phi(t) (or one population f_i(t)) at every node into a dense FP64 array.
template <typename F>
__global__ __launch_bounds__(kBlock) void gather_field_kernel(GatherArgs<typename F::T> a)
{
    using T = typename F::T;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= static_cast<int64_t>(a.s.nx) * a.s.ny) return;
    const int y = static_cast<int>(k / a.s.nx);
    const int x = static_cast<int>(k - static_cast<int64_t>(y) * a.s.nx);
    T f[9];
    pull_any<F>(a.s, x, y, f);
    T v = T(0);
    if (a.population < 0) {
        v = sum9(f);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (i == a.population) v = f[i];
    }
    a.out[k] = static_cast<double>(v);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// Deterministic block reduction of kReducePartials values: wavefront shuffles, then the
// four wave results combined in a fixed order by thread 0. Result valid in thread 0.
__device__ __forceinline__ void block_reduce(double v[kReducePartials])
{
    __shared__ double lds[kBlock / 64][kReducePartials];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kReducePartials; ++j) v[j] = (j == 4) ? wave_max(v[j]) : wave_sum(v[j]);
    if (lane == 0)
        for (int j = 0; j < kReducePartials; ++j) lds[wave][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < kReducePartials; ++j) {
            double acc = lds[0][j];
            for (int w = 1; w < kBlock / 64; ++w) acc = (j == 4) ? fmax(acc, lds[w][j]) : acc + lds[w][j];
            v[j] = acc;
        }
    }
}

// First pass: each block covers a fixed grid-stride subset of the nodes and writes its
// partial sums. kResidual: a = |phi - snap|, b = |phi|, snap := phi (Eq. (64)).
// kError: a = |phi - ref|, b = |ref|, c = (phi - ref)^2, d = ref^2, max |phi - ref| (Eq. (63)).
template <typename F, int MODE>
__global__ __launch_bounds__(kBlock) void reduce_kernel(GatherArgs<typename F::T> a)
{
    using T = typename F::T;
    double v[kReducePartials] = {0, 0, 0, 0, 0, 0};
    const int64_t nn = static_cast<int64_t>(a.s.nx) * a.s.ny;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; k < nn; k += stride) {
        const int y = static_cast<int>(k / a.s.nx);
        const int x = static_cast<int>(k - static_cast<int64_t>(y) * a.s.nx);
        T f[9];
        pull_any<F>(a.s, x, y, f);
        const double phi = static_cast<double>(sum9(f));
        if (!isfinite(phi)) v[5] += 1.0;
        if constexpr (MODE == kResidual) {
            v[0] += fabs(phi - a.snap[k]);
            v[1] += fabs(phi);
            a.snap[k] = phi;
        } else {
            const double r = a.ref[k];
            const double d = phi - r;
            v[0] += fabs(d);
            v[1] += fabs(r);
            v[2] += d * d;
            v[3] += r * r;
            v[4] = fmax(v[4], fabs(d));
        }
    }
    block_reduce(v);
    if (threadIdx.x == 0)
        for (int j = 0; j < kReducePartials; ++j) a.partial[blockIdx.x * kReducePartials + j] = v[j];
}

// Second pass: one block folds the per-block partials in a fixed order.
__global__ __launch_bounds__(kBlock) void reduce_final_kernel(const double* __restrict__ partial, int nblocks,
                                                              double* __restrict__ result)
{
    double v[kReducePartials] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int j = 0; j < kReducePartials; ++j)
            v[j] = (j == 4) ? fmax(v[j], partial[b * kReducePartials + j]) : v[j] + partial[b * kReducePartials + j];
    block_reduce(v);
    if (threadIdx.x == 0)
        for (int j = 0; j < kReducePartials; ++j) result[j] = v[j];
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

template <typename F>
hipError_t init_with(const SweepArgs<typename F::T>& a, const double* phi0, const double wall[4], const double ab[4],
                     const double cq[3], const double dq[4], hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(a.nx) * a.ny;
    InitConsts c{};
    for (int q = 0; q < 4; ++q) c.wall[q] = wall[q];
    for (int q = 0; q < 4; ++q) c.ab[q] = ab[q];
    for (int q = 0; q < 3; ++q) c.cq[q] = cq[q];
    for (int q = 0; q < 4; ++q) c.dq[q] = dq[q];
    hipLaunchKernelGGL((init_kernel<F>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, a, phi0, c);
    return hipGetLastError();
}

template <typename F>
hipError_t gather_with_fmt(const GatherArgs<typename F::T>& a, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(a.s.nx) * a.s.ny;
    hipLaunchKernelGGL((gather_field_kernel<F>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <typename F>
hipError_t reduce_with(const GatherArgs<typename F::T>& a, int mode, double* result, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(a.s.nx) * a.s.ny;
    const unsigned nb = static_cast<unsigned>(std::min<int64_t>(kReduceBlocks, (nn + kBlock - 1) / kBlock));
    if (mode == kResidual)
        hipLaunchKernelGGL((reduce_kernel<F, kResidual>), dim3(nb), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((reduce_kernel<F, kError>), dim3(nb), dim3(kBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kBlock), 0, s, a.partial, static_cast<int>(nb), result);
    return hipGetLastError();
}

}  // namespace

// Format dispatch: double has only the plain format; float has plain, FP16 and BF16 deviations.
#define BTRT_BY_FORMAT(T, FN, ...)                                                                       \
    do {                                                                                                 \
        if constexpr (sizeof(T) == 8) {                                                                  \
            if (fmt != kFmtPlain) return hipErrorInvalidValue;                                           \
            return FN<Plain<T>>(__VA_ARGS__);                                                            \
        } else {                                                                                         \
            if (fmt == kFmtF16Dev) return FN<Dev<F16Codec>>(__VA_ARGS__);                                \
            if (fmt == kFmtBF16Dev) return FN<Dev<BF16Codec>>(__VA_ARGS__);                              \
            return FN<Plain<T>>(__VA_ARGS__);                                                            \
        }                                                                                                \
    } while (0)

template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, int fmt, int src_kind, int kmode, const LaunchCfg& cfg,
                        hipStream_t s)
{
    if ((kmode & kGen) != 0) {  // the general node model: plain storage only
        if (fmt != kFmtPlain) return hipErrorInvalidValue;
        if constexpr (sizeof(T) == 8)
            return sweep_gen_f64(a, src_kind, kmode & ~kK0One, cfg, s);
        else
            return sweep_gen_f32(a, src_kind, kmode & ~kK0One, cfg, s);
    }
    if ((kmode & kK0One) != 0) {
        if constexpr (sizeof(T) == 8) {
            if (fmt != kFmtPlain) return hipErrorInvalidValue;
            return sweep_k0_f64(a, src_kind, kmode, cfg, s);
        } else {
            if (fmt == kFmtF16Dev) return sweep_k0_f16dev(a, src_kind, kmode, cfg, s);
            if (fmt == kFmtBF16Dev) return sweep_k0_bf16dev(a, src_kind, kmode, cfg, s);
            return sweep_k0_f32(a, src_kind, kmode, cfg, s);
        }
    }
    kmode &= ~kK0One;
    if constexpr (sizeof(T) == 8) {
        if (fmt != kFmtPlain) return hipErrorInvalidValue;
        return sweep_f64(a, src_kind, kmode, cfg, s);
    } else {
        if (fmt == kFmtF16Dev) return sweep_f16dev(a, src_kind, kmode, cfg, s);
        if (fmt == kFmtBF16Dev) return sweep_bf16dev(a, src_kind, kmode, cfg, s);
        return sweep_f32(a, src_kind, kmode, cfg, s);
    }
}

template <typename T>
LaunchCfg resolve_launch(const SweepArgs<T>& a, int fmt, int src_kind, int kmode, LaunchCfg cfg)
{
    if ((kmode & kGen) != 0) {
        if constexpr (sizeof(T) == 8)
            return resolve_gen_f64(a, src_kind, kmode & ~kK0One, cfg);
        else
            return resolve_gen_f32(a, src_kind, kmode & ~kK0One, cfg);
    }
    if ((kmode & kK0One) != 0) {
        if constexpr (sizeof(T) == 8) {
            return resolve_k0_f64(a, src_kind, kmode, cfg);
        } else {
            if (fmt == kFmtF16Dev) return resolve_k0_f16dev(a, src_kind, kmode, cfg);
            if (fmt == kFmtBF16Dev) return resolve_k0_bf16dev(a, src_kind, kmode, cfg);
            return resolve_k0_f32(a, src_kind, kmode, cfg);
        }
    }
    kmode &= ~kK0One;
    if constexpr (sizeof(T) == 8) {
        return resolve_f64(a, src_kind, kmode, cfg);
    } else {
        if (fmt == kFmtF16Dev) return resolve_f16dev(a, src_kind, kmode, cfg);
        if (fmt == kFmtBF16Dev) return resolve_bf16dev(a, src_kind, kmode, cfg);
        return resolve_f32(a, src_kind, kmode, cfg);
    }
}

template <typename T>
hipError_t launch_init(const SweepArgs<T>& a, int fmt, const double* phi0, const double wall[4], const double ab[4],
                       const double cq[3], const double dq[4], hipStream_t s)
{
    BTRT_BY_FORMAT(T, init_with, a, phi0, wall, ab, cq, dq, s);
}

template <typename T>
hipError_t launch_gather_field(const GatherArgs<T>& a, int fmt, hipStream_t s)
{
    BTRT_BY_FORMAT(T, gather_with_fmt, a, s);
}

template <typename T>
hipError_t launch_reduce(const GatherArgs<T>& a, int fmt, int mode, double* result, hipStream_t s)
{
    BTRT_BY_FORMAT(T, reduce_with, a, mode, result, s);
}

#undef BTRT_BY_FORMAT

template <typename T>
hipError_t launch_convert(const double* in, T* out, int nx, int ny, int pitch, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(nx) * ny;
    hipLaunchKernelGGL((convert_kernel<T>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, in, out, nx, ny, pitch);
    return hipGetLastError();
}

#define BTRT_INSTANTIATE(T)                                                                                        \
    template hipError_t launch_sweep<T>(const SweepArgs<T>&, int, int, int, const LaunchCfg&, hipStream_t);       \
    template LaunchCfg resolve_launch<T>(const SweepArgs<T>&, int, int, int, LaunchCfg);                         \
    template hipError_t launch_init<T>(const SweepArgs<T>&, int, const double*, const double[4], const double[4],  \
                                       const double[3], const double[4], hipStream_t);                             \
    template hipError_t launch_gather_field<T>(const GatherArgs<T>&, int, hipStream_t);                           \
    template hipError_t launch_reduce<T>(const GatherArgs<T>&, int, int, double*, hipStream_t);                   \
    template hipError_t launch_convert<T>(const double*, T*, int, int, int, hipStream_t);                         \


BTRT_INSTANTIATE(double)
BTRT_INSTANTIATE(float)

}  // namespace btrtk

