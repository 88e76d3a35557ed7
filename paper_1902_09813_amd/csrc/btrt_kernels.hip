// gfx950 kernels of the B-TriRT D2Q9 sweep (Zhao, Wu, Chai & Shi, arXiv:1902.09813).
//
// State between steps: the post-collision populations f+(t-1) in 9 SoA planes
// (f[i][y][pitch], i in the velocity order of Eq. (85)) and phi(t-1) in one plane.
// One sweep per time step, one thread per node:
//   1. pull  f_i(x, t) = f_i+(x - c_i, t-1)                         (Eq. (38))
//      or, when x - c_i lies beyond a Dirichlet wall,
//            f_i(x, t) = -f_opp(i)+(x, t-1) + 2 w_i phi_w             (Eqs. (54)-(56))
//   2. moments m = T f (Eq. (88)), phi = m_0 (Eq. (9))
//   3. block relaxation in moment space with S_f of Eq. (99), the equilibrium moments
//      of Eq. (7) with D = phi I, the source of Eq. (8) and G of Eq. (11)
//   4. f+ = T^-1 m+ and aligned stores of f+(t) and phi(t)
// Reads and writes are disjoint (two population buffers), so no synchronisation is needed.
// The 9x9 transform is a handful of adds per node and stays in registers: the sweep is
// bound by HBM bandwidth, not by arithmetic, so there is no matrix-core work here.

#include "btrt_internal.h"
#include "btrt_node.h"

#include <algorithm>

namespace btrtk {
namespace {

constexpr int kTileX = 64;  // one wavefront along a row: coalesced 64-wide accesses
constexpr int kTileY = kBlock / kTileX;

// Block index -> tile index, grouping consecutive tiles on one XCD. Workgroups are
// dispatched round-robin over the 8 XCDs; this gives XCD k a contiguous run of tiles so
// the cache lines shared by horizontally adjacent tiles (the x-1 / x+1 pulls) meet in
// the same L2.
__device__ __forceinline__ int xcd_tile()
{
    const int b = static_cast<int>(blockIdx.x);
    const int nb = static_cast<int>(gridDim.x);
    const int q = nb >> 3, r = nb & 7, k = b & 7, j = b >> 3;
    return k * q + (k < r ? k : r) + j;
}

template <typename T, int SRC, bool KPHI>
__global__ __launch_bounds__(kBlock) void sweep_kernel(SweepArgs<T> a)
{
    const int tile = xcd_tile();
    const int ty = tile / a.tiles_x;
    const int tx = tile - ty * a.tiles_x;
    const int x = tx * kTileX + static_cast<int>(threadIdx.x % kTileX);
    const int y = ty * kTileY + static_cast<int>(threadIdx.x / kTileX);
    if (x >= a.nx || y >= a.ny) return;

    T f[9];
    gather(a.fin, a.plane, x, y, a.nx, a.ny, a.pitch, a.perx, a.pery, a.wall, f);
    const int n = y * a.pitch + x;
    const T phi_prev = a.phi_prev[n];
    T s = T(0);
    if constexpr (SRC == kSrcField) s = a.src[n];
    if constexpr (SRC == kSrcSep) s = a.src_amp * a.src[x] * a.src_y[y];

    const T phi = collide<T, SRC, KPHI>(a, f, phi_prev, s);

    T* __restrict__ o = a.fout;
    const int64_t p = a.plane;
#pragma unroll
    for (int i = 0; i < 9; ++i) o[i * p + n] = f[i];
    a.phi_out[n] = phi;
}

// f+(-1) such that the first pull yields f(0) = f^eq(phi0) (Section 4 initialisation).
template <typename T>
__global__ __launch_bounds__(kBlock) void init_kernel(T* __restrict__ f, T* __restrict__ phi_prev,
                                                      const double* __restrict__ phi0, int64_t plane,
                                                      int nx, int ny, int pitch, int perx, int pery,
                                                      double w0, double w1, double w2, double w3,
                                                      double ax, double ay, double bx, double by)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= static_cast<int64_t>(nx) * ny) return;
    const int y = static_cast<int>(k / nx);
    const int x = static_cast<int>(k - static_cast<int64_t>(y) * nx);
    const double wall[4] = {w0, w1, w2, w3};
    init_node(f, phi_prev, phi0, plane, x, y, nx, ny, pitch, perx, pery, wall, ax, ay, bx, by);
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

// phi(t) (or one population f_i(t)) at every node into a dense FP64 array.
template <typename T>
__global__ __launch_bounds__(kBlock) void gather_field_kernel(GatherArgs<T> a)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= static_cast<int64_t>(a.nx) * a.ny) return;
    const int y = static_cast<int>(k / a.nx);
    const int x = static_cast<int>(k - static_cast<int64_t>(y) * a.nx);
    T f[9];
    gather(a.fin, a.plane, x, y, a.nx, a.ny, a.pitch, a.perx, a.pery, a.wall, f);
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
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void reduce_kernel(GatherArgs<T> a)
{
    double v[kReducePartials] = {0, 0, 0, 0, 0, 0};
    const int64_t nn = static_cast<int64_t>(a.nx) * a.ny;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; k < nn; k += stride) {
        const int y = static_cast<int>(k / a.nx);
        const int x = static_cast<int>(k - static_cast<int64_t>(y) * a.nx);
        T f[9];
        gather(a.fin, a.plane, x, y, a.nx, a.ny, a.pitch, a.perx, a.pery, a.wall, f);
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

}  // namespace

template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, int src_kind, bool k1_per_node, hipStream_t s)
{
    const unsigned grid = static_cast<unsigned>(a.tiles_x) * static_cast<unsigned>(a.tiles_y);
#define BTRT_SWEEP(SRC, KP) hipLaunchKernelGGL((sweep_kernel<T, SRC, KP>), dim3(grid), dim3(kBlock), 0, s, a)
    if (k1_per_node) {
        if (src_kind == kSrcField) BTRT_SWEEP(kSrcField, true);
        else if (src_kind == kSrcSep) BTRT_SWEEP(kSrcSep, true);
        else BTRT_SWEEP(kSrcNone, true);
    } else {
        if (src_kind == kSrcField) BTRT_SWEEP(kSrcField, false);
        else if (src_kind == kSrcSep) BTRT_SWEEP(kSrcSep, false);
        else BTRT_SWEEP(kSrcNone, false);
    }
#undef BTRT_SWEEP
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init(const T*, T* f, T* phi_prev, const double* phi0, int64_t plane, int nx, int ny,
                       int pitch, int perx, int pery, const double wall[4], double ax, double ay,
                       double bx, double by, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(nx) * ny;
    hipLaunchKernelGGL((init_kernel<T>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, f, phi_prev, phi0, plane,
                       nx, ny, pitch, perx, pery, wall[0], wall[1], wall[2], wall[3], ax, ay, bx, by);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_field(const GatherArgs<T>& a, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(a.nx) * a.ny;
    hipLaunchKernelGGL((gather_field_kernel<T>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce(const GatherArgs<T>& a, int mode, double* result, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(a.nx) * a.ny;
    const unsigned nb = static_cast<unsigned>(std::min<int64_t>(kReduceBlocks, (nn + kBlock - 1) / kBlock));
    if (mode == kResidual)
        hipLaunchKernelGGL((reduce_kernel<T, kResidual>), dim3(nb), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((reduce_kernel<T, kError>), dim3(nb), dim3(kBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kBlock), 0, s, a.partial, static_cast<int>(nb), result);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_convert(const double* in, T* out, int nx, int ny, int pitch, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(nx) * ny;
    hipLaunchKernelGGL((convert_kernel<T>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, in, out, nx, ny, pitch);
    return hipGetLastError();
}

#define BTRT_INSTANTIATE(T)                                                                                  \
    template hipError_t launch_sweep<T>(const SweepArgs<T>&, int, bool, hipStream_t);                       \
    template hipError_t launch_init<T>(const T*, T*, T*, const double*, int64_t, int, int, int, int, int,    \
                                       const double[4], double, double, double, double, hipStream_t);        \
    template hipError_t launch_gather_field<T>(const GatherArgs<T>&, hipStream_t);                          \
    template hipError_t launch_reduce<T>(const GatherArgs<T>&, int, double*, hipStream_t);                  \
    template hipError_t launch_convert<T>(const double*, T*, int, int, int, hipStream_t);

BTRT_INSTANTIATE(double)
BTRT_INSTANTIATE(float)

}  // namespace btrtk
