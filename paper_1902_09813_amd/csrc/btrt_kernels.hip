// gfx950 kernels of the B-TriRT D2Q9 sweep (Zhao, Wu, Chai & Shi, arXiv:1902.09813).
//
// State between steps: the post-collision populations f+(t-1) in 9 SoA planes
// (f[i][y][pitch], i in the velocity order of Eq. (85)) and phi(t-1) in one plane.
// One node update:
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
//
// Storage formats: plain FP64 or FP32 planes, or 16-bit planes (FP16 or BF16) of scaled
// deviations from equilibrium, h_i = q(s (f_i+ - f_i^eq(phi))), with phi(t) in FP32 at the
// same node (the phi plane the sweep writes anyway) and FP32 arithmetic.

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

template <typename T>
__device__ __forceinline__ void store(T* p, T v, bool nontemporal)
{
    // Non-temporal stores keep a grid much larger than the caches from evicting the data
    // the next tiles are about to pull; small grids keep them cached (they fit in the MALL).
    if (nontemporal)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <typename T, int SRC>
__device__ __forceinline__ T source_at(const SweepArgs<T>& a, int n, int x, int y)
{
    if constexpr (SRC == kSrcField) return a.src[n];
    if constexpr (SRC == kSrcSep) return a.src_amp * a.src[x] * a.src_y[y];
    return T(0);
}

// ---- storage formats ---------------------------------------------------------------------
// pull(a, x, y, f): f_i(x, t) from the stored f+(t-1) (with wrap / bounce-back);
// settle(a, f, phi): f+ as the next pull will see it (identity, or the 16-bit round trip);
// put(a, n, f, phi): store f+(t) and phi(t) at node index n.

template <typename T_>
struct Plain {
    using T = T_;
    __device__ static void pull(const SweepArgs<T>& a, int x, int y, T f[9])
    {
        gather(a.fin, a.plane, x, y, a.nx, a.ny, a.pitch, a.perx, a.pery, a.wall, f);
    }
    __device__ static void settle(const SweepArgs<T>&, T*, T) {}
    __device__ static void put(const SweepArgs<T>& a, int n, const T f[9], T phi)
    {
        const int64_t p = a.plane;
#pragma unroll
        for (int i = 0; i < 9; ++i) store(a.fout + i * p + n, f[i], a.nts);
        store(a.phi_out + n, phi, a.nts);
    }
};

// IEEE binary16, round to nearest even.
struct F16Codec {
    __device__ static unsigned short enc(float v) { return __builtin_bit_cast(unsigned short, static_cast<_Float16>(v)); }
    __device__ static float dec(unsigned short h) { return static_cast<float>(__builtin_bit_cast(_Float16, h)); }
};

// bfloat16 (the upper half of an FP32), round to nearest even.
struct BF16Codec {
    __device__ static unsigned short enc(float v)
    {
        unsigned u = __builtin_bit_cast(unsigned, v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<unsigned short>((u >> 16) | 0x40u);  // NaN stays NaN
        u += 0x7fffu + ((u >> 16) & 1u);
        return static_cast<unsigned short>(u >> 16);
    }
    __device__ static float dec(unsigned short h) { return __builtin_bit_cast(float, static_cast<unsigned>(h) << 16); }
};

template <typename C>
struct Dev {
    using T = float;
    __device__ static float rebuild(const SweepArgs<float>& a, int i, float phi, unsigned short h)
    {
        return fmadd(C::dec(h), a.dev_inv, feq_dir(i, phi, a.ax, a.ay, a.bx, a.by));
    }
    __device__ static unsigned short quant(const SweepArgs<float>& a, int i, float f, float phi)
    {
        return C::enc((f - feq_dir(i, phi, a.ax, a.ay, a.bx, a.by)) * a.dev_scale);
    }
    __device__ static void pull(const SweepArgs<float>& a, int x, int y, float f[9])
    {
        const unsigned short* __restrict__ H = reinterpret_cast<const unsigned short*>(a.fin);
        const float* __restrict__ P = a.phi_prev;
        const int64_t p = a.plane;
        gather_with<float>([&](int i, int idx) { return rebuild(a, i, P[idx], H[i * p + idx]); }, x, y, a.nx, a.ny,
                           a.pitch, a.perx, a.pery, a.wall, f);
    }
    __device__ static void settle(const SweepArgs<float>& a, float f[9], float phi)
    {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = rebuild(a, i, phi, quant(a, i, f[i], phi));
    }
    __device__ static void put(const SweepArgs<float>& a, int n, const float f[9], float phi)
    {
        unsigned short* __restrict__ H = reinterpret_cast<unsigned short*>(a.fout);
        const int64_t p = a.plane;
#pragma unroll
        for (int i = 0; i < 9; ++i) store(H + i * p + n, quant(a, i, f[i], phi), a.nts);
        store(a.phi_out + n, phi, a.nts);
    }
};

// ---- one time step --------------------------------------------------------------------------

// One time step on tile (tx, ty) of kTileX x kTileY nodes, one node per thread.
template <typename F, int SRC, bool KPHI>
__device__ __forceinline__ void tile1(const SweepArgs<typename F::T>& a, int tx, int ty)
{
    using T = typename F::T;
    const int x = tx * kTileX + static_cast<int>(threadIdx.x % kTileX);
    const int y = ty * kTileY + static_cast<int>(threadIdx.x / kTileX);
    if (x >= a.nx || y >= a.ny) return;
    T f[9];
    F::pull(a, x, y, f);
    const int n = y * a.pitch + x;
    const T phi = collide<T, SRC, KPHI>(a, f, a.phi_prev[n], source_at<T, SRC>(a, n, x, y));
    F::put(a, n, f, phi);
}

template <typename F, int SRC, bool KPHI>
__global__ __launch_bounds__(kBlock) void sweep_kernel(SweepArgs<typename F::T> a)
{
    const int tile = xcd_tile();
    const int ty = tile / a.tiles_x;
    tile1<F, SRC, KPHI>(a, tile - ty * a.tiles_x, ty);
}

// Wrap a coordinate of a periodic direction into [0, n) (any distance).
__device__ __forceinline__ int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// ---- two time steps per launch --------------------------------------------------------------
// Step 1 runs on a kTile2X x TY tile plus a one-node ring, pulling f+(t-1) from global memory,
// and leaves f+(t) (as the next pull would see it) and phi(t) in LDS; step 2 runs on the tile,
// pulling f+(t) from LDS (bounce-back at Dirichlet walls uses the node's own LDS values), and
// stores f+(t+1) and phi(t+1). Every node update is the same arithmetic as in sweep_kernel, so
// results are bitwise identical to two single steps; HBM traffic per node update is halved.
constexpr int kTile2X = 64;
constexpr int kBlock2 = 512;

template <typename T>
struct Tile2 {
    static constexpr int TY = sizeof(T) == 8 ? 8 : 16;  // LDS: FP64 52.8 KB, FP32 47.5 KB
    static constexpr int EX = kTile2X + 2, EY = TY + 2, E = EX * EY;
    static constexpr int S1 = (E + kBlock2 - 1) / kBlock2;
    static constexpr int S2 = (kTile2X * TY + kBlock2 - 1) / kBlock2;
};

template <typename F, int SRC, bool KPHI>
__device__ __forceinline__ void tile2(const SweepArgs<typename F::T>& a, int tx, int ty,
                                      typename F::T (&lf)[9][Tile2<typename F::T>::E],
                                      typename F::T (&lphi)[Tile2<typename F::T>::E])
{
    using T = typename F::T;
    using G = Tile2<T>;
    constexpr int TX = kTile2X, TY = G::TY, EX = G::EX, E = G::E;
    const int nx = a.nx, ny = a.ny;
    const int x0 = tx * TX - 1, y0 = ty * TY - 1;  // global position of LDS slot (0, 0)

    // Step 1 on the extended tile; all loads are issued before any collision.
    T f[G::S1][9];
    T pp[G::S1];
    int gxs[G::S1], gys[G::S1];
    bool live[G::S1];
#pragma unroll
    for (int j = 0; j < G::S1; ++j) {
        const int s = static_cast<int>(threadIdx.x) + j * kBlock2;
        const int ly = s / EX, lx = s - ly * EX;
        int gx = x0 + lx, gy = y0 + ly;
        bool e = s < E;
        if (gx < 0 || gx >= nx) {
            if (a.perx) gx = wrap(gx, nx); else e = false;
        }
        if (gy < 0 || gy >= ny) {
            if (a.pery) gy = wrap(gy, ny); else e = false;
        }
        live[j] = e;
        gxs[j] = gx;
        gys[j] = gy;
        if (e) {
            F::pull(a, gx, gy, f[j]);
            pp[j] = a.phi_prev[gy * a.pitch + gx];
        }
    }
#pragma unroll
    for (int j = 0; j < G::S1; ++j) {
        if (!live[j]) continue;
        const int s = static_cast<int>(threadIdx.x) + j * kBlock2;
        const int n = gys[j] * a.pitch + gxs[j];
        const T phi = collide<T, SRC, KPHI>(a, f[j], pp[j], source_at<T, SRC>(a, n, gxs[j], gys[j]));
        F::settle(a, f[j], phi);
#pragma unroll
        for (int i = 0; i < 9; ++i) lf[i][s] = f[j][i];
        lphi[s] = phi;
    }
    __syncthreads();

    // Step 2 on the tile, pulling from LDS.
    const T tw1 = T(2) * Lat<T>::w1, tw5 = T(2) * Lat<T>::w5;
#pragma unroll
    for (int j = 0; j < G::S2; ++j) {
        const int s = static_cast<int>(threadIdx.x) + j * kBlock2;
        if (s >= TX * TY) continue;
        const int iy = s / TX, ix = s - iy * TX;
        const int gx = tx * TX + ix, gy = ty * TY + iy;
        if (gx >= nx || gy >= ny) continue;
        const int l = (iy + 1) * EX + ix + 1;
        const bool okxm = a.perx || gx > 0, okxp = a.perx || gx < nx - 1;
        const bool okym = a.pery || gy > 0, okyp = a.pery || gy < ny - 1;
        T g[9];
        g[0] = lf[0][l];
        g[1] = okxm ? lf[1][l - 1] : bounce(lf[3][l], tw1, a.wall[0]);
        g[2] = okym ? lf[2][l - EX] : bounce(lf[4][l], tw1, a.wall[2]);
        g[3] = okxp ? lf[3][l + 1] : bounce(lf[1][l], tw1, a.wall[1]);
        g[4] = okyp ? lf[4][l + EX] : bounce(lf[2][l], tw1, a.wall[3]);
        g[5] = (okxm && okym) ? lf[5][l - EX - 1] : bounce(lf[7][l], tw5, wall_value(!okxm, !okym, a.wall[0], a.wall[2]));
        g[6] = (okxp && okym) ? lf[6][l - EX + 1] : bounce(lf[8][l], tw5, wall_value(!okxp, !okym, a.wall[1], a.wall[2]));
        g[7] = (okxp && okyp) ? lf[7][l + EX + 1] : bounce(lf[5][l], tw5, wall_value(!okxp, !okyp, a.wall[1], a.wall[3]));
        g[8] = (okxm && okyp) ? lf[8][l + EX - 1] : bounce(lf[6][l], tw5, wall_value(!okxm, !okyp, a.wall[0], a.wall[3]));
        const int n = gy * a.pitch + gx;
        const T phi = collide<T, SRC, KPHI>(a, g, lphi[l], source_at<T, SRC>(a, n, gx, gy));
        F::put(a, n, g, phi);
    }
}

template <typename F, int SRC, bool KPHI>
__global__ __launch_bounds__(kBlock2) void sweep2_kernel(SweepArgs<typename F::T> a)
{
    using T = typename F::T;
    __shared__ T lf[9][Tile2<T>::E];
    __shared__ T lphi[Tile2<T>::E];
    const int tile = xcd_tile();
    const int ty = tile / a.tiles_x;
    tile2<F, SRC, KPHI>(a, tile - ty * a.tiles_x, ty, lf, lphi);
}

// ---- many instances in one launch -------------------------------------------------------
// The tiles of all instances form one list (instance i owns tiles begin[i] .. begin[i+1]-1).
// A persistent grid walks the list; each tile reads its instance's arguments (uniform per
// block, so they land in scalar registers) and runs the same tile body as a single solve.
// Instance i's buffers swap every launch: it uses a[par[i] ^ flip].

// Instance index owning tile t: the last i with begin[i] <= t.
__device__ __forceinline__ int owner(const int* __restrict__ begin, int ninst, int t)
{
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void batch1_kernel(const BatchEntry<T>* __restrict__ ent,
                                                        const int* __restrict__ begin, const int* __restrict__ par,
                                                        int ninst, int total, int flip)
{
    using F = Plain<T>;
    const int g = static_cast<int>(gridDim.x);
    for (int t = xcd_tile(); t < total; t += g) {
        const int i = owner(begin, ninst, t);
        const SweepArgs<T> a = ent[i].a[par[i] ^ flip];
        const int local = t - begin[i];
        const int tiles_x = (a.nx + kTileX - 1) / kTileX;
        const int ty = local / tiles_x, tx = local - ty * tiles_x;
        switch (ent[i].variant) {
            case 0: tile1<F, kSrcNone, false>(a, tx, ty); break;
            case 1: tile1<F, kSrcNone, true>(a, tx, ty); break;
            case 2: tile1<F, kSrcField, false>(a, tx, ty); break;
            case 3: tile1<F, kSrcField, true>(a, tx, ty); break;
            case 4: tile1<F, kSrcSep, false>(a, tx, ty); break;
            default: tile1<F, kSrcSep, true>(a, tx, ty); break;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock2) void batch2_kernel(const BatchEntry<T>* __restrict__ ent,
                                                         const int* __restrict__ begin, const int* __restrict__ par,
                                                         int ninst, int total, int flip)
{
    using F = Plain<T>;
    __shared__ T lf[9][Tile2<T>::E];
    __shared__ T lphi[Tile2<T>::E];
    const int g = static_cast<int>(gridDim.x);
    for (int t = xcd_tile(); t < total; t += g) {
        const int i = owner(begin, ninst, t);
        const SweepArgs<T> a = ent[i].a[par[i] ^ flip];
        const int local = t - begin[i];
        const int tiles_x = (a.nx + kTile2X - 1) / kTile2X;
        const int ty = local / tiles_x, tx = local - ty * tiles_x;
        switch (ent[i].variant) {
            case 0: tile2<F, kSrcNone, false>(a, tx, ty, lf, lphi); break;
            case 1: tile2<F, kSrcNone, true>(a, tx, ty, lf, lphi); break;
            case 2: tile2<F, kSrcField, false>(a, tx, ty, lf, lphi); break;
            case 3: tile2<F, kSrcField, true>(a, tx, ty, lf, lphi); break;
            case 4: tile2<F, kSrcSep, false>(a, tx, ty, lf, lphi); break;
            default: tile2<F, kSrcSep, true>(a, tx, ty, lf, lphi); break;
        }
        __syncthreads();  // the next tile reuses the LDS
    }
}

// ---- set-up, field reads and reductions -------------------------------------------------

// f+(-1) such that the first pull yields f(0) = f^eq(phi0) (Section 4 initialisation), and
// phi(-1) := phi0; written through the format's put into a.fout / a.phi_out.
template <typename F>
__global__ __launch_bounds__(kBlock) void init_kernel(SweepArgs<typename F::T> a, const double* __restrict__ phi0,
                                                      double w0, double w1, double w2, double w3, double ax,
                                                      double ay, double bx, double by)
{
    using T = typename F::T;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= static_cast<int64_t>(a.nx) * a.ny) return;
    const int y = static_cast<int>(k / a.nx);
    const int x = static_cast<int>(k - static_cast<int64_t>(y) * a.nx);
    const double wall[4] = {w0, w1, w2, w3};
    T f[9];
    init_values(phi0, x, y, a.nx, a.ny, a.perx, a.pery, wall, ax, ay, bx, by,
                [&](int i, double v) { f[i] = static_cast<T>(v); });
    F::put(a, y * a.pitch + x, f, static_cast<T>(phi0[k]));
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
template <typename F>
__global__ __launch_bounds__(kBlock) void gather_field_kernel(GatherArgs<typename F::T> a)
{
    using T = typename F::T;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= static_cast<int64_t>(a.s.nx) * a.s.ny) return;
    const int y = static_cast<int>(k / a.s.nx);
    const int x = static_cast<int>(k - static_cast<int64_t>(y) * a.s.nx);
    T f[9];
    F::pull(a.s, x, y, f);
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
        F::pull(a.s, x, y, f);
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
hipError_t sweep_with(const SweepArgs<typename F::T>& a_in, int src_kind, bool k1_per_node, int steps, hipStream_t s)
{
    using T = typename F::T;
    SweepArgs<T> a = a_in;
    if (steps == 2) {
        a.tiles_x = (a.nx + kTile2X - 1) / kTile2X;
        a.tiles_y = (a.ny + Tile2<T>::TY - 1) / Tile2<T>::TY;
    } else {
        a.tiles_x = (a.nx + kTileX - 1) / kTileX;
        a.tiles_y = (a.ny + kTileY - 1) / kTileY;
    }
    const unsigned grid = static_cast<unsigned>(a.tiles_x) * static_cast<unsigned>(a.tiles_y);
#define BTRT_SWEEP(SRC, KP)                                                                                \
    do {                                                                                                   \
        if (steps == 2)                                                                                    \
            hipLaunchKernelGGL((sweep2_kernel<F, SRC, KP>), dim3(grid), dim3(kBlock2), 0, s, a);          \
        else                                                                                               \
            hipLaunchKernelGGL((sweep_kernel<F, SRC, KP>), dim3(grid), dim3(kBlock), 0, s, a);            \
    } while (0)
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

template <typename F>
hipError_t init_with(const SweepArgs<typename F::T>& a, const double* phi0, const double wall[4], double ax, double ay,
                     double bx, double by, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(a.nx) * a.ny;
    hipLaunchKernelGGL((init_kernel<F>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, a, phi0, wall[0], wall[1], wall[2],
                       wall[3], ax, ay, bx, by);
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
hipError_t launch_sweep(const SweepArgs<T>& a, int fmt, int src_kind, bool k1_per_node, int steps, hipStream_t s)
{
    BTRT_BY_FORMAT(T, sweep_with, a, src_kind, k1_per_node, steps, s);
}

template <typename T>
hipError_t launch_init(const SweepArgs<T>& a, int fmt, const double* phi0, const double wall[4], double ax, double ay,
                       double bx, double by, hipStream_t s)
{
    BTRT_BY_FORMAT(T, init_with, a, phi0, wall, ax, ay, bx, by, s);
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
hipError_t launch_batch_sweep(const BatchEntry<T>* ent, const int* begin, const int* par, int ninst, int total_tiles,
                              int flip, int steps, int grid, hipStream_t s)
{
    if (total_tiles <= 0 || ninst <= 0) return hipSuccess;
    const unsigned g = static_cast<unsigned>(grid > 0 ? std::min(grid, total_tiles) : total_tiles);
    if (steps == 2)
        hipLaunchKernelGGL((batch2_kernel<T>), dim3(g), dim3(kBlock2), 0, s, ent, begin, par, ninst, total_tiles, flip);
    else
        hipLaunchKernelGGL((batch1_kernel<T>), dim3(g), dim3(kBlock), 0, s, ent, begin, par, ninst, total_tiles, flip);
    return hipGetLastError();
}

int tile_rows(int steps, int precision_bytes)
{
    if (steps == 2) return precision_bytes == 8 ? Tile2<double>::TY : Tile2<float>::TY;
    return kTileY;
}

template <typename T>
hipError_t launch_convert(const double* in, T* out, int nx, int ny, int pitch, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(nx) * ny;
    hipLaunchKernelGGL((convert_kernel<T>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, in, out, nx, ny, pitch);
    return hipGetLastError();
}

#define BTRT_INSTANTIATE(T)                                                                                        \
    template hipError_t launch_sweep<T>(const SweepArgs<T>&, int, int, bool, int, hipStream_t);                   \
    template hipError_t launch_init<T>(const SweepArgs<T>&, int, const double*, const double[4], double, double,   \
                                       double, double, hipStream_t);                                               \
    template hipError_t launch_gather_field<T>(const GatherArgs<T>&, int, hipStream_t);                           \
    template hipError_t launch_reduce<T>(const GatherArgs<T>&, int, int, double*, hipStream_t);                   \
    template hipError_t launch_convert<T>(const double*, T*, int, int, int, hipStream_t);                         \
    template hipError_t launch_batch_sweep<T>(const BatchEntry<T>*, const int*, const int*, int, int, int, int, int, \
                                              hipStream_t);

BTRT_INSTANTIATE(double)
BTRT_INSTANTIATE(float)

}  // namespace btrtk
