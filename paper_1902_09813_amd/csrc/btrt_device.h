// gfx950 kernels of the B-TriRT D2Q9 sweep (Zhao, Wu, Chai & Shi, arXiv:1902.09813).
//
// State between steps: the post-collision populations f+(t-1) in 9 SoA planes
// (f[i][y][pitch], i in the velocity order of Eq. (85)) and phi(t-1) in one plane.
// One node update:
//   1. pull  f_i(x, t) = f_i+(x - c_i, t-1)                         (Eq. (38))
//      or, when x - c_i lies beyond a Dirichlet wall,
//            f_i(x, t) = -f_opp(i)+(x, t-1) + 2 w_i phi_w             (Eqs. (54)-(56))
//   2. phi, j and P (rows of Eq. (88)) from sums and differences of opposite populations
//   3. Eq. (6): f_i+ = (1 - k0) f_i + w_i [E_i + 3 c_i . q], the moments the block relaxation
//      of Eq. (99) changes (j with K1, P with K2) folded into q and E_i, with the equilibrium
//      of Eq. (7), the source of Eq. (8) and G of Eq. (11)
//   4. aligned stores of f+(t) and phi(t)
// Reads and writes are disjoint (two population buffers), so no synchronisation is needed.
// A node update is about a hundred FP64 operations in registers, with no dense contraction:
// there is no matrix-core work here.
//
// Storage formats: plain FP64 or FP32 planes, or 16-bit planes (FP16 or BF16) of scaled
// deviations from equilibrium, h_i = q(s (f_i+ - f_i^eq(phi))), with phi(t) in FP32 at the
// same node (the phi plane the sweep writes anyway) and FP32 arithmetic.
//
// This header holds the device code (storage formats, the one-step, two-step and strip-walker
// sweeps, the batched kernels) and the host templates that shape and launch the sweeps. It is
// included by several translation units, each instantiating its own part (one per storage
// format, one for batches), so the library builds in parallel.
#pragma once

#include "btrt_internal.h"
#include "btrt_node.h"

#include <algorithm>
#include <type_traits>

namespace btrtk {
namespace {


constexpr int kTileX = 64;  // one wavefront along a row: coalesced 64-wide accesses
constexpr int kTileY = kBlock / kTileX;
constexpr int kMaxBlock1 = 1024;  // one-step kernel: tiles of up to 64 x 16 nodes

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

// NT: a non-temporal store (the caches do not keep the line). On grids much larger than the
// caches it keeps the written state from evicting what the next tiles are about to pull (the
// one-step and two-step tile kernels, single grids and batches, run 4-9 % faster on MI355X);
// grids that fit in the Infinity Cache keep their stores cached for the next step. The strip
// walkers store normally at every size: they write once per K steps, and non-temporal stores
// made the FP32 seven-step walker 15 % slower. A compile-time choice: with a run-time flag the
// compiler merges the two stores of the branch into one and drops the non-temporal hint.
template <bool NT, typename T>
__device__ __forceinline__ void store(T* p, T v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <typename T, int SRC>
// Source term of step `lvl` of the launch at node n = (x, y): the time-independent part times
// that step's factor (Scheme 2 folded in, 1 for a source constant in time).
__device__ __forceinline__ T source_at(const SweepArgs<T>& a, int n, int x, int y, int lvl)
{
    if constexpr (SRC == kSrcField) return a.src[n] * a.sfac[lvl];
    if constexpr (SRC == kSrcSep) return (a.src_amp * a.src[x] * a.src_y[y]) * a.sfac[lvl];
    return T(0);
}

// ---- storage formats ---------------------------------------------------------------------
// pull(a, x, y, f): f_i(x, t) from the stored f+(t-1) (with wrap / bounce-back);
// settle(a, f, phi): f+ as the next pull will see it (identity, or the 16-bit round trip);
// put<NT>(a, n, f, phi): store f+(t) and phi(t) at node index n (NT: non-temporal stores).

template <typename T_>
struct Plain {
    using T = T_;
    // With a wall table (TABLE: the general node model) an edge node takes its Dirichlet values
    // from the table entry of the launch's first step.
    template <bool TABLE>
    __device__ __forceinline__ static void pull(const SweepArgs<T>& a, int x, int y, T f[9])
    {
        gather(a.fin, a.plane, x, y, a.nx, a.ny, a.pitch, a.perx, a.pery,
               [&](int i, bool ox, bool oy) {
                   if constexpr (TABLE)
                       return table_wall(a, x, y, 0, i, ox, oy);
                   else
                       return side_wall(a.wall, i, ox, oy);
               },
               f);
    }
    __device__ __forceinline__ static void settle(const SweepArgs<T>&, T*, T) {}
    // Raw loads of one node's pull (see walk_load): value read for each direction.
    struct Raw {
        T v[9];
    };
    __device__ __forceinline__ static void fetch(const SweepArgs<T>& a, const int plane[9], const int idx[9], Raw& r)
    {
        const int64_t p = a.plane;
#pragma unroll
        for (int i = 0; i < 9; ++i) r.v[i] = a.fin[plane[i] * p + idx[i]];
    }
    __device__ __forceinline__ static T value(const SweepArgs<T>&, const Raw& r, int i, int, bool) { return r.v[i]; }
    template <bool NT>
    __device__ __forceinline__ static void put(const SweepArgs<T>& a, int n, const T f[9], T phi)
    {
        const int64_t p = a.plane;
#pragma unroll
        for (int i = 0; i < 9; ++i) store<NT>(a.fout + i * p + n, f[i]);
        store<NT>(a.phi_out + n, phi);
    }
};

// Plain FP64/FP32 storage (as opposed to the 16-bit deviation formats).
template <typename F>
constexpr bool plain_format()
{
    return std::is_same<F, Plain<typename F::T>>::value;
}

// The collision's mode for storage format F: the kernel mode, plus kRcp1 for the 16-bit formats.
template <typename F, int KM>
constexpr int collide_mode()
{
    return plain_format<F>() ? KM : (KM | kRcp1);
}

// IEEE binary16, round to nearest even.
struct F16Codec {
    __device__ __forceinline__ static unsigned short enc(float v) { return __builtin_bit_cast(unsigned short, static_cast<_Float16>(v)); }
    __device__ __forceinline__ static float dec(unsigned short h) { return static_cast<float>(__builtin_bit_cast(_Float16, h)); }
};

// bfloat16 (the upper half of an FP32), round to nearest even. gfx950 converts in one
// instruction (v_cvt_pk_bf16_f32); over all 2^32 FP32 inputs it gives the bits of the integer
// rounding u + 0x7fff + (bit 16 of u), NaNs kept quiet (u | 0x400000) -- checked exhaustively on
// the device.
struct BF16Codec {
    __device__ __forceinline__ static unsigned short enc(float v)
    {
        return __builtin_bit_cast(unsigned short, static_cast<__bf16>(v));
    }
    __device__ __forceinline__ static float dec(unsigned short h) { return __builtin_bit_cast(float, static_cast<unsigned>(h) << 16); }
};

template <typename C>
struct Dev {
    using T = float;
    __device__ __forceinline__ static float rebuild(const SweepArgs<float>& a, int i, float phi, unsigned short h)
    {
        return fmadd(C::dec(h), a.dev_inv, feq_dir(i, phi, a.ax, a.ay, a.bx, a.by));
    }
    __device__ __forceinline__ static unsigned short quant(const SweepArgs<float>& a, int i, float f, float phi)
    {
        return C::enc((f - feq_dir(i, phi, a.ax, a.ay, a.bx, a.by)) * a.dev_scale);
    }
    template <bool TABLE>  // the 16-bit formats take per-side constants only
    __device__ __forceinline__ static void pull(const SweepArgs<float>& a, int x, int y, float f[9])
    {
        const unsigned short* __restrict__ H = reinterpret_cast<const unsigned short*>(a.fin);
        const float* __restrict__ P = a.phi_prev;
        const int64_t p = a.plane;
        gather_with<float>([&](int i, int idx) { return rebuild(a, i, P[idx], H[i * p + idx]); }, x, y, a.nx, a.ny,
                           a.pitch, a.perx, a.pery,
                           [&](int i, bool ox, bool oy) { return side_wall(a.wall, i, ox, oy); }, f);
    }
    // Raw loads of one node's pull: the 16-bit code and phi(t-1) of the node it comes from.
    struct Raw {
        unsigned short h[9];
        float p[9];
    };
    __device__ __forceinline__ static void fetch(const SweepArgs<float>& a, const int plane[9], const int idx[9],
                                                 Raw& r)
    {
        const unsigned short* __restrict__ H = reinterpret_cast<const unsigned short*>(a.fin);
        const int64_t p = a.plane;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            r.h[i] = H[plane[i] * p + idx[i]];
            r.p[i] = a.phi_prev[idx[i]];
        }
    }
    // Value read for direction i: population i of the source node, or, when `own`
    // (bounce-back), population o (the opposite direction) of the node itself.
    __device__ __forceinline__ static float value(const SweepArgs<float>& a, const Raw& r, int i, int o, bool own)
    {
        const float e = own ? feq_dir(o, r.p[i], a.ax, a.ay, a.bx, a.by) : feq_dir(i, r.p[i], a.ax, a.ay, a.bx, a.by);
        return fmadd(C::dec(r.h[i]), a.dev_inv, e);
    }
    __device__ __forceinline__ static void settle(const SweepArgs<float>& a, float f[9], float phi)
    {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = rebuild(a, i, phi, quant(a, i, f[i], phi));
    }
    template <bool NT>
    __device__ __forceinline__ static void put(const SweepArgs<float>& a, int n, const float f[9], float phi)
    {
        unsigned short* __restrict__ H = reinterpret_cast<unsigned short*>(a.fout);
        const int64_t p = a.plane;
#pragma unroll
        for (int i = 0; i < 9; ++i) store<NT>(H + i * p + n, quant(a, i, f[i], phi));
        store<NT>(a.phi_out + n, phi);
    }
};

// ---- one time step --------------------------------------------------------------------------

// One time step on tile (tx, ty) of kTileX x rows nodes, one node per thread.
template <typename F, int SRC, int KM, bool NT>
__device__ __forceinline__ void tile1(const SweepArgs<typename F::T>& a, int tx, int ty, int rows)
{
    using T = typename F::T;
    const int x = tx * kTileX + static_cast<int>(threadIdx.x % kTileX);
    const int y = ty * rows + static_cast<int>(threadIdx.x / kTileX);
    if (x >= a.nx || y >= a.ny) return;
    T f[9];
    F::template pull<(KM & kGen) != 0>(a, x, y, f);
    const int n = y * a.pitch + x;
    const T phi = collide<T, SRC, collide_mode<F, KM>()>(a, f, a.phi_prev[n], source_at<T, SRC>(a, n, x, y, 0), n);
    F::template put<NT>(a, n, f, phi);
}

// Tiles of 64 x (blockDim.x / 64) nodes; taller tiles re-read fewer halo rows of their
// neighbours above and below.
template <typename F, int SRC, int KM, bool NT>
__global__ __launch_bounds__(kMaxBlock1) void sweep_kernel(SweepArgs<typename F::T> a)
{
    const int tile = xcd_tile();
    const int ty = tile / a.tiles_x;
    tile1<F, SRC, KM, NT>(a, tile - ty * a.tiles_x, ty, static_cast<int>(blockDim.x) / kTileX);
}

// Wrap a coordinate of a periodic direction into [0, n) (any distance).
__device__ __forceinline__ int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// ---- two time steps per tile through LDS -------------------------------------------------------
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

template <typename F, int SRC, int KM, bool NT>
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
            F::template pull<(KM & kGen) != 0>(a, gx, gy, f[j]);
            pp[j] = a.phi_prev[gy * a.pitch + gx];
        }
    }
#pragma unroll
    for (int j = 0; j < G::S1; ++j) {
        if (!live[j]) continue;
        const int s = static_cast<int>(threadIdx.x) + j * kBlock2;
        const int n = gys[j] * a.pitch + gxs[j];
        const T phi = collide<T, SRC, collide_mode<F, KM>()>(a, f[j], pp[j], source_at<T, SRC>(a, n, gxs[j], gys[j], 0), n);
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
        auto wv = [&](int i, bool ox, bool oy) {
            if constexpr ((KM & kGen) != 0)
                return table_wall(a, gx, gy, 1, i, ox, oy);
            else
                return side_wall(a.wall, i, ox, oy);
        };
        T g[9];
        g[0] = lf[0][l];
        g[1] = okxm ? lf[1][l - 1] : bounce(lf[3][l], tw1, wv(1, true, false));
        g[2] = okym ? lf[2][l - EX] : bounce(lf[4][l], tw1, wv(2, false, true));
        g[3] = okxp ? lf[3][l + 1] : bounce(lf[1][l], tw1, wv(3, true, false));
        g[4] = okyp ? lf[4][l + EX] : bounce(lf[2][l], tw1, wv(4, false, true));
        g[5] = (okxm && okym) ? lf[5][l - EX - 1] : bounce(lf[7][l], tw5, wv(5, !okxm, !okym));
        g[6] = (okxp && okym) ? lf[6][l - EX + 1] : bounce(lf[8][l], tw5, wv(6, !okxp, !okym));
        g[7] = (okxp && okyp) ? lf[7][l + EX + 1] : bounce(lf[5][l], tw5, wv(7, !okxp, !okyp));
        g[8] = (okxm && okyp) ? lf[8][l + EX - 1] : bounce(lf[6][l], tw5, wv(8, !okxm, !okyp));
        const int n = gy * a.pitch + gx;
        const T phi = collide<T, SRC, collide_mode<F, KM>()>(a, g, lphi[l], source_at<T, SRC>(a, n, gx, gy, 1), n);
        F::template put<NT>(a, n, g, phi);
    }
}

template <typename F, int SRC, int KM, bool NT>
__global__ __launch_bounds__(kBlock2) void sweep2_kernel(SweepArgs<typename F::T> a)
{
    using T = typename F::T;
    __shared__ T lf[9][Tile2<T>::E];
    __shared__ T lphi[Tile2<T>::E];
    const int tile = xcd_tile();
    const int ty = tile / a.tiles_x;
    tile2<F, SRC, KM, NT>(a, tile - ty * a.tiles_x, ty, lf, lphi);
}

// ---- K time steps per launch: strip walkers ------------------------------------------------
// One wavefront owns a strip of W = 64 - 2(K-1) columns by a.rows rows and walks down it one row
// per iteration; its 64 lanes hold the strip plus K-1 halo columns on each side. In iteration r,
// step 1 of the launch updates row r from the populations in global memory, and step l
// (l = 2..K) updates row r-(l-1) from rows r-l .. r-l+2 of step l-1, which stay in registers
// (the row below, the row itself and the row step l-1 has just produced); the x-1 / x+1
// neighbours come from the adjacent lanes through DPP wavefront shifts. Step K stores. Each
// step narrows the valid region by one node per side, so step l is valid on lanes l-1 .. 64-l
// and rows ys-(K-l) .. ys+L-1+(K-l). There is no LDS and no barrier; the state is read and
// written once per launch, plus the halo columns (64/W) and rows ((L+2(K-1))/L) on the read side.
// Every node update is the same arithmetic as in sweep_kernel (collide and the format's round
// trip), so K steps in one launch give the bits of K single steps.

constexpr int kWave = 64;
constexpr int kShr1 = 0x138;  // DPP wave_shr:1, lane j receives lane j-1
constexpr int kShl1 = 0x130;  // DPP wave_shl:1, lane j receives lane j+1

template <int CTRL>
__device__ __forceinline__ int lane_shift_b32(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ float lane_shift(float v)
{
    return __builtin_bit_cast(float, lane_shift_b32<CTRL>(__builtin_bit_cast(int, v)));
}

template <int CTRL>
__device__ __forceinline__ double lane_shift(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = static_cast<unsigned>(lane_shift_b32<CTRL>(static_cast<int>(static_cast<unsigned>(u))));
    const unsigned hi = static_cast<unsigned>(lane_shift_b32<CTRL>(static_cast<int>(static_cast<unsigned>(u >> 32))));
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

template <int K>
struct Walk {
    static constexpr int W = kWave - 2 * (K - 1);  // output columns per strip
};

// One row of one time level as the next level pulls it: f+ (after the format's round trip)
// and phi.
template <typename T>
struct Level {
    T f[9];
    T phi;
};

// What a walker lane keeps between rows. For each level l < K: the populations of the row
// below the one level l+1 updates next that move up (2, 5, 6), and that row itself, in one of
// two buffers that alternate from row to row (so no row is copied); and the last level's row
// waiting to be stored.
template <typename T, int K>
struct WalkState {
    T up[K - 1][3];
    Level<T> mid[2][K - 1];
    Level<T> out;
    int out_n;  // node index of `out`, -1 when nothing waits
};

// Row coordinate of a walker: wrapped into the grid (periodic), with validity and wall flags.
struct WalkRow {
    int y;       // row inside [0, ny) (clamped when invalid)
    bool ok;     // a node row of the grid
    bool okm;    // the y-1 pull is a node (else bounce-back at the y- wall)
    bool okp;    // the y+1 pull is a node (else bounce-back at the y+ wall)
};

__device__ __forceinline__ WalkRow walk_row(int q, int ny, int pery)
{
    WalkRow w;
    if (pery) {
        w.y = wrap(q, ny);
        w.ok = true;
        w.okm = w.okp = true;
    } else {
        w.ok = q >= 0 && q < ny;
        w.y = q < 0 ? 0 : (q >= ny ? ny - 1 : q);
        w.okm = w.y > 0;
        w.okp = w.y < ny - 1;
    }
    return w;
}

// Level l >= 2 at one node: pull from level l-1's rows below (up: populations 2, 5, 6), at
// (mid) and above (fresh, just produced), then collide. All lanes must be active here (the
// wavefront shifts read the neighbouring lanes).
template <typename T, int SRC, int KM, bool WALLS>
__device__ __forceinline__ T walk_collide(const SweepArgs<T>& a, const T up[3], const Level<T>& mid,
                                          const Level<T>& fresh, int x, bool okxm, bool okxp, const WalkRow& row,
                                          int lvl, T g[9])
{
    const T* m = mid.f;
    const T s1 = lane_shift<kShr1>(m[1]);
    const T s3 = lane_shift<kShl1>(m[3]);
    const T s5 = lane_shift<kShr1>(up[1]);
    const T s6 = lane_shift<kShl1>(up[2]);
    const T s7 = lane_shift<kShl1>(fresh.f[7]);
    const T s8 = lane_shift<kShr1>(fresh.f[8]);
    if constexpr (!WALLS) {  // periodic in both directions: no bounce-back
        okxm = okxp = true;
    }
    const bool okym = WALLS ? row.okm : true, okyp = WALLS ? row.okp : true;
    const T tw1 = T(2) * Lat<T>::w1, tw5 = T(2) * Lat<T>::w5;
    auto wv = [&](int i, bool ox, bool oy) {
        if constexpr (WALLS && (KM & kGen) != 0)
            return table_wall(a, x, row.y, lvl, i, ox, oy);
        else
            return side_wall(a.wall, i, ox, oy);
    };
    g[0] = m[0];
    g[1] = okxm ? s1 : bounce(m[3], tw1, wv(1, true, false));
    g[2] = okym ? up[0] : bounce(m[4], tw1, wv(2, false, true));
    g[3] = okxp ? s3 : bounce(m[1], tw1, wv(3, true, false));
    g[4] = okyp ? fresh.f[4] : bounce(m[2], tw1, wv(4, false, true));
    g[5] = (okxm && okym) ? s5 : bounce(m[7], tw5, wv(5, !okxm, !okym));
    g[6] = (okxp && okym) ? s6 : bounce(m[8], tw5, wv(6, !okxp, !okym));
    g[7] = (okxp && okyp) ? s7 : bounce(m[5], tw5, wv(7, !okxp, !okyp));
    g[8] = (okxm && okyp) ? s8 : bounce(m[6], tw5, wv(8, !okxm, !okyp));
    const int n = row.y * a.pitch + x;
    return collide<T, SRC, KM>(a, g, mid.phi, source_at<T, SRC>(a, n, x, row.y, lvl), n);
}

// Level-1 inputs of row r at column x, as raw loads: for each direction the source address is
// the neighbour x - c_i (wrapped on periodic sides) or, when that lies beyond a Dirichlet wall,
// the node's own opposite population (bounce-back); every load is issued unconditionally from a
// valid address and the values are only used (bounce-back, decoding) an iteration later.
template <typename F>
struct WalkIn {
    typename F::Raw raw;
    typename F::T phi;   // phi(t-1) of the node
    typename F::T w[9];  // general model: the Dirichlet value of each pull that crosses a wall
    //                        (directions 1..8, from the wall table; 0 where the pull is a node)
    int ok;              // bit 0: x-1 is a node, 1: x+1, 2: y-1, 3: y+1; bit 4: (x, r) is a node
};

// Rows of a periodic walk past its fill rows, as counters kept inside [0, ny): y[0] the row of
// the next loads, y[l] the row level l updates. Every step moves each by one row, which needs a
// compare and a select for any grid height, where wrapping a row number afresh needs a division.
template <int K>
struct WalkCursor {
    int y[K + 1];
};

template <int K>
__device__ __forceinline__ void cursor_start(WalkCursor<K>& c, int r, int ahead, int ny)
{
    c.y[0] = wrap(r + ahead, ny);
#pragma unroll
    for (int l = 1; l <= K; ++l) c.y[l] = wrap(r - (l - 1), ny);
}

template <int K>
__device__ __forceinline__ void cursor_next(WalkCursor<K>& c, int ny)
{
#pragma unroll
    for (int l = 0; l <= K; ++l) c.y[l] = c.y[l] + 1 == ny ? 0 : c.y[l] + 1;
}

__device__ __forceinline__ WalkRow periodic_row(int y) { return WalkRow{y, true, true, true}; }

template <typename F, bool WALLS, bool GEN>
__device__ __forceinline__ void walk_load_row(const SweepArgs<typename F::T>& a, int x, bool colok, const WalkRow& w,
                                              WalkIn<F>& in)
{
    const int nx = a.nx, ny = a.ny, pitch = a.pitch, y = w.y;
    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
    bool okxm = true, okxp = true, okym = true, okyp = true;
    if constexpr (WALLS) {
        if (xm < 0) { if (a.perx) xm += nx; else { okxm = false; xm = x; } }
        if (xp >= nx) { if (a.perx) xp -= nx; else { okxp = false; xp = x; } }
        if (ym < 0) { if (a.pery) ym += ny; else { okym = false; ym = y; } }
        if (yp >= ny) { if (a.pery) yp -= ny; else { okyp = false; yp = y; } }
    } else {
        if (xm < 0) xm += nx;
        if (xp >= nx) xp -= nx;
        if (ym < 0) ym += ny;
        if (yp >= ny) yp -= ny;
    }
    const int n = y * pitch + x, r0 = y * pitch, rm = ym * pitch, rp = yp * pitch;
    const bool ok5 = okxm && okym, ok6 = okxp && okym, ok7 = okxp && okyp, ok8 = okxm && okyp;
    const int plane[9] = {0, okxm ? 1 : 3, okym ? 2 : 4, okxp ? 3 : 1, okyp ? 4 : 2,
                          ok5 ? 5 : 7, ok6 ? 6 : 8, ok7 ? 7 : 5, ok8 ? 8 : 6};
    const int idx[9] = {n, okxm ? r0 + xm : n, okym ? rm + x : n, okxp ? r0 + xp : n, okyp ? rp + x : n,
                        ok5 ? rm + xm : n, ok6 ? rm + xp : n, ok7 ? rp + xp : n, ok8 ? rp + xm : n};
    F::fetch(a, plane, idx, in.raw);
    in.phi = a.phi_prev[n];
    if constexpr (WALLS && GEN) {  // x, y are in the grid, so every table index is in range
        using T = typename F::T;
        const bool oxm = !okxm, oxp = !okxp, oym = !okym, oyp = !okyp;
        in.w[1] = oxm ? table_wall(a, x, y, 0, 1, true, false) : T(0);
        in.w[2] = oym ? table_wall(a, x, y, 0, 2, false, true) : T(0);
        in.w[3] = oxp ? table_wall(a, x, y, 0, 3, true, false) : T(0);
        in.w[4] = oyp ? table_wall(a, x, y, 0, 4, false, true) : T(0);
        in.w[5] = (oxm || oym) ? table_wall(a, x, y, 0, 5, oxm, oym) : T(0);
        in.w[6] = (oxp || oym) ? table_wall(a, x, y, 0, 6, oxp, oym) : T(0);
        in.w[7] = (oxp || oyp) ? table_wall(a, x, y, 0, 7, oxp, oyp) : T(0);
        in.w[8] = (oxm || oyp) ? table_wall(a, x, y, 0, 8, oxm, oyp) : T(0);
    }
    in.ok = (okxm ? 1 : 0) | (okxp ? 2 : 0) | (okym ? 4 : 0) | (okyp ? 8 : 0) | ((colok && w.ok) ? 16 : 0);
}

template <typename F, bool WALLS, bool GEN>
__device__ __forceinline__ void walk_load(const SweepArgs<typename F::T>& a, int x, bool colok, int r, WalkIn<F>& in)
{
    walk_load_row<F, WALLS, GEN>(a, x, colok, walk_row(r, a.ny, WALLS ? a.pery : 1), in);
}

// f(x, t) from the raw loads (bounce-back at Dirichlet walls, Eqs. (54)-(56)); zeros where the
// lane is not a node.
template <typename F, bool WALLS, bool GEN>
__device__ __forceinline__ void walk_finish(const SweepArgs<typename F::T>& a, const WalkIn<F>& in,
                                            typename F::T f[9], typename F::T& phi_prev)
{
    using T = typename F::T;
    if constexpr (!WALLS) {  // periodic in both directions: every lane pulls from its neighbours
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = F::value(a, in.raw, i, i, false);
        phi_prev = in.phi;
        return;
    }
    const bool okxm = in.ok & 1, okxp = in.ok & 2, okym = in.ok & 4, okyp = in.ok & 8, node = in.ok & 16;
    const T tw1 = T(2) * Lat<T>::w1, tw5 = T(2) * Lat<T>::w5;
    const bool ok[9] = {true, okxm, okym, okxp, okyp, okxm && okym, okxp && okym, okxp && okyp, okxm && okyp};
    constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    T v[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = F::value(a, in.raw, i, opp[i], !ok[i]);
    auto wv = [&](int i, bool ox, bool oy) {
        if constexpr (GEN)
            return in.w[i];
        else
            return side_wall(a.wall, i, ox, oy);
    };
    f[0] = v[0];
    f[1] = ok[1] ? v[1] : bounce(v[1], tw1, wv(1, true, false));
    f[2] = ok[2] ? v[2] : bounce(v[2], tw1, wv(2, false, true));
    f[3] = ok[3] ? v[3] : bounce(v[3], tw1, wv(3, true, false));
    f[4] = ok[4] ? v[4] : bounce(v[4], tw1, wv(4, false, true));
    f[5] = ok[5] ? v[5] : bounce(v[5], tw5, wv(5, !okxm, !okym));
    f[6] = ok[6] ? v[6] : bounce(v[6], tw5, wv(6, !okxp, !okym));
    f[7] = ok[7] ? v[7] : bounce(v[7], tw5, wv(7, !okxp, !okyp));
    f[8] = ok[8] ? v[8] : bounce(v[8], tw5, wv(8, !okxm, !okyp));
    phi_prev = in.phi;
    if (!node) {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = T(0);
        phi_prev = T(0);
    }
}

// Where a walker lane sits: its column, the band of rows of its strip and what it stores.
struct WalkLane {
    int x;                  // grid column of the lane (wrapped; clamped when not a node)
    bool colok;             // the lane's column is a node of a live strip
    bool okxm, okxp;        // x-1 / x+1 are nodes (else bounce-back at the x- / x+ wall)
    bool store_col;         // the lane's column is an output column of its strip
    int ys, ye;             // output rows ys .. ye-1
};

// Rows of level-1 loads in flight per walker: two for the 4- and 2-byte formats; one for FP64,
// whose registers already limit a SIMD to two wavefronts (measured on gfx950: a second FP64 row
// buys nothing and costs an occupancy step with Dirichlet walls).
template <typename T>
constexpr int kAhead = sizeof(T) == 8 ? 1 : 2;

// One row of the walk: level 1 on row r, levels 2..K on rows r-1 .. r-(K-1). PH picks which
// of the two row buffers per level is current; the next call uses the other. `in` holds the
// loads of row r and receives those of row r + kAhead. FULL: every level's row is valid and the
// last level's row is an output row (the walk past its first 2 (K - 1) rows), so no row is
// checked: the loop body has no branch per level.
// With FULL on a grid periodic in both directions, rows come from the cursor `rows` (advanced
// here) instead of being wrapped afresh.
template <typename F, int SRC, int KM, int K, bool WALLS, int PH, bool FULL>
__device__ __forceinline__ void walk_step(const SweepArgs<typename F::T>& a, const WalkLane& L, int r, int r1,
                                          WalkIn<F>& in, WalkState<typename F::T, K>& st, WalkCursor<K>& rows)
{
    using T = typename F::T;
    constexpr bool GEN = (KM & kGen) != 0;
    constexpr bool CURSOR = FULL && !WALLS;
    __builtin_amdgcn_s_barrier();
    Level<T> lev;
    walk_finish<F, WALLS, GEN>(a, in, lev.f, lev.phi);

    // Level 1: row r from global memory.
    {
        const WalkRow w = CURSOR ? periodic_row(rows.y[1]) : walk_row(r, a.ny, a.pery);
        const int n = w.y * a.pitch + L.x;
        const T phi = collide<T, SRC, collide_mode<F, KM>()>(a, lev.f, lev.phi, source_at<T, SRC>(a, n, L.x, w.y, 0), n);
        F::settle(a, lev.f, phi);
        lev.phi = phi;
        // Keep level 1 (and so the wait for its loads) ahead of the stores below.
        asm volatile("" ::"v"(lev.f[0]), "v"(lev.f[1]), "v"(lev.f[2]), "v"(lev.f[3]), "v"(lev.f[4]), "v"(lev.f[5]),
                     "v"(lev.f[6]), "v"(lev.f[7]), "v"(lev.f[8]), "v"(phi)
                     : "memory");
    }
    // The last level's row from the previous call, then the loads two rows ahead: every wait
    // covers memory operations issued at least one row earlier.
    if (st.out_n >= 0) F::template put<false>(a, st.out_n, st.out.f, st.out.phi);
    st.out_n = -1;
    if (r + kAhead<T> < r1) {
        if constexpr (CURSOR)
            walk_load_row<F, WALLS, GEN>(a, L.x, L.colok, periodic_row(rows.y[0]), in);
        else
            walk_load<F, WALLS, GEN>(a, L.x, L.colok, r + kAhead<T>, in);
    }

    // Levels 2..K: row r-(l-1) from the rows of level l-1. Level l is valid from row
    // ys-(K-l) on; the first rows of the walk (while the levels fill) are skipped, which leaves
    // only rows that no valid node reads.
#pragma unroll
    for (int l = 2; l <= K; ++l) {
        const int q = r - (l - 1);
        const WalkRow w = CURSOR ? periodic_row(rows.y[l]) : walk_row(q, a.ny, a.pery);
        Level<T>& cur = st.mid[PH][l - 2];
        T g[9];
        T phi;
        if (FULL || q >= L.ys - (K - l)) {
            phi = walk_collide<T, SRC, collide_mode<F, KM>(), WALLS>(a, st.up[l - 2], cur, lev, L.x, L.okxm, L.okxp, w, l - 1, g);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = lev.f[i];
            phi = lev.phi;
        }
        st.up[l - 2][0] = cur.f[2];
        st.up[l - 2][1] = cur.f[5];
        st.up[l - 2][2] = cur.f[6];
        st.mid[1 - PH][l - 2] = lev;
        if (l < K) {
            F::settle(a, g, phi);
#pragma unroll
            for (int i = 0; i < 9; ++i) lev.f[i] = g[i];
            lev.phi = phi;
        } else if (L.store_col && (FULL || (q >= L.ys && q < L.ye))) {
#pragma unroll
            for (int i = 0; i < 9; ++i) st.out.f[i] = g[i];
            st.out.phi = phi;
            st.out_n = w.y * a.pitch + L.x;
        }
    }
    if constexpr (CURSOR) cursor_next(rows, a.ny);
}

// A workgroup of G = blockDim.x / 64 wavefronts (1 or kWalkGroup) holds G strips side by side
// in one band of rows; they walk in lockstep (one barrier per row, no memory fence: they share
// no data), so the rows they read and write at a time are contiguous across the group.
// Strip sx of band sy (a.rows rows) walked by the calling wavefront. A wavefront without a
// strip (live false: the last group of a band) walks along without loads or stores, so it
// meets the group's barriers.
template <typename F, int SRC, int KM, int K, bool WALLS>
__device__ __forceinline__ void walk_strip(const SweepArgs<typename F::T>& a, int sx, int sy, bool live, int lane)
{
    using T = typename F::T;
    constexpr int W = Walk<K>::W;
    const int nx = a.nx, ny = a.ny;

    // Column of this lane (K-1 halo columns on each side of the strip).
    WalkLane L;
    const int cx = sx * W - (K - 1) + lane;
    if (a.perx) {
        L.x = wrap(cx, nx);
        L.colok = live;
    } else {
        L.colok = live && cx >= 0 && cx < nx;
        L.x = cx < 0 ? 0 : (cx >= nx ? nx - 1 : cx);
    }
    L.okxm = a.perx || L.x > 0;
    L.okxp = a.perx || L.x < nx - 1;
    L.store_col = live && lane >= K - 1 && lane < kWave - (K - 1) && cx < nx;
    L.ys = sy * a.rows;
    L.ye = min(L.ys + a.rows, ny);  // uniform over the group
    const int r0 = L.ys - (K - 1), r1 = L.ye + (K - 1);

    WalkState<T, K> st;
#pragma unroll
    for (int l = 0; l < K - 1; ++l) {
        st.up[l][0] = st.up[l][1] = st.up[l][2] = T(0);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int i = 0; i < 9; ++i) st.mid[b][l].f[i] = T(0);
            st.mid[b][l].phi = T(0);
        }
    }
    st.out_n = -1;

    // Loads of rows r0, r0+2, ... go to in[0] and of rows r0+1, r0+3, ... to in[1] with two
    // rows in flight; with one row in flight in[0] serves every row.
    constexpr bool GEN = (KM & kGen) != 0;
    WalkIn<F> in[kAhead<T>];
    walk_load<F, WALLS, GEN>(a, L.x, L.colok, r0, in[0]);
    if (kAhead<T> == 2 && r0 + 1 < r1) walk_load<F, WALLS, GEN>(a, L.x, L.colok, r0 + 1, in[kAhead<T> - 1]);
    // The first 2 (K - 1) rows fill the levels: level l computes its first valid row at row
    // r0 + 2 (l - 1) (its rows before that are not needed) and the last level stores from there on.
    // That many rows (an even count, so the row buffers keep their parity) run with the checks;
    // the rest of the walk has every level valid and stores every row. Its loop renames the row
    // buffers instead of copying them, at the price of more registers: the 16-bit formats, which
    // would lose a wavefront per SIMD (measured 3.8 % slower at four steps), walk every row with
    // the checks.
    constexpr bool kSteady = plain_format<F>();
    const int fill = !kSteady ? r1 : (r0 + 2 * (K - 1) < r1 ? r0 + 2 * (K - 1) : r1);
    WalkCursor<K> rows;
    int r = r0;
    for (; r < fill; r += 2) {
        walk_step<F, SRC, KM, K, WALLS, 0, false>(a, L, r, r1, in[0], st, rows);
        if (r + 1 < r1) walk_step<F, SRC, KM, K, WALLS, 1, false>(a, L, r + 1, r1, in[kAhead<T> - 1], st, rows);
    }
    if constexpr (kSteady) {
        if constexpr (!WALLS) cursor_start(rows, r, kAhead<T>, ny);
        for (; r + 1 < r1; r += 2) {
            walk_step<F, SRC, KM, K, WALLS, 0, true>(a, L, r, r1, in[0], st, rows);
            walk_step<F, SRC, KM, K, WALLS, 1, true>(a, L, r + 1, r1, in[kAhead<T> - 1], st, rows);
        }
        if (r < r1) walk_step<F, SRC, KM, K, WALLS, 0, true>(a, L, r, r1, in[0], st, rows);
    }
    if (st.out_n >= 0) F::template put<false>(a, st.out_n, st.out.f, st.out.phi);
}

// A workgroup of G = blockDim.x / 64 wavefronts (1 or kWalkGroup) holds G strips side by side
// in one band of rows; they walk in lockstep (one barrier per row, no memory fence: they share
// no data), so the rows they read and write at a time are contiguous across the group.
// Whether strip (sx, sy) of a K-step walk stays clear of the grid's edges: every lane's column
// and every row the walk loads, with their pulls at +-1, lie inside the grid, so no link wraps
// or bounces back and the walk without wall handling computes the same bits.
template <int K, typename T>
__device__ __forceinline__ bool walk_clear_of_edges(const SweepArgs<T>& a, int sx, int sy)
{
    const int cx0 = sx * Walk<K>::W - (K - 1);
    const int ys = sy * a.rows;
    const int ye = min(ys + a.rows, a.ny);
    return cx0 >= 1 && cx0 + kWave - 1 <= a.nx - 2 && ys - K >= 0 && ye + K - 1 <= a.ny - 1;
}

template <typename F, int SRC, int KM, int K, bool WALLS>
__global__ __launch_bounds__(kWave* kWalkGroup) void walk_kernel(SweepArgs<typename F::T> a)
{
    const int gsize = static_cast<int>(blockDim.x) / kWave;
    const int group = xcd_tile();
    const int groups_x = (a.tiles_x + gsize - 1) / gsize;
    const int sy = group / groups_x;
    const int sx = (group - sy * groups_x) * gsize + static_cast<int>(threadIdx.x / kWave);
    const bool live = sx < a.tiles_x;
    const int lane = static_cast<int>(threadIdx.x % kWave);
    if constexpr (WALLS) {
        // Strips away from every edge (almost all of a large grid) skip the bounce-back code;
        // the choice is uniform per wavefront, and both walks meet the group's barriers row by
        // row alike.
        if (live && walk_clear_of_edges<K>(a, sx, sy)) {
            walk_strip<F, SRC, KM, K, false>(a, sx, sy, true, lane);
            return;
        }
    }
    walk_strip<F, SRC, KM, K, WALLS>(a, sx, sy, live, lane);
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

template <typename T, int K0, bool NT>
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
            case 0: tile1<F, kSrcNone, kK1Const | K0, NT>(a, tx, ty, kTileY); break;
            case 1: tile1<F, kSrcNone, kK1Phi | K0, NT>(a, tx, ty, kTileY); break;
            case 2: tile1<F, kSrcField, kK1Const | K0, NT>(a, tx, ty, kTileY); break;
            case 3: tile1<F, kSrcField, kK1Phi | K0, NT>(a, tx, ty, kTileY); break;
            case 4: tile1<F, kSrcSep, kK1Const | K0, NT>(a, tx, ty, kTileY); break;
            default: tile1<F, kSrcSep, kK1Phi | K0, NT>(a, tx, ty, kTileY); break;
        }
    }
}

template <typename T, int K0, bool NT>
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
            case 0: tile2<F, kSrcNone, kK1Const | K0, NT>(a, tx, ty, lf, lphi); break;
            case 1: tile2<F, kSrcNone, kK1Phi | K0, NT>(a, tx, ty, lf, lphi); break;
            case 2: tile2<F, kSrcField, kK1Const | K0, NT>(a, tx, ty, lf, lphi); break;
            case 3: tile2<F, kSrcField, kK1Phi | K0, NT>(a, tx, ty, lf, lphi); break;
            case 4: tile2<F, kSrcSep, kK1Const | K0, NT>(a, tx, ty, lf, lphi); break;
            default: tile2<F, kSrcSep, kK1Phi | K0, NT>(a, tx, ty, lf, lphi); break;
        }
        __syncthreads();  // the next tile reuses the LDS
    }
}

// Four steps per launch for a batch: the strips of every instance (58 columns by `rows` rows)
// form the list; one wavefront per strip, no lockstep groups (instances differ in length).
template <typename T, int K, int K0>
__global__ __launch_bounds__(kWave) void batchw_kernel(const BatchEntry<T>* __restrict__ ent,
                                                       const int* __restrict__ begin, const int* __restrict__ par,
                                                       int ninst, int total, int flip, int rows)
{
    using F = Plain<T>;
    const int g = static_cast<int>(gridDim.x);
    const int lane = static_cast<int>(threadIdx.x);
    for (int t = xcd_tile(); t < total; t += g) {
        const int i = owner(begin, ninst, t);
        SweepArgs<T> a = ent[i].a[par[i] ^ flip];
        a.rows = rows;
        a.tiles_x = (a.nx + Walk<K>::W - 1) / Walk<K>::W;
        const int local = t - begin[i];
        const int sy = local / a.tiles_x, sx = local - sy * a.tiles_x;
        const bool walls = !(a.perx && a.pery);
        switch (2 * ent[i].variant + (walls ? 1 : 0)) {
            case 0: walk_strip<F, kSrcNone, kK1Const | K0, K, false>(a, sx, sy, true, lane); break;
            case 1: walk_strip<F, kSrcNone, kK1Const | K0, K, true>(a, sx, sy, true, lane); break;
            case 2: walk_strip<F, kSrcNone, kK1Phi | K0, K, false>(a, sx, sy, true, lane); break;
            case 3: walk_strip<F, kSrcNone, kK1Phi | K0, K, true>(a, sx, sy, true, lane); break;
            case 4: walk_strip<F, kSrcField, kK1Const | K0, K, false>(a, sx, sy, true, lane); break;
            case 5: walk_strip<F, kSrcField, kK1Const | K0, K, true>(a, sx, sy, true, lane); break;
            case 6: walk_strip<F, kSrcField, kK1Phi | K0, K, false>(a, sx, sy, true, lane); break;
            case 7: walk_strip<F, kSrcField, kK1Phi | K0, K, true>(a, sx, sy, true, lane); break;
            case 8: walk_strip<F, kSrcSep, kK1Const | K0, K, false>(a, sx, sy, true, lane); break;
            case 9: walk_strip<F, kSrcSep, kK1Const | K0, K, true>(a, sx, sy, true, lane); break;
            case 10: walk_strip<F, kSrcSep, kK1Phi | K0, K, false>(a, sx, sy, true, lane); break;
            default: walk_strip<F, kSrcSep, kK1Phi | K0, K, true>(a, sx, sy, true, lane); break;
        }
    }
}

// Compute units of the current device (cached per device ordinal).
inline int device_cus()
{
    static int cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] <= 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// Resident wavefronts per CU of one walker instantiation (its registers decide).
template <typename F, int SRC, int KP, int K>
int walk_waves_per_cu()
{
    static const int waves = [] {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_kernel<F, SRC, KP, K, true>, kWave, 0) != hipSuccess ||
            nb <= 0)
            nb = 8;
        return nb;
    }();
    return waves;
}

// Automatic launch shape (measured on gfx950 over 256^2 .. 4096^2 grids):
//  - steps: kAutoDeep (7) per launch with plain FP64/FP32 storage and the standard node model
//    from 2^22 nodes up (there the walkers are issue-bound and every further level saves a pass
//    over the state: 4096^2 FP64 155k against 110k MLUPS at four steps, FP32 287k against 203k;
//    2048^2 FP64 120k against 93k), kAutoDeepWalls (6) for FP64 with a Dirichlet wall (its
//    seven-step walker carries the bounce-back registers: with the single-round strips below,
//    4096^2 walled 123k MLUPS at six steps, 113k at seven, 110k at four; 2048^2 107k at six,
//    95k at four), and for FP32 with a wall from 2^24 nodes up (4096^2 239k at seven steps
//    against 201k at four, but 2048^2 160k against 173k); else kAutoFuse (4) per launch from
//    2^20 nodes up (the state no longer fits the caches and the strip walkers cut its traffic),
//    one per launch below;
//  - strip rows: walkers that hold one wavefront per SIMD (FP64 from six steps on) take the
//    height that fits all strips in the resident slots at once, when that is 64 rows or more:
//    one round of long strips, so the 2(K - 1) fill rows of each strip are a small part of it
//    and no second round starts on a partly idle chip (4096^2 FP64, K = 7: 342-row strips, 948
//    strips for 1024 slots, 174k MLUPS against 163k with 64-row strips; K = 6: 316 rows, 159k
//    against 147k); FP32 walkers (two wavefronts per SIMD) ran slower that way (4096^2, K = 7:
//    164 rows 282k, 64 rows 285k). Otherwise the largest of 64 (from six steps on), 32, 16, 8
//    that still gives every resident wavefront slot about two strips (rows at least 8);
//  - strips per group: from six steps on 1 (one wavefront per SIMD); else kWalkGroup with 32-row
//    strips (large grids), else 1.
constexpr int kAutoDeep = 7;
constexpr int kAutoDeepWalls = 6;


template <typename F, int SRC, int KP, int K>
void walk_shape(const SweepArgs<typename F::T>& a, LaunchCfg& cfg)
{
    constexpr int W = Walk<K>::W;
    const int64_t strips_x = (a.nx + W - 1) / W;
    if (cfg.rows <= 0 && K >= 6 && walk_waves_per_cu<F, SRC, KP, K>() <= 4) {
        const int64_t slots = static_cast<int64_t>(device_cus()) * walk_waves_per_cu<F, SRC, KP, K>();
        const int64_t per_column = slots / strips_x;
        if (per_column >= 1) {
            const int64_t rows = (a.ny + per_column - 1) / per_column;
            if (rows >= 64) cfg.rows = static_cast<int>(rows);
        }
    }
    if (cfg.rows <= 0) {
        const int64_t want = 2LL * device_cus() * walk_waves_per_cu<F, SRC, KP, K>();
        cfg.rows = 8;
        for (int r : {64, 32, 16}) {
            if (r == 64 && K < 6) continue;
            if (strips_x * ((a.ny + r - 1) / r) >= want) {
                cfg.rows = r;
                break;
            }
        }
    }
    if (cfg.group <= 0) cfg.group = (K < 6 && cfg.rows >= 32) ? kWalkGroup : 1;
}

template <typename F, int SRC, int KP>
LaunchCfg resolve_variant(const SweepArgs<typename F::T>& a, LaunchCfg cfg)
{
    if (cfg.steps <= 0) {
        const int64_t nodes = static_cast<int64_t>(a.nx) * a.ny;
        const bool fp64 = sizeof(typename F::T) == 8, periodic = a.perx && a.pery;
        const bool deep = plain_format<F>() && (KP & kGen) == 0 && nodes >= (periodic || fp64 ? (1LL << 22) : (1LL << 24));
        cfg.steps = deep ? (fp64 && !periodic ? kAutoDeepWalls : kAutoDeep) : (nodes >= (1LL << 20) ? kAutoFuse : 1);
    }
    if (cfg.steps != 2) cfg.tile = 0;
    if (cfg.steps == 1) {  // rows: tile height of the one-step kernel
        if (cfg.rows <= 0) cfg.rows = kTileY;
        cfg.group = 0;
        return cfg;
    }
    if (cfg.tile) {
        cfg.rows = cfg.group = 0;
        return cfg;
    }
    switch (cfg.steps) {
        case 2: walk_shape<F, SRC, KP, 2>(a, cfg); break;
        case 3: walk_shape<F, SRC, KP, 3>(a, cfg); break;
        case 4: walk_shape<F, SRC, KP, 4>(a, cfg); break;
        case 5: walk_shape<F, SRC, KP, 5>(a, cfg); break;
        case 6: walk_shape<F, SRC, KP, 6>(a, cfg); break;
        default: walk_shape<F, SRC, KP, 7>(a, cfg); break;
    }
    return cfg;
}

template <typename F, int SRC, int KP, int K>
hipError_t walk_launch(SweepArgs<typename F::T> a, const LaunchCfg& cfg, hipStream_t s)
{
    constexpr int W = Walk<K>::W;
    a.tiles_x = (a.nx + W - 1) / W;
    a.rows = cfg.rows;
    a.tiles_y = (a.ny + a.rows - 1) / a.rows;
    const int groups_x = (a.tiles_x + cfg.group - 1) / cfg.group;
    const unsigned grid = static_cast<unsigned>(groups_x) * static_cast<unsigned>(a.tiles_y);
    if (a.perx && a.pery)
        hipLaunchKernelGGL((walk_kernel<F, SRC, KP, K, false>), dim3(grid), dim3(kWave * cfg.group), 0, s, a);
    else
        hipLaunchKernelGGL((walk_kernel<F, SRC, KP, K, true>), dim3(grid), dim3(kWave * cfg.group), 0, s, a);
    return hipGetLastError();
}

template <typename F, int SRC, int KP>
hipError_t sweep_variant(SweepArgs<typename F::T> a, LaunchCfg cfg, hipStream_t s)
{
    using T = typename F::T;
    cfg = resolve_variant<F, SRC, KP>(a, cfg);
    if (cfg.steps < 1 || cfg.steps > kMaxFuse || cfg.rows < 0 || (cfg.steps >= 2 && !cfg.tile && cfg.rows < 1) ||
        (cfg.steps == 1 && (cfg.rows < 1 || cfg.rows > kMaxBlock1 / kTileX || (cfg.rows & (cfg.rows - 1)))) ||
        (cfg.group != 0 && cfg.group != 1 && cfg.group != kWalkGroup))
        return hipErrorInvalidValue;
    if (cfg.steps == 1) {
        a.tiles_x = (a.nx + kTileX - 1) / kTileX;
        a.tiles_y = (a.ny + cfg.rows - 1) / cfg.rows;
        const unsigned grid = static_cast<unsigned>(a.tiles_x) * static_cast<unsigned>(a.tiles_y);
        if (a.nts)
            hipLaunchKernelGGL((sweep_kernel<F, SRC, KP, true>), dim3(grid), dim3(kTileX * cfg.rows), 0, s, a);
        else
            hipLaunchKernelGGL((sweep_kernel<F, SRC, KP, false>), dim3(grid), dim3(kTileX * cfg.rows), 0, s, a);
        return hipGetLastError();
    }
    if (cfg.tile) {
        a.tiles_x = (a.nx + kTile2X - 1) / kTile2X;
        a.tiles_y = (a.ny + Tile2<T>::TY - 1) / Tile2<T>::TY;
        const unsigned grid = static_cast<unsigned>(a.tiles_x) * static_cast<unsigned>(a.tiles_y);
        if (a.nts)
            hipLaunchKernelGGL((sweep2_kernel<F, SRC, KP, true>), dim3(grid), dim3(kBlock2), 0, s, a);
        else
            hipLaunchKernelGGL((sweep2_kernel<F, SRC, KP, false>), dim3(grid), dim3(kBlock2), 0, s, a);
        return hipGetLastError();
    }
    switch (cfg.steps) {
        case 2: return walk_launch<F, SRC, KP, 2>(a, cfg, s);
        case 3: return walk_launch<F, SRC, KP, 3>(a, cfg, s);
        case 4: return walk_launch<F, SRC, KP, 4>(a, cfg, s);
        case 5: return walk_launch<F, SRC, KP, 5>(a, cfg, s);
        case 6: return walk_launch<F, SRC, KP, 6>(a, cfg, s);
        default: return walk_launch<F, SRC, KP, 7>(a, cfg, s);
    }
}

// Source kind x K1 mode dispatch of FN<F, SRC, KM>(args...).
#define BTRT_BY_SRC(KMV, FN, ...)                                                \
    do {                                                                         \
        if (src_kind == kSrcField) return FN<F, kSrcField, KMV>(__VA_ARGS__);    \
        if (src_kind == kSrcSep) return FN<F, kSrcSep, KMV>(__VA_ARGS__);        \
        return FN<F, kSrcNone, KMV>(__VA_ARGS__);                                \
    } while (0)
#define BTRT_BY_VARIANT(FN, ...)                                                 \
    do {                                                                         \
        if (kmode == kK1Field) BTRT_BY_SRC(kK1Field, FN, __VA_ARGS__);           \
        if (kmode == kK1Phi) BTRT_BY_SRC(kK1Phi, FN, __VA_ARGS__);               \
        BTRT_BY_SRC(kK1Const, FN, __VA_ARGS__);                                  \
    } while (0)

// The same over the general node model (K1 mode | kGen).
#define BTRT_BY_VARIANT_GEN(FN, ...)                                             \
    do {                                                                         \
        if (kmode == (kK1Field | kGen)) BTRT_BY_SRC(kK1Field | kGen, FN, __VA_ARGS__); \
        if (kmode == (kK1Phi | kGen)) BTRT_BY_SRC(kK1Phi | kGen, FN, __VA_ARGS__);     \
        BTRT_BY_SRC(kK1Const | kGen, FN, __VA_ARGS__);                           \
    } while (0)

template <typename F>
hipError_t sweep_with(const SweepArgs<typename F::T>& a, int src_kind, int kmode, const LaunchCfg& cfg,
                      hipStream_t s)
{
    BTRT_BY_VARIANT(sweep_variant, a, cfg, s);
}

template <typename F>
LaunchCfg resolve_with(const SweepArgs<typename F::T>& a, int src_kind, int kmode, const LaunchCfg& cfg)
{
    BTRT_BY_VARIANT(resolve_variant, a, cfg);
}

// k0 = 1 kernels (kK0One): the standard node model's variants with the bit set.
#define BTRT_BY_VARIANT_K0(FN, ...)                                              \
    do {                                                                         \
        if ((kmode & kK1Mask) == kK1Field) BTRT_BY_SRC(kK1Field | kK0One, FN, __VA_ARGS__); \
        if ((kmode & kK1Mask) == kK1Phi) BTRT_BY_SRC(kK1Phi | kK0One, FN, __VA_ARGS__);     \
        BTRT_BY_SRC(kK1Const | kK0One, FN, __VA_ARGS__);                         \
    } while (0)

template <typename F>
hipError_t sweep_with_k0(const SweepArgs<typename F::T>& a, int src_kind, int kmode, const LaunchCfg& cfg,
                         hipStream_t s)
{
    BTRT_BY_VARIANT_K0(sweep_variant, a, cfg, s);
}

template <typename F>
LaunchCfg resolve_with_k0(const SweepArgs<typename F::T>& a, int src_kind, int kmode, const LaunchCfg& cfg)
{
    BTRT_BY_VARIANT_K0(resolve_variant, a, cfg);
}

template <typename F>
hipError_t sweep_with_gen(const SweepArgs<typename F::T>& a, int src_kind, int kmode, const LaunchCfg& cfg,
                          hipStream_t s)
{
    BTRT_BY_VARIANT_GEN(sweep_variant, a, cfg, s);
}

template <typename F>
LaunchCfg resolve_with_gen(const SweepArgs<typename F::T>& a, int src_kind, int kmode, const LaunchCfg& cfg)
{
    BTRT_BY_VARIANT_GEN(resolve_variant, a, cfg);
}

#undef BTRT_BY_VARIANT_K0
#undef BTRT_BY_VARIANT_GEN
#undef BTRT_BY_VARIANT
#undef BTRT_BY_SRC

}  // namespace

// Sweeps of one storage format: launch (cfg resolved here) and shape resolution. Each is
// defined in its own translation unit (btrt_sweep_<format>.hip).
hipError_t sweep_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
hipError_t sweep_f32(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
hipError_t sweep_f16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
hipError_t sweep_bf16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
LaunchCfg resolve_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg);
LaunchCfg resolve_f32(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg);
LaunchCfg resolve_f16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg);
LaunchCfg resolve_bf16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg);
// The general node model (kmode carries kGen), plain storage only (btrt_sweep_gen_<format>.hip).
hipError_t sweep_gen_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
// k0 = 1 variants (btrt_sweep_k0_<format>.hip).
hipError_t sweep_k0_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
hipError_t sweep_k0_f32(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
hipError_t sweep_k0_f16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
hipError_t sweep_k0_bf16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
LaunchCfg resolve_k0_f16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg);
LaunchCfg resolve_k0_bf16dev(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg);
LaunchCfg resolve_k0_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg);
LaunchCfg resolve_k0_f32(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg);
hipError_t sweep_gen_f32(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg, hipStream_t s);
LaunchCfg resolve_gen_f64(const SweepArgs<double>& a, int src_kind, int kmode, const LaunchCfg& cfg);
LaunchCfg resolve_gen_f32(const SweepArgs<float>& a, int src_kind, int kmode, const LaunchCfg& cfg);

}  // namespace btrtk
