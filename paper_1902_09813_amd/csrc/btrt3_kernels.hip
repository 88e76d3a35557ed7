// gfx950 kernels of the three-dimensional B-TriRT sweep on the D3Q19 lattice (Zhao, Wu, Chai &
// Shi, arXiv:1902.09813, Eq. (6) on the lattice of Eq. (86)).
//
// State between steps: f+(t-1) in 19 SoA planes (f[i][z][y][pitch]) and phi(t-1) in one plane.
// One node update, one thread per node:
//   1. pull f_i(x, t) = f_i+(x - c_i, t-1) (Eq. (38)), or, when x - c_i lies beyond a Dirichlet
//      face, f_i = -f_opp+(x, t-1) + 2 w_i phi_w (Eqs. (54)-(56); two faces: mean value);
//   2. phi, j and the second moments Pi of f; M1 = j - B, M2_neq = Pi - phi/3 I (Eq. (9));
//   3. Eq. (6) rearranged per direction: with q = k0 j + dB - K1 (M1 + dB/2) (the first-moment
//      relaxation, the equilibrium flux and G of Eq. (11) together) and Q = (K2s - k0) o M2_neq
//      (K2s: off-diagonal rates symmetrised, Eq. (100)),
//          f_i+ = (1 - k0) f_i + w_i [k0 phi + s + 3/2 tr Q + 3 c_i . q - 9/2 c_i^T Q c_i],
//      which is f_i - k0 f_neq_i - R f_neq - P f_neq + G_i + S_i of Eqs. (6), (77) for D = phi I;
//      opposite directions share the even part and flip the odd one;
//   4. store f+(t) and phi(t).
// HBM traffic per node and step: 19 populations and phi read and written once, plus the source;
// the arithmetic is ~200 flops against 320 B (FP64), so the sweep is bandwidth-bound and there is
// no matrix-core work.

#include "btrt3_internal.h"

#include <algorithm>

namespace btrt3k {
namespace {

constexpr int kTileX = 64;
constexpr int kTileY = 4;
constexpr int kBlock = kTileX * kTileY;

// D3Q19 velocities in the column order of C in Eq. (86), and the opposite of each.
__host__ __device__ constexpr int cxv(int i)
{
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int cyv(int i)
{
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int czv(int i)
{
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
    return v[i];
}
__host__ __device__ constexpr int oppv(int i)
{
    constexpr int v[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
    return v[i];
}
template <typename T>
__host__ __device__ constexpr T wv(int i)
{
    return i == 0 ? T(1) / T(3) : (i <= 6 ? T(1) / T(18) : T(1) / T(36));
}

template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c)
{
    if constexpr (sizeof(T) == 4)
        return fmaf(a, b, c);
    else
        return fma(a, b, c);
}

// Block -> tile, consecutive tiles on one XCD (workgroups are dispatched round-robin over the 8
// XCDs), so neighbouring tiles' shared cache lines meet in the same L2.
__device__ __forceinline__ int xcd_tile()
{
    const int b = static_cast<int>(blockIdx.x);
    const int nb = static_cast<int>(gridDim.x);
    const int q = nb >> 3, r = nb & 7, k = b & 7, j = b >> 3;
    return k * q + (k < r ? k : r) + j;
}

// NT: a non-temporal store, for the one-step kernel on boxes much larger than the caches. A
// compile-time choice: with a run-time flag the compiler merges the two stores of the branch
// into one and drops the hint. The two-step kernel stores normally.
template <bool NT, typename T>
__device__ __forceinline__ void store(T* p, T v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Step 1: f_i(x, t) for all 19 directions at node (x, y, z).
template <typename T>
__device__ __forceinline__ void pull3(const Sweep3<T>& a, int x, int y, int z, T f[kQ])
{
    const int64_t p = a.plane;
    const int n = z * a.slab + y * a.pitch + x;
    if (x > 0 && x < a.nx - 1 && y > 0 && y < a.ny - 1 && z > 0 && z < a.nz - 1) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) f[i] = a.fin[i * p + n - (cxv(i) + cyv(i) * a.pitch + czv(i) * a.slab)];
        return;
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        int xs = x - cxv(i), ys = y - cyv(i), zs = z - czv(i);
        int faces = 0;
        T wsum = T(0);
        if (xs < 0) {
            if (a.per[0]) xs += a.nx; else { ++faces; wsum += a.wall[0]; }
        } else if (xs >= a.nx) {
            if (a.per[0]) xs -= a.nx; else { ++faces; wsum += a.wall[1]; }
        }
        if (ys < 0) {
            if (a.per[1]) ys += a.ny; else { ++faces; wsum += a.wall[2]; }
        } else if (ys >= a.ny) {
            if (a.per[1]) ys -= a.ny; else { ++faces; wsum += a.wall[3]; }
        }
        if (zs < 0) {
            if (a.per[2]) zs += a.nz; else { ++faces; wsum += a.wall[4]; }
        } else if (zs >= a.nz) {
            if (a.per[2]) zs -= a.nz; else { ++faces; wsum += a.wall[5]; }
        }
        if (faces == 0) {
            f[i] = a.fin[i * p + zs * a.slab + ys * a.pitch + xs];
        } else {
            const T phiw = faces == 1 ? wsum : T(0.5) * wsum;
            f[i] = fmadd(T(2) * wv<T>(i), phiw, -a.fin[oppv(i) * p + n]);
        }
    }
}

// Steps 2-3: f (f(x, t) on entry, f+(x, t) on return); returns phi(t).
template <typename T, bool KPHI>
__device__ __forceinline__ T collide3(const Sweep3<T>& a, T f[kQ], T phi_prev, T s)
{
    constexpr T third = T(1) / T(3), half = T(0.5);
    const T d1 = (f[1] + f[2]), d3 = (f[3] + f[4]), d5 = (f[5] + f[6]);
    const T sxy = (f[7] + f[8]) + (f[9] + f[10]);
    const T sxz = (f[11] + f[12]) + (f[13] + f[14]);
    const T syz = (f[15] + f[16]) + (f[17] + f[18]);
    const T phi = (((f[0] + d1) + (d3 + d5)) + sxy) + (sxz + syz);
    const T jx = ((f[1] - f[2]) + (f[7] - f[8])) + ((f[9] - f[10]) + ((f[11] - f[12]) + (f[13] - f[14])));
    const T jy = ((f[3] - f[4]) + ((f[7] + f[8]) - (f[9] + f[10]))) + ((f[15] - f[16]) + (f[17] - f[18]));
    const T jz = ((f[5] - f[6]) + ((f[11] + f[12]) - (f[13] + f[14]))) + ((f[15] + f[16]) - (f[17] + f[18]));
    const T pxx = (d1 + sxy) + sxz, pyy = (d3 + sxy) + syz, pzz = (d5 + sxz) + syz;
    const T pxy = (f[7] - f[8]) - (f[9] - f[10]);
    const T pxz = (f[11] - f[12]) - (f[13] - f[14]);
    const T pyz = (f[15] - f[16]) - (f[17] - f[18]);

    // B(phi) = phi (a + b phi / 2) and its backward difference over one step (G, Eq. (11)).
    T B[3], dB[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T hb = half * a.b[c];
        B[c] = phi * fmadd(hb, phi, a.a[c]);
        dB[c] = fmadd(-phi_prev, fmadd(hb, phi_prev, a.a[c]), B[c]);
    }

    // K1 = (A / c_s^2 + I/2)^-1 (Eq. (30)); symmetric, kept as (11, 12, 13, 22, 23, 33).
    T k11 = a.K1[0], k12 = a.K1[1], k13 = a.K1[2], k22 = a.K1[3], k23 = a.K1[4], k33 = a.K1[5];
    if constexpr (KPHI) {
        const T g = fmadd(a.beta, phi * phi, T(1));
        const T m11 = fmadd(T(3) * a.A0[0], g, half), m12 = (T(3) * a.A0[1]) * g, m13 = (T(3) * a.A0[2]) * g;
        const T m22 = fmadd(T(3) * a.A0[3], g, half), m23 = (T(3) * a.A0[4]) * g;
        const T m33 = fmadd(T(3) * a.A0[5], g, half);
        const T c11 = fmadd(m22, m33, -(m23 * m23)), c12 = fmadd(m13, m23, -(m12 * m33));
        const T c13 = fmadd(m12, m23, -(m13 * m22));
        const T rdet = T(1) / fmadd(m11, c11, fmadd(m12, c12, m13 * c13));
        k11 = c11 * rdet;
        k12 = c12 * rdet;
        k13 = c13 * rdet;
        k22 = fmadd(m11, m33, -(m13 * m13)) * rdet;
        k23 = fmadd(m12, m13, -(m11 * m23)) * rdet;
        k33 = fmadd(m11, m22, -(m12 * m12)) * rdet;
    }

    // q = k0 j + dB - K1 (M1 + dB/2), M1 = j - B.
    const T vx = fmadd(half, dB[0], jx - B[0]), vy = fmadd(half, dB[1], jy - B[1]), vz = fmadd(half, dB[2], jz - B[2]);
    const T qx = fmadd(a.k0, jx, dB[0]) - fmadd(k11, vx, fmadd(k12, vy, k13 * vz));
    const T qy = fmadd(a.k0, jy, dB[1]) - fmadd(k12, vx, fmadd(k22, vy, k23 * vz));
    const T qz = fmadd(a.k0, jz, dB[2]) - fmadd(k13, vx, fmadd(k23, vy, k33 * vz));

    // Q = (K2s - k0) o M2_neq; M2_neq = Pi - phi/3 I.
    const T phi3 = third * phi;
    const T Qxx = (a.q2[0] - a.k0) * (pxx - phi3), Qyy = (a.q2[3] - a.k0) * (pyy - phi3);
    const T Qzz = (a.q2[5] - a.k0) * (pzz - phi3);
    const T Qxy = (a.q2[1] - a.k0) * pxy, Qxz = (a.q2[2] - a.k0) * pxz, Qyz = (a.q2[4] - a.k0) * pyz;
    const T E0 = fmadd(a.cq[0], (Qxx + Qyy) + Qzz, fmadd(a.k0, phi, s));

    const T om = T(1) - a.k0;
    const T w0 = wv<T>(0), w1 = wv<T>(1), w2 = wv<T>(7);
    f[0] = fmadd(om, f[0], w0 * E0);
    // Axis pairs: c^T Q c = Q_aa, c . q = +-q_a.
    const T ex = fmadd(a.cq[1], Qxx, E0), ey = fmadd(a.cq[1], Qyy, E0), ez = fmadd(a.cq[1], Qzz, E0);
    f[1] = fmadd(om, f[1], w1 * fmadd(a.cq[2], qx, ex));
    f[2] = fmadd(om, f[2], w1 * fmadd(a.cq[3], qx, ex));
    f[3] = fmadd(om, f[3], w1 * fmadd(a.cq[2], qy, ey));
    f[4] = fmadd(om, f[4], w1 * fmadd(a.cq[3], qy, ey));
    f[5] = fmadd(om, f[5], w1 * fmadd(a.cq[2], qz, ez));
    f[6] = fmadd(om, f[6], w1 * fmadd(a.cq[3], qz, ez));
    // Face-diagonal pairs: c^T Q c = Q_aa + Q_bb +- 2 Q_ab, c . q = +-q_a +- q_b.
    const T xy = fmadd(a.cq[1], Qxx + Qyy, E0), xz = fmadd(a.cq[1], Qxx + Qzz, E0), yz = fmadd(a.cq[1], Qyy + Qzz, E0);
    const T xyp = fmadd(a.cq[5], Qxy, xy), xym = fmadd(a.cq[4], Qxy, xy);
    const T xzp = fmadd(a.cq[5], Qxz, xz), xzm = fmadd(a.cq[4], Qxz, xz);
    const T yzp = fmadd(a.cq[5], Qyz, yz), yzm = fmadd(a.cq[4], Qyz, yz);
    f[7] = fmadd(om, f[7], w2 * fmadd(a.cq[2], qx + qy, xyp));    // ( 1,  1,  0)
    f[10] = fmadd(om, f[10], w2 * fmadd(a.cq[3], qx + qy, xyp)); // (-1, -1,  0)
    f[8] = fmadd(om, f[8], w2 * fmadd(a.cq[2], qy - qx, xym));    // (-1,  1,  0)
    f[9] = fmadd(om, f[9], w2 * fmadd(a.cq[3], qy - qx, xym));   // ( 1, -1,  0)
    f[11] = fmadd(om, f[11], w2 * fmadd(a.cq[2], qx + qz, xzp));  // ( 1,  0,  1)
    f[14] = fmadd(om, f[14], w2 * fmadd(a.cq[3], qx + qz, xzp)); // (-1,  0, -1)
    f[12] = fmadd(om, f[12], w2 * fmadd(a.cq[2], qz - qx, xzm));  // (-1,  0,  1)
    f[13] = fmadd(om, f[13], w2 * fmadd(a.cq[3], qz - qx, xzm)); // ( 1,  0, -1)
    f[15] = fmadd(om, f[15], w2 * fmadd(a.cq[2], qy + qz, yzp));  // ( 0,  1,  1)
    f[18] = fmadd(om, f[18], w2 * fmadd(a.cq[3], qy + qz, yzp)); // ( 0, -1, -1)
    f[16] = fmadd(om, f[16], w2 * fmadd(a.cq[2], qz - qy, yzm));  // ( 0, -1,  1)
    f[17] = fmadd(om, f[17], w2 * fmadd(a.cq[3], qz - qy, yzm)); // ( 0,  1, -1)
    return phi;
}

// Node coordinates of tile t (64 x 4 nodes of one z-slice) for the calling thread.
template <typename T>
__device__ __forceinline__ bool node_of(const Sweep3<T>& a, int t, int& x, int& y, int& z)
{
    const int per_slice = a.tiles_x * a.tiles_y;
    z = t / per_slice;
    const int r = t - z * per_slice;
    const int ty = r / a.tiles_x, tx = r - ty * a.tiles_x;
    x = tx * kTileX + static_cast<int>(threadIdx.x % kTileX);
    y = ty * kTileY + static_cast<int>(threadIdx.x / kTileX);
    return x < a.nx && y < a.ny;
}

template <typename T, bool SRC, bool KPHI, bool NT>
__global__ __launch_bounds__(kBlock) void sweep3_kernel(Sweep3<T> a)
{
    int x, y, z;
    if (!node_of(a, xcd_tile(), x, y, z)) return;
    T f[kQ];
    pull3(a, x, y, z, f);
    const int n = z * a.slab + y * a.pitch + x;
    const T s = SRC ? a.src[n] : T(0);
    const T phi = collide3<T, KPHI>(a, f, a.phi_prev[n], s);
#pragma unroll
    for (int i = 0; i < kQ; ++i) store<NT>(a.fout + i * a.plane + n, f[i]);
    store<NT>(a.phi_out + n, phi);
}

// ---- two time steps per launch --------------------------------------------------------------
// A workgroup of TXH x TYH threads owns an xy tile of (TXH - 2) x (TYH - 2) columns and walks z
// over a chunk of zc output planes. Each thread holds one column of the tile plus its one-column
// halo ring. Iteration it updates plane uz = z0 - 1 + it at step 1 (level 1: pull from f+(t-1)
// in global memory, collide) and, from it = 2 on, plane uz - 1 at step 2 (level 2) on the
// interior columns, pulling the level-1 populations of planes uz - 2 .. uz: those with c_xy != 0
// from the neighbouring columns through LDS, those along z (0, 5, 6) and the bounce-back partners
// from the thread's own registers. Level-1 values a neighbour pulls are published in LDS per
// group of c_z: c_z = -1 (read in the same iteration, one slot), c_z = 0 (read one iteration
// later, two slots), c_z = +1 (read two iterations later, three slots). Two barriers per
// iteration (after publishing, after the level-2 reads). Both levels run pull3/collide3's
// arithmetic, so a launch gives the bits of two one-step launches.
//
// Halo columns outside a Dirichlet face and planes outside the box along a Dirichlet z axis are
// not nodes: they compute nothing, and no node reads them (it bounces back instead).

// LDS slot of each direction's level-1 value (-1: kept in registers).
__host__ __device__ constexpr int lds_pos(int i)
{
    //                        0   1  2  3  4   5   6  7  8  9 10 11 12 13 14 15 16 17 18
    constexpr int v[19] = {-1, 0, 1, 2, 3, -1, -1, 4, 5, 6, 7, 0, 1, 0, 1, 2, 3, 2, 3};
    return v[i];
}
constexpr int kSlotsD = 4;       // c_z = -1: directions 13, 14, 17, 18
constexpr int kSlotsM = 2 * 8;   // c_z = 0: 1, 2, 3, 4, 7, 8, 9, 10, two planes
constexpr int kSlotsU = 3 * 4;   // c_z = +1: 11, 12, 15, 16, three planes
constexpr int kSlots = kSlotsD + kSlotsM + kSlotsU;

template <int TXH, int TYH>
struct Tile3x2 {
    static constexpr int TX = TXH - 2, TY = TYH - 2, N = TXH * TYH;
};

// v mod n in [0, n) (a halo column of a ragged tile can lie more than one period away on a
// grid narrower than the tile).
__device__ __forceinline__ int wrap3(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Slot of direction i's level-1 value written in iteration `it` (a reader passes the iteration
// that wrote it: plane pz - c_z was level 1's plane in iteration it - 1 - c_z).
__device__ __forceinline__ int lds_slot(int i, int it)
{
    const int cz = czv(i);
    if (cz < 0) return lds_pos(i);
    if (cz == 0) return kSlotsD + 8 * (it & 1) + lds_pos(i);
    return kSlotsD + kSlotsM + 4 * (it % 3) + lds_pos(i);
}

// Level-1 inputs of one column and plane as raw loads, issued an iteration before they are used:
// each direction's value comes from x - c_i (wrapped on periodic axes) or, where that lies beyond
// a Dirichlet face, from the node's own opposite population (resolved by raw3_resolve).
template <typename T>
struct Raw3 {
    T v[kQ];
    T phi;  // phi(t-1) of the node
    T s;    // source
};

template <typename T, bool SRC, bool WALLS>
__device__ __forceinline__ void raw3_issue(const Sweep3<T>& a, bool node, int x, int y, int z, Raw3<T>& r)
{
    if (!node) {  // not a node: nothing to load (the values are never read)
#pragma unroll
        for (int i = 0; i < kQ; ++i) r.v[i] = T(0);
        r.phi = r.s = T(0);
        return;
    }
    const int64_t p = a.plane;
    const int n = z * a.slab + y * a.pitch + x;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        int xs = x - cxv(i), ys = y - cyv(i), zs = z - czv(i);
        bool out = false;
        if (WALLS) {
            if (xs < 0 || xs >= a.nx) { if (a.per[0]) xs = xs < 0 ? xs + a.nx : xs - a.nx; else out = true; }
            if (ys < 0 || ys >= a.ny) { if (a.per[1]) ys = ys < 0 ? ys + a.ny : ys - a.ny; else out = true; }
            if (zs < 0 || zs >= a.nz) { if (a.per[2]) zs = zs < 0 ? zs + a.nz : zs - a.nz; else out = true; }
        } else {
            xs = xs < 0 ? xs + a.nx : (xs >= a.nx ? xs - a.nx : xs);
            ys = ys < 0 ? ys + a.ny : (ys >= a.ny ? ys - a.ny : ys);
            zs = zs < 0 ? zs + a.nz : (zs >= a.nz ? zs - a.nz : zs);
        }
        r.v[i] = out ? a.fin[oppv(i) * p + n] : a.fin[i * p + zs * a.slab + ys * a.pitch + xs];
    }
    r.phi = a.phi_prev[n];
    r.s = SRC ? a.src[n] : T(0);
}

// f_i(x, t) from the raw loads: the bounce-back rule where x - c_i lies beyond Dirichlet faces
// (one face: its phi_w; two: their mean), the arithmetic of pull3.
template <typename T, bool WALLS>
__device__ __forceinline__ void raw3_resolve(const Sweep3<T>& a, int x, int y, int z, const Raw3<T>& r, T f[kQ])
{
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        f[i] = r.v[i];
        if constexpr (WALLS) {
            const int xs = x - cxv(i), ys = y - cyv(i), zs = z - czv(i);
            int faces = 0;
            T wsum = T(0);
            if (!a.per[0]) {
                if (xs < 0) { ++faces; wsum += a.wall[0]; }
                else if (xs >= a.nx) { ++faces; wsum += a.wall[1]; }
            }
            if (!a.per[1]) {
                if (ys < 0) { ++faces; wsum += a.wall[2]; }
                else if (ys >= a.ny) { ++faces; wsum += a.wall[3]; }
            }
            if (!a.per[2]) {
                if (zs < 0) { ++faces; wsum += a.wall[4]; }
                else if (zs >= a.nz) { ++faces; wsum += a.wall[5]; }
            }
            if (faces > 0) {
                const T phiw = faces == 1 ? wsum : T(0.5) * wsum;
                f[i] = fmadd(T(2) * wv<T>(i), phiw, -r.v[i]);
            }
        }
    }
}

// Registers a column keeps of its own level-1 values for the next iteration: the directions no
// LDS slot holds any more by then (0, 5, 6 and the c_z = -1 group), for i = 0, for the pull of
// direction 5 one plane later and for bounce-back partners; -1: read back from LDS.
__host__ __device__ constexpr int keep_pos(int i)
{
    //                        0   1   2   3   4  5  6   7   8   9  10  11  12 13 14  15  16 17 18
    constexpr int v[19] = {0, -1, -1, -1, -1, 1, 2, -1, -1, -1, -1, -1, -1, 3, 4, -1, -1, 5, 6};
    return v[i];
}
constexpr int kKeep = 7;

template <typename T, bool SRC, bool KPHI, bool WALLS, int TXH, int TYH>
__global__ __launch_bounds__(TXH* TYH) void sweep3x2_kernel(Sweep3<T> a)
{
    using G = Tile3x2<TXH, TYH>;
    __shared__ T lds[kSlots][TYH][TXH];

    const int t = xcd_tile();
    const int per_chunk = a.tiles_x * a.tiles_y;
    const int chunk = t / per_chunk;
    const int rr = t - chunk * per_chunk;
    const int tyi = rr / a.tiles_x, txi = rr - tyi * a.tiles_x;
    const int lx = static_cast<int>(threadIdx.x % TXH), ly = static_cast<int>(threadIdx.x / TXH);

    // This thread's column: unwrapped (ux, uy) and the grid node (x, y) it stands for.
    const int ux = txi * G::TX - 1 + lx, uy = tyi * G::TY - 1 + ly;
    bool col = true;
    int x = ux, y = uy;
    if (!WALLS || a.per[0]) x = wrap3(ux, a.nx); else col = col && ux >= 0 && ux < a.nx;
    if (!WALLS || a.per[1]) y = wrap3(uy, a.ny); else col = col && uy >= 0 && uy < a.ny;
    // Level 2 runs on interior columns that are nodes of the grid (not wrapped copies).
    const bool interior = lx >= 1 && lx <= TXH - 2 && ly >= 1 && ly <= TYH - 2 && ux >= 0 && ux < a.nx && uy >= 0 &&
                          uy < a.ny;
    const int z0 = chunk * a.zc;
    const int z1 = min(z0 + a.zc, a.nz);

    T keep[kKeep];  // own level-1 values (keep_pos) of plane uz - 1
    T prev_phi = T(0);
    T f5pp = T(0);  // own level-1 f_5+ of plane uz - 2
#pragma unroll
    for (int k = 0; k < kKeep; ++k) keep[k] = T(0);

    // Plane uz of the walk: wrapped plane index and whether (x, y, uz) is a node.
    auto plane_of = [&](int uz, int& zz) {
        zz = uz;
        if (!WALLS || a.per[2]) {
            zz = wrap3(uz, a.nz);
            return col;
        }
        return col && uz >= 0 && uz < a.nz;
    };
    Raw3<T> raw;  // level-1 inputs of the next plane, loaded an iteration ahead
    {
        int zz;
        const bool nd = plane_of(z0 - 1, zz);
        raw3_issue<T, SRC, WALLS>(a, nd, x, y, zz, raw);
    }

    for (int it = 0; it <= z1 - z0 + 1; ++it) {
        const int uz = z0 - 1 + it;
        // Level 1 at (x, y, uz) from the loads issued an iteration ago.
        T f[kQ];
        T phi1 = T(0);
        int zz;
        const bool node1 = plane_of(uz, zz);
        if (node1) {
            raw3_resolve<T, WALLS>(a, x, y, zz, raw, f);
            phi1 = collide3<T, KPHI>(a, f, raw.phi, raw.s);
        } else {
#pragma unroll
            for (int i = 0; i < kQ; ++i) f[i] = T(0);
        }
        if (it <= z1 - z0) {  // the loads of the next plane, in flight during level 2
            int zn;
            const bool nd = plane_of(uz + 1, zn);
            raw3_issue<T, SRC, WALLS>(a, nd, x, y, zn, raw);
        }
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            if (lds_pos(i) >= 0) lds[lds_slot(i, it)][ly][lx] = f[i];
        __syncthreads();

        // Level 2 at plane pz = uz - 1 (an output plane of the chunk from it = 2 on).
        if (it >= 2 && interior) {
            const int pz = uz - 1;
            const int pzz = (!WALLS || a.per[2]) ? wrap3(pz, a.nz) : pz;
            T g[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const int cx = cxv(i), cy = cyv(i), cz = czv(i);
                int faces = 0;
                T wsum = T(0);
                if constexpr (WALLS) {
                    if (!a.per[0]) {
                        if (ux - cx < 0) { ++faces; wsum += a.wall[0]; }
                        else if (ux - cx >= a.nx) { ++faces; wsum += a.wall[1]; }
                    }
                    if (!a.per[1]) {
                        if (uy - cy < 0) { ++faces; wsum += a.wall[2]; }
                        else if (uy - cy >= a.ny) { ++faces; wsum += a.wall[3]; }
                    }
                    if (!a.per[2]) {
                        if (pz - cz < 0) { ++faces; wsum += a.wall[4]; }
                        else if (pz - cz >= a.nz) { ++faces; wsum += a.wall[5]; }
                    }
                }
                if (faces > 0) {
                    // Half-way bounce-back against the node's own level-1 value of the opposite
                    // direction at plane pz (written to LDS in iteration it - 1, or kept).
                    const int o = oppv(i);
                    const T own = keep_pos(o) >= 0 ? keep[keep_pos(o)] : lds[lds_slot(o, it - 1)][ly][lx];
                    const T phiw = faces == 1 ? wsum : T(0.5) * wsum;
                    g[i] = fmadd(T(2) * wv<T>(i), phiw, -own);
                } else if (i == 0) {
                    g[i] = keep[0];
                } else if (i == 5) {
                    g[i] = f5pp;
                } else if (i == 6) {
                    g[i] = f[6];
                } else {
                    g[i] = lds[lds_slot(i, it - 1 - cz)][ly - cy][lx - cx];
                }
            }
            const int n = pzz * a.slab + y * a.pitch + x;
            const T phi2 = collide3<T, KPHI>(a, g, prev_phi, SRC ? a.src[n] : T(0));
#pragma unroll
            for (int i = 0; i < kQ; ++i) store<false>(a.fout + i * a.plane + n, g[i]);
            store<false>(a.phi_out + n, phi2);
        }
        __syncthreads();
        f5pp = keep[keep_pos(5)];
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            if (keep_pos(i) >= 0) keep[keep_pos(i)] = f[i];
        prev_phi = phi1;
    }
}

// f+(-1): a value pulled by an interior neighbour is f^eq (Eq. (7), D = phi I) of that neighbour;
// a value the bounce-back consumes at its own node is 2 w phi_w - f^eq of the opposite direction,
// so the first pull yields f(0) = f^eq(phi0). FP64 arithmetic.
template <typename T>
__global__ __launch_bounds__(kBlock) void init3_kernel(Sweep3<T> a, const double* __restrict__ phi0, double a0,
                                                       double a1, double a2, double b0, double b1, double b2,
                                                       double w0, double w1, double w2, double w3, double w4,
                                                       double w5)
{
    const int64_t nn = static_cast<int64_t>(a.nx) * a.ny * a.nz;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= nn) return;
    const int x = static_cast<int>(k % a.nx);
    const int y = static_cast<int>((k / a.nx) % a.ny);
    const int z = static_cast<int>(k / (static_cast<int64_t>(a.nx) * a.ny));
    const double wall[6] = {w0, w1, w2, w3, w4, w5};
    const double av[3] = {a0, a1, a2}, bv[3] = {b0, b1, b2};
    auto feq = [&](int i, double p) {
        double cB = 0.0;
        const int c[3] = {cxv(i), cyv(i), czv(i)};
        for (int d = 0; d < 3; ++d) cB += c[d] * (p * (av[d] + 0.5 * bv[d] * p));
        return wv<double>(i) * (p + 3.0 * cB);
    };
    const int n = z * a.slab + y * a.pitch + x;
    for (int i = 0; i < kQ; ++i) {
        int d[3] = {x + cxv(i), y + cyv(i), z + czv(i)};
        const int dim[3] = {a.nx, a.ny, a.nz};
        int faces = 0;
        double wsum = 0.0;
        for (int c = 0; c < 3; ++c) {
            if (d[c] < 0) {
                if (a.per[c]) d[c] += dim[c]; else { ++faces; wsum += wall[2 * c]; }
            } else if (d[c] >= dim[c]) {
                if (a.per[c]) d[c] -= dim[c]; else { ++faces; wsum += wall[2 * c + 1]; }
            }
        }
        double v;
        if (faces == 0) {
            v = feq(i, phi0[(static_cast<int64_t>(d[2]) * a.ny + d[1]) * a.nx + d[0]]);
        } else {
            const double pw = faces == 1 ? wsum : 0.5 * wsum;
            v = 2.0 * wv<double>(i) * pw - feq(oppv(i), phi0[k]);
        }
        a.fout[i * a.plane + n] = static_cast<T>(v);
    }
    a.phi_out[n] = static_cast<T>(phi0[k]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void convert3_kernel(const double* __restrict__ in, T* __restrict__ out, int nx,
                                                          int ny, int nz, int pitch)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= static_cast<int64_t>(nx) * ny * nz) return;
    const int64_t row = k / nx;
    const int x = static_cast<int>(k - row * nx);
    out[row * pitch + x] = static_cast<T>(in[k]);
}

// Dense index k -> (x, y, z) and the node index of the planes.
template <typename T>
__device__ __forceinline__ void dense_node(const Sweep3<T>& a, int64_t k, int& x, int& y, int& z)
{
    x = static_cast<int>(k % a.nx);
    y = static_cast<int>((k / a.nx) % a.ny);
    z = static_cast<int>(k / (static_cast<int64_t>(a.nx) * a.ny));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void gather3_kernel(Gather3<T> g)
{
    const Sweep3<T>& a = g.s;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= static_cast<int64_t>(a.nx) * a.ny * a.nz) return;
    int x, y, z;
    dense_node(a, k, x, y, z);
    T f[kQ];
    pull3(a, x, y, z, f);
    T v = T(0);
    if (g.population < 0) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) v += f[i];
    } else {
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            if (i == g.population) v = f[i];
    }
    g.out[k] = static_cast<double>(v);
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

// Fixed-order block reduction of kPartials values (entry 4 is a max); result in thread 0.
__device__ __forceinline__ void block_reduce(double v[kPartials])
{
    __shared__ double lds[kBlock / 64][kPartials];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kPartials; ++j) v[j] = (j == 4) ? wave_max(v[j]) : wave_sum(v[j]);
    if (lane == 0)
        for (int j = 0; j < kPartials; ++j) lds[wave][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < kPartials; ++j) {
            double acc = lds[0][j];
            for (int w = 1; w < kBlock / 64; ++w) acc = (j == 4) ? fmax(acc, lds[w][j]) : acc + lds[w][j];
            v[j] = acc;
        }
    }
}

// Residual (mode 0): a = |phi - snap|, b = |phi|, snap := phi. Error (mode 1): a = |phi - ref|,
// b = |ref|, c = (phi - ref)^2, d = ref^2, max |phi - ref|. Entry 5 counts non-finite phi.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void reduce3_kernel(Gather3<T> g)
{
    const Sweep3<T>& a = g.s;
    double v[kPartials] = {0, 0, 0, 0, 0, 0};
    const int64_t nn = static_cast<int64_t>(a.nx) * a.ny * a.nz;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; k < nn; k += stride) {
        int x, y, z;
        dense_node(a, k, x, y, z);
        T f[kQ];
        pull3(a, x, y, z, f);
        T s = T(0);
#pragma unroll
        for (int i = 0; i < kQ; ++i) s += f[i];
        const double phi = static_cast<double>(s);
        if (!isfinite(phi)) v[5] += 1.0;
        if constexpr (MODE == 0) {
            v[0] += fabs(phi - g.snap[k]);
            v[1] += fabs(phi);
            g.snap[k] = phi;
        } else {
            const double r = g.ref[k], d = phi - r;
            v[0] += fabs(d);
            v[1] += fabs(r);
            v[2] += d * d;
            v[3] += r * r;
            v[4] = fmax(v[4], fabs(d));
        }
    }
    block_reduce(v);
    if (threadIdx.x == 0)
        for (int j = 0; j < kPartials; ++j) g.partial[blockIdx.x * kPartials + j] = v[j];
}

__global__ __launch_bounds__(kBlock) void reduce3_final_kernel(const double* __restrict__ partial, int nblocks,
                                                               double* __restrict__ result)
{
    double v[kPartials] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int j = 0; j < kPartials; ++j)
            v[j] = (j == 4) ? fmax(v[j], partial[b * kPartials + j]) : v[j] + partial[b * kPartials + j];
    block_reduce(v);
    if (threadIdx.x == 0)
        for (int j = 0; j < kPartials; ++j) result[j] = v[j];
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

}  // namespace

template <typename T, bool NT>
hipError_t launch3_one(const Sweep3<T>& a, bool src, bool k1_per_node, dim3 grid, dim3 block, hipStream_t s)
{
    if (src) {
        if (k1_per_node)
            hipLaunchKernelGGL((sweep3_kernel<T, true, true, NT>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((sweep3_kernel<T, true, false, NT>), grid, block, 0, s, a);
    } else {
        if (k1_per_node)
            hipLaunchKernelGGL((sweep3_kernel<T, false, true, NT>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((sweep3_kernel<T, false, false, NT>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch3_sweep(const Sweep3<T>& in, bool src, bool k1_per_node, hipStream_t s)
{
    Sweep3<T> a = in;
    a.tiles_x = (a.nx + kTileX - 1) / kTileX;
    a.tiles_y = (a.ny + kTileY - 1) / kTileY;
    const int64_t tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.nz;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(tiles)), block(kBlock);
    return a.nts ? launch3_one<T, true>(a, src, k1_per_node, grid, block, s)
                 : launch3_one<T, false>(a, src, k1_per_node, grid, block, s);
}

int64_t sweep2_workgroups(int nx, int ny, int nz, int tile, int zc)
{
    if (tile < 1 || tile >= kTiles2 || zc < 1) return 0;
    constexpr int txs[5] = {0, 62, 30, 30, 14}, tys[5] = {0, 6, 14, 6, 14};
    const int tx = txs[tile], ty = tys[tile];
    return static_cast<int64_t>((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + zc - 1) / zc);
}

template <typename T, bool WALLS, int TXH, int TYH>
int blocks_per_cu_shape(bool src, bool k1_per_node)
{
    using G = Tile3x2<TXH, TYH>;
    int nb = 0;
    hipError_t e;
    if (src)
        e = k1_per_node ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep3x2_kernel<T, true, true, WALLS, TXH, TYH>, G::N, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep3x2_kernel<T, true, false, WALLS, TXH, TYH>, G::N, 0);
    else
        e = k1_per_node ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep3x2_kernel<T, false, true, WALLS, TXH, TYH>, G::N, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep3x2_kernel<T, false, false, WALLS, TXH, TYH>, G::N, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

template <typename T>
int sweep2_blocks_per_cu(bool walls, bool src, bool k1_per_node, int tile)
{
    switch (tile) {
        case 2: return walls ? blocks_per_cu_shape<T, true, 32, 16>(src, k1_per_node) : blocks_per_cu_shape<T, false, 32, 16>(src, k1_per_node);
        case 3: return walls ? blocks_per_cu_shape<T, true, 32, 8>(src, k1_per_node) : blocks_per_cu_shape<T, false, 32, 8>(src, k1_per_node);
        case 4: return walls ? blocks_per_cu_shape<T, true, 16, 16>(src, k1_per_node) : blocks_per_cu_shape<T, false, 16, 16>(src, k1_per_node);
        default: return walls ? blocks_per_cu_shape<T, true, 64, 8>(src, k1_per_node) : blocks_per_cu_shape<T, false, 64, 8>(src, k1_per_node);
    }
}

template <typename T, bool WALLS, int TXH, int TYH>
hipError_t launch3_sweep2_shape(Sweep3<T> a, bool src, bool k1_per_node, int zc, hipStream_t s)
{
    using G = Tile3x2<TXH, TYH>;
    a.tiles_x = (a.nx + G::TX - 1) / G::TX;
    a.tiles_y = (a.ny + G::TY - 1) / G::TY;
    a.zc = zc;
    const int64_t wg = static_cast<int64_t>(a.tiles_x) * a.tiles_y * ((a.nz + zc - 1) / zc);
    if (zc < 1 || wg > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(wg)), block(G::N);
    if (src) {
        if (k1_per_node)
            hipLaunchKernelGGL((sweep3x2_kernel<T, true, true, WALLS, TXH, TYH>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((sweep3x2_kernel<T, true, false, WALLS, TXH, TYH>), grid, block, 0, s, a);
    } else {
        if (k1_per_node)
            hipLaunchKernelGGL((sweep3x2_kernel<T, false, true, WALLS, TXH, TYH>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((sweep3x2_kernel<T, false, false, WALLS, TXH, TYH>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch3_sweep2(const Sweep3<T>& a, bool src, bool k1_per_node, int tile, int zc, hipStream_t s)
{
    const bool walls = !(a.per[0] && a.per[1] && a.per[2]);
    switch (tile) {
        case 1:
            return walls ? launch3_sweep2_shape<T, true, 64, 8>(a, src, k1_per_node, zc, s)
                         : launch3_sweep2_shape<T, false, 64, 8>(a, src, k1_per_node, zc, s);
        case 2:
            return walls ? launch3_sweep2_shape<T, true, 32, 16>(a, src, k1_per_node, zc, s)
                         : launch3_sweep2_shape<T, false, 32, 16>(a, src, k1_per_node, zc, s);
        case 3:
            return walls ? launch3_sweep2_shape<T, true, 32, 8>(a, src, k1_per_node, zc, s)
                         : launch3_sweep2_shape<T, false, 32, 8>(a, src, k1_per_node, zc, s);
        case 4:
            return walls ? launch3_sweep2_shape<T, true, 16, 16>(a, src, k1_per_node, zc, s)
                         : launch3_sweep2_shape<T, false, 16, 16>(a, src, k1_per_node, zc, s);
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch3_init(const Sweep3<T>& a, const double* phi0, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(a.nx) * a.ny * a.nz;
    hipLaunchKernelGGL((init3_kernel<T>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, a, phi0,
                       static_cast<double>(a.a[0]), static_cast<double>(a.a[1]), static_cast<double>(a.a[2]),
                       static_cast<double>(a.b[0]), static_cast<double>(a.b[1]), static_cast<double>(a.b[2]),
                       static_cast<double>(a.wall[0]), static_cast<double>(a.wall[1]), static_cast<double>(a.wall[2]),
                       static_cast<double>(a.wall[3]), static_cast<double>(a.wall[4]),
                       static_cast<double>(a.wall[5]));
    return hipGetLastError();
}

template <typename T>
hipError_t launch3_gather(const Gather3<T>& g, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(g.s.nx) * g.s.ny * g.s.nz;
    hipLaunchKernelGGL((gather3_kernel<T>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, g);
    return hipGetLastError();
}

template <typename T>
hipError_t launch3_reduce(const Gather3<T>& g, int mode, double* result, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(g.s.nx) * g.s.ny * g.s.nz;
    const unsigned nb = static_cast<unsigned>(std::min<int64_t>(kReduceBlocks3, (nn + kBlock - 1) / kBlock));
    if (mode == 0)
        hipLaunchKernelGGL((reduce3_kernel<T, 0>), dim3(nb), dim3(kBlock), 0, s, g);
    else
        hipLaunchKernelGGL((reduce3_kernel<T, 1>), dim3(nb), dim3(kBlock), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce3_final_kernel, dim3(1), dim3(kBlock), 0, s, g.partial, static_cast<int>(nb), result);
    return hipGetLastError();
}

template <typename T>
hipError_t launch3_convert(const double* in, T* out, int nx, int ny, int nz, int pitch, hipStream_t s)
{
    const int64_t nn = static_cast<int64_t>(nx) * ny * nz;
    hipLaunchKernelGGL((convert3_kernel<T>), dim3(blocks_for(nn)), dim3(kBlock), 0, s, in, out, nx, ny, nz, pitch);
    return hipGetLastError();
}

#define BTRT3_INSTANTIATE(T)                                                                        \
    template hipError_t launch3_sweep<T>(const Sweep3<T>&, bool, bool, hipStream_t);                \
    template hipError_t launch3_sweep2<T>(const Sweep3<T>&, bool, bool, int, int, hipStream_t);     \
    template int sweep2_blocks_per_cu<T>(bool, bool, bool, int);                                    \
    template hipError_t launch3_init<T>(const Sweep3<T>&, const double*, hipStream_t);              \
    template hipError_t launch3_gather<T>(const Gather3<T>&, hipStream_t);                          \
    template hipError_t launch3_reduce<T>(const Gather3<T>&, int, double*, hipStream_t);            \
    template hipError_t launch3_convert<T>(const double*, T*, int, int, int, int, hipStream_t);

BTRT3_INSTANTIATE(double)
BTRT3_INSTANTIATE(float)

}  // namespace btrt3k
