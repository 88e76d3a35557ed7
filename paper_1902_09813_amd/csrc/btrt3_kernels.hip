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

template <typename T>
__device__ __forceinline__ void store(T* p, T v, bool nontemporal)
{
    if (nontemporal)
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
    const T E0 = fmadd(T(1.5), (Qxx + Qyy) + Qzz, fmadd(a.k0, phi, s));

    const T om = T(1) - a.k0;
    const T w0 = wv<T>(0), w1 = wv<T>(1), w2 = wv<T>(7);
    f[0] = fmadd(om, f[0], w0 * E0);
    // Axis pairs: c^T Q c = Q_aa, c . q = +-q_a.
    const T ex = fmadd(T(-4.5), Qxx, E0), ey = fmadd(T(-4.5), Qyy, E0), ez = fmadd(T(-4.5), Qzz, E0);
    f[1] = fmadd(om, f[1], w1 * fmadd(T(3), qx, ex));
    f[2] = fmadd(om, f[2], w1 * fmadd(T(-3), qx, ex));
    f[3] = fmadd(om, f[3], w1 * fmadd(T(3), qy, ey));
    f[4] = fmadd(om, f[4], w1 * fmadd(T(-3), qy, ey));
    f[5] = fmadd(om, f[5], w1 * fmadd(T(3), qz, ez));
    f[6] = fmadd(om, f[6], w1 * fmadd(T(-3), qz, ez));
    // Face-diagonal pairs: c^T Q c = Q_aa + Q_bb +- 2 Q_ab, c . q = +-q_a +- q_b.
    const T xy = fmadd(T(-4.5), Qxx + Qyy, E0), xz = fmadd(T(-4.5), Qxx + Qzz, E0), yz = fmadd(T(-4.5), Qyy + Qzz, E0);
    const T xyp = fmadd(T(-9), Qxy, xy), xym = fmadd(T(9), Qxy, xy);
    const T xzp = fmadd(T(-9), Qxz, xz), xzm = fmadd(T(9), Qxz, xz);
    const T yzp = fmadd(T(-9), Qyz, yz), yzm = fmadd(T(9), Qyz, yz);
    f[7] = fmadd(om, f[7], w2 * fmadd(T(3), qx + qy, xyp));    // ( 1,  1,  0)
    f[10] = fmadd(om, f[10], w2 * fmadd(T(-3), qx + qy, xyp)); // (-1, -1,  0)
    f[8] = fmadd(om, f[8], w2 * fmadd(T(3), qy - qx, xym));    // (-1,  1,  0)
    f[9] = fmadd(om, f[9], w2 * fmadd(T(-3), qy - qx, xym));   // ( 1, -1,  0)
    f[11] = fmadd(om, f[11], w2 * fmadd(T(3), qx + qz, xzp));  // ( 1,  0,  1)
    f[14] = fmadd(om, f[14], w2 * fmadd(T(-3), qx + qz, xzp)); // (-1,  0, -1)
    f[12] = fmadd(om, f[12], w2 * fmadd(T(3), qz - qx, xzm));  // (-1,  0,  1)
    f[13] = fmadd(om, f[13], w2 * fmadd(T(-3), qz - qx, xzm)); // ( 1,  0, -1)
    f[15] = fmadd(om, f[15], w2 * fmadd(T(3), qy + qz, yzp));  // ( 0,  1,  1)
    f[18] = fmadd(om, f[18], w2 * fmadd(T(-3), qy + qz, yzp)); // ( 0, -1, -1)
    f[16] = fmadd(om, f[16], w2 * fmadd(T(3), qz - qy, yzm));  // ( 0, -1,  1)
    f[17] = fmadd(om, f[17], w2 * fmadd(T(-3), qz - qy, yzm)); // ( 0,  1, -1)
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

template <typename T, bool SRC, bool KPHI>
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
    for (int i = 0; i < kQ; ++i) store(a.fout + i * a.plane + n, f[i], a.nts);
    store(a.phi_out + n, phi, a.nts);
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

template <typename T>
hipError_t launch3_sweep(const Sweep3<T>& in, bool src, bool k1_per_node, hipStream_t s)
{
    Sweep3<T> a = in;
    a.tiles_x = (a.nx + kTileX - 1) / kTileX;
    a.tiles_y = (a.ny + kTileY - 1) / kTileY;
    const int64_t tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.nz;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(tiles)), block(kBlock);
    if (src) {
        if (k1_per_node)
            hipLaunchKernelGGL((sweep3_kernel<T, true, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((sweep3_kernel<T, true, false>), grid, block, 0, s, a);
    } else {
        if (k1_per_node)
            hipLaunchKernelGGL((sweep3_kernel<T, false, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((sweep3_kernel<T, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
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
    template hipError_t launch3_init<T>(const Sweep3<T>&, const double*, hipStream_t);              \
    template hipError_t launch3_gather<T>(const Gather3<T>&, hipStream_t);                          \
    template hipError_t launch3_reduce<T>(const Gather3<T>&, int, double*, hipStream_t);            \
    template hipError_t launch3_convert<T>(const double*, T*, int, int, int, int, hipStream_t);

BTRT3_INSTANTIATE(double)
BTRT3_INSTANTIATE(float)

}  // namespace btrt3k
