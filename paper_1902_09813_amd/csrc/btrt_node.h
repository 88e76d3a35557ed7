// Per-node pieces of the B-TriRT D2Q9 sweep (Zhao, Wu, Chai & Shi, arXiv:1902.09813):
// the pull with half-way bounce-back (Eq. (38), Eqs. (54)-(56)) and the collision of Eq. (6)
// (with Eqs. (7), (8), (11), (30)). Host-callable as well, so the same code can be
// exercised on the CPU; the library itself only runs it inside its kernels.
#pragma once

#include "btrt_internal.h"

namespace btrtk {

// a*b + c with a single rounding, in the storage type.
template <typename T>
__host__ __device__ inline T fmadd(T a, T b, T c)
{
    if constexpr (sizeof(T) == 4)
        return fmaf(a, b, c);
    else
        return fma(a, b, c);
}

// |x|^y in the storage type (the power-law flux and the phi-dependent source).
template <typename T>
__host__ __device__ inline T abspow(T x, T y)
{
    if constexpr (sizeof(T) == 4)
        return powf(fabsf(x), y);
    else
        return pow(fabs(x), y);
}

// 1/d for the per-node K1 (d = det M >= 1/4). FP64: the hardware reciprocal refined by two
// Newton steps, about half the instructions of an IEEE division, which matters in the fused
// walkers where every level repeats it; measured on gfx950 over 2^24 divisors log-uniform in
// [1/4, 64), it gives the IEEE quotient every time (the reciprocal alone is off by up to 2.5e8
// ulp, one Newton step by up to 11). FP32: a division,
// or with ONE_NEWTON the hardware reciprocal and one Newton step (within an ulp, a third of the
// instructions; the 16-bit deviation formats, whose walkers keep the VALU busy every cycle, run
// 5-6.5 % faster with it, while the FP32 seven-step walker's schedule ran 2 % slower).
template <typename T, bool ONE_NEWTON = false>
__host__ __device__ inline T recip(T d)
{
    if constexpr (sizeof(T) == 4) {
        if constexpr (ONE_NEWTON) {
#if defined(__HIP_DEVICE_COMPILE__)
            const T r = __builtin_amdgcn_rcpf(d);
#else
            const T r = T(1) / d;
#endif
            return fmadd(r, fmadd(-d, r, T(1)), r);
        } else {
            return T(1) / d;
        }
    } else {
#if defined(__HIP_DEVICE_COMPILE__)
        T r = __builtin_amdgcn_rcp(d);
#else
        T r = T(1) / d;
#endif
        T e = fmadd(-d, r, T(1));
        r = fmadd(r, e, r);
        e = fmadd(-d, r, T(1));
        return fmadd(r, e, r);
    }
}

// Half-way bounce-back value (Eqs. (54)-(56)): -f_opp+ + 2 w phi_w.
template <typename T>
__host__ __device__ inline T bounce(T f_opp, T two_w, T phi_w)
{
    return fmadd(two_w, phi_w, -f_opp);
}

template <typename T>
struct Lat {
    static constexpr T w0 = T(4) / T(9);
    static constexpr T w1 = T(1) / T(9);
    static constexpr T w5 = T(1) / T(36);
};

template <typename T>
__host__ __device__ inline T wall_value(bool out_x, bool out_y, T vx, T vy)
{
    // A link crossing both walls (a corner point) takes the mean of the two values.
    return (out_x && out_y) ? T(0.5) * (vx + vy) : (out_x ? vx : vy);
}

// Velocity components of direction i (the order of Eq. (85)); i is a constant wherever these
// are used, so they fold away.
__host__ __device__ constexpr int dir_cx(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0); }
__host__ __device__ constexpr int dir_cy(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0); }

// Dirichlet value phi_w for the pull of direction i at a node whose pull crosses a wall, from
// the per-side constants w = (x-, x+, y-, y+): the population bounced back left the node along
// -c_i, through side x- when c_ix > 0 (x+ when < 0) and y- when c_iy > 0 (y+ when < 0).
template <typename T>
__host__ __device__ inline T side_wall(const T w[4], int i, bool out_x, bool out_y)
{
    return wall_value(out_x, out_y, w[dir_cx(i) > 0 ? 0 : 1], w[dir_cy(i) > 0 ? 2 : 3]);
}

// The same from the wall table entry of step lvl of a launch (general node model). Half-way
// bounce-back (Eqs. (54)-(56)) puts a wall half a spacing beyond the last node, so the link from
// node (x, y) (at x + 1/2, y + 1/2) along -c_i meets it at x + 1/2 - c_ix/2, y + 1/2 - c_iy/2.
// An entry holds each side sampled every half spacing from corner to corner: x- (2 ny + 1
// samples), x+ (2 ny + 1), y- (2 nx + 1), y+ (2 nx + 1), sample s at position s/2; the link then
// reads sample 2y + 1 - c_iy of its x side or 2x + 1 - c_ix of its y side. Four more slots hold,
// for the links that meet a corner point, the mean of the two sides' corner samples (corners
// x-y-, x+y-, x+y+, x-y+; filled by the library). Every index lies inside its side for a node
// of the grid.
template <typename T>
__host__ __device__ inline T table_wall(const SweepArgs<T>& a, int x, int y, int lvl, int i, bool out_x, bool out_y)
{
    const T* e = a.wtab + lvl * a.wstride;
    const int cx = dir_cx(i), cy = dir_cy(i);
    const int sx = 2 * a.ny + 1, sy = 2 * a.nx + 1;
    if (out_x && out_y) return e[2 * sx + 2 * sy + (cy > 0 ? (cx > 0 ? 0 : 1) : (cx > 0 ? 3 : 2))];
    if (out_x) return e[(cx > 0 ? 0 : sx) + 2 * y + 1 - cy];
    return e[2 * sx + (cy > 0 ? 0 : sy) + 2 * x + 1 - cx];
}

// Pull f_i(x, t) for all nine directions: load(i, idx) returns the post-collision value
// f_i+(t-1) stored at in-plane index idx (for a storage format of the caller's choice);
// wall(i, out_x, out_y) the Dirichlet value of a pull that crosses a wall (side_wall, table_wall).
template <typename T, typename Load, typename Wall>
__host__ __device__ inline void gather_with(Load load, int x, int y, int nx, int ny, int pitch, int perx, int pery,
                                            Wall wall, T f[9])
{
    const int n = y * pitch + x;
    if (x > 0 && x < nx - 1 && y > 0 && y < ny - 1) {
        f[0] = load(0, n);
        f[1] = load(1, n - 1);
        f[2] = load(2, n - pitch);
        f[3] = load(3, n + 1);
        f[4] = load(4, n + pitch);
        f[5] = load(5, n - pitch - 1);
        f[6] = load(6, n - pitch + 1);
        f[7] = load(7, n + pitch + 1);
        f[8] = load(8, n + pitch - 1);
        return;
    }
    // Edge node: wrap periodic directions, bounce back at Dirichlet walls.
    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
    bool okxm = true, okxp = true, okym = true, okyp = true;
    if (xm < 0) { if (perx) xm += nx; else okxm = false; }
    if (xp >= nx) { if (perx) xp -= nx; else okxp = false; }
    if (ym < 0) { if (pery) ym += ny; else okym = false; }
    if (yp >= ny) { if (pery) yp -= ny; else okyp = false; }
    const int r0 = y * pitch, rm = ym * pitch, rp = yp * pitch;
    const T tw1 = T(2) * Lat<T>::w1, tw5 = T(2) * Lat<T>::w5;
    f[0] = load(0, n);
    f[1] = okxm ? load(1, r0 + xm) : bounce(load(3, n), tw1, wall(1, true, false));
    f[2] = okym ? load(2, rm + x) : bounce(load(4, n), tw1, wall(2, false, true));
    f[3] = okxp ? load(3, r0 + xp) : bounce(load(1, n), tw1, wall(3, true, false));
    f[4] = okyp ? load(4, rp + x) : bounce(load(2, n), tw1, wall(4, false, true));
    f[5] = (okxm && okym) ? load(5, rm + xm) : bounce(load(7, n), tw5, wall(5, !okxm, !okym));
    f[6] = (okxp && okym) ? load(6, rm + xp) : bounce(load(8, n), tw5, wall(6, !okxp, !okym));
    f[7] = (okxp && okyp) ? load(7, rp + xp) : bounce(load(5, n), tw5, wall(7, !okxp, !okyp));
    f[8] = (okxm && okyp) ? load(8, rp + xm) : bounce(load(6, n), tw5, wall(8, !okxm, !okyp));
}

// Pull from nine planes of T (plane stride `plane`).
template <typename T, typename Wall>
__host__ __device__ inline void gather(const T* __restrict__ fin, int64_t plane, int x, int y, int nx,
                                       int ny, int pitch, int perx, int pery, Wall wall, T f[9])
{
    gather_with<T>([fin, plane](int i, int idx) { return fin[i * plane + idx]; }, x, y, nx, ny, pitch, perx, pery,
                   wall, f);
}

// Equilibrium of Eq. (7) with D = phi I for direction i: w_i (phi + 3 c_i . B(phi)), with
// B(phi) = phi (a + b phi / 2).
template <typename T>
__host__ __device__ inline T feq_dir(int i, T phi, T ax, T ay, T bx, T by)
{
    const T Bx = phi * fmadd(T(0.5) * bx, phi, ax);
    const T By = phi * fmadd(T(0.5) * by, phi, ay);
    switch (i) {
        case 0: return Lat<T>::w0 * phi;
        case 1: return Lat<T>::w1 * fmadd(T(3), Bx, phi);
        case 2: return Lat<T>::w1 * fmadd(T(3), By, phi);
        case 3: return Lat<T>::w1 * fmadd(T(-3), Bx, phi);
        case 4: return Lat<T>::w1 * fmadd(T(-3), By, phi);
        case 5: return Lat<T>::w5 * fmadd(T(3), Bx + By, phi);
        case 6: return Lat<T>::w5 * fmadd(T(3), By - Bx, phi);
        case 7: return Lat<T>::w5 * fmadd(T(-3), Bx + By, phi);
        default: return Lat<T>::w5 * fmadd(T(3), Bx - By, phi);
    }
}

// phi = sum_i f_i (Eq. (9)), summed over pairs of opposite directions; collide forms the same
// sums, so the phi a sweep writes and the phi a gather returns have the same bits.
template <typename T>
__host__ __device__ inline T sum9(const T f[9])
{
    return (f[0] + (f[1] + f[3])) + ((f[2] + f[4]) + ((f[5] + f[7]) + (f[6] + f[8])));
}

// One node of the B-TriRT collision; f holds f(x, t) on entry and f+(x, t) on return. Returns
// phi(t). Eq. (6) with f^neq = f - f^eq is used in the form
//     f_i+ = (1 - k0) f_i + w_i [E_i + 3 c_i . q],
//     q    = k0 j + dB - K1 (M1 + dB/2),                      (M1 = j - B, Eq. (10); G of Eq. (11))
//     E_i  = k0 phi + s + 3/2 tr Q - 9/2 c_i^T Q c_i,        Q = (K2 - k0) o M2,
// where M2 = P - (d/3) I is the second moment of f^neq (P = sum c c f, Eq. (9)) and, for
// D = d I != phi I, Q gains -k0 (d - phi)/3 on the diagonal (the D term of f^eq in Eq. (7)), so
// only phi, j and P are needed: the moments the block relaxation (Eq. (99)) changes; all others
// relax with k0 through (1 - k0) f_i. The library is built without floating-point contraction:
// every fused multiply-add below is written out, so a node update rounds the same way in every
// kernel that inlines it.
// KM (K1Mode, plus kGen) selects where K1 comes from and the node model; n is the node's
// in-plane index (read only for an A0 field). s is the part of the source term of the step that
// does not depend on phi, with the Scheme 2 correction folded in.
template <typename T, int SRC, int KM>
__host__ __device__ inline T collide(const SweepArgs<T>& a, T f[9], T phi_prev, T s, int n)
{
    constexpr int K1M = KM & kK1Mask;
    constexpr bool GEN = (KM & kGen) != 0;
    constexpr bool K0ONE = (KM & kK0One) != 0;  // k0 = 1: no (1 - k0) f_i term
    constexpr T third = T(1) / T(3);
    constexpr T half = T(0.5);

    // phi, j and P (rows of Eq. (88)) from sums and differences of opposite populations.
    const T s13 = f[1] + f[3], s24 = f[2] + f[4], s57 = f[5] + f[7], s68 = f[6] + f[8];
    const T d13 = f[1] - f[3], d24 = f[2] - f[4], d57 = f[5] - f[7], d68 = f[6] - f[8];
    const T sd = s57 + s68;
    const T phi = sum9(f);  // (f0 + s13) + (s24 + sd)
    const T jx = d13 + (d57 - d68);
    const T jy = d24 + (d57 + d68);
    const T pxx = s13 + sd;
    const T pyy = s24 + sd;
    const T pxy = s57 - s68;

    // Flux B(phi) = phi (a + b phi / 2) and its backward difference over one step (the
    // correction G of Eq. (11)).
    const T hbx = half * a.bx, hby = half * a.by;
    T Bx = phi * fmadd(hbx, phi, a.ax);
    T By = phi * fmadd(hby, phi, a.ay);
    T dBx, dBy;
    if (GEN && (a.fcx != T(0) || a.fcy != T(0))) {
        // General model: B gains c |phi|^q.
        const T pw = abspow(phi, a.fq), pwp = abspow(phi_prev, a.fq);
        const T Bxp = fmadd(a.fcx, pwp, phi_prev * fmadd(hbx, phi_prev, a.ax));
        const T Byp = fmadd(a.fcy, pwp, phi_prev * fmadd(hby, phi_prev, a.ay));
        Bx = fmadd(a.fcx, pw, Bx);
        By = fmadd(a.fcy, pw, By);
        dBx = Bx - Bxp;
        dBy = By - Byp;
    } else {
        dBx = fmadd(-phi_prev, fmadd(hbx, phi_prev, a.ax), Bx);
        dBy = fmadd(-phi_prev, fmadd(hby, phi_prev, a.ay), By);
    }
    if (GEN && a.rr != T(0)) {
        // General model: S(phi) = r phi (1 - |phi|^p) with the Scheme 2 correction,
        // S(t) + (S(t) - S(t-1))/2, S(t-1) taken at phi(t-1).
        const T R = (a.rr * phi) * (T(1) - abspow(phi, a.rp));
        const T Rp = (a.rr * phi_prev) * (T(1) - abspow(phi_prev, a.rp));
        s = s + fmadd(T(1.5), R, -half * Rp);
    }

    // Odd part: q = k0 j + dB - K1 h, h = j - B + dB/2, with K1 = (A / c_s^2 + I/2)^-1 (Eq. (30)).
    // Per node when A depends on phi or on x (A = A0(x) (1 + beta phi^2), Eq. (73)): with
    // M = 3 A + I/2, K1 h = adj(M) h / det M, the adjugate applied first and 1/det M taken into
    // the last multiply-add (three multiplies fewer than forming K1).
    const T k0 = K0ONE ? T(1) : a.k0;
    const T hx = fmadd(half, dBx, jx - Bx), hy = fmadd(half, dBy, jy - By);
    T qx, qy;
    if constexpr (K1M != kK1Const) {
        T a11 = a.a11, a12 = a.a12, a22 = a.a22;
        if constexpr (K1M == kK1Field) {
            a11 = a.afield[n];
            a12 = a.afield[a.plane + n];
            a22 = a.afield[2 * a.plane + n];
        }
        const T g = fmadd(a.beta, phi * phi, T(1));
        const T m11 = fmadd(T(3) * a11, g, half);
        const T m12 = (T(3) * a12) * g;
        const T m22 = fmadd(T(3) * a22, g, half);
        const T rdet = recip<T, (KM & kRcp1) != 0>(fmadd(m11, m22, -(m12 * m12)));
        const T ux = fmadd(m22, hx, -(m12 * hy));
        const T uy = fmadd(m11, hy, -(m12 * hx));
        qx = fmadd(-rdet, ux, fmadd(k0, jx, dBx));
        qy = fmadd(-rdet, uy, fmadd(k0, jy, dBy));
    } else {
        qx = fmadd(k0, jx, dBx) - fmadd(a.K11, hx, a.K12 * hy);
        qy = fmadd(k0, jy, dBy) - fmadd(a.K12, hx, a.K22 * hy);
    }

    // Even part: Q = (K2 - k0) o (P - d/3 I) with d = phi (D = phi I) or the general model's d.
    T d3 = third * phi;
    T diag = T(0);
    if (GEN && a.dpoly) {
        // General model: D = d(phi) I; the equilibrium of P is d/3 I (Eq. (9)) and f^eq of
        // Eq. (7) gains 3/2 (d - phi)(|c|^2 - 2/3) w_i, i.e. -k0 (d - phi)/3 on Q's diagonal.
        const T d = a.de != T(0) ? fmadd(a.dg, phi, a.de * abspow(phi, a.ds)) : a.dg * phi;
        d3 = third * d;
        diag = (-k0 * third) * (d - phi);
    }
    T Qxx = (a.k2xx - k0) * (pxx - d3);
    T Qyy = (a.k2yy - k0) * (pyy - d3);
    const T Qxy = (a.k2xy - k0) * pxy;
    if (GEN && a.dpoly) {
        Qxx = Qxx + diag;
        Qyy = Qyy + diag;
    }
    const T trQ = Qxx + Qyy;
    // Without a source s is zero, and k0 phi is the product itself (no "+ 0" instruction).
    const T ks = (SRC == kSrcNone && !GEN) ? k0 * phi : fmadd(k0, phi, s);
    const T base = fmadd(a.cq[0], trQ, ks);

    // f+ per direction pair: (1 - k0) f_i + w_i E_i +- 3 w_i c_i . q. With k0 = 1 the first
    // term is dropped (fma(0, f, v) is v but for the sign of a zero v).
    const T om0 = T(1) - k0;
    auto relax = [&](T fi, T v) { return K0ONE ? v : fmadd(om0, fi, v); };
    constexpr T w0 = Lat<T>::w0, w1 = Lat<T>::w1, w5 = Lat<T>::w5;
    f[0] = relax(f[0], w0 * base);
    const T ex = w1 * fmadd(a.cq[1], Qxx, base), ox = (T(3) * w1) * qx;
    f[1] = relax(f[1], ex + ox);
    f[3] = relax(f[3], ex - ox);
    const T ey = w1 * fmadd(a.cq[1], Qyy, base), oy = (T(3) * w1) * qy;
    f[2] = relax(f[2], ey + oy);
    f[4] = relax(f[4], ey - oy);
    const T ed = fmadd(a.cq[1], trQ, base);
    const T e57 = w5 * fmadd(a.cq[2], Qxy, ed), o57 = (T(3) * w5) * (qx + qy);
    f[5] = relax(f[5], e57 + o57);
    f[7] = relax(f[7], e57 - o57);
    const T e68 = w5 * fmadd(a.cq[3], Qxy, ed), o68 = (T(3) * w5) * (qy - qx);
    f[6] = relax(f[6], e68 + o68);
    f[8] = relax(f[8], e68 - o68);
    return phi;
}

// f+(-1) at node (x, y) such that the first pull yields f(0) = f^eq(phi0) (Section 4): a value
// whose consumer is an interior pull gets f^eq of Eq. (7) (D = phi I) at its destination; a
// value whose consumer is the bounce-back rule gets 2 w phi_w - f^eq_opp at its own node.
// ab = (ax, ay, bx, by), cq = (cx, cy, q): B(phi) = a phi + b phi^2 / 2 + c |phi|^q; dq = (kind,
// g, e, s): D(phi) = phi I (kind 0) or (g phi + e |phi|^s) I.
// put(i, v) receives the value for direction i (FP64).
__host__ __device__ inline void init_flux(double p, const double ab[4], const double cq[3], double& Bx, double& By)
{
    Bx = p * (ab[0] + 0.5 * ab[2] * p);
    By = p * (ab[1] + 0.5 * ab[3] * p);
    if (cq[0] != 0.0 || cq[1] != 0.0) {
        const double pw = pow(fabs(p), cq[2]);
        Bx += cq[0] * pw;
        By += cq[1] * pw;
    }
}

// w_i (phi + 3 c_i . B + 3/2 (d - phi)(|c_i|^2 - 2/3)) of Eq. (7) for D = d I.
__host__ __device__ inline double init_feq(int i, double p, double Bx, double By, const double dq[4])
{
    constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double wt[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    double v = p + 3.0 * (cx[i] * Bx + cy[i] * By);
    if (dq[0] != 0.0) {
        const double d = dq[1] * p + (dq[2] != 0.0 ? dq[2] * pow(fabs(p), dq[3]) : 0.0);
        v += 1.5 * (d - p) * (cx[i] * cx[i] + cy[i] * cy[i] - 2.0 / 3.0);
    }
    return wt[i] * v;
}

template <typename Put>
__host__ __device__ inline void init_values(const double* __restrict__ phi0, int x, int y, int nx, int ny, int perx,
                                            int pery, const double wall[4], const double ab[4], const double cq[3],
                                            const double dq[4], Put put)
{
    constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    const double wt[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const double here = phi0[static_cast<int64_t>(y) * nx + x];
    for (int i = 0; i < 9; ++i) {
        int xd = x + cx[i], yd = y + cy[i];
        bool outx = false, outy = false;
        if (xd < 0) { if (perx) xd += nx; else outx = true; }
        if (xd >= nx) { if (perx) xd -= nx; else outx = true; }
        if (yd < 0) { if (pery) yd += ny; else outy = true; }
        if (yd >= ny) { if (pery) yd -= ny; else outy = true; }
        double v;
        if (!outx && !outy) {
            const double p = phi0[static_cast<int64_t>(yd) * nx + xd];
            double Bx, By;
            init_flux(p, ab, cq, Bx, By);
            v = init_feq(i, p, Bx, By, dq);
        } else {
            // The link leaves through x- or x+ (y- or y+) according to the sign of c_i.
            const double vx = wall[cx[i] < 0 ? 0 : 1];
            const double vy = wall[cy[i] < 0 ? 2 : 3];
            const double pw = (outx && outy) ? 0.5 * (vx + vy) : (outx ? vx : vy);
            const int o = opp[i];
            double Bx, By;
            init_flux(here, ab, cq, Bx, By);
            const double feq_o = init_feq(o, here, Bx, By, dq);
            v = 2.0 * wt[i] * pw - feq_o;
        }
        put(i, v);
    }
}

}  // namespace btrtk
