// Device-side building blocks of the GRPIC hot path for gfx950 (CDNA4).
//
// Metric: Kerr in Cartesian Kerr-Schild form, g = eta + f k k with
// eta = diag(1,1,1,-1), f = 2 m r^3 / (r^4 + a^2 z^2) and the null one-form
// k = ((r x - a y)/(r^2+a^2), (r y + a x)/(r^2+a^2), z/r, 1) (Sec. 2.1, eq.
// kerr_metric and the expression for k), r the root of
// r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0 (eq. radius_eqn).  Because k is null,
// g^{-1} = eta - f k^a k^b with k^a = (k_1, k_2, k_3, -1), and det g = -1.
// The Christoffel contraction Gamma^a_{mn} u^m u^n is formed directly from
// f, k and their gradients (rank-one structure), never as a 4x4x4 array.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grpic {

constexpr int kMaxSpecies = 8;
constexpr uint8_t kDead = 0xFF;

// Ghosted field layout shared by every staggered component: index
// (i,j,k) with i in [-1, nx+1] at ((k+1)*sy + (j+1))*sx + (i+1).
struct Grid {
    int nx, ny, nz;
    int64_t sx, sy;  // strides: sx = nx+3, sy = (ny+3)*(nx+3)
    __host__ __device__ inline int64_t g(int i, int j, int k) const {
        return (int64_t)(k + 1) * sy + (int64_t)(j + 1) * sx + (i + 1);
    }
    __host__ __device__ inline int64_t node(int i, int j, int k) const {
        return ((int64_t)k * (ny + 1) + j) * (nx + 1) + i;
    }
    __host__ __device__ inline int64_t gsize() const { return sy * (nz + 3); }
    __host__ __device__ inline int64_t nnodes() const {
        return (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    }
    __host__ __device__ inline int dim(int ax) const { return ax == 0 ? nx : (ax == 1 ? ny : nz); }
};

// Hole parameters every kernel needs.
struct Hole {
    double m, a;
    double cx, cy, cz;
    double r_exc;
};

// Square root, reciprocal square root, reciprocal and quotient from the
// hardware estimates (about 2^-23 relative) refined by one third-order step:
// with e = 1 - x y^2 the error of y = x^-1/2, y (1 + e/2 + 3 e^2 / 8) has
// error O(e^3); with e = 1 - d r, r (1 + e + e^2) has error O(e^3); the
// quotient adds a residual correction.  A few ulps instead of the correctly
// rounded result, at about a third of the instructions.  sqrt_nr takes
// x >= 0 and raises it to the smallest normal first (so 0 gives about
// 1.5e-154, which vanishes against anything it is added to); rsqrt_nr takes
// a finite positive normal x; rcp_nr and div_nr a finite non-zero normal d.
__device__ __forceinline__ double sqrt_nr(double x) {
    x = fmax(x, 2.2250738585072014e-308);
    const double y = __builtin_amdgcn_rsq(x);
    const double s = x * y;
    const double e = fma(-s, y, 1.0);
    return fma(s * e, fma(e, 0.375, 0.5), s);
}
// sqrt_nr without the raise to the smallest normal: for x > 0 (normal or
// subnormal) the same value; 0 gives NaN, which callers must treat as such.
__device__ __forceinline__ double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double s = x * y;
    const double e = fma(-s, y, 1.0);
    return fma(s * e, fma(e, 0.375, 0.5), s);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ double rcp_nr(double d) {
    const double r = __builtin_amdgcn_rcp(d);
    const double e = fma(-d, r, 1.0);
    return fma(r, fma(e, e, e), r);
}
__device__ __forceinline__ double div_nr(double n, double d) {
    const double r = rcp_nr(d);
    const double q = n * r;
    return fma(fma(-d, q, n), r, q);
}
// 1/d in the pusher's type: the refined FP64 estimate, or the FP32 hardware
// reciprocal with one Newton step.
template <typename T> __device__ __forceinline__ T recip(T d);
template <> __device__ __forceinline__ double recip<double>(double d) { return rcp_nr(d); }
template <> __device__ __forceinline__ float recip<float>(float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    return fmaf(fmaf(-d, r, 1.0f), r, r);
}

// Radius from the quartic, always in FP64: the cancellation-free root for
// r^2 on each side of R^2 = a^2.
__device__ __forceinline__ double ks_radius(double a, double x, double y, double z) {
    double R2 = x * x + y * y + z * z;
    double b = R2 - a * a;
    double a2z2 = a * a * z * z;
    double s = sqrt(b * b + 4.0 * a2z2);
    double r2 = (b >= 0.0) ? 0.5 * (b + s) : (2.0 * a2z2) / (s - b);
    return sqrt(r2);
}

// The same root with the refined square roots and quotient (the hot paths:
// every RK4 stage and every deposit face point); r2 receives r^2 as the
// quartic gives it.  The quotient branch (R < |a|, deep inside the horizon)
// is a real branch so the common case does not pay for it.
__device__ __forceinline__ double ks_radius_nr(double a, double x, double y, double z, double &r2) {
    const double b = x * x + y * y + z * z - a * a, a2z2 = a * a * (z * z);
    const double s = sqrt_nr(fma(b, b, 4.0 * a2z2));
    if (b >= 0.0)
        r2 = 0.5 * (b + s);
    else
        r2 = div_nr(2.0 * a2z2, s - b);
    return sqrt_nr(r2);
}
__device__ __forceinline__ double ks_radius_nr(double a, double x, double y, double z) {
    double r2;
    return ks_radius_nr(a, x, y, z, r2);
}
// The same root with sqrt_pos: NaN where the quartic's discriminant or r^2
// is exactly 0 (the ring r = 0, z = 0 and, for a = 0, the centre); the
// area density below treats NaN as inside r_exc.
__device__ __forceinline__ double ks_radius_pos(double a, double x, double y, double z, double &r2) {
    const double b = x * x + y * y + z * z - a * a, a2z2 = a * a * (z * z);
    const double s = sqrt_pos(fma(b, b, 4.0 * a2z2));
    if (b >= 0.0)
        r2 = 0.5 * (b + s);
    else
        r2 = div_nr(2.0 * a2z2, s - b);
    return sqrt_pos(r2);
}

// Area density of a K-face at a hole-relative point (m > 0):
// sqrt(g_II g_JJ - g_IJ^2) = sqrt(1 + f (1 - k_K^2)) (I, J the other two
// axes; k null, so k_1^2 + k_2^2 + k_3^2 = 1), 1 inside r < r_exc.  With
// f = 2 m r^3 / S4, S4 = r^4 + a^2 z^2, and
//   K = 2:    1 - k_K^2 = (r - z)(r + z) / r^2,
//   K = 0, 1: 1 - k_K^2 = (Dn - n)(Dn + n) / Dn^2, Dn = r^2 + a^2,
//             n = r x - a y (K = 0) or r y + a x (K = 1),
// the density is sqrt(N / den) = N / sqrt(N den) with f (1 - k_K^2) =
// num / den and N = den + num: one reciprocal square root, no quotient.
__device__ __forceinline__ double ks_area_density(double m, double a, double r_exc, int K, double x, double y,
                                                  double z) {
    double r2;
    const double r = ks_radius_pos(a, x, y, z, r2);
    if (!(r >= r_exc)) return 1.0;  // also the NaN of r = 0
    const double S4 = fma(r2, r2, a * a * (z * z)), m2r = 2.0 * m * r;
    double num, den;
    if (K == 2) {
        num = m2r * ((r - z) * (r + z));
        den = S4;
    } else {
        const double Dn = r2 + a * a;
        const double nK = K == 0 ? r * x - a * y : r * y + a * x;
        num = m2r * r2 * ((Dn - nK) * (Dn + nK));
        den = S4 * (Dn * Dn);
    }
    const double N = den + num;
    return N * rsqrt_nr(N * den);
}

// r < r_lim decided exactly as the correctly rounded radius decides it: the
// refined radius (a few ulps from it) settles every case farther than 1e-12
// relative from the limit, the correctly rounded one the rest.
__device__ __forceinline__ bool ks_radius_below(double a, double x, double y, double z, double r_lim) {
    const double r = ks_radius_nr(a, x, y, z);
    if (fabs(r - r_lim) > 1e-12 * r_lim) return r < r_lim;
    return ks_radius(a, x, y, z) < r_lim;
}

// Spatial volume density sqrt(det g_ij) = sqrt(1 + f) (|k| = 1 for the
// spatial part of the null k) at a hole-relative point (m > 0), 1 inside
// r < r_exc: with S4 = r^4 + a^2 z^2 and N = S4 + 2 m r^3 it is
// sqrt(N / S4) = N / sqrt(N S4).
__device__ __forceinline__ double ks_volume_density(double m, double a, double r_exc, double x, double y, double z) {
    double r2;
    const double r = ks_radius_nr(a, x, y, z, r2);
    if (r < r_exc) return 1.0;
    const double S4 = fma(r2, r2, a * a * (z * z));
    const double N = fma(2.0 * m * r, r2, S4);
    return N * rsqrt_nr(N * S4);
}

// f and the spatial part of k at a hole-relative point (m > 0, r > 0).
template <typename T>
struct KSPoint {
    T r, f, k0, k1, k2;
};

__device__ __forceinline__ void ks_point(double m, double a, double x, double y, double z,
                                         KSPoint<double> &o) {
    double r = ks_radius(a, x, y, z);
    double rr = r * r;
    double iden = 1.0 / (rr + a * a);
    double S4 = rr * rr + a * a * z * z;
    o.r = r;
    o.f = 2.0 * m * r * rr / S4;
    o.k0 = (r * x - a * y) * iden;
    o.k1 = (r * y + a * x) * iden;
    o.k2 = z / r;
}

// Inverse metric components g^{ab} = eta^{ab} - f k^a k^b (packed symmetric
// 4x4, order 00 01 02 03 11 12 13 22 23 33) at a grid point; flat inside
// r_exc or when m = 0.
struct Sym4 {
    double v[10];
};

__host__ __device__ constexpr int sym4(int a, int b) {
    // index of (a,b) in the packed upper triangle
    return (a < b ? a : b) * 4 - ((a < b ? a : b) * ((a < b ? a : b) - 1)) / 2 + ((a < b ? b : a) - (a < b ? a : b));
}

// g_{ab} and g^{ab} at a grid point (node coordinates X, Y, Z).
__device__ inline void grid_metric(const Hole &h, double X, double Y, double Z, Sym4 &g, Sym4 &gi) {
    double x = X - h.cx, y = Y - h.cy, z = Z - h.cz;
    double k[4] = {0.0, 0.0, 0.0, 1.0};
    double f = 0.0;
    if (h.m != 0.0) {
        double r = ks_radius(h.a, x, y, z);
        if (!(r < h.r_exc)) {
            KSPoint<double> p;
            ks_point(h.m, h.a, x, y, z, p);
            f = p.f;
            k[0] = p.k0;
            k[1] = p.k1;
            k[2] = p.k2;
        }
    }
    const double eta[4] = {1.0, 1.0, 1.0, -1.0};
    const double ku[4] = {k[0], k[1], k[2], -1.0};
    for (int a = 0; a < 4; a++)
        for (int b = a; b < 4; b++) {
            int s = sym4(a, b);
            g.v[s] = (a == b ? eta[a] : 0.0) + f * k[a] * k[b];
            gi.v[s] = (a == b ? eta[a] : 0.0) - f * ku[a] * ku[b];
        }
}

__device__ __forceinline__ bool grid_excised(const Hole &h, double X, double Y, double Z) {
    if (h.m == 0.0) return false;
    return ks_radius(h.a, X - h.cx, Y - h.cy, Z - h.cz) < h.r_exc;
}

// Kerr-Schild point with the gradients the pusher needs, in type T, from a
// radius r already solved (in FP64):
//   d_i r = x_i r^3/(r^4+a^2 z^2) (x, y),  z r (r^2+a^2)/(r^4+a^2 z^2) (z);
//   d_i f = f (3 d_i r / r - d_i S4 / S4),  S4 = r^4 + a^2 z^2;
//   dk[j][i] = d_i k_j.
template <typename T>
struct KSGradT {
    T r, f, k[3];
    T df[3];
    T dk[3][3];
};
using KSGrad = KSGradT<double>;

template <typename T>
__device__ __forceinline__ void ks_grad_r(T m, T a, T x, T y, T z, T r, KSGradT<T> &o) {
    const T one = (T)1;
    T rr = r * r;
    T a2 = a * a;
    T S4 = rr * rr + a2 * z * z;
    T iS4 = recip<T>(S4);
    T iden = recip<T>(rr + a2);
    T ir = recip<T>(r);
    T f = (T)2 * m * r * rr * iS4;
    T k0 = (r * x - a * y) * iden;
    T k1 = (r * y + a * x) * iden;
    T k2 = z * ir;
    T c = r * rr * iS4;
    T dr[3] = {x * c, y * c, z * r * (rr + a2) * iS4};
    T f3r = (T)3 * f * ir;
    T f4 = (T)4 * f * rr * r * iS4;
    for (int i = 0; i < 3; i++) o.df[i] = (f3r - f4) * dr[i];
    o.df[2] -= f * (T)2 * a2 * z * iS4;
    T two_r = (T)2 * r;
    for (int i = 0; i < 3; i++) {
        T dd = two_r * dr[i];
        o.dk[0][i] = (dr[i] * x - k0 * dd) * iden;
        o.dk[1][i] = (dr[i] * y - k1 * dd) * iden;
        o.dk[2][i] = -k2 * dr[i] * ir;
    }
    o.dk[0][0] += r * iden;
    o.dk[0][1] -= a * iden;
    o.dk[1][1] += r * iden;
    o.dk[1][0] += a * iden;
    o.dk[2][2] += ir;
    o.r = r;
    o.f = f;
    o.k[0] = k0;
    o.k[1] = k1;
    o.k[2] = k2;
}

__device__ __forceinline__ void ks_grad(double m, double a, double x, double y, double z, KSGrad &o) {
    ks_grad_r<double>(m, a, x, y, z, ks_radius_nr(a, x, y, z), o);
}

// G^a = Gamma^a_{mn} u^m u^n for g = eta + f k k (stationary, k_4 = 1):
//   G_b = s (Df k_b + f Dk_b) + f q k_b - s^2/2 d_b f - f s w_b   (b spatial)
//   G_4 = s Df + f q
// with s = k.u, D = u^i d_i, Dk_j = u^i d_i k_j, q = u^j Dk_j,
// w_b = u^j d_b k_j, then G^a = g^{ab} G_b = eta^{ab} G_b - f k^a (k^b G_b).
template <typename T>
__device__ __forceinline__ void gamma_uu(const KSGradT<T> &p, const T u[4], T G[4]) {
    const T f = p.f;
    T s = p.k[0] * u[0] + p.k[1] * u[1] + p.k[2] * u[2] + u[3];
    T Df = p.df[0] * u[0] + p.df[1] * u[1] + p.df[2] * u[2];
    T Dk[3], w[3];
    for (int j = 0; j < 3; j++) Dk[j] = p.dk[j][0] * u[0] + p.dk[j][1] * u[1] + p.dk[j][2] * u[2];
    for (int b = 0; b < 3; b++) w[b] = p.dk[0][b] * u[0] + p.dk[1][b] * u[1] + p.dk[2][b] * u[2];
    T q = Dk[0] * u[0] + Dk[1] * u[1] + Dk[2] * u[2];
    T Gl[4];
    T hs2 = (T)0.5 * s * s;
    T fs = f * s;
    T sDf_fq = s * Df + f * q;
    for (int b = 0; b < 3; b++) Gl[b] = sDf_fq * p.k[b] + fs * Dk[b] - hs2 * p.df[b] - fs * w[b];
    Gl[3] = sDf_fq;
    T kG = p.k[0] * Gl[0] + p.k[1] * Gl[1] + p.k[2] * Gl[2] - Gl[3];
    T fkG = f * kG;
    G[0] = Gl[0] - fkG * p.k[0];
    G[1] = Gl[1] - fkG * p.k[1];
    G[2] = Gl[2] - fkG * p.k[2];
    G[3] = -Gl[3] + fkG;
}

// l / d for 0 <= l < 2^20 and d >= 1 through a float reciprocal inv_d of d
// accurate to one ulp (the hardware estimate): (l + 1/2)/d lies at least
// 1/(2d) from an integer while the float roundings move it by less than
// (l + 1/2)/d * 2^-22, so the truncation is the exact quotient.
__device__ __forceinline__ int small_div(int l, float inv_d) { return (int)(((float)l + 0.5f) * inv_d); }

// Round-to-nearest-even int64 of v for |v| < 2^51: v + 1.5 * 2^52 lies in
// [2^52, 2^53), where the ulp is 1, so the addition rounds v to an integer
// and the difference of the bit patterns is that integer (3 instructions
// instead of the general conversion sequence).  Current and charge
// contributions are below 2^(fp_bits + 1) with fp_bits <= 50.
__device__ __forceinline__ long long fixed_rn(double v) {
    const double magic = 6755399441055744.0;  // 1.5 * 2^52
    return __double_as_longlong(v + magic) - __double_as_longlong(magic);
}

}  // namespace grpic
