// Device building blocks shared by the expansion, power-spectrum and
// adjoint kernels: cutoff, radial spline, and real spherical harmonics with
// their Cartesian gradients.
//
// Harmonics (Sec. 4.E).  For a unit vector u = (x, y, z) the real harmonic
// of degree l and order m is a polynomial Z_lm(u) = K_lm Qt_l^|m|(u) T_m(x, y)
// with T_m = Re (x + i y)^m for m >= 0 and Im (x + i y)^|m| for m < 0, and
// Qt_l^m the associated Legendre polynomial without its sin^m factor,
// written as a solid (homogeneous) polynomial.  Qt obeys
//   Qt_m^m = (2m-1)!!,  Qt_{m+1}^m = (2m+1) z Qt_m^m,
//   (l-m) Qt_l^m = (2l-1) z Qt_{l-1}^m - (l+m-1) r^2 Qt_{l-2}^m,
// and its derivatives close on the same table:
//   d/dx Qt_l^m = -x Qt_{l-1}^{m+1},  d/dy Qt_l^m = -y Qt_{l-1}^{m+1},
//   d/dz Qt_l^m = (l+m) Qt_{l-1}^m,
// while d/dx Re/Im (x+iy)^m = m Re/Im (x+iy)^{m-1}, d/dy Re = -m Im(m-1),
// d/dy Im = m Re(m-1).  The gradient of Y_lm(r^) with respect to the pair
// vector of length r is (grad Z_lm(u) - l Y_lm u) / r (Euler's identity for
// a degree-l homogeneous polynomial removes the radial part).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace soap {
namespace dev {

constexpr double kPi = 3.141592653589793238462643383279502884;

__device__ __forceinline__ void sin_cos_pi(float x, float& s, float& c) { sincospif(x, &s, &c); }
__device__ __forceinline__ void sin_cos_pi(double x, double& s, double& c) { sincospi(x, &s, &c); }

template <typename T>
__device__ __forceinline__ T fcut(T r, T rcut, T width, T& df)
{
    if (r >= rcut) { df = T(0); return T(0); }
    T r0 = rcut - width;
    if (r <= r0) { df = T(0); return T(1); }
    // sin and cos of pi x for x in (0, 1): no large-argument reduction
    T x = (r - r0) / width, s, c;
    sin_cos_pi(x, s, c);
    df = T(-0.5) * s * T(kPi) / width;
    return T(0.5) * (T(1) + c);
}

// Index of (l, m >= 0) in the lower-triangular Qt table.
__host__ __device__ __forceinline__ int qidx(int l, int m) { return l * (l + 1) / 2 + m; }

// Degree of a packed lm index: l = floor(sqrt(lm)).
__host__ __device__ __forceinline__ int l_of(int lm)
{
    int l = int(sqrtf(float(lm)));
    while (l * l > lm) --l;
    while ((l + 1) * (l + 1) <= lm) ++l;
    return l;
}

// Column m of the Qt table (l = m..lmax) at the unit vector with z
// component z, and T_m = (x + i y)^m, written into the per-pair arrays.
template <typename T>
__device__ __forceinline__ void q_column(int m, int lmax, T x, T y, T z, T* qt, T* cre, T* cim)
{
    T q_mm = T(1);
    for (int k = 1; k <= m; ++k) q_mm *= T(2 * k - 1);
    qt[qidx(m, m)] = q_mm;
    if (m + 1 <= lmax) {
        T q1 = T(2 * m + 1) * z * q_mm;
        qt[qidx(m + 1, m)] = q1;
        T q2 = q_mm;
        for (int l = m + 2; l <= lmax; ++l) {
            T q = (T(2 * l - 1) * z * q1 - T(l + m - 1) * q2) / T(l - m);
            qt[qidx(l, m)] = q;
            q2 = q1;
            q1 = q;
        }
    }
    T re = T(1), im = T(0);
    for (int k = 0; k < m; ++k) {
        T nre = re * x - im * y;
        im = re * y + im * x;
        re = nre;
    }
    cre[m] = re;
    cim[m] = im;
}

// Y_lm and d Y_lm / d r_ji (3 components) of one pair, from its Qt table and
// (x+iy)^m values; l is the degree of lm, K its normalisation, u the unit
// vector and rinv = 1/r.
template <typename T>
__device__ __forceinline__ void ylm_and_grad(int lm, int l, T K, const T* qt, const T* cre, const T* cim, T ux, T uy,
                                             T uz, T rinv, T& Y, T& gx, T& gy, T& gz)
{
    int m = lm - l * l - l;
    int am = m < 0 ? -m : m;
    T Q = qt[qidx(l, am)];
    T Qa = (l >= 1 && am <= l - 1) ? qt[qidx(l - 1, am)] : T(0);          // Qt_{l-1}^m
    T Qb = (l >= 1 && am + 1 <= l - 1) ? qt[qidx(l - 1, am + 1)] : T(0);  // Qt_{l-1}^{m+1}
    T Tm, Tx, Ty;
    if (m > 0) {
        Tm = cre[am];
        Tx = T(am) * cre[am - 1];
        Ty = -T(am) * cim[am - 1];
    } else if (m < 0) {
        Tm = cim[am];
        Tx = T(am) * cim[am - 1];
        Ty = T(am) * cre[am - 1];
    } else {
        Tm = T(1);
        Tx = T(0);
        Ty = T(0);
    }
    T Z = K * Q * Tm;
    T zx = K * (-ux * Qb * Tm + Q * Tx);
    T zy = K * (-uy * Qb * Tm + Q * Ty);
    T zz = K * T(l + am) * Qa * Tm;
    Y = Z;
    T lz = T(l) * Z;
    gx = (zx - lz * ux) * rinv;
    gy = (zy - lz * uy) * rinv;
    gz = (zz - lz * uz) * rinv;
}

// Interval k of the radial spline that holds r and the local coordinate
// t = r / delta - k in [0, 1] (clamped to the table).
template <typename T>
__device__ __forceinline__ void spline_locate(int64_t M, T inv_delta, T r, int64_t& k, T& t)
{
    T x = r * inv_delta;
    T xmax = T(M) - T(0.5);
    k = int64_t(x < xmax ? x : xmax);
    if (k < 0) k = 0;
    if (k > M - 1) k = M - 1;
    t = x - T(k);
}

// Value and r-derivative of the interval's cubic a0 + t (a1 + t (a2 + t a3)).
template <typename T>
__device__ __forceinline__ void spline_poly(T a0, T a1, T a2, T a3, T t, T inv_delta, T& v, T& dv)
{
    v = a0 + t * (a1 + t * (a2 + t * a3));
    dv = (a1 + t * (T(2) * a2 + T(3) * t * a3)) * inv_delta;
}

// Splined orthogonalised radial integral and its r-derivative for one
// (n, l) channel j (table [M][nl][4]).
template <typename T>
__device__ __forceinline__ void spline_eval(const T* coef, int64_t M, T inv_delta, int nl, int j, T r, T& v, T& dv)
{
    int64_t k;
    T t;
    spline_locate<T>(M, inv_delta, r, k, t);
    const T* cf = coef + (k * nl + j) * 4;
    spline_poly<T>(cf[0], cf[1], cf[2], cf[3], t, inv_delta, v, dv);
}

// Packed upper-triangle index -> (k1, k2), k1 <= k2 < K.
__device__ __forceinline__ void tri_decode(int K, int kk, int& k1, int& k2)
{
    // start(k) = k K - k (k-1) / 2
    float b = float(2 * K + 1);
    int r = int((b - sqrtf(b * b - 8.0f * float(kk))) * 0.5f);
    if (r < 0) r = 0;
    if (r > K - 1) r = K - 1;
    while (r > 0 && r * K - r * (r - 1) / 2 > kk) --r;
    while (r + 1 < K && (r + 1) * K - (r + 1) * r / 2 <= kk) ++r;
    k1 = r;
    k2 = kk - (r * K - r * (r - 1) / 2) + r;
}

}  // namespace dev
}  // namespace soap
