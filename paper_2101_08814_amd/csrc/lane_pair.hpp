// Per-lane evaluation of one pair, fully unrolled in the degree lmax.
//
// The kernels built on this header give each lane a whole pair: its
// geometry, cutoff, splined radial integrals and real harmonics are formed in
// registers with every index a compile-time constant, so no lane decodes a
// packed index or divides by a run-time extent (the per-item index work of
// the LDS-staged kernels is what bounded them).
//
// Harmonics (Sec. 4.E) come out degree by degree: YlmStream::degree<L>()
// produces Y_lm, m = -L..L, and the gradient of the solid polynomial
// Z_lm(u) = K_lm Qt_L^|m|(u) T_m(x, y) from the Qt columns of degrees L-1
// and L-2 (the same recurrence and derivative identities as sph.hpp, with the
// coefficients (2L-1)/(L-m) and (L+m-1)/(L-m) folded into constants).  The
// gradient of Y_lm(r^) with respect to the pair vector is
// (grad Z_lm - L Y_lm u) / r.
//
// The radial table read here is the interval-major, degree-major copy
// [M][lmax+1][nmax] of float4/double4 local cubics, so the nmax coefficients
// of one (interval, l) are contiguous.
#pragma once

#include <type_traits>

#include "chunk.hpp"

namespace soap {
namespace dev {

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// (2m-1)!! = 1 * 3 * ... * (2m-1), 1 for m = 0
constexpr double odd_factorial(int m)
{
    double v = 1.0;
    for (int k = 1; k <= m; ++k) v *= double(2 * k - 1);
    return v;
}

// Normalisation K_lm of the real harmonics,
// sqrt((2 - delta_m0) (2l+1)/(4 pi) (l-|m|)!/(l+|m|)!), as compile-time
// constants for lm = l^2 + l + m < 169.
constexpr double ce_sqrt(double x)
{
    if (!(x > 0.0)) return 0.0;
    double r = x > 1.0 ? x : 1.0;
    for (int k = 0; k < 200; ++k) r = 0.5 * (r + x / r);
    return r;
}

struct HarmonicNorms {
    double v[169];
    constexpr HarmonicNorms() : v()
    {
        for (int l = 0; l <= 12; ++l)
            for (int m = -l; m <= l; ++m) {
                const int am = m < 0 ? -m : m;
                double ratio = 1.0;   // (l-|m|)! / (l+|m|)!
                for (int k = l - am + 1; k <= l + am; ++k) ratio /= double(k);
                v[l * l + l + m] = ce_sqrt((am == 0 ? 1.0 : 2.0) * (2 * l + 1) / (4.0 * kPi) * ratio);
            }
    }
};
constexpr HarmonicNorms kHarmonicNorms{};

// Gradient of the solid harmonic Z_lm in terms of the harmonics of degree
// l - 1.  With F_l^M = Qt_l^M (x + i y)^M (M >= 0) the raising and lowering
// identities
//   (d_x + i d_y) F_l^M = -F_{l-1}^{M+1},
//   (d_x - i d_y) F_l^M = (l+M)(l+M-1) F_{l-1}^{M-1}   (M >= 1),
//   d_z F_l^M = (l+M) F_{l-1}^M
// (the first from d_{x,y} Qt_l^M = -{x, y} Qt_{l-1}^{M+1}, the others from the
// Legendre recurrences) give, for Z_lm = K_lm Re F_l^M (m > 0), K_lm Im F_l^M
// (m < 0) or K_l0 F_l^0, each component as at most two harmonics Y_{l-1,m'}
// (= Z_{l-1,m'} at a unit vector).  Term j of component x of lm is
// gx[lm][j] * Y[ix[lm][j]]; absent terms have coefficient 0 and index 0.
struct HarmonicGradTerms {
    int ix[169][2], iy[169][2], iz[169];
    double gx[169][2], gy[169][2], gz[169];

    // Re F_{l}^{M} and Im F_{l}^{M} as (index of Y_{l,m'}, factor 1/K_{l,m'})
    static constexpr void re_f(int l, int M, int& idx, double& s)
    {
        idx = 0;
        s = 0.0;
        if (l < 0 || M > l) return;
        idx = l * l + l + M;
        s = 1.0 / kHarmonicNorms.v[idx];
    }
    static constexpr void im_f(int l, int M, int& idx, double& s)
    {
        idx = 0;
        s = 0.0;
        if (l < 0 || M < 1 || M > l) return;
        idx = l * l + l - M;
        s = 1.0 / kHarmonicNorms.v[idx];
    }

    constexpr HarmonicGradTerms() : ix(), iy(), iz(), gx(), gy(), gz()
    {
        for (int l = 1; l <= 12; ++l)
            for (int m = -l; m <= l; ++m) {
                const int lm = l * l + l + m, M = m < 0 ? -m : m;
                const double K = kHarmonicNorms.v[lm];
                const double beta = double(l + M) * double(l + M - 1);
                int a = 0, b = 0, c = 0;
                double sa = 0.0, sb = 0.0, sc = 0.0;
                if (m > 0) {
                    re_f(l - 1, M + 1, a, sa);
                    re_f(l - 1, M - 1, b, sb);
                    ix[lm][0] = a; gx[lm][0] = -0.5 * K * sa;
                    ix[lm][1] = b; gx[lm][1] = 0.5 * K * beta * sb;
                    im_f(l - 1, M + 1, a, sa);
                    im_f(l - 1, M - 1, b, sb);
                    iy[lm][0] = a; gy[lm][0] = -0.5 * K * sa;
                    iy[lm][1] = b; gy[lm][1] = -0.5 * K * beta * sb;
                    re_f(l - 1, M, c, sc);
                } else if (m < 0) {
                    im_f(l - 1, M + 1, a, sa);
                    im_f(l - 1, M - 1, b, sb);
                    ix[lm][0] = a; gx[lm][0] = -0.5 * K * sa;
                    ix[lm][1] = b; gx[lm][1] = 0.5 * K * beta * sb;
                    re_f(l - 1, M + 1, a, sa);
                    re_f(l - 1, M - 1, b, sb);
                    iy[lm][0] = a; gy[lm][0] = 0.5 * K * sa;
                    iy[lm][1] = b; gy[lm][1] = 0.5 * K * beta * sb;
                    im_f(l - 1, M, c, sc);
                } else {
                    re_f(l - 1, 1, a, sa);
                    ix[lm][0] = a; gx[lm][0] = -K * sa;
                    im_f(l - 1, 1, a, sa);
                    iy[lm][0] = a; gy[lm][0] = -K * sa;
                    re_f(l - 1, 0, c, sc);
                }
                iz[lm] = c;
                gz[lm] = K * double(l + M) * sc;
            }
    }
};
constexpr HarmonicGradTerms kHarmonicGrad{};

template <typename T, int LMAX>
struct YlmStream {
    T x, y, z;
    T cr[LMAX + 1], ci[LMAX + 1];   // Re and Im of (x + i y)^m
    T q1[LMAX + 2], q2[LMAX + 2];   // Qt_{L-1}^m and Qt_{L-2}^m

    __device__ __forceinline__ YlmStream(T ux, T uy, T uz) : x(ux), y(uy), z(uz)
    {
        cr[0] = T(1);
        ci[0] = T(0);
#pragma unroll
        for (int m = 1; m <= LMAX; ++m) {
            cr[m] = cr[m - 1] * x - ci[m - 1] * y;
            ci[m] = cr[m - 1] * y + ci[m - 1] * x;
        }
#pragma unroll
        for (int m = 0; m < LMAX + 2; ++m) q1[m] = q2[m] = T(0);
    }

    // Degree L; call for L = 0, 1, ..., LMAX in turn.  f(mi, Y, zx, zy, zz)
    // for mi = m + L = 0..2L: Y = Y_{L,m}(u) and, with GRAD, z = grad Z_{L,m}
    // at u (zero otherwise).
    template <int L, bool GRAD, typename F>
    __device__ __forceinline__ void degree(F&& f)
    {
        T q[L + 1];
#pragma unroll
        for (int m = 0; m <= L; ++m) {
            if (m == L) q[m] = T(odd_factorial(L));
            else if (m == L - 1) q[m] = T(2 * m + 1) * z * q1[m];
            else
                q[m] = T(double(2 * L - 1) / double(L - m)) * z * q1[m] -
                       T(double(L + m - 1) / double(L - m)) * q2[m];
        }
#pragma unroll
        for (int mi = 0; mi <= 2 * L; ++mi) {
            const int m = mi - L;
            const int am = m < 0 ? -m : m;
            const T K = T(kHarmonicNorms.v[L * L + mi]);
            T Tm, Tx = T(0), Ty = T(0);
            if (m > 0) {
                Tm = cr[am];
                if (GRAD) { Tx = T(am) * cr[am - 1]; Ty = -T(am) * ci[am - 1]; }
            } else if (m < 0) {
                Tm = ci[am];
                if (GRAD) { Tx = T(am) * ci[am - 1]; Ty = T(am) * cr[am - 1]; }
            } else {
                Tm = T(1);
            }
            const T KQ = K * q[am];
            const T Y = KQ * Tm;
            if constexpr (GRAD) {
                const T Qa = am <= L - 1 ? q1[am] : T(0);       // Qt_{L-1}^|m|
                const T Qb = am + 1 <= L - 1 ? q1[am + 1] : T(0); // Qt_{L-1}^{|m|+1}
                const T KQbT = K * Qb * Tm;
                f(mi, Y, KQ * Tx - x * KQbT, KQ * Ty - y * KQbT, K * T(L + am) * Qa * Tm);
            } else {
                f(mi, Y, T(0), T(0), T(0));
            }
        }
#pragma unroll
        for (int m = 0; m <= L; ++m) {
            q2[m] = q1[m];
            q1[m] = q[m];
        }
    }
};

// Geometry of one pair: unit vector, 1/r, cutoff and its derivative, the
// spline interval and local coordinate; a status on coincident atoms.
template <typename T>
struct PairGeom {
    T ux, uy, uz, r, rinv, f, df, t;
    int k;
};

template <typename T>
__device__ __forceinline__ PairGeom<T> pair_geometry(const FeatureArgs& a, T vx, T vy, T vz)
{
    PairGeom<T> g;
    g.r = sqrt(vx * vx + vy * vy + vz * vz);
    g.f = T(0);
    g.df = T(0);
    if (!(g.r > T(1e-8))) {
        put_status(a.status, SOAP_EGEOMETRY);
        g.ux = T(0); g.uy = T(0); g.uz = T(1); g.rinv = T(0);
    } else {
        g.rinv = T(1) / g.r;
        g.ux = vx * g.rinv; g.uy = vy * g.rinv; g.uz = vz * g.rinv;
        g.f = fcut<T>(g.r, T(a.rcut), T(a.width), g.df);
    }
    const T xs = g.r * T(a.inv_delta);
    const T xmax = T(a.M) - T(0.5);
    int k = int(xs < xmax ? xs : xmax);
    k = k < 0 ? 0 : (k > int(a.M) - 1 ? int(a.M) - 1 : k);
    g.k = k;
    g.t = xs - T(k);
    return g;
}

// Species of the neighbour of pair q, checked (an invalid j stores
// SOAP_EINVAL, an invalid species SOAP_ESPECIES; both count as species 0).
__device__ __forceinline__ int pair_species(const FeatureArgs& a, int64_t q)
{
    const int j = a.pair_j[q];
    if (j < 0 || j >= a.n_atoms) {
        put_status(a.status, SOAP_EINVAL);
        return 0;
    }
    const int sp = a.species[j];
    if (sp < 0 || sp >= a.S) {
        put_status(a.status, SOAP_ESPECIES);
        return 0;
    }
    return sp;
}

// lmax as a template parameter for both float and double
template <typename T, template <typename, int> class Fn, typename... Args>
hipError_t by_degree(int lmax, Args&&... args)
{
    switch (lmax) {
    case 0: return Fn<T, 0>::run(args...);
    case 1: return Fn<T, 1>::run(args...);
    case 2: return Fn<T, 2>::run(args...);
    case 3: return Fn<T, 3>::run(args...);
    case 4: return Fn<T, 4>::run(args...);
    case 5: return Fn<T, 5>::run(args...);
    case 6: return Fn<T, 6>::run(args...);
    case 7: return Fn<T, 7>::run(args...);
    case 8: return Fn<T, 8>::run(args...);
    case 9: return Fn<T, 9>::run(args...);
    case 10: return Fn<T, 10>::run(args...);
    case 11: return Fn<T, 11>::run(args...);
    case 12: return Fn<T, 12>::run(args...);
    default: return hipErrorNotSupported;
    }
}

}  // namespace dev
}  // namespace soap
