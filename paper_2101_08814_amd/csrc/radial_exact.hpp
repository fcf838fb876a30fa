// Radial integrals of a Gaussian atom density evaluated directly (no
// spline), host and device.
//
// GTO basis (Sec. 4.B Eq. rad-int-gto-1, App. A): per n the restricted
// function G(a, b, r) = Gamma(a)/Gamma(b) exp(-c r^2) 1F1(a; b; alpha r^2),
// alpha = c^2/(c + d_n), is summed directly at the two largest l (power
// series below a switch point, the large-z asymptotic expansion above it)
// together with H = G(a+1, b+1); the two-step downward recurrence of App. A
// gives every smaller l, and dG/dr = 2 alpha r H - 2 c r G.  Then
// I_nl = pref_nl r^l G and the orthogonalisation I~ = S^{-1/2} I (Sec. 4.B).
//
// DVR basis (Sec. 4.C Eq. rad-int-dvr, with the factor 4 pi exp(-c r^2) of
// Eq. radial-integral-gaussian-density): on the Gauss-Legendre points x_n of
// [0, rcut + 3 sigma] with weights w_n,
//   I_nl(r) = 4 pi x_n sqrt(w_n) exp(-c (x_n - r)^2) e^{-z} i_l(z),
//   z = 2 c x_n r,
// with the scaled modified spherical Bessel functions e^{-z} i_l(z) from
// their power series for small z and from the closed forms of l = 0, 1 and
// the upward recurrence i_{l+1} = i_{l-1} - (2l+1)/z i_l (stable for l
// below z) above.
//
// Templates in the degree lmax keep every per-lane array in registers on
// the device; the host instantiates the same code.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace soap {
namespace rad {

constexpr double kPi = 3.141592653589793238462643383279502884;

// ------------------------------------------------------------ 1F1 pieces
// 1F1(a; b; z) by its power series (a, b, z > 0: positive terms)
__host__ __device__ inline double hyp1f1_series(double a, double b, double z)
{
    double term = 1.0, sum = 1.0;
    for (int s = 1; s < 100000; ++s) {
        term *= (a + s - 1) * z / ((b + s - 1) * s);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// sum_s (b-a)_s (1-a)_s / s! z^-s of the large-z expansion, stopped at the
// smallest term
__host__ __device__ inline double hyp1f1_asym_sum(double a, double b, double z)
{
    double term = 1.0, sum = 1.0, prev = 1e300;
    for (int s = 1; s < 1000; ++s) {
        term *= (b - a + s - 1) * (1.0 - a + s - 1) / (s * z);
        if (fabs(term) >= prev || term == 0.0) break;
        sum += term;
        prev = fabs(term);
        if (prev < 1e-17 * fabs(sum)) break;
    }
    return sum;
}

// Parameters of one restricted function G(a, b, .): lgr = log Gamma(a) -
// log Gamma(b), zswitch = switch point between series and asymptotic forms.
struct GParams {
    double a, b, lgr, zswitch;
};

__host__ __device__ inline double g_value(const GParams& g, double c, double alpha, double r)
{
    const double z = alpha * r * r;
    if (z < g.zswitch) return exp(g.lgr - c * r * r) * hyp1f1_series(g.a, g.b, z);
    // the Gamma ratio of the asymptotic form cancels the one in G
    return exp(z - c * r * r + (g.a - g.b) * log(z)) * hyp1f1_asym_sum(g.a, g.b, z);
}

// Per-calculator constants of the direct GTO evaluation (host or device
// arrays): alpha [nmax]; pref [nmax][lmax+1] = pi^{3/2} N_n c^l (c+d_n)^{-a};
// top [nmax][4]: G at lmax, H at lmax, G at lmax-1, H at lmax-1;
// X [nmax][nmax] = S^{-1/2}.
struct GtoTables {
    int nmax;
    double c;
    const double* alpha;
    const double* pref;
    const GParams* top;
    const double* X;
};

// Raw GTO integrals of one n for every l = 0..LMAX (and d/dr).
template <int LMAX>
__host__ __device__ inline void gto_raw_n(const GtoTables& t, int n, double r, double* I, double* dI)
{
    constexpr int LM1 = LMAX + 1;
    double G[LM1 + 2], H[LM1 + 2];
    const double alpha = t.alpha[n], c = t.c, z = alpha * r * r;
    const GParams* top = t.top + 4 * n;
    G[LMAX] = g_value(top[0], c, alpha, r);
    H[LMAX] = g_value(top[1], c, alpha, r);
    if (LMAX >= 1) {
        G[LMAX - 1] = g_value(top[2], c, alpha, r);
        H[LMAX - 1] = g_value(top[3], c, alpha, r);
    }
    // two-step downward recurrence (App. A Eq. 1f1-recurrence)
#pragma unroll
    for (int l = LMAX - 2; l >= 0; --l) {
        const double a = 0.5 * (n + l + 3), b = l + 1.5;
        H[l] = z * H[l + 2] + (b + 1) * G[l + 2];
        G[l] = z * (a - b) / a * G[l + 2] + (b / a) * H[l];
    }
    double rl = 1.0, rl1 = 0.0;   // r^l and l r^(l-1)
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) {
        const double P = t.pref[n * LM1 + l];
        I[l] = P * rl * G[l];
        const double dG = 2.0 * alpha * r * H[l] - 2.0 * c * r * G[l];
        dI[l] = P * (rl1 * G[l] + rl * dG);
        rl1 = (l + 1) * rl;
        rl *= r;
    }
}

// ---------------------------------------------------------------- DVR
// e^{-z} i_l(z) and d/dz [e^{-z} i_l(z)] for l = 0..LMAX, z >= 0
template <int LMAX>
__host__ __device__ inline void scaled_bessel_i(double z, double* s, double* ds)
{
    constexpr double kSeriesBelow = 2.0 * LMAX + 16.0;
    if (z < kSeriesBelow) {
        const double ez = exp(-z);
        double lead = 1.0;   // z^l / (2l+1)!!
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
            double term = lead, sum = 0.0, dsum = 0.0;
            for (int k = 0; k < 400; ++k) {
                sum += term;
                dsum += term * (l + 2 * k);   // times z^-1 below
                const double nt = term * z * z / (2.0 * (k + 1) * (2 * l + 2 * k + 3));
                if (nt < 1e-17 * sum || nt == 0.0) break;
                term = nt;
            }
            const double di = z > 0.0 ? dsum / z : (l == 1 ? 1.0 / 3.0 : 0.0);
            s[l] = ez * sum;
            ds[l] = ez * (di - sum);
            lead *= z / (2 * l + 3);
        }
        return;
    }
    const double e2 = exp(-2.0 * z), iz = 1.0 / z;
    s[0] = 0.5 * (1.0 - e2) * iz;
    if (LMAX >= 1) s[1] = (0.5 * (1.0 + e2) - s[0]) * iz;
#pragma unroll
    for (int l = 1; l < LMAX; ++l) s[l + 1] = s[l - 1] - (2 * l + 1) * iz * s[l];
    // d/dz e^{-z} i_l = e^{-z} (i_l' - i_l); i_0' = i_1, i_l' = i_{l-1} - (l+1)/z i_l
    const double s1 = LMAX >= 1 ? s[1] : (0.5 * (1.0 + e2) - s[0]) * iz;
    ds[0] = s1 - s[0];
#pragma unroll
    for (int l = 1; l <= LMAX; ++l) ds[l] = s[l - 1] - (l + 1) * iz * s[l] - s[l];
}

// Constants of the direct DVR evaluation: points x [nmax] and amplitudes
// A [nmax] = 4 pi x_n sqrt(w_n).
struct DvrTables {
    int nmax;
    double c;
    const double* x;
    const double* A;
};

template <int LMAX>
__host__ __device__ inline void dvr_n(const DvrTables& t, int n, double r, double* I, double* dI)
{
    double s[LMAX + 1], ds[LMAX + 1];
    const double x = t.x[n], c = t.c, z = 2.0 * c * x * r;
    scaled_bessel_i<LMAX>(z, s, ds);
    const double g = t.A[n] * exp(-c * (x - r) * (x - r));
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) {
        I[l] = g * s[l];
        dI[l] = g * (-2.0 * c * (r - x) * s[l] + 2.0 * c * x * ds[l]);
    }
}

}  // namespace rad
}  // namespace soap
