// Host-side FP64 construction of the radial spline tables.
//
// Sec. 4.B: GTO radial basis, analytic overlap, Loewdin orthogonalisation
//           S^{-1/2} (here: Householder tridiagonalisation followed by
//           shifted QR sweeps on the tridiagonal matrix).
// App. A:   the radial integral through the restricted function
//             G(a, b, r) = Gamma(a)/Gamma(b) exp(-c r^2) 1F1(a; b; alpha r^2),
//           alpha = c^2 / (c + d_n), evaluated directly only at the two
//           largest l of each n (power series below a switch point found by
//           bisection, the large-z asymptotic expansion above it) and by the
//           two-step downward recurrence in l for the rest; dG/dr from G at
//           (a+1, b+1).
// Sec. 4.C: DVR radial basis (radial_basis = 1): Gauss-Legendre points of
//           [0, rcut + 3 sigma] by the Golub-Welsch method (eigenvalues of the
//           Jacobi matrix of the Legendre recurrence), the radial integral in
//           the closed form of radial_exact.hpp; orthonormal, so no S^{-1/2}.
// Sec. 4.D: the orthogonalised radial integral tabulated on a uniform grid
//           over [0, rcut] and interpolated by a cubic spline (clamped with
//           the exact end derivatives).  The grid is doubled, from 1024
//           intervals, until the spline error at four interior points of
//           every interval is below the requested accuracy.  Each interval
//           is stored as the cubic a0 + t (a1 + t (a2 + t a3)) in the local
//           coordinate t = (r - r_k) / delta, the form the kernels evaluate.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "radial_exact.hpp"
#include "soap_internal.hpp"

namespace soap {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// ---------------------------------------------------------------- basis
struct Gto {
    std::vector<double> sigma, d, norm;
    explicit Gto(int nmax, double rcut) : sigma(nmax), d(nmax), norm(nmax)
    {
        for (int n = 0; n < nmax; ++n) {
            double s = rcut * std::max(std::sqrt(double(n)), 1.0) / nmax;
            sigma[n] = s;
            d[n] = 0.5 / (s * s);
            // N_n^2 = 2 / (sigma_n^(2n+3) Gamma(n + 3/2))
            norm[n] = std::exp(0.5 * (std::log(2.0) - (2.0 * n + 3.0) * std::log(s) - std::lgamma(n + 1.5)));
        }
    }
};

// S_nm = N_n N_m Gamma((n+m+3)/2) / (2 (d_n + d_m)^((n+m+3)/2))
std::vector<double> gto_overlap(const Gto& g, int nmax)
{
    std::vector<double> S(nmax * nmax);
    for (int n = 0; n < nmax; ++n)
        for (int m = 0; m < nmax; ++m) {
            double e = 0.5 * (n + m + 3);
            S[n * nmax + m] = g.norm[n] * g.norm[m] * std::exp(std::lgamma(e) - e * std::log(g.d[n] + g.d[m])) / 2.0;
        }
    return S;
}


// ------------------------------------------------------- restricted 1F1
// G(a, b, r) = Gamma(a)/Gamma(b) exp(-c r^2) 1F1(a; b; alpha r^2).
class GFunction {
public:
    GFunction(double a, double b, double c, double alpha) : a_(a), b_(b), c_(c), alpha_(alpha)
    {
        lgr_ = std::lgamma(a) - std::lgamma(b);
        // Switch point: smallest z (found by bisection) above which the
        // truncated asymptotic expansion agrees with the series to 1e-14.
        double lo = 0.0, hi = 690.0;
        if (!agree(hi)) {
            zswitch_ = hi;
        } else {
            for (int it = 0; it < 60; ++it) {
                double mid = 0.5 * (lo + hi);
                (agree(mid) ? hi : lo) = mid;
            }
            zswitch_ = hi;
        }
    }
    double zswitch() const { return zswitch_; }
    // series below the switch point, exp(z - c r^2) z^(a-b) sum_s
    // (b-a)_s (1-a)_s / s! z^-s above it (the Gamma ratio of the asymptotic
    // form cancels the one in G)
    rad::GParams params() const { return rad::GParams{a_, b_, lgr_, zswitch_}; }

private:
    double series(double z) const { return rad::hyp1f1_series(a_, b_, z); }
    double asym_sum(double z) const { return rad::hyp1f1_asym_sum(a_, b_, z); }
    bool agree(double z) const
    {
        if (z <= 0) return false;
        // compare e^{-z} 1F1 in both forms (Gamma(a)/Gamma(b) scaled out)
        double s = series(z) * std::exp(-z);
        double as = std::exp((a_ - b_) * std::log(z) - lgr_) * asym_sum(z);
        return std::fabs(as - s) <= 1e-14 * std::fabs(s);
    }
    double a_, b_, c_, alpha_, lgr_, zswitch_;
};

// lmax as a template parameter for the shared direct evaluation
template <typename F>
void with_degree(int lmax, F&& f)
{
    switch (lmax) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    case 11: f(std::integral_constant<int, 11>{}); break;
    default: f(std::integral_constant<int, 12>{}); break;
    }
}

}  // namespace

// Constants of the direct evaluation of either basis (also uploaded for the
// device's direct path).
void build_exact_radial(const soap_hypers& h, const std::vector<double>& orth, ExactRadial& e)
{
    const int nmax = h.nmax, lmax = h.lmax;
    e.basis = h.radial_basis;
    e.nmax = nmax;
    e.lmax = lmax;
    e.c = 0.5 / (h.sigma * h.sigma);
    if (h.radial_basis == 1) {
        // Golub-Welsch: the Gauss-Legendre points are the eigenvalues of the
        // symmetric Jacobi matrix with off-diagonal k / sqrt(4 k^2 - 1), the
        // weights 2 (first eigenvector component)^2
        std::vector<double> J(nmax * nmax, 0.0), w, Q;
        for (int k = 1; k < nmax; ++k) J[(k - 1) * nmax + k] = J[k * nmax + k - 1] = k / std::sqrt(4.0 * k * k - 1.0);
        sym_eigen(nmax, J, w, Q);
        std::vector<int> order(nmax);
        for (int i = 0; i < nmax; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return w[x] < w[y]; });
        const double bmax = h.rcut + 3.0 * h.sigma;
        e.x.resize(nmax);
        e.A.resize(nmax);
        for (int i = 0; i < nmax; ++i) {
            const int k = order[i];
            const double t = nmax == 1 ? 0.0 : w[k];
            const double wt = nmax == 1 ? 2.0 : 2.0 * Q[0 * nmax + k] * Q[0 * nmax + k];
            e.x[i] = 0.5 * bmax * (t + 1.0);
            const double wn = 0.5 * bmax * wt;
            e.A[i] = 4.0 * kPi * e.x[i] * std::sqrt(wn);
        }
        return;
    }
    Gto gto(nmax, h.rcut);
    e.alpha.resize(nmax);
    e.pref.resize(nmax * (lmax + 1));
    e.top.clear();
    for (int n = 0; n < nmax; ++n) {
        e.alpha[n] = e.c * e.c / (e.c + gto.d[n]);
        for (int l = 0; l <= lmax; ++l) {
            double a = 0.5 * (n + l + 3);
            // pi^{3/2} N_n c^l (c + d_n)^{-a}
            e.pref[n * (lmax + 1) + l] = std::pow(kPi, 1.5) * gto.norm[n] *
                                         std::exp(l * std::log(e.c) - a * std::log(e.c + gto.d[n]));
        }
        for (int L = lmax; L >= lmax - 1; --L) {
            if (L < 0) {   // lmax = 0: unused slots
                e.top.push_back(rad::GParams{1.0, 1.0, 0.0, 0.0});
                e.top.push_back(rad::GParams{1.0, 1.0, 0.0, 0.0});
                continue;
            }
            double a = 0.5 * (n + L + 3), b = L + 1.5;
            e.top.push_back(GFunction(a, b, e.c, e.alpha[n]).params());           // G(a, b)
            e.top.push_back(GFunction(a + 1, b + 1, e.c, e.alpha[n]).params());   // H = G(a+1, b+1)
        }
    }
    e.X = orth;
}

// I~_nl(r) and d/dr [nmax][lmax+1] (dI may be NULL)
void exact_radial_eval(const ExactRadial& e, double r, double* I, double* dI)
{
    const int nmax = e.nmax, lm1 = e.lmax + 1;
    std::vector<double> tI(lm1), tdI(lm1);
    if (e.basis == 1) {
        rad::DvrTables t{nmax, e.c, e.x.data(), e.A.data()};
        with_degree(e.lmax, [&](auto Lc) {
            constexpr int L = decltype(Lc)::value;
            for (int n = 0; n < nmax; ++n) {
                rad::dvr_n<L>(t, n, r, tI.data(), tdI.data());
                for (int l = 0; l < lm1; ++l) {
                    I[n * lm1 + l] = tI[l];
                    if (dI) dI[n * lm1 + l] = tdI[l];
                }
            }
        });
        return;
    }
    rad::GtoTables t{nmax, e.c, e.alpha.data(), e.pref.data(), e.top.data(), e.X.data()};
    std::vector<double> raw(nmax * lm1), draw(nmax * lm1);
    with_degree(e.lmax, [&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        for (int n = 0; n < nmax; ++n) rad::gto_raw_n<L>(t, n, r, &raw[n * lm1], &draw[n * lm1]);
    });
    for (int n = 0; n < nmax; ++n)
        for (int l = 0; l < lm1; ++l) {
            double s = 0.0, ds = 0.0;
            for (int m = 0; m < nmax; ++m) {
                s += e.X[n * nmax + m] * raw[m * lm1 + l];
                ds += e.X[n * nmax + m] * draw[m * lm1 + l];
            }
            I[n * lm1 + l] = s;
            if (dI) dI[n * lm1 + l] = ds;
        }
}

namespace {

// Clamped cubic spline through y_0..y_M on a uniform grid of step h; returns
// the second derivatives at the knots (tridiagonal solve).
std::vector<double> clamped_second_derivatives(const std::vector<double>& y, double h, double d0, double dM)
{
    size_t M = y.size() - 1;
    std::vector<double> diag(M + 1), rhs(M + 1), sub(M + 1), sup(M + 1);
    diag[0] = h / 3.0; sup[0] = h / 6.0;
    rhs[0] = (y[1] - y[0]) / h - d0;
    for (size_t k = 1; k < M; ++k) {
        sub[k] = h / 6.0; diag[k] = 2.0 * h / 3.0; sup[k] = h / 6.0;
        rhs[k] = (y[k + 1] - 2.0 * y[k] + y[k - 1]) / h;
    }
    sub[M] = h / 6.0; diag[M] = h / 3.0;
    rhs[M] = dM - (y[M] - y[M - 1]) / h;
    // Thomas algorithm
    for (size_t k = 1; k <= M; ++k) {
        double w = sub[k] / diag[k - 1];
        diag[k] -= w * sup[k - 1];
        rhs[k] -= w * rhs[k - 1];
    }
    std::vector<double> m2(M + 1);
    m2[M] = rhs[M] / diag[M];
    for (size_t k = M; k-- > 0;) m2[k] = (rhs[k] - sup[k] * m2[k + 1]) / diag[k];
    return m2;
}

}  // namespace

// Symmetric eigen-decomposition A = Q diag(w) Q^T of a small dense matrix.
// Householder reflections bring A to tridiagonal form; implicit QR sweeps
// with a Wilkinson shift (Golub & Van Loan, Sec. 8.3) diagonalise it.  The
// rotations are applied to the dense matrix (n is at most a few hundred
// here), which keeps the code short at O(n^3) cost.
void sym_eigen(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& Q)
{
    auto at = [n](std::vector<double>& M, int i, int j) -> double& { return M[i * n + j]; };
    Q.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
    // Householder: zero column k below the subdiagonal.
    for (int k = 0; k + 2 < n; ++k) {
        std::vector<double> v(n, 0.0);
        double norm = 0.0;
        for (int i = k + 1; i < n; ++i) { v[i] = at(A, i, k); norm += v[i] * v[i]; }
        norm = std::sqrt(norm);
        if (norm == 0.0) continue;
        double alpha = v[k + 1] > 0 ? -norm : norm;
        v[k + 1] -= alpha;
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
        if (vn == 0.0) continue;
        vn = std::sqrt(vn);
        for (int i = k + 1; i < n; ++i) v[i] /= vn;
        // A <- (I - 2vv^T) A (I - 2vv^T);  Q <- Q (I - 2vv^T)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int i = k + 1; i < n; ++i) s += v[i] * at(A, i, j);
            for (int i = k + 1; i < n; ++i) at(A, i, j) -= 2.0 * v[i] * s;
        }
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += at(A, i, j) * v[j];
            for (int j = k + 1; j < n; ++j) at(A, i, j) -= 2.0 * s * v[j];
        }
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += at(Q, i, j) * v[j];
            for (int j = k + 1; j < n; ++j) at(Q, i, j) -= 2.0 * s * v[j];
        }
    }
    // rotation in the (p, p+1) plane applied as A <- G A G^T, Q <- Q G^T
    auto rotate = [&](int p, double c, double s) {
        for (int j = 0; j < n; ++j) {
            double x = at(A, p, j), y = at(A, p + 1, j);
            at(A, p, j) = c * x + s * y;
            at(A, p + 1, j) = -s * x + c * y;
        }
        for (int i = 0; i < n; ++i) {
            double x = at(A, i, p), y = at(A, i, p + 1);
            at(A, i, p) = c * x + s * y;
            at(A, i, p + 1) = -s * x + c * y;
        }
        for (int i = 0; i < n; ++i) {
            double x = at(Q, i, p), y = at(Q, i, p + 1);
            at(Q, i, p) = c * x + s * y;
            at(Q, i, p + 1) = -s * x + c * y;
        }
    };
    const double eps = 2.220446049250313e-16;
    // A subdiagonal entry is negligible next to its two diagonal neighbours
    // or next to the whole matrix: the second test deflates blocks of
    // (near-)zero eigenvalues, whose neighbours are themselves rounding
    // noise, at a backward error of eps |A|.
    double anorm = 0.0;
    for (int i = 0; i < n; ++i) {
        anorm += at(A, i, i) * at(A, i, i);
        if (i + 1 < n) anorm += 2.0 * at(A, i + 1, i) * at(A, i + 1, i);
    }
    anorm = std::sqrt(anorm);
    int hi = n - 1;
    for (int iter = 0; hi > 0 && iter < 100 * n; ++iter) {
        // deflate negligible subdiagonal entries
        for (int i = 0; i < hi; ++i)
            if (std::fabs(at(A, i + 1, i)) <= eps * (std::fabs(at(A, i, i)) + std::fabs(at(A, i + 1, i + 1))) ||
                std::fabs(at(A, i + 1, i)) <= eps * anorm) {
                at(A, i + 1, i) = at(A, i, i + 1) = 0.0;
            }
        while (hi > 0 && at(A, hi, hi - 1) == 0.0) --hi;
        if (hi == 0) break;
        int lo = hi - 1;
        while (lo > 0 && at(A, lo, lo - 1) != 0.0) --lo;
        // Wilkinson shift from the trailing 2x2 block
        double a = at(A, hi - 1, hi - 1), b = at(A, hi, hi - 1), cc = at(A, hi, hi);
        double delta = 0.5 * (a - cc);
        double sgn = delta >= 0 ? 1.0 : -1.0;
        double mu = cc - b * b / (delta + sgn * std::sqrt(delta * delta + b * b));
        double x = at(A, lo, lo) - mu, z = at(A, lo + 1, lo);
        for (int k = lo; k < hi; ++k) {
            double r = std::hypot(x, z);
            double c = r == 0 ? 1.0 : x / r, s = r == 0 ? 0.0 : z / r;
            rotate(k, c, s);
            if (k + 1 < hi) { x = at(A, k + 1, k); z = at(A, k + 2, k); }
        }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = at(A, i, i);
}

soap_status build_tables(soap_calculator* calc)
{
    const soap_hypers& h = calc->h;
    int nmax = h.nmax, lmax = h.lmax, nl = nmax * (lmax + 1);
    calc->orth.assign(nmax * nmax, 0.0);
    if (h.radial_basis == 1) {
        for (int i = 0; i < nmax; ++i) calc->orth[i * nmax + i] = 1.0;
        calc->info.overlap_condition = 1.0;
    } else {
        Gto gto(nmax, h.rcut);
        std::vector<double> S = gto_overlap(gto, nmax), w, Q;
        sym_eigen(nmax, S, w, Q);
        double wmin = *std::min_element(w.begin(), w.end()), wmax = *std::max_element(w.begin(), w.end());
        if (!(wmin > 0)) return fail(SOAP_EINVAL, "GTO overlap matrix is not positive definite (nmax=%d)", nmax);
        for (int i = 0; i < nmax; ++i)
            for (int j = 0; j < nmax; ++j) {
                double s = 0.0;
                for (int k = 0; k < nmax; ++k) s += Q[i * nmax + k] * Q[j * nmax + k] / std::sqrt(w[k]);
                calc->orth[i * nmax + j] = s;
            }
        calc->info.overlap_condition = wmax / wmin;
    }
    build_exact_radial(h, calc->orth, calc->exact);
    struct {
        const ExactRadial& e;
        void orth(double r, double* I, double* dI) const { exact_radial_eval(e, r, I, dI); }
    } ex{calc->exact};
    std::vector<double> I0(nl), dI0(nl);
    ex.orth(0.0, I0.data(), dI0.data());
    // device constants: [nmax] centre terms I~_n0(0) Y_00, then [(lmax+1)^2]
    // harmonic normalisations K_lm = sqrt((2 - delta_m0)(2l+1)/4pi (l-|m|)!/(l+|m|)!)
    calc->center.resize(nmax + (lmax + 1) * (lmax + 1));
    for (int n = 0; n < nmax; ++n) calc->center[n] = I0[n * (lmax + 1)] / std::sqrt(4.0 * kPi);
    for (int l = 0; l <= lmax; ++l)
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double lr = std::lgamma(l - am + 1.0) - std::lgamma(l + am + 1.0);
            calc->center[nmax + l * l + l + m] = std::sqrt((am == 0 ? 1.0 : 2.0) * (2 * l + 1) / (4.0 * kPi) * std::exp(lr));
        }

    double acc = h.spline_accuracy;
    for (int64_t M = 1024; M <= (int64_t(1) << 16); M *= 2) {
        double dr = h.rcut / double(M);
        // exact values on the knots, derivatives at both ends
        std::vector<double> knots((M + 1) * nl), dend0(nl), dendM(nl), tmp(nl);
        for (int64_t k = 0; k <= M; ++k) {
            double r = (k == M) ? h.rcut : k * dr;
            ex.orth(r, &knots[k * nl], k == 0 ? dend0.data() : (k == M ? dendM.data() : nullptr));
        }
        std::vector<double> coef(M * nl * 4);
        std::vector<double> y(M + 1);
        for (int j = 0; j < nl; ++j) {
            for (int64_t k = 0; k <= M; ++k) y[k] = knots[k * nl + j];
            std::vector<double> m2 = clamped_second_derivatives(y, dr, dend0[j], dendM[j]);
            double h26 = dr * dr / 6.0;
            for (int64_t k = 0; k < M; ++k) {
                double* cf = &coef[(k * nl + j) * 4];
                // y(t) = A y_k + B y_k+1 + ((A^3-A) y''_k + (B^3-B) y''_k+1) h^2/6,
                // A = 1 - t, B = t, expanded in powers of t
                cf[0] = y[k];
                cf[1] = (y[k + 1] - y[k]) - h26 * (2.0 * m2[k] + m2[k + 1]);
                cf[2] = 3.0 * h26 * m2[k];
                cf[3] = h26 * (m2[k + 1] - m2[k]);
            }
        }
        // error at four interior points per interval
        double err = 0.0, derr = 0.0;
        std::vector<double> Ie(nl), dIe(nl);
        for (int64_t k = 0; k < M; ++k)
            for (int q = 1; q <= 4; ++q) {
                double t = q / 5.0, r = (k + t) * dr;
                ex.orth(r, Ie.data(), dIe.data());
                for (int j = 0; j < nl; ++j) {
                    const double* cf = &coef[(k * nl + j) * 4];
                    double v = cf[0] + t * (cf[1] + t * (cf[2] + t * cf[3]));
                    double dv = (cf[1] + t * (2.0 * cf[2] + 3.0 * t * cf[3])) / dr;
                    err = std::max(err, std::fabs(v - Ie[j]));
                    derr = std::max(derr, std::fabs(dv - dIe[j]));
                }
            }
        if (err <= acc || M == (int64_t(1) << 16)) {
            if (err > acc) return fail(SOAP_EINVAL, "spline accuracy %.3g not reached (%.3g at M=%lld)", acc, err, (long long)M);
            calc->M = M;
            calc->delta = dr;
            calc->inv_delta = double(M) / h.rcut;
            calc->coef64 = std::move(coef);
            calc->coef32.resize(calc->coef64.size());
            for (size_t i = 0; i < calc->coef64.size(); ++i) calc->coef32[i] = float(calc->coef64[i]);
            calc->info.n_intervals = M;
            calc->info.delta = dr;
            calc->info.max_error = err;
            calc->info.max_error_deriv = derr;
            calc->info.table_bytes_f64 = int64_t(calc->coef64.size() * sizeof(double));
            calc->info.table_bytes_f32 = int64_t(calc->coef32.size() * sizeof(float));
            return SOAP_OK;
        }
    }
    return fail(SOAP_EINVAL, "spline refinement failed");
}

void radial_exact(const soap_calculator* calc, int64_t n, const double* r, double* I, double* dI)
{
    for (int64_t k = 0; k < n; ++k) exact_radial_eval(calc->exact, r[k], I + k * calc->nl, dI ? dI + k * calc->nl : nullptr);
}

void radial_spline_host(const soap_calculator* calc, double r, double* I, double* dI)
{
    int nl = calc->nl;
    double x = r * calc->inv_delta;
    int64_t k = std::min<int64_t>(std::max<int64_t>(int64_t(std::floor(x)), 0), calc->M - 1);
    double t = x - double(k);
    for (int j = 0; j < nl; ++j) {
        const double* cf = &calc->coef64[(k * nl + j) * 4];
        I[j] = cf[0] + t * (cf[1] + t * (cf[2] + t * cf[3]));
        if (dI) dI[j] = (cf[1] + t * (2.0 * cf[2] + 3.0 * t * cf[3])) * calc->inv_delta;
    }
}

}  // namespace soap
