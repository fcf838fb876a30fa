/*
 * soap_oracle.c -- plain FP64 CPU oracle of the SOAP hot path.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The GPU library neither
 * links nor calls it and the two share no source, header, table or helper.
 *
 * Everything here is written from the definitions in Musil et al.,
 * "Efficient implementation of atom-density representations" (arXiv
 * 2101.08814), in the most direct form available, in double precision:
 *   - neighbours: brute force over every atom and every periodic image shift
 *     that can lie inside the cutoff (App. B: environments hold every j, with
 *     periodic images, with r_ji < rcut);
 *   - radial integral: the closed form of Eq. (rad-int-gto-1) with the
 *     confluent hypergeometric function summed as its defining power series
 *     (App. A, first equation) -- no recurrence, no asymptotic switch, no
 *     spline;
 *   - orthogonalisation: S^{-1/2} from a cyclic Jacobi eigen-decomposition of
 *     the analytic GTO overlap (Sec. 4.B);
 *   - DVR radial basis (Sec. 4.C Eq. rad-int-dvr): Gauss-Legendre points by
 *     Newton iteration on the Legendre polynomial, the modified spherical
 *     Bessel function by its defining power series;
 *   - real spherical harmonics: explicit polynomials (binomial sum of the
 *     Legendre polynomial, differentiated term by term), not a recurrence;
 *   - coefficients, power spectrum, gradients and the vector-Jacobian
 *     product: direct sums (Eqs. density-coefficients, nu2-basis-coupled,
 *     Sec. 4.G, App. B Eq. energy-derivative).
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   cutoff function  : shifted cosine of width w (the paper only asks for a
 *                      smooth function);
 *   Gaussian density : exp(-|x|^2 / 2 sigma^2), unnormalised -- the only
 *                      normalisation under which Eq. radial-integral-gaussian-
 *                      density and Eq. rad-int-gto-1 agree;
 *   harmonics        : real, orthonormal, m = -l..l stored at l*l+l+m,
 *                      Y_{1,-1}, Y_{1,0}, Y_{1,1} proportional to y, z, x;
 *   power spectrum   : p_{l,k1<=k2} = sum_m c_{k1 lm} c_{k2 lm} with
 *                      k = species*nmax + n; the paper's Eq. nu2-basis-coupled
 *                      is this divided by sqrt(2l+1);
 *   centre atom      : include_center adds the r = 0 term of the central atom
 *                      to its own species channel;
 *   DVR radial basis : I_nl(r) = 4 pi exp(-c r^2) x_n sqrt(w_n) exp(-c x_n^2)
 *                      i_l(2 c x_n r) on the nmax Gauss-Legendre points x_n
 *                      (weights w_n) of [0, rcut + 3 sigma]: Eq. rad-int-dvr
 *                      with the factor 4 pi exp(-c r^2) of Eq. radial-
 *                      integral-gaussian-density restored; the single power
 *                      of x_n is that of DVR functions normalised with the
 *                      radial measure x^2 dx (value 1 / (x_n sqrt(w_n)) at
 *                      their own point), which are orthonormal, so no S^-1/2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.141592653589793238462643383279502884

/* Number of threads the parallel loops over centres use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of threads of later parallel loops (n >= 1). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------------- */
/* Cutoff function (reading: shifted cosine of width w, see header).        */
/* ---------------------------------------------------------------------- */
double orc_fcut(double r, double rcut, double width, double* dfdr)
{
    if (r >= rcut) { *dfdr = 0.0; return 0.0; }
    if (r <= rcut - width) { *dfdr = 0.0; return 1.0; }
    double t = ORC_PI * (r - rcut + width) / width;
    *dfdr = -0.5 * sin(t) * ORC_PI / width;
    return 0.5 * (1.0 + cos(t));
}

/* ---------------------------------------------------------------------- */
/* GTO radial basis, Sec. 4.B Eq. (GTO):                                   */
/*   R_n(r) = N_n r^n exp(-d_n r^2), d_n = 1/(2 sigma_n^2),                */
/*   sigma_n = rcut max(sqrt(n),1)/nmax, N_n^2 = 2/(sigma_n^(2n+3) G(n+3/2)) */
/* ---------------------------------------------------------------------- */
void orc_gto_constants(int nmax, double rcut, double* sigma_n, double* d_n, double* norm_n)
{
    for (int n = 0; n < nmax; ++n) {
        double s = rcut * fmax(sqrt((double)n), 1.0) / nmax;
        sigma_n[n] = s;
        d_n[n] = 1.0 / (2.0 * s * s);
        norm_n[n] = sqrt(2.0 / (pow(s, 2.0 * n + 3.0) * tgamma(n + 1.5)));
    }
}

/* Overlap S_nn' = int_0^inf r^2 R_n(r) R_n'(r) dr.  With
 * int_0^inf r^k exp(-a r^2) dr = Gamma((k+1)/2) / (2 a^((k+1)/2)) and
 * k = n+n'+2, a = d_n + d_n' this is
 *   N_n N_n' Gamma((n+n'+3)/2) / (2 (d_n+d_n')^((n+n'+3)/2)).           */
void orc_overlap(int nmax, double rcut, double* S)
{
    double sg[64], d[64], nn[64];
    orc_gto_constants(nmax, rcut, sg, d, nn);
    for (int n = 0; n < nmax; ++n)
        for (int m = 0; m < nmax; ++m) {
            double k = 0.5 * (n + m + 3.0);
            S[n * nmax + m] = nn[n] * nn[m] * tgamma(k) / (2.0 * pow(d[n] + d[m], k));
        }
}

/* Symmetric inverse square root X = V diag(1/sqrt(lambda)) V^T of a
 * symmetric positive definite matrix, by cyclic Jacobi rotations.
 * Returns 0 on success, -1 if the matrix is not positive definite.      */
int orc_inverse_sqrt(int n, const double* A, double* X)
{
    double* a = (double*)malloc(sizeof(double) * n * n);
    double* V = (double*)malloc(sizeof(double) * n * n);
    memcpy(a, A, sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < n; ++p) {
            diag += a[p * n + p] * a[p * n + p];
            for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
        }
        if (off <= 1e-34 * diag) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = a[p * n + q];
                if (apq == 0.0) continue;
                double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {       /* columns p, q of a */
                    double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = c * akp - s * akq;
                    a[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {       /* rows p, q of a */
                    double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = c * apk - s * aqk;
                    a[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {       /* accumulate V = V J */
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    int status = 0;
    for (int i = 0; i < n && !status; ++i)
        if (!(a[i * n + i] > 0.0)) status = -1;
    if (!status)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += V[i * n + k] * V[j * n + k] / sqrt(a[k * n + k]);
                X[i * n + j] = s;
            }
    free(a);
    free(V);
    return status;
}

/* Confluent hypergeometric function 1F1(a;b;z), App. A first equation:
 * the power series sum_s (a)_s / ((b)_s s!) z^s, each term obtained from
 * the previous one by the factor (a+s-1) z / ((b+s-1) s).  For a, b, z > 0
 * every term is positive, so the series is summed until a term no longer
 * changes the sum in double precision.                                  */
double orc_hyp1f1(double a, double b, double z)
{
    double term = 1.0, sum = 1.0;
    for (int s = 1; s < 1000000; ++s) {
        term *= (a + s - 1.0) * z / ((b + s - 1.0) * s);
        sum += term;
        if (fabs(term) < 1e-17 * fabs(sum)) break;
    }
    return sum;
}

/* Raw (non-orthogonal) GTO radial integral of a Gaussian density,
 * Eq. (rad-int-gto-1), for all 0 <= n < nmax, 0 <= l <= lmax:
 *   I_nl(r) = pi^{3/2} exp(-c r^2) N_n G((n+l+3)/2)/G(l+3/2) c^l r^l
 *             (c+d_n)^{-(n+l+3)/2} 1F1((n+l+3)/2; l+3/2; c^2 r^2/(c+d_n)),
 * c = 1/(2 sigma^2).  Layout I[n*(lmax+1)+l].  dI (nullable) is d/dr,
 * using d 1F1(a;b;z)/dz = (a/b) 1F1(a+1;b+1;z) and the product rule.    */
void orc_radial_integral(int nmax, int lmax, double rcut, double sigma, double r,
                         double* I, double* dI)
{
    double sg[64], d[64], nn[64];
    orc_gto_constants(nmax, rcut, sg, d, nn);
    double c = 1.0 / (2.0 * sigma * sigma);
    for (int n = 0; n < nmax; ++n)
        for (int l = 0; l <= lmax; ++l) {
            double a = 0.5 * (n + l + 3.0), b = l + 1.5;
            double alpha = c * c / (c + d[n]);
            double z = alpha * r * r;
            double pref = pow(ORC_PI, 1.5) * nn[n] * exp(lgamma(a) - lgamma(b)) *
                          pow(c, (double)l) * pow(c + d[n], -a);
            double F = orc_hyp1f1(a, b, z);
            double e = exp(-c * r * r);
            double rl = (l == 0) ? 1.0 : pow(r, (double)l);
            I[n * (lmax + 1) + l] = pref * e * rl * F;
            if (dI) {
                double F1 = orc_hyp1f1(a + 1.0, b + 1.0, z);
                double drl = (l == 0) ? 0.0 : l * ((l == 1) ? 1.0 : pow(r, (double)(l - 1)));
                double dz = 2.0 * alpha * r;
                dI[n * (lmax + 1) + l] =
                    pref * e * (drl * F - 2.0 * c * r * rl * F + rl * dz * (a / b) * F1);
            }
        }
}

/* Orthogonalised radial integral: I~_nl = sum_n' [S^{-1/2}]_nn' I_n'l
 * (Sec. 4.B; the orthogonalisation is linear so it may be applied to the
 * radial integral directly).  X is S^{-1/2}.                             */
static void orth_apply(int nmax, int lmax, const double* X, const double* I, double* out)
{
    for (int n = 0; n < nmax; ++n)
        for (int l = 0; l <= lmax; ++l) {
            double s = 0.0;
            for (int m = 0; m < nmax; ++m) s += X[n * nmax + m] * I[m * (lmax + 1) + l];
            out[n * (lmax + 1) + l] = s;
        }
}

int orc_orth_matrix(int nmax, double rcut, double* X)
{
    double* S = (double*)malloc(sizeof(double) * nmax * nmax);
    orc_overlap(nmax, rcut, S);
    int st = orc_inverse_sqrt(nmax, S, X);
    free(S);
    return st;
}

int orc_radial_integral_orth(int nmax, int lmax, double rcut, double sigma, double r,
                             double* It, double* dIt)
{
    int nl = nmax * (lmax + 1);
    double* X = (double*)malloc(sizeof(double) * nmax * nmax);
    double* I = (double*)malloc(sizeof(double) * nl);
    double* dI = (double*)malloc(sizeof(double) * nl);
    int st = orc_orth_matrix(nmax, rcut, X);
    orc_radial_integral(nmax, lmax, rcut, sigma, r, I, dIt ? dI : NULL);
    orth_apply(nmax, lmax, X, I, It);
    if (dIt) orth_apply(nmax, lmax, X, dI, dIt);
    free(X); free(I); free(dI);
    return st;
}

/* ---------------------------------------------------------------------- */
/* DVR radial basis, Sec. 4.C Eq. (rad-int-dvr).                          */
/* ---------------------------------------------------------------------- */
/* Gauss-Legendre points t_k and weights w_k on [-1, 1]: the roots of P_n by
 * Newton iteration from cos(pi (k - 1/4) / (n + 1/2)), P_n and P_n' from the
 * three-term recurrence j P_j = (2j-1) t P_{j-1} - (j-1) P_{j-2},
 * w = 2 / ((1 - t^2) P_n'(t)^2).  Ascending order.                       */
void orc_gauss_legendre(int n, double* t, double* w)
{
    for (int k = 1; k <= n; ++k) {
        double x = cos(ORC_PI * (k - 0.25) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            if (n == 0) p1 = 1.0;
            for (int j = 2; j <= n; ++j) {
                double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            /* p1 = P_n(x), p0 = P_{n-1}(x) */
            dp = (n == 1) ? 1.0 : n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int j = 2; j <= n; ++j) {
            double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = (n == 1) ? 1.0 : n * (x * p1 - p0) / (x * x - 1.0);
        t[n - k] = x;
        w[n - k] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

/* Modified spherical Bessel function of the first kind by its defining
 * power series,
 *   i_l(z) = sum_k z^(l+2k) / (2^k k! (2l+2k+1)!!),
 * each term from the previous one by z^2 / (2 (k+1) (2l+2k+3)) (all terms
 * positive).  *d (nullable) receives d i_l / dz = sum_k (l+2k) z^(l+2k-1)
 * / (2^k k! (2l+2k+1)!!).                                                */
double orc_sph_bessel_i(int l, double z, double* d)
{
    double t = 1.0;
    for (int k = 1; k <= l; ++k) t *= z / (2.0 * k + 1.0);   /* z^l / (2l+1)!! */
    double sum = 0.0, dsum = 0.0;
    for (int k = 0; k < 100000; ++k) {
        sum += t;
        if (d && z > 0.0) dsum += t * (l + 2.0 * k) / z;
        double nt = t * z * z / (2.0 * (k + 1.0) * (2.0 * l + 2.0 * k + 3.0));
        if (nt < 1e-17 * sum || nt == 0.0) break;
        t = nt;
    }
    if (d) *d = (z > 0.0) ? dsum : (l == 1 ? 1.0 / 3.0 : 0.0);
    return sum;
}

void orc_dvr_points(int nmax, double rcut, double sigma, double* x, double* w)
{
    double* t = (double*)malloc(sizeof(double) * nmax);
    double* wt = (double*)malloc(sizeof(double) * nmax);
    orc_gauss_legendre(nmax, t, wt);
    double b = rcut + 3.0 * sigma;
    for (int n = 0; n < nmax; ++n) {
        x[n] = 0.5 * b * (t[n] + 1.0);
        w[n] = 0.5 * b * wt[n];
    }
    free(t); free(wt);
}

/* I_nl(r) = 4 pi x_n sqrt(w_n) exp(-c (x_n^2 + r^2)) i_l(2 c x_n r) and
 * d/dr, c = 1/(2 sigma^2) (the reading in the file header).  The Gaussian
 * and Bessel factors are combined in logarithms (the Bessel factor grows
 * like e^z).  Layout I[n*(lmax+1)+l].                                    */
void orc_dvr_radial_integral(int nmax, int lmax, double rcut, double sigma, double r, double* I, double* dI)
{
    double x[64], w[64];
    orc_dvr_points(nmax, rcut, sigma, x, w);
    double c = 1.0 / (2.0 * sigma * sigma);
    for (int n = 0; n < nmax; ++n) {
        double z = 2.0 * c * x[n] * r;
        double g = -c * (x[n] * x[n] + r * r);
        double A = 4.0 * ORC_PI * x[n] * sqrt(w[n]);
        for (int l = 0; l <= lmax; ++l) {
            double di;
            double bi = orc_sph_bessel_i(l, z, &di);
            double v = (bi > 0.0) ? A * exp(g + log(bi)) : 0.0;
            I[n * (lmax + 1) + l] = v;
            if (dI) {
                double dterm = (di > 0.0) ? A * exp(g + log(di)) * 2.0 * c * x[n] : 0.0;
                dI[n * (lmax + 1) + l] = -2.0 * c * r * v + dterm;
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Real spherical harmonics from explicit polynomials.                    */
/* P_l(x) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) x^(l-2k); Q_lm = d^m P_l/dx^m */
/* For a unit vector u: Y_l0 = K_l0 Q_l0(u_z),                             */
/*   Y_{l,m}  = K_lm Q_lm(u_z) Re((u_x + i u_y)^m),  m > 0,                */
/*   Y_{l,-m} = K_lm Q_lm(u_z) Im((u_x + i u_y)^m),                        */
/*   K_l0 = sqrt((2l+1)/4pi), K_lm = sqrt(2 (2l+1)/4pi (l-m)!/(l+m)!).     */
/* (sin^m theta cos m phi = Re((u_x+iu_y)^m); P_l^m without the           */
/*  Condon-Shortley phase is (1-x^2)^(m/2) Q_lm(x).)                       */
/* ---------------------------------------------------------------------- */
static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

static double factorial(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

static double ipow(double x, int e) /* x^e for e >= 0, with 0^0 = 1 */
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

/* value of d^m P_l / dx^m at x */
static double legendre_deriv(int l, int m, double x)
{
    double s = 0.0;
    for (int k = 0; 2 * k <= l; ++k) {
        int deg = l - 2 * k;
        if (deg < m) continue;
        double coef = ((k & 1) ? -1.0 : 1.0) * binom(l, k) * binom(2 * l - 2 * k, l) / ipow(2.0, l);
        s += coef * factorial(deg) / factorial(deg - m) * ipow(x, deg - m);
    }
    return s;
}

/* Re/Im of (x + i y)^m and their x, y derivatives, by the binomial sum. */
static void cplx_power(int m, double x, double y, double out[6])
{
    /* out: re, im, dre/dx, dre/dy, dim/dx, dim/dy */
    for (int i = 0; i < 6; ++i) out[i] = 0.0;
    for (int k = 0; k <= m; ++k) {
        double cb = binom(m, k);
        /* i^k: k%4 = 0 -> 1, 1 -> i, 2 -> -1, 3 -> -i */
        int r4 = k % 4;
        double re_f = (r4 == 0) ? 1.0 : (r4 == 2) ? -1.0 : 0.0;
        double im_f = (r4 == 1) ? 1.0 : (r4 == 3) ? -1.0 : 0.0;
        double v = cb * ipow(x, m - k) * ipow(y, k);
        double vx = (m - k > 0) ? cb * (m - k) * ipow(x, m - k - 1) * ipow(y, k) : 0.0;
        double vy = (k > 0) ? cb * k * ipow(x, m - k) * ipow(y, k - 1) : 0.0;
        out[0] += re_f * v;  out[1] += im_f * v;
        out[2] += re_f * vx; out[3] += re_f * vy;
        out[4] += im_f * vx; out[5] += im_f * vy;
    }
}

/* Y[l*l+l+m] for the direction of v (any length > 0); dY (nullable) is the
 * Cartesian gradient with respect to v, layout dY[axis*(lmax+1)^2 + lm].
 * With F(u) the polynomial above, grad_v Y = (grad_u F - u (u . grad_u F))/|v|. */
void orc_ylm(int lmax, const double* v, double* Y, double* dY)
{
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double u[3] = {v[0] / r, v[1] / r, v[2] / r};
    int L2 = (lmax + 1) * (lmax + 1);
    for (int l = 0; l <= lmax; ++l)
        for (int m = 0; m <= l; ++m) {
            double K = (m == 0) ? sqrt((2 * l + 1) / (4.0 * ORC_PI))
                                : sqrt(2.0 * (2 * l + 1) / (4.0 * ORC_PI) * factorial(l - m) / factorial(l + m));
            double Q = legendre_deriv(l, m, u[2]);
            double dQ = legendre_deriv(l, m + 1, u[2]);
            double cp[6];
            cplx_power(m, u[0], u[1], cp);
            /* m >= 0 uses the real part (m = 0: (x+iy)^0 = 1); -m the imaginary part */
            for (int sgn = 0; sgn < ((m == 0) ? 1 : 2); ++sgn) {
                int mm = sgn ? -m : m;
                double T = sgn ? cp[1] : cp[0];
                double Tx = sgn ? cp[4] : cp[2];
                double Ty = sgn ? cp[5] : cp[3];
                int idx = l * l + l + mm;
                Y[idx] = K * Q * T;
                if (dY) {
                    double g[3] = {K * Q * Tx, K * Q * Ty, K * dQ * T};
                    double ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
                    for (int a = 0; a < 3; ++a) dY[a * L2 + idx] = (g[a] - u[a] * ug) / r;
                }
            }
        }
}

/* ---------------------------------------------------------------------- */
/* Neighbour list by brute force (App. B: A_i holds every j, including     */
/* periodic images, with 0 < r_ji < rcut; images of i itself are kept).   */
/* A pair is (i, j, s) with r_ji = r_j + s1 h1 + s2 h2 + s3 h3 - r_i.      */
/* Pairs of a centre are ordered by (species_j, j, s1, s2, s3).            */
/* ---------------------------------------------------------------------- */
typedef struct { int32_t a, j, s0, s1, s2; double v[3]; } orc_pair;

static int pair_cmp(const void* x, const void* y)
{
    const orc_pair* p = (const orc_pair*)x;
    const orc_pair* q = (const orc_pair*)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->j != q->j) return p->j < q->j ? -1 : 1;
    if (p->s0 != q->s0) return p->s0 < q->s0 ? -1 : 1;
    if (p->s1 != q->s1) return p->s1 < q->s1 ? -1 : 1;
    if (p->s2 != q->s2) return p->s2 < q->s2 ? -1 : 1;
    return 0;
}

static int inverse3(const double* H, double* Hi)
{
    double det = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                 H[2] * (H[3] * H[7] - H[4] * H[6]);
    if (fabs(det) < 1e-12) return -1;
    Hi[0] = (H[4] * H[8] - H[5] * H[7]) / det;
    Hi[1] = (H[2] * H[7] - H[1] * H[8]) / det;
    Hi[2] = (H[1] * H[5] - H[2] * H[4]) / det;
    Hi[3] = (H[5] * H[6] - H[3] * H[8]) / det;
    Hi[4] = (H[0] * H[8] - H[2] * H[6]) / det;
    Hi[5] = (H[2] * H[3] - H[0] * H[5]) / det;
    Hi[6] = (H[3] * H[7] - H[4] * H[6]) / det;
    Hi[7] = (H[1] * H[6] - H[0] * H[7]) / det;
    Hi[8] = (H[0] * H[4] - H[1] * H[3]) / det;
    return 0;
}

/* All pairs of centre i (global index) of structure s, sorted; returns the
 * count (or -1 for coincident distinct atoms).  *out is malloc'ed.         */
static int64_t centre_pairs(int64_t i, int64_t lo, int64_t hi, const double* pos,
                            const double* H, const uint8_t* pbc, const int32_t* species,
                            double rcut, orc_pair** out)
{
    double Hi[9];
    int any = pbc[0] || pbc[1] || pbc[2];
    int range_lo[3] = {0, 0, 0}, range_hi[3] = {0, 0, 0};
    double width[3] = {0, 0, 0};
    if (any) {
        if (inverse3(H, Hi)) return -2;
        /* perpendicular width along axis k is 1/|column k of H^-1| */
        for (int k = 0; k < 3; ++k)
            width[k] = 1.0 / sqrt(Hi[0 * 3 + k] * Hi[0 * 3 + k] + Hi[1 * 3 + k] * Hi[1 * 3 + k] +
                                  Hi[2 * 3 + k] * Hi[2 * 3 + k]);
    }
    int64_t cap = 64, n = 0;
    orc_pair* list = (orc_pair*)malloc(sizeof(orc_pair) * cap);
    for (int64_t j = lo; j < hi; ++j) {
        double d[3] = {pos[3 * j] - pos[3 * i], pos[3 * j + 1] - pos[3 * i + 1], pos[3 * j + 2] - pos[3 * i + 2]};
        if (any) {
            /* any image inside the cutoff satisfies |f_k + s_k| * width_k < rcut */
            for (int k = 0; k < 3; ++k) {
                if (!pbc[k]) { range_lo[k] = range_hi[k] = 0; continue; }
                double f = d[0] * Hi[0 * 3 + k] + d[1] * Hi[1 * 3 + k] + d[2] * Hi[2 * 3 + k];
                range_lo[k] = (int)floor(-f - rcut / width[k]) - 1;
                range_hi[k] = (int)ceil(-f + rcut / width[k]) + 1;
            }
        }
        for (int s0 = range_lo[0]; s0 <= range_hi[0]; ++s0)
            for (int s1 = range_lo[1]; s1 <= range_hi[1]; ++s1)
                for (int s2 = range_lo[2]; s2 <= range_hi[2]; ++s2) {
                    double v[3];
                    for (int a = 0; a < 3; ++a)
                        v[a] = d[a] + s0 * H[0 * 3 + a] + s1 * H[1 * 3 + a] + s2 * H[2 * 3 + a];
                    double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                    if (j == i && s0 == 0 && s1 == 0 && s2 == 0) continue;
                    if (r2 >= rcut * rcut) continue;
                    if (r2 == 0.0) { free(list); return -1; }
                    if (n == cap) { cap *= 2; list = (orc_pair*)realloc(list, sizeof(orc_pair) * cap); }
                    orc_pair* p = &list[n++];
                    p->a = species[j]; p->j = (int32_t)j; p->s0 = s0; p->s1 = s1; p->s2 = s2;
                    p->v[0] = v[0]; p->v[1] = v[1]; p->v[2] = v[2];
                }
    }
    qsort(list, n, sizeof(orc_pair), pair_cmp);
    *out = list;
    return n;
}

/* Two-phase use: call with pair_j == NULL to get pair_offsets (the total is
 * pair_offsets[N]); allocate; call again to fill.  Returns 0, or -1 for
 * coincident distinct atoms, -2 for a singular periodic cell.              */
int orc_neighbors(int n_struct, const int64_t* atom_offsets, const double* pos, const double* cells,
                  const uint8_t* pbc, const int32_t* species, double rcut, int64_t* pair_offsets,
                  int32_t* pair_j, int32_t* pair_shift, double* pair_vec)
{
    int64_t N = atom_offsets[n_struct];
    int status = 0;
    int64_t* counts = (int64_t*)calloc(N + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < N; ++i) {
        int s = 0;
        while (atom_offsets[s + 1] <= i) ++s;
        orc_pair* list = NULL;
        int64_t n = centre_pairs(i, atom_offsets[s], atom_offsets[s + 1], pos, cells + 9 * s,
                                 pbc + 3 * s, species, rcut, &list);
        if (n < 0) {
#pragma omp critical
            status = (int)n;
            continue;
        }
        counts[i] = n;
        if (pair_j) {
            int64_t off = pair_offsets[i];
            for (int64_t k = 0; k < n; ++k) {
                pair_j[off + k] = list[k].j;
                pair_shift[3 * (off + k) + 0] = list[k].s0;
                pair_shift[3 * (off + k) + 1] = list[k].s1;
                pair_shift[3 * (off + k) + 2] = list[k].s2;
                for (int a = 0; a < 3; ++a) pair_vec[3 * (off + k) + a] = list[k].v[a];
            }
        }
        free(list);
    }
    if (!pair_j) {
        pair_offsets[0] = 0;
        for (int64_t i = 0; i < N; ++i) pair_offsets[i + 1] = pair_offsets[i] + counts[i];
    }
    free(counts);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Density expansion coefficients, Eq. (spherical_expansion_coefficients_   */
/* gaussians):  c_{i,a,n,lm} = sum_{j in A_i, a_j = a} f_cut(r_ji)          */
/*                              I~_nl(r_ji) Y_lm(r^_ji)                    */
/* plus, with include_center, the central atom's r = 0 term in channel a_i */
/* (only l = 0 survives at r = 0).  Layout c[centre][a][n][lm].            */
/* ---------------------------------------------------------------------- */
/* Radial basis: 0 = orthogonalised GTO (Sec. 4.B), 1 = DVR (Sec. 4.C). */
typedef struct {
    int S, nmax, lmax, include_center, basis;
    double rcut, width, sigma;
    double* X;
} orc_ctx;

static int ctx_init(orc_ctx* c, int S, int nmax, int lmax, int include_center, double rcut,
                    double width, double sigma, int basis)
{
    c->S = S; c->nmax = nmax; c->lmax = lmax; c->include_center = include_center;
    c->rcut = rcut; c->width = width; c->sigma = sigma; c->basis = basis;
    c->X = (double*)malloc(sizeof(double) * nmax * nmax);
    if (basis == 1) {   /* DVR: orthonormal by construction */
        for (int i = 0; i < nmax * nmax; ++i) c->X[i] = (i % (nmax + 1) == 0) ? 1.0 : 0.0;
        return 0;
    }
    return orc_orth_matrix(nmax, rcut, c->X);
}

/* raw radial integral of the context's basis */
static void ctx_radial(const orc_ctx* c, double r, double* I, double* dI)
{
    if (c->basis == 1) orc_dvr_radial_integral(c->nmax, c->lmax, c->rcut, c->sigma, r, I, dI);
    else orc_radial_integral(c->nmax, c->lmax, c->rcut, c->sigma, r, I, dI);
}

/* The per-pair radial and angular factors of one neighbour vector. */
static void pair_terms(const orc_ctx* c, const double* v, double* f, double* df, double* It,
                       double* dIt, double* Y, double* dY)
{
    int nl = c->nmax * (c->lmax + 1);
    double* I = (double*)malloc(sizeof(double) * nl);
    double* dI = (double*)malloc(sizeof(double) * nl);
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    *f = orc_fcut(r, c->rcut, c->width, df);
    ctx_radial(c, r, I, dIt ? dI : NULL);
    orth_apply(c->nmax, c->lmax, c->X, I, It);
    if (dIt) orth_apply(c->nmax, c->lmax, c->X, dI, dIt);
    orc_ylm(c->lmax, v, Y, dY);
    free(I); free(dI);
}

static void centre_coeffs(const orc_ctx* c, int64_t i, const int32_t* species,
                          const int64_t* pair_offsets, const int32_t* pair_j,
                          const double* pair_vec, double* out)
{
    int nmax = c->nmax, lmax = c->lmax, L2 = (lmax + 1) * (lmax + 1);
    int nl = nmax * (lmax + 1);
    memset(out, 0, sizeof(double) * c->S * nmax * L2);
    double* It = (double*)malloc(sizeof(double) * nl);
    double* Y = (double*)malloc(sizeof(double) * L2);
    if (c->include_center) {
        double* I0 = (double*)malloc(sizeof(double) * nl);
        ctx_radial(c, 0.0, I0, NULL);
        orth_apply(nmax, lmax, c->X, I0, It);
        double y00 = 1.0 / sqrt(4.0 * ORC_PI);
        for (int n = 0; n < nmax; ++n)
            out[(species[i] * nmax + n) * L2 + 0] += It[n * (lmax + 1) + 0] * y00;
        free(I0);
    }
    for (int64_t q = pair_offsets[i]; q < pair_offsets[i + 1]; ++q) {
        double f, df;
        pair_terms(c, pair_vec + 3 * q, &f, &df, It, NULL, Y, NULL);
        int a = species[pair_j[q]];
        for (int n = 0; n < nmax; ++n)
            for (int l = 0; l <= lmax; ++l)
                for (int m = -l; m <= l; ++m)
                    out[(a * nmax + n) * L2 + l * l + l + m] += f * It[n * (lmax + 1) + l] * Y[l * l + l + m];
    }
    free(It); free(Y);
}

int orc_expansion(int S, int nmax, int lmax, int include_center, double rcut, double width, double sigma,
                  int basis, const int32_t* species, const int64_t* pair_offsets, const int32_t* pair_j,
                  const double* pair_vec, int64_t n_centres, const int64_t* centres, double* coeffs)
{
    orc_ctx c;
    int st = ctx_init(&c, S, nmax, lmax, include_center, rcut, width, sigma, basis);
    int64_t blk = (int64_t)S * nmax * (lmax + 1) * (lmax + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < n_centres; ++t)
        centre_coeffs(&c, centres[t], species, pair_offsets, pair_j, pair_vec, coeffs + t * blk);
    free(c.X);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Power spectrum (Eq. nu2-basis-coupled with real coefficients, up to the */
/* 1/sqrt(2l+1) factor): p_{l, k1<=k2} = sum_m c_{k1,lm} c_{k2,lm},        */
/* k = a*nmax + n, packed row-major over the upper triangle k1 <= k2.      */
/* ---------------------------------------------------------------------- */
static int64_t tri_index(int K, int k1, int k2) /* k1 <= k2 */
{
    return (int64_t)k1 * K - (int64_t)k1 * (k1 - 1) / 2 + (k2 - k1);
}

void orc_power_spectrum(int S, int nmax, int lmax, int64_t n, const double* coeffs, double* p)
{
    int K = S * nmax, L2 = (lmax + 1) * (lmax + 1);
    int64_t KK = (int64_t)K * (K + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double* c = coeffs + i * (int64_t)K * L2;
        for (int l = 0; l <= lmax; ++l)
            for (int k1 = 0; k1 < K; ++k1)
                for (int k2 = k1; k2 < K; ++k2) {
                    double s = 0.0;
                    for (int m = -l; m <= l; ++m) s += c[k1 * L2 + l * l + l + m] * c[k2 * L2 + l * l + l + m];
                    p[(i * (lmax + 1) + l) * KK + tri_index(K, k1, k2)] = s;
                }
    }
}

/* ---------------------------------------------------------------------- */
/* Gradients (Sec. 4.G; App. B Eq. energy-derivative).                      */
/* For pair q = (i, j, s) the row dc_q[x][n][lm] = d c_{i,a_j,n,lm}/d r_ji,x */
/*   = d/dr_x [ f(r) I~_nl(r) Y_lm(r^) ]                                     */
/*   = (f' I~ + f I~') Y r^_x + f I~ dY/dr_x.                               */
/* The self row of centre i, species block a, is -sum over pairs of i with  */
/* a_j = a (r_ji = r_j + sH - r_i, so d r_ji / d r_i = -1).                 */
/* dp rows follow from the product rule,                                    */
/*   dp_{x,l,k1k2} = sum_m dc_{x,k1,lm} c_{k2,lm} + c_{k1,lm} dc_{x,k2,lm}, */
/* with dc nonzero only in the a_j block.  The self dp row is the same      */
/* contraction of the full self dc row.                                     */
/* Rows are produced for the listed centres, pair rows in the centres'      */
/* pair order, concatenated.                                                */
/* ---------------------------------------------------------------------- */
static void contract_dp(int K, int lmax, const double* c, const double* dcfull, double* dp)
{
    /* c [K][L2], dcfull [3][K][L2] -> dp [3][lmax+1][KK] */
    int L2 = (lmax + 1) * (lmax + 1);
    int64_t KK = (int64_t)K * (K + 1) / 2;
    for (int x = 0; x < 3; ++x)
        for (int l = 0; l <= lmax; ++l)
            for (int k1 = 0; k1 < K; ++k1)
                for (int k2 = k1; k2 < K; ++k2) {
                    double s = 0.0;
                    for (int m = -l; m <= l; ++m) {
                        int lm = l * l + l + m;
                        s += dcfull[(x * K + k1) * L2 + lm] * c[k2 * L2 + lm] +
                             c[k1 * L2 + lm] * dcfull[(x * K + k2) * L2 + lm];
                    }
                    dp[(x * (lmax + 1) + l) * KK + tri_index(K, k1, k2)] = s;
                }
}

int orc_gradients(int S, int nmax, int lmax, int include_center, double rcut, double width, double sigma,
                  int basis, const int32_t* species, const int64_t* pair_offsets, const int32_t* pair_j,
                  const double* pair_vec, int64_t n_centres, const int64_t* centres,
                  double* dc, double* dc_self, double* dp, double* dp_self)
{
    orc_ctx c;
    int st = ctx_init(&c, S, nmax, lmax, include_center, rcut, width, sigma, basis);
    int K = S * nmax, L2 = (lmax + 1) * (lmax + 1), nl = nmax * (lmax + 1);
    int64_t KK = (int64_t)K * (K + 1) / 2;
    int64_t blk = (int64_t)nmax * L2;            /* one species block */
    int64_t dprow = 3 * (int64_t)(lmax + 1) * KK;
    /* row offsets of each listed centre */
    int64_t* row0 = (int64_t*)malloc(sizeof(int64_t) * (n_centres + 1));
    row0[0] = 0;
    for (int64_t t = 0; t < n_centres; ++t)
        row0[t + 1] = row0[t] + pair_offsets[centres[t] + 1] - pair_offsets[centres[t]];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < n_centres; ++t) {
        int64_t i = centres[t];
        double* cc = (double*)malloc(sizeof(double) * K * L2);
        double* full = (double*)malloc(sizeof(double) * 3 * K * L2);
        double* self = dc_self + t * 3 * (int64_t)K * L2;
        double* It = (double*)malloc(sizeof(double) * nl);
        double* dIt = (double*)malloc(sizeof(double) * nl);
        double* Y = (double*)malloc(sizeof(double) * L2);
        double* dY = (double*)malloc(sizeof(double) * 3 * L2);
        centre_coeffs(&c, i, species, pair_offsets, pair_j, pair_vec, cc);
        memset(self, 0, sizeof(double) * 3 * K * L2);
        for (int64_t q = pair_offsets[i]; q < pair_offsets[i + 1]; ++q) {
            int64_t row = row0[t] + (q - pair_offsets[i]);
            const double* v = pair_vec + 3 * q;
            double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            double f, df;
            pair_terms(&c, v, &f, &df, It, dIt, Y, dY);
            int a = species[pair_j[q]];
            double* drow = dc + row * 3 * blk;
            memset(full, 0, sizeof(double) * 3 * K * L2);
            for (int x = 0; x < 3; ++x)
                for (int n = 0; n < nmax; ++n)
                    for (int l = 0; l <= lmax; ++l)
                        for (int m = -l; m <= l; ++m) {
                            int lm = l * l + l + m;
                            double I = It[n * (lmax + 1) + l], dI = dIt[n * (lmax + 1) + l];
                            double g = (df * I + f * dI) * Y[lm] * v[x] / r + f * I * dY[x * L2 + lm];
                            drow[(x * nmax + n) * L2 + lm] = g;
                            full[(x * K + a * nmax + n) * L2 + lm] = g;
                            self[(x * K + a * nmax + n) * L2 + lm] -= g;
                        }
            contract_dp(K, lmax, cc, full, dp + row * dprow);
        }
        contract_dp(K, lmax, cc, self, dp_self + t * dprow);
        free(cc); free(full); free(It); free(dIt); free(Y); free(dY);
    }
    free(row0);
    free(c.X);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Vector-Jacobian product of the power spectrum with respect to positions */
/* (App. B Eq. energy-derivative with E = sum_i <W_i, p_i>):               */
/*   dL/dr_k = sum_i sum_{pairs q of i} <W_i, dp_q> ([atom(j_q) = k] - [i = k]) */
/* grad_pair (nullable) receives g_q = <W_i, dp_q>, the derivative of L with */
/* respect to the pair vector r_ji (the input of the virial, App. B).       */
/* ---------------------------------------------------------------------- */
int orc_vjp(int S, int nmax, int lmax, int include_center, double rcut, double width, double sigma,
            int basis, int64_t n_atoms, const int32_t* species, const int64_t* pair_offsets, const int32_t* pair_j,
            const double* pair_vec, const double* grad_p, double* grad_pos, double* grad_pair)
{
    int K = S * nmax, L2 = (lmax + 1) * (lmax + 1);
    int64_t KK = (int64_t)K * (K + 1) / 2;
    int64_t dprow = 3 * (int64_t)(lmax + 1) * KK;
    int64_t P = pair_offsets[n_atoms];
    double* g = (double*)malloc(sizeof(double) * 3 * (P > 0 ? P : 1));
    int status = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n_atoms; ++i) {
        int64_t np = pair_offsets[i + 1] - pair_offsets[i];
        double* dc = (double*)malloc(sizeof(double) * (np > 0 ? np : 1) * 3 * nmax * L2);
        double* dcs = (double*)malloc(sizeof(double) * 3 * K * L2);
        double* dp = (double*)malloc(sizeof(double) * (np > 0 ? np : 1) * dprow);
        double* dps = (double*)malloc(sizeof(double) * dprow);
        int st = orc_gradients(S, nmax, lmax, include_center, rcut, width, sigma, basis, species, pair_offsets,
                               pair_j, pair_vec, 1, &i, dc, dcs, dp, dps);
        if (st) {
#pragma omp critical
            status = st;
        }
        const double* w = grad_p + i * (int64_t)(lmax + 1) * KK;
        for (int64_t k = 0; k < np; ++k)
            for (int x = 0; x < 3; ++x) {
                double s = 0.0;
                for (int64_t f = 0; f < (lmax + 1) * KK; ++f) s += w[f] * dp[k * dprow + x * (lmax + 1) * KK + f];
                g[3 * (pair_offsets[i] + k) + x] = s;
            }
        free(dc); free(dcs); free(dp); free(dps);
    }
    for (int64_t k = 0; k < 3 * n_atoms; ++k) grad_pos[k] = 0.0;
    for (int64_t i = 0; i < n_atoms; ++i)
        for (int64_t q = pair_offsets[i]; q < pair_offsets[i + 1]; ++q)
            for (int x = 0; x < 3; ++x) {
                grad_pos[3 * (int64_t)pair_j[q] + x] += g[3 * q + x];
                grad_pos[3 * i + x] -= g[3 * q + x];
            }
    if (grad_pair)
        for (int64_t k = 0; k < 3 * P; ++k) grad_pair[k] = g[k];
    free(g);
    return status;
}
