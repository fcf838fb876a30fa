// The radial integrals I~_nl(r) and d/dr for a batch of radii on the device,
// one lane per radius, from the spline table (the evaluation the expansion
// kernels inline) or evaluated directly: GTO through the restricted 1F1 of
// App. A and S^{-1/2} (Sec. 4.B), DVR through the closed form with the
// modified spherical Bessel function (Sec. 4.C).  Outputs [nl][n_r] with the
// radius fastest, so the lanes of a wave store consecutive addresses.  Used
// to compare the cost of the three evaluations (Sec. 4.D) and to check the
// table against the direct values on the device.
#include "lane_pair.hpp"

namespace soap {
namespace {

using namespace dev;

template <typename T, int LMAX>
__global__ void __launch_bounds__(256) k_radial_spline(int nmax, int64_t M, double inv_delta, const V4<T>* coef,
                                                       int64_t n_r, const double* r, T* I, T* dI)
{
    constexpr int LM1 = LMAX + 1;
    const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (q >= n_r) return;
    const int nl = nmax * LM1;
    const T rr = T(r[q]);
    int64_t k;
    T t;
    spline_locate<T>(M, T(inv_delta), rr, k, t);
    const V4<T>* cf = coef + k * nl;
    for (int j0 = 0; j0 < nl; j0 += 4) {
        V4<T> c4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c4[u] = cf[j0 + u < nl ? j0 + u : nl - 1];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (j0 + u < nl) {
                T v, dv;
                spline_poly<T>(c4[u].x, c4[u].y, c4[u].z, c4[u].w, t, T(inv_delta), v, dv);
                I[(j0 + u) * n_r + q] = v;
                if (dI) dI[(j0 + u) * n_r + q] = dv;
            }
        }
    }
}

// direct GTO: raw values of each n to the outputs, then S^{-1/2} applied in
// place per l (each lane reads back only what it wrote)
template <int LMAX>
__global__ void __launch_bounds__(256) k_radial_gto(rad::GtoTables tab, int64_t n_r, const double* r, double* I,
                                                    double* dI)
{
    constexpr int LM1 = LMAX + 1;
    const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (q >= n_r) return;
    const double rr = r[q];
    const int nmax = tab.nmax;
    for (int n = 0; n < nmax; ++n) {
        double v[LM1], dv[LM1];
        rad::gto_raw_n<LMAX>(tab, n, rr, v, dv);
#pragma unroll
        for (int l = 0; l < LM1; ++l) {
            I[(n * LM1 + l) * n_r + q] = v[l];
            if (dI) dI[(n * LM1 + l) * n_r + q] = dv[l];
        }
    }
    constexpr int kMaxN = 16;
#pragma unroll
    for (int l = 0; l < LM1; ++l) {
        double col[kMaxN], dcol[kMaxN];
        for (int m = 0; m < nmax; ++m) {
            col[m] = I[(m * LM1 + l) * n_r + q];
            dcol[m] = dI ? dI[(m * LM1 + l) * n_r + q] : 0.0;
        }
        for (int n = 0; n < nmax; ++n) {
            double s = 0.0, ds = 0.0;
            for (int m = 0; m < nmax; ++m) {
                s += tab.X[n * nmax + m] * col[m];
                ds += tab.X[n * nmax + m] * dcol[m];
            }
            I[(n * LM1 + l) * n_r + q] = s;
            if (dI) dI[(n * LM1 + l) * n_r + q] = ds;
        }
    }
}

template <int LMAX>
__global__ void __launch_bounds__(256) k_radial_dvr(rad::DvrTables tab, int64_t n_r, const double* r, double* I,
                                                    double* dI)
{
    constexpr int LM1 = LMAX + 1;
    const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (q >= n_r) return;
    const double rr = r[q];
    for (int n = 0; n < tab.nmax; ++n) {
        double v[LM1], dv[LM1];
        rad::dvr_n<LMAX>(tab, n, rr, v, dv);
#pragma unroll
        for (int l = 0; l < LM1; ++l) {
            I[(n * LM1 + l) * n_r + q] = v[l];
            if (dI) dI[(n * LM1 + l) * n_r + q] = dv[l];
        }
    }
}

template <typename T, int LM>
struct SplineFn {
    static hipError_t run(const RadialArgs& a, hipStream_t st)
    {
        const unsigned blocks = unsigned((a.n_r + 255) / 256);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_radial_spline<T, LM>), dim3(blocks), dim3(256), 0, st, a.nmax, a.M,
                           a.inv_delta, static_cast<const V4<T>*>(a.coef), a.n_r, a.r, static_cast<T*>(a.I),
                           static_cast<T*>(a.dI));
        return hipGetLastError();
    }
};

template <typename T, int LM>
struct ExactFn {
    static hipError_t run(const RadialArgs& a, hipStream_t st)
    {
        const unsigned blocks = unsigned((a.n_r + 255) / 256);
        if (a.basis == SOAP_RADIAL_DVR)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_radial_dvr<LM>), dim3(blocks), dim3(256), 0, st, a.dvr, a.n_r, a.r,
                               static_cast<double*>(a.I), static_cast<double*>(a.dI));
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_radial_gto<LM>), dim3(blocks), dim3(256), 0, st, a.gto, a.n_r, a.r,
                               static_cast<double*>(a.I), static_cast<double*>(a.dI));
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_radial(const RadialArgs& a, bool f64, hipStream_t stream)
{
    if (a.n_r == 0) return hipSuccess;
    if (a.exact) return by_degree<double, ExactFn>(a.lmax, a, stream);
    return f64 ? by_degree<double, SplineFn>(a.lmax, a, stream) : by_degree<float, SplineFn>(a.lmax, a, stream);
}

}  // namespace soap
