// Selected invariants (Sec. 4.H): for each centre and each chosen
// q = (k1, k2, l), the sum over m of c[k1, l^2 + m] c[k2, l^2 + m], m < 2l+1.
//
// One 256-lane work-group per centre stages the centre's K x (lmax+1)^2
// coefficients in LDS with coalesced loads, then lanes take the selected
// invariants in turn, so a centre's outputs leave as one contiguous row.
// The work per centre is sum over q of (2 l_q + 1) products instead of the
// full spectrum's (lmax+1)^2 K(K+1)/2.
#include "soap_internal.hpp"

namespace soap {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void report(int32_t* st, int v)
{
    if (st) *st = v;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_ps_selected(int K, int lmax, const T* __restrict__ c, int64_t n_sel,
                                                          const int32_t* __restrict__ sel, T* __restrict__ out,
                                                          int32_t* status)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* cs = reinterpret_cast<T*>(smem_raw);
    const int L2 = (lmax + 1) * (lmax + 1);
    const int KL2 = K * L2;
    const int64_t i = blockIdx.x;
    const T* ci = c + i * KL2;
    for (int e = threadIdx.x; e < KL2; e += kThreads) cs[e] = ci[e];
    __syncthreads();
    T* oi = out + i * n_sel;
    for (int64_t q = threadIdx.x; q < n_sel; q += kThreads) {
        const int k1 = sel[3 * q], k2 = sel[3 * q + 1], l = sel[3 * q + 2];
        if (k1 < 0 || k1 >= K || k2 < 0 || k2 >= K || l < 0 || l > lmax) {
            report(status, SOAP_EINVAL);
            oi[q] = T(0);
            continue;
        }
        const T* a = cs + k1 * L2 + l * l;
        const T* b = cs + k2 * L2 + l * l;
        T s = T(0);
        for (int m = 0; m <= 2 * l; ++m) s += a[m] * b[m];
        oi[q] = s;
    }
}

template <typename T>
hipError_t selected_t(int64_t n, int K, int lmax, const void* c, int64_t n_sel, const int32_t* sel, void* out,
                      int32_t* status, hipStream_t stream)
{
    const size_t lds = size_t(K) * (lmax + 1) * (lmax + 1) * sizeof(T);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ps_selected<T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ps_selected<T>), dim3(unsigned(n)), dim3(kThreads), lds, stream, K, lmax,
                       static_cast<const T*>(c), n_sel, sel, static_cast<T*>(out), status);
    return hipGetLastError();
}

}  // namespace

size_t power_spectrum_selected_lds(bool f64, int K, int lmax)
{
    return size_t(K) * (lmax + 1) * (lmax + 1) * (f64 ? 8 : 4);
}

hipError_t launch_power_spectrum_selected(bool f64, int64_t n, int K, int lmax, const void* c, int64_t n_sel,
                                          const int32_t* sel, void* out, int32_t* status, hipStream_t stream)
{
    if (n == 0 || n_sel == 0) return hipSuccess;
    return f64 ? selected_t<double>(n, K, lmax, c, n_sel, sel, out, status, stream)
               : selected_t<float>(n, K, lmax, c, n_sel, sel, out, status, stream);
}

}  // namespace soap
