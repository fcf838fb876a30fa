// Selected invariants (Sec. 4.H): for each centre and each chosen
// q = (k1, k2, l), the sum over m of c[k1, l^2 + m] c[k2, l^2 + m], m < 2l+1.
//
// One 256-lane work-group per centre stages the centre's K x (lmax+1)^2
// coefficients in LDS with coalesced loads, then lanes take the selected
// invariants in turn (eight per lane per round, their triples loaded
// together), so a centre's outputs leave as one contiguous row.
// The work per centre is sum over q of (2 l_q + 1) products instead of the
// full spectrum's (lmax+1)^2 K(K+1)/2.
#include "soap_internal.hpp"

#include <vector>

namespace soap {
namespace {

constexpr int kThreads = 256;
constexpr int kQBatch = 8;       // invariants per lane whose triples are loaded together
constexpr int kStageBatch = 8;   // coefficient loads per lane in flight

__device__ __forceinline__ void report(int32_t* st, int v)
{
    if (st) *st = v;
}

// copy n elements to LDS with kStageBatch 16-byte loads per lane in flight
// (scalar loads when the row is not a whole number of aligned vectors)
template <typename T>
__device__ __forceinline__ void stage(const T* __restrict__ src, T* dst, int n)
{
    typedef __attribute__((ext_vector_type(16 / sizeof(T)))) T V;
    constexpr int VW = 16 / sizeof(T);
    if (n % VW == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        const V* s = reinterpret_cast<const V*>(src);
        V* d = reinterpret_cast<V*>(dst);
        const int nv = n / VW;
        for (int e0 = threadIdx.x; e0 < nv; e0 += kStageBatch * kThreads) {
            V v[kStageBatch];
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) {
                const int e = e0 + u * kThreads;
                v[u] = s[e < nv ? e : nv - 1];
            }
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) {
                const int e = e0 + u * kThreads;
                if (e < nv) d[e] = v[u];
            }
        }
    } else {
        for (int e = threadIdx.x; e < n; e += kThreads) dst[e] = src[e];
    }
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
    T* oi = out + i * n_sel;
    stage(ci, cs, KL2);
    // the triples of kQBatch invariants per lane are loaded together (index
    // clamped, so no load waits behind a branch); the first batch is in
    // flight across the barrier
    int t1[kQBatch], t2[kQBatch], tl[kQBatch];
    auto load = [&](int64_t qb) {
#pragma unroll
        for (int u = 0; u < kQBatch; ++u) {
            const int64_t q = qb + int64_t(u) * kThreads;
            const int64_t qq = q < n_sel ? q : n_sel - 1;
            t1[u] = sel[3 * qq];
            t2[u] = sel[3 * qq + 1];
            tl[u] = sel[3 * qq + 2];
        }
    };
    int64_t qb = threadIdx.x;
    if (qb < n_sel) load(qb);
    __syncthreads();
    for (; qb < n_sel; qb += int64_t(kQBatch) * kThreads) {
#pragma unroll
        for (int u = 0; u < kQBatch; ++u) {
            const int64_t q = qb + int64_t(u) * kThreads;
            if (q >= n_sel) break;
            const int k1 = t1[u], k2 = t2[u], l = tl[u];
            if (k1 < 0 || k1 >= K || k2 < 0 || k2 >= K || l < 0 || l > lmax) {
                report(status, SOAP_EINVAL);
                oi[q] = T(0);
                continue;
            }
            const T* a = cs + k1 * L2 + l * l;
            const T* b = cs + k2 * L2 + l * l;
            T sum = T(0);
            for (int m = 0; m <= 2 * l; ++m) sum += a[m] * b[m];
            oi[q] = sum;
        }
        const int64_t next = qb + int64_t(kQBatch) * kThreads;
        if (next < n_sel) load(next);
    }
}

// dL/dc of one centre per work-group: coefficients and the centre's
// gradient row in LDS, the plan read through L2 (staging it in LDS as well
// halves the work-groups per CU and was measured slower); lane e = k L2 + lm
// sums, over the plan entries of row (k, l), grad[q] c[partner, lm] in plan
// order; lane steps carry (k, lm) forward and l comes from an LDS table.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_ps_selected_backward(int K, int lmax, const T* __restrict__ c,
                                                                   int64_t n_sel, const T* __restrict__ grad,
                                                                   const int32_t* __restrict__ row_offsets,
                                                                   const int32_t* __restrict__ entries,
                                                                   T* __restrict__ grad_c, int32_t* status)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L2 = (lmax + 1) * (lmax + 1);
    const int KL2 = K * L2;
    T* cs = reinterpret_cast<T*>(smem_raw);
    T* gs = cs + ((KL2 + 3) & ~3);
    int32_t* ltab = reinterpret_cast<int32_t*>(gs + ((n_sel + 3) & ~int64_t(3)));   // l of each lm
    const int64_t i = blockIdx.x;
    stage(c + i * KL2, cs, KL2);
    stage(grad + i * n_sel, gs, int(n_sel));
    for (int lm = threadIdx.x; lm < L2; lm += kThreads) {
        int l = 0;
        while ((l + 1) * (l + 1) <= lm) ++l;
        ltab[lm] = l;
    }
    __syncthreads();
    // e = k L2 + lm advances by kThreads per step: (k, lm) is carried
    // forward instead of divided out again
    const int step_k = kThreads / L2, step_lm = kThreads - step_k * L2;
    int k = int(threadIdx.x) / L2, lm = int(threadIdx.x) - k * L2;
    T* gi = grad_c + i * KL2;
    for (int e = threadIdx.x; e < KL2; e += kThreads) {
        const int l = ltab[lm];
        const int r = k * (lmax + 1) + l;
        T s = T(0);
        const int t0 = row_offsets[r], t1 = row_offsets[r + 1];
        if (t0 < 0 || t1 < t0 || int64_t(t1) > 2 * n_sel) {   // not a plan of these triples
            report(status, SOAP_EINVAL);
        } else {
            for (int t = t0; t < t1; ++t) {
                const int q = entries[2 * t], partner = entries[2 * t + 1];
                if (q < 0 || q >= n_sel || partner < 0 || partner >= K) {
                    report(status, SOAP_EINVAL);
                    continue;
                }
                s += gs[q] * cs[partner * L2 + lm];
            }
        }
        gi[e] = s;
        lm += step_lm;
        k += step_k;
        if (lm >= L2) {
            lm -= L2;
            ++k;
        }
    }
}

// LDS bytes: coefficients, gradient row, table of l per lm
size_t backward_lds(size_t es, int K, int lmax, int64_t n_sel)
{
    const size_t KL2 = size_t(K) * (lmax + 1) * (lmax + 1);
    const size_t L2 = size_t(lmax + 1) * (lmax + 1);
    return (((KL2 + 3) & ~size_t(3)) + ((size_t(n_sel) + 3) & ~size_t(3))) * es + L2 * 4;
}

template <typename T>
hipError_t selected_backward_t(int64_t n, int K, int lmax, const void* c, int64_t n_sel, const void* grad,
                               const int32_t* row_offsets, const int32_t* entries, void* grad_c, int32_t* status,
                               hipStream_t stream)
{
    const size_t lds = backward_lds(sizeof(T), K, lmax, n_sel);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ps_selected_backward<T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ps_selected_backward<T>), dim3(unsigned(n)), dim3(kThreads), lds, stream, K,
                       lmax, static_cast<const T*>(c), n_sel, static_cast<const T*>(grad), row_offsets, entries,
                       static_cast<T*>(grad_c), status);
    return hipGetLastError();
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

size_t power_spectrum_selected_backward_lds(bool f64, int K, int lmax, int64_t n_sel)
{
    return backward_lds(f64 ? 8 : 4, K, lmax, n_sel);
}

void selected_backward_plan(int K, int lmax, int64_t n_sel, const int32_t* selected, int32_t* row_offsets,
                            int32_t* entries)
{
    // counting sort of the 2 n_sel (row, q, partner) entries by row, q order
    // kept within a row; row = k (lmax + 1) + l
    const int rows = K * (lmax + 1);
    for (int r = 0; r <= rows; ++r) row_offsets[r] = 0;
    for (int64_t q = 0; q < n_sel; ++q) {
        const int k1 = selected[3 * q], k2 = selected[3 * q + 1], l = selected[3 * q + 2];
        ++row_offsets[k1 * (lmax + 1) + l + 1];
        ++row_offsets[k2 * (lmax + 1) + l + 1];
    }
    for (int r = 0; r < rows; ++r) row_offsets[r + 1] += row_offsets[r];
    std::vector<int32_t> fill(row_offsets, row_offsets + rows);
    for (int64_t q = 0; q < n_sel; ++q) {
        const int k1 = selected[3 * q], k2 = selected[3 * q + 1], l = selected[3 * q + 2];
        int32_t t = fill[k1 * (lmax + 1) + l]++;
        entries[2 * t] = int32_t(q);
        entries[2 * t + 1] = k2;
        t = fill[k2 * (lmax + 1) + l]++;
        entries[2 * t] = int32_t(q);
        entries[2 * t + 1] = k1;
    }
}

hipError_t launch_power_spectrum_selected_backward(bool f64, int64_t n, int K, int lmax, const void* c,
                                                   int64_t n_sel, const void* grad, const int32_t* row_offsets,
                                                   const int32_t* entries, void* grad_c, int32_t* status,
                                                   hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    return f64 ? selected_backward_t<double>(n, K, lmax, c, n_sel, grad, row_offsets, entries, grad_c, status, stream)
               : selected_backward_t<float>(n, K, lmax, c, n_sel, grad, row_offsets, entries, grad_c, status, stream);
}

hipError_t launch_power_spectrum_selected(bool f64, int64_t n, int K, int lmax, const void* c, int64_t n_sel,
                                          const int32_t* sel, void* out, int32_t* status, hipStream_t stream)
{
    if (n == 0 || n_sel == 0) return hipSuccess;
    return f64 ? selected_t<double>(n, K, lmax, c, n_sel, sel, out, status, stream)
               : selected_t<float>(n, K, lmax, c, n_sel, sel, out, status, stream);
}

}  // namespace soap
