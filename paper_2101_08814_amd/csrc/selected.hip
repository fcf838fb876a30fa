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

#include <algorithm>
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

// The same adjoint with the plan held in LDS by persistent work-groups.
// A work-group loads and checks the plan once (row bounds, entry ranges:
// anything outside them is reported and contributes nothing) and lays it
// out again in LDS: every row padded to a multiple of four entries with
// entries that point at a zero after the gradient row, each entry packed
// as the byte offsets (q, partner row) of its two operands.  It then walks
// its centres i = blockIdx.x, blockIdx.x + gridDim.x, ..., the next
// centre's coefficients and gradient row prefetched into registers while
// the current one is summed.  Lane e = k L2 + lm reads its row's entries
// four at a time (one 16-byte LDS read; the 2l+1 lanes of a row read the
// same ones) and sums grad[q] c[partner, lm] in plan order, as the kernel
// above.
constexpr int kPrefetch = 8;   // 16-byte vectors of c per lane held for the next centre
constexpr int kPrefetchG = 4;  // and of the gradient row

struct PlanLayout {
    int rows;                  // K (lmax + 1)
    int64_t n_entries;         // 2 n_sel
    int64_t cap;               // entries with each row padded to a multiple of four
    size_t off_bounds, off_entries, off_c, off_g, total;
};

inline PlanLayout plan_layout(size_t es, int K, int lmax, int64_t n_sel)
{
    PlanLayout P{};
    P.rows = K * (lmax + 1);
    P.n_entries = 2 * n_sel;
    P.cap = P.n_entries + 3 * int64_t(P.rows);
    size_t o = 0;
    P.off_bounds = o; o += size_t(2 * P.rows) * 4;
    o = (o + 15) & ~size_t(15);
    P.off_entries = o; o += size_t(P.cap) * 4;
    o = (o + 15) & ~size_t(15);
    P.off_c = o; o += ((size_t(K) * (lmax + 1) * (lmax + 1) * es + 15) & ~size_t(15));
    P.off_g = o; o += (((size_t(n_sel) + 1) * es + 15) & ~size_t(15));
    P.total = o;
    return P;
}

// operand byte offsets fit 16 bits each
inline bool plan_packable(size_t es, int K, int lmax, int64_t n_sel)
{
    return (n_sel + 1) * int64_t(es) < 65536 && int64_t(K) * (lmax + 1) * (lmax + 1) * int64_t(es) < 65536;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_ps_selected_backward_plan(int64_t n, int K, int lmax,
                                                                        const T* __restrict__ c, int64_t n_sel,
                                                                        const T* __restrict__ grad,
                                                                        const int32_t* __restrict__ row_offsets,
                                                                        const int32_t* __restrict__ entries,
                                                                        T* __restrict__ grad_c, int32_t* status,
                                                                        PlanLayout P)
{
    typedef __attribute__((ext_vector_type(16 / sizeof(T)))) T V;
    constexpr int VW = 16 / sizeof(T);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int2* bounds = reinterpret_cast<int2*>(smem_raw + P.off_bounds);
    uint32_t* ent = reinterpret_cast<uint32_t*>(smem_raw + P.off_entries);
    T* cs = reinterpret_cast<T*>(smem_raw + P.off_c);
    T* gs = reinterpret_cast<T*>(smem_raw + P.off_g);
    const int L2 = (lmax + 1) * (lmax + 1);
    const int KL2 = K * L2;
    const int tid = threadIdx.x;
    const uint32_t none = uint32_t(n_sel) * uint32_t(sizeof(T));   // the zero after the gradient row
    // padded row starts: an exclusive scan of the padded counts by the
    // first wave, 64 rows at a time
    if (tid < 64) {
        int carry = 0;
        for (int r0 = 0; r0 < P.rows; r0 += 64) {
            const int r = r0 + tid;
            int pc = 0, t0 = 0, t1 = 0;
            if (r < P.rows) {
                t0 = row_offsets[r];
                t1 = row_offsets[r + 1];
                if (t0 < 0 || t1 < t0 || int64_t(t1) > P.n_entries) {
                    report(status, SOAP_EINVAL);
                    t0 = t1 = 0;
                }
                pc = (t1 - t0 + 3) & ~3;
            }
            int inc = pc;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int up = __shfl_up(inc, d, 64);
                if (tid >= d) inc += up;
            }
            if (r < P.rows) bounds[r] = make_int2(carry + inc - pc, t1 - t0);
            carry += __shfl(inc, 63, 64);
        }
    }
    __syncthreads();
    // entries: row r's go to [start, start + count), the rest of its padded
    // span points at the zero
    for (int r = tid; r < P.rows; r += kThreads) {
        const int2 b = bounds[r];
        const int t0 = b.y > 0 ? row_offsets[r] : 0;
        for (int u = 0; u < ((b.y + 3) & ~3); ++u) {
            uint32_t e = none;
            if (u < b.y) {
                const int q = entries[2 * (t0 + u)], partner = entries[2 * (t0 + u) + 1];
                if (q < 0 || q >= n_sel || partner < 0 || partner >= K) report(status, SOAP_EINVAL);
                else e = uint32_t(q) * uint32_t(sizeof(T)) | (uint32_t(partner * L2) * uint32_t(sizeof(T)) << 16);
            }
            ent[b.x + u] = e;
        }
        bounds[r] = make_int2(b.x, b.x + ((b.y + 3) & ~3));
    }
    if (tid == 0) gs[n_sel] = T(0);
    // rows of whole 16-byte vectors go through registers; others directly
    const bool vec_c = KL2 % VW == 0 && KL2 / VW <= kPrefetch * kThreads;
    const bool vec_g = n_sel % VW == 0 && n_sel / VW <= kPrefetchG * kThreads;
    const int ncv = KL2 / VW, ngv = int(n_sel / VW);
    V pre[kPrefetch], preg[kPrefetchG];
    auto prefetch = [&](int64_t i) {
        if (vec_c) {
            const V* src = reinterpret_cast<const V*>(c + i * KL2);
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) {
                const int e = tid + u * kThreads;
                if (e < ncv) pre[u] = src[e];
            }
        }
        if (vec_g) {
            const V* src = reinterpret_cast<const V*>(grad + i * n_sel);
#pragma unroll
            for (int u = 0; u < kPrefetchG; ++u) {
                const int e = tid + u * kThreads;
                if (e < ngv) preg[u] = src[e];
            }
        }
    };
    int64_t i = blockIdx.x;
    if (i < n) prefetch(i);
    const int step_k = kThreads / L2, step_lm = kThreads - step_k * L2;
    const unsigned char* gsb = reinterpret_cast<const unsigned char*>(gs);
    const unsigned char* csb = reinterpret_cast<const unsigned char*>(cs);
    for (; i < n; i += gridDim.x) {
        __syncthreads();   // the previous centre's sums are done with cs and gs
        if (vec_c) {
            V* dst = reinterpret_cast<V*>(cs);
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) {
                const int e = tid + u * kThreads;
                if (e < ncv) dst[e] = pre[u];
            }
        } else {
            for (int e = tid; e < KL2; e += kThreads) cs[e] = c[i * KL2 + e];
        }
        if (vec_g) {
            V* dst = reinterpret_cast<V*>(gs);
#pragma unroll
            for (int u = 0; u < kPrefetchG; ++u) {
                const int e = tid + u * kThreads;
                if (e < ngv) dst[e] = preg[u];
            }
        } else {
            for (int64_t e = tid; e < n_sel; e += kThreads) gs[e] = grad[i * n_sel + e];
        }
        __syncthreads();
        if (i + gridDim.x < n) prefetch(i + gridDim.x);
        int k = tid / L2, lm = tid - k * L2;
        T* gi = grad_c + i * KL2;
        for (int e = tid; e < KL2; e += kThreads) {
            // floor(sqrt(lm + 1/2)) is l for lm in [l^2, (l+1)^2)
            const int l = int(sqrtf(float(lm) + 0.5f));
            const int2 b = bounds[k * (lmax + 1) + l];
            const unsigned char* cl = csb + lm * int(sizeof(T));
            T sum = T(0);
            for (int t = b.x; t < b.y; t += 4) {
                const uint4 q4 = *reinterpret_cast<const uint4*>(ent + t);
                const uint32_t qe[4] = {q4.x, q4.y, q4.z, q4.w};
                T gv[4], cv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    gv[u] = *reinterpret_cast<const T*>(gsb + (qe[u] & 0xFFFFu));
                    cv[u] = *reinterpret_cast<const T*>(cl + (qe[u] >> 16));
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) sum += gv[u] * cv[u];
            }
            gi[e] = sum;
            lm += step_lm;
            k += step_k;
            if (lm >= L2) {
                lm -= L2;
                ++k;
            }
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
    // the plan in LDS when it fits beside one centre's rows with at least
    // two work-groups per CU
    const PlanLayout P = plan_layout(sizeof(T), K, lmax, n_sel);
    if (P.total <= 80 * 1024 && plan_packable(sizeof(T), K, lmax, n_sel)) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
            if (P.total > 65536) {
                hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ps_selected_backward_plan<T>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(P.total));
                if (e != hipSuccess) return e;
            }
            const int64_t per_cu = int64_t(160 * 1024 / P.total);
            const int64_t blocks = std::min<int64_t>(n, int64_t(cus) * per_cu);
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ps_selected_backward_plan<T>), dim3(unsigned(blocks)),
                               dim3(kThreads), P.total, stream, n, K, lmax, static_cast<const T*>(c), n_sel,
                               static_cast<const T*>(grad), row_offsets, entries, static_cast<T*>(grad_c), status, P);
            return hipGetLastError();
        }
    }
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
