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
#include <type_traits>
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

// The same adjoint for FP32 with the plan held in LDS by persistent
// 512-lane work-groups, two per CU when their LDS allows.  A work-group
// loads and checks the plan once (row bounds, entry ranges: anything
// outside them is reported and contributes nothing) and lays it out again
// in LDS: each row padded to a multiple of four entries whose padding
// points at a zero after the gradient row, each entry packed as the LDS
// byte addresses of grad[q] and of c[partner, l^2].  A lane then takes
// whole rows (k, l) (at most two) and sums each row's 2l+1 outputs
// together: per entry one gradient value and the partner's 2l+1
// coefficients, read at immediate offsets, added in plan order as in the
// kernel above.  Rows go to lanes grouped by l and, within a group, sorted
// by entry count (groups alternately descending and ascending, so a wave
// that straddles two groups meets rows of similar length), so the lanes of
// a wave run loops of near-equal length; the wave unrolls the sum over m to
// the largest 2l+1 among its rows.  The sums stay in registers until every
// lane is done reading the centre's coefficients, then overwrite them in
// LDS and leave with 16-byte stores; the next centre's coefficients and
// gradient row are loaded into registers during the sums.  With no
// separate output buffer two work-groups fit a CU, so one computes while
// the other stages and stores.
constexpr int kRowThreads = 512;
constexpr int kTasksPerLane = 2;
constexpr int kPrefetch = 4;    // 16-byte vectors of c per lane held for the next centre
constexpr int kPrefetchG = 2;   // and of the gradient row

struct PlanLayout {
    int rows;                    // K (lmax + 1)
    int waves;                   // rows / 64, rounded up
    int64_t n_entries;           // 2 n_sel
    int64_t cap;                 // entries with each row padded to a multiple of four
    // c at offset 0; while the plan is built, the padded row bounds sit there
    size_t off_g, off_entries, off_tasks, off_wnm, total;
};

inline size_t round16(size_t v)
{
    return (v + 15) & ~size_t(15);
}

inline PlanLayout plan_layout(int K, int lmax, int64_t n_sel)
{
    PlanLayout P{};
    const size_t row_bytes = size_t(K) * (lmax + 1) * (lmax + 1) * sizeof(float);
    P.rows = K * (lmax + 1);
    P.waves = (P.rows + 63) / 64;
    P.n_entries = 2 * n_sel;
    P.cap = P.n_entries + 3 * int64_t(P.rows);
    size_t o = round16(std::max(row_bytes, size_t(P.rows) * 8));
    P.off_g = o; o += round16((size_t(n_sel) + 1) * sizeof(float));
    P.off_entries = o; o += round16(size_t(P.cap) * 4);
    P.off_tasks = o; o += size_t(P.rows) * 8;
    P.off_wnm = o; o += round16(size_t(P.waves) * 4);
    P.total = o;
    return P;
}

// the packed entries and tasks hold LDS byte addresses and entry indices
// in 16 bits; a lane holds the sums of at most kTasksPerLane rows
inline bool plan_fits(const PlanLayout& P, int K, int lmax, int64_t n_sel)
{
    return P.off_g + (size_t(n_sel) + 1) * sizeof(float) <= 65536 &&
           size_t(K) * (lmax + 1) * (lmax + 1) * sizeof(float) <= 65536 && P.cap <= 65535 &&
           P.rows <= kTasksPerLane * kRowThreads && P.total <= 160 * 1024 && lmax <= 12;
}

// the sums of one row into acc[0, NM), its loop over m unrolled to the
// wave's NM >= 2l+1
template <int NM, int NMAX>
__device__ __forceinline__ void row_sums(const unsigned char* lds, const uint4* __restrict__ ent4, int s0, int s1,
                                         float (&acc)[NMAX])
{
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[m] = 0.0f;
    for (int t = s0; t < s1; t += 4) {
        const uint4 q4 = ent4[t >> 2];
        const uint32_t qe[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float g = *reinterpret_cast<const float*>(lds + (qe[u] & 0xFFFFu));
            const float* cp = reinterpret_cast<const float*>(lds + (qe[u] >> 16));
#pragma unroll
            for (int m = 0; m < NM; ++m) acc[m] = fmaf(g, cp[m], acc[m]);
        }
    }
}

template <int NM, int NMAX>
__device__ __forceinline__ void row_sums_for(int nmw, const unsigned char* lds, const uint4* __restrict__ ent4,
                                             int s0, int s1, float (&acc)[NMAX])
{
    if constexpr (NM <= NMAX) {
        if (nmw <= NM) row_sums<NM, NMAX>(lds, ent4, s0, s1, acc);
        else row_sums_for<NM + 2, NMAX>(nmw, lds, ent4, s0, s1, acc);
    }
}

// NMAX >= 2 lmax + 1
template <int NMAX>
__global__ void __launch_bounds__(kRowThreads, 2) k_ps_selected_backward_rows(int64_t n, int K, int lmax,
                                                                              const float* __restrict__ c,
                                                                              int64_t n_sel,
                                                                              const float* __restrict__ grad,
                                                                              const int32_t* __restrict__ row_offsets,
                                                                              const int32_t* __restrict__ entries,
                                                                              float* __restrict__ grad_c,
                                                                              int32_t* status, PlanLayout P)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* cs = reinterpret_cast<float*>(smem_raw);
    float* gs = reinterpret_cast<float*>(smem_raw + P.off_g);
    uint32_t* ent = reinterpret_cast<uint32_t*>(smem_raw + P.off_entries);
    int2* bounds = reinterpret_cast<int2*>(smem_raw);   // until the first centre is staged
    uint2* tasks = reinterpret_cast<uint2*>(smem_raw + P.off_tasks);
    int32_t* wnm = reinterpret_cast<int32_t*>(smem_raw + P.off_wnm);
    const int L1 = lmax + 1, L2 = L1 * L1, KL2 = K * L2;
    const int tid = threadIdx.x;
    const uint32_t zero_g = uint32_t(P.off_g + size_t(n_sel) * sizeof(float));   // the zero after the gradient row
    // padded row starts and counts: an exclusive scan by the first wave, 64
    // rows at a time
    if (tid < 64) {
        int carry = 0;
        for (int r0 = 0; r0 < P.rows; r0 += 64) {
            const int r = r0 + tid;
            int pc = 0;
            if (r < P.rows) {
                const int t0 = row_offsets[r], t1 = row_offsets[r + 1];
                if (t0 < 0 || t1 < t0 || int64_t(t1) > P.n_entries) report(status, SOAP_EINVAL);
                else pc = min((t1 - t0 + 3) & ~3, 65536);   // more overruns the capacity; the sums stay in int
            }
            int inc = pc;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int up = __shfl_up(inc, d, 64);
                if (tid >= d) inc += up;
            }
            if (r < P.rows) bounds[r] = make_int2(carry + inc - pc, pc);
            carry += __shfl(inc, 63, 64);
        }
    }
    if (tid == 0) gs[n_sel] = 0.0f;
    __syncthreads();
    // row r = k (lmax+1) + l: its entries, then its place among the rows of
    // the same l (more entries first, ties by k) and its task
    const bool sorted = K <= 512;
    for (int r = tid; r < P.rows; r += kRowThreads) {
        const int k = r / L1, l = r - k * L1;
        int2 b = bounds[r];
        const int pc = b.y;   // as the other rows see it
        // rows that each pass the check can still overlap and overrun the
        // padded capacity when the offsets are not monotonic
        if (int64_t(b.x) + b.y > P.cap) {
            report(status, SOAP_EINVAL);
            b = make_int2(0, 0);
        }
        const int t0 = b.y > 0 ? row_offsets[r] : 0;
        const int cnt = b.y > 0 ? row_offsets[r + 1] - t0 : 0;
        for (int u = 0; u < b.y; ++u) {
            uint32_t e = zero_g;   // c address 0 for padding
            if (u < cnt) {
                const int q = entries[2 * (t0 + u)], partner = entries[2 * (t0 + u) + 1];
                if (q < 0 || q >= n_sel || partner < 0 || partner >= K) report(status, SOAP_EINVAL);
                else e = (uint32_t(P.off_g) + uint32_t(q) * 4u) | (uint32_t(partner * L2 + l * l) * 4u << 16);
            }
            ent[b.x + u] = e;
        }
        int rank = k;
        if (sorted) {
            rank = 0;
            for (int k2 = 0; k2 < K; ++k2) {
                const int pc2 = bounds[k2 * L1 + l].y;
                rank += (pc2 > pc || (pc2 == pc && k2 < k)) ? 1 : 0;
            }
        }
        const int grp = lmax - l;   // larger l first
        const int slot = grp * K + ((grp & 1) ? K - 1 - rank : rank);
        tasks[slot] = make_uint2(uint32_t(b.x) | (uint32_t(b.x + b.y) << 16),
                                 uint32_t((k * L2 + l * l) * 4) | (uint32_t(2 * l + 1) << 16));
    }
    __syncthreads();
    // the largest 2l+1 among each wave's rows
    for (int w = tid; w < P.waves; w += kRowThreads) {
        int mx = 1;
        for (int t = w * 64; t < min(w * 64 + 64, P.rows); ++t) mx = max(mx, int(tasks[t].y >> 16));
        wnm[w] = mx;
    }
    // rows of whole aligned 16-byte vectors go through registers; others directly
    typedef __attribute__((ext_vector_type(4))) float V;
    const bool vec_c = KL2 % 4 == 0 && KL2 / 4 <= kPrefetch * kRowThreads &&
                       (reinterpret_cast<uintptr_t>(c) & 15) == 0 && (reinterpret_cast<uintptr_t>(grad_c) & 15) == 0;
    const bool vec_g = n_sel % 4 == 0 && n_sel / 4 <= kPrefetchG * kRowThreads &&
                       (reinterpret_cast<uintptr_t>(grad) & 15) == 0;
    const int ncv = KL2 / 4, ngv = int(n_sel / 4);
    V pre[kPrefetch], preg[kPrefetchG];
    auto prefetch = [&](int64_t i) {
        if (vec_c) {
            const V* src = reinterpret_cast<const V*>(c + i * KL2);
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) {
                const int e = tid + u * kRowThreads;
                if (e < ncv) pre[u] = src[e];
            }
        }
        if (vec_g) {
            const V* src = reinterpret_cast<const V*>(grad + i * n_sel);
#pragma unroll
            for (int u = 0; u < kPrefetchG; ++u) {
                const int e = tid + u * kRowThreads;
                if (e < ngv) preg[u] = src[e];
            }
        }
    };
    const uint4* ent4 = reinterpret_cast<const uint4*>(ent);
    int64_t i = blockIdx.x;
    if (i < n) prefetch(i);
    for (; i < n; i += gridDim.x) {
        __syncthreads();   // the previous centre has left cs; the plan is built
        if (vec_c) {
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) {
                const int e = tid + u * kRowThreads;
                if (e < ncv) reinterpret_cast<V*>(cs)[e] = pre[u];
            }
        } else {
            for (int e = tid; e < KL2; e += kRowThreads) cs[e] = c[i * KL2 + e];
        }
        if (vec_g) {
#pragma unroll
            for (int u = 0; u < kPrefetchG; ++u) {
                const int e = tid + u * kRowThreads;
                if (e < ngv) reinterpret_cast<V*>(gs)[e] = preg[u];
            }
        } else {
            for (int64_t e = tid; e < n_sel; e += kRowThreads) gs[e] = grad[i * n_sel + e];
        }
        __syncthreads();
        if (i + gridDim.x < n) prefetch(i + gridDim.x);
        float acc[kTasksPerLane][NMAX];
#pragma unroll
        for (int j = 0; j < kTasksPerLane; ++j) {
            const int t = tid + j * kRowThreads;
            if (t < P.rows) {
                const uint2 tk = tasks[t];
                const int nmw = __builtin_amdgcn_readfirstlane(wnm[t >> 6]);
                row_sums_for<1, NMAX>(nmw, smem_raw, ent4, int(tk.x & 0xFFFFu), int(tk.x >> 16), acc[j]);
            }
        }
        __syncthreads();   // every read of this centre's coefficients is done
#pragma unroll
        for (int j = 0; j < kTasksPerLane; ++j) {
            const int t = tid + j * kRowThreads;
            if (t < P.rows) {
                const uint2 tk = tasks[t];
                const int nm = int(tk.y >> 16);
                float* orow = reinterpret_cast<float*>(smem_raw + (tk.y & 0xFFFFu));
#pragma unroll
                for (int m = 0; m < NMAX; ++m)
                    if (m < nm) orow[m] = acc[j][m];
            }
        }
        __syncthreads();
        float* gi = grad_c + i * KL2;
        if (vec_c) {
            for (int e = tid; e < ncv; e += kRowThreads)
                reinterpret_cast<V*>(gi)[e] = reinterpret_cast<const V*>(cs)[e];
        } else {
            for (int e = tid; e < KL2; e += kRowThreads) gi[e] = cs[e];
        }
    }
}

template <int NMAX>
hipError_t launch_rows(const PlanLayout& P, int per_cu, int cus, int64_t n, int K, int lmax, const void* c,
                       int64_t n_sel, const void* grad, const int32_t* row_offsets, const int32_t* entries,
                       void* grad_c, int32_t* status, hipStream_t stream)
{
    if (P.total > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ps_selected_backward_rows<NMAX>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(P.total));
        if (e != hipSuccess) return e;
    }
    const int64_t blocks = std::min<int64_t>(n, int64_t(cus) * per_cu);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ps_selected_backward_rows<NMAX>), dim3(unsigned(blocks)), dim3(kRowThreads),
                       P.total, stream, n, K, lmax, static_cast<const float*>(c), n_sel,
                       static_cast<const float*>(grad), row_offsets, entries, static_cast<float*>(grad_c), status, P);
    return hipGetLastError();
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
    // FP32: the plan in LDS, persistent work-groups (two per CU when they fit)
    if constexpr (std::is_same<T, float>::value) {
        const PlanLayout P = plan_layout(K, lmax, n_sel);
        int dev = 0, cus = 0;
        if (plan_fits(P, K, lmax, n_sel) && hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
            const int per_cu = int(std::min<size_t>(2, 160 * 1024 / P.total));
            const int nm = 2 * lmax + 1;
            if (nm <= 9)
                return launch_rows<9>(P, per_cu, cus, n, K, lmax, c, n_sel, grad, row_offsets, entries, grad_c,
                                      status, stream);
            if (nm <= 17)
                return launch_rows<17>(P, per_cu, cus, n, K, lmax, c, n_sel, grad, row_offsets, entries, grad_c,
                                       status, stream);
            return launch_rows<25>(P, per_cu, cus, n, K, lmax, c, n_sel, grad, row_offsets, entries, grad_c, status,
                                   stream);
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
