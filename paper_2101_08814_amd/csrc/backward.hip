// Reverse mode (vector-Jacobian products) of the power spectrum and of the
// expansion with respect to the positions.
//
// Power spectrum (chain rule of Sec. 4.G): with W_l the packed upstream
// gradient of p_{i,l,.} unpacked into a symmetric K x K matrix whose
// diagonal is doubled,
//   dL/dc_{k,lm} = sum_k' W_{l,k k'} c_{k',lm}.
// One work-group per centre: W_l unpacked into full blocks in LDS when K is
// a multiple of 4 and they fit, else read from the packed triangle.
//
// Expansion (App. B Eq. energy-derivative): for pair q = (i, j, s)
//   g_q = dL/dr_ji = sum_{n,lm} G_{i,a_j,n,lm} [(f I~)'_nl Y_lm u + f I~_nl grad Y_lm],
// formed as a sum over lm after the sum over n,
// with G = dL/dc.  The per-pair factors are recomputed (the same LDS staging
// as the forward pass) instead of being stored: the model-side sum is
// contracted first, as the paper recommends for forces.  Then
//   dL/dr_k = sum_{q: j_q = k} g_q - sum_{q of centre k} g_q,
// and because the full neighbour list holds (j, i, -s) for every (i, j, s),
// the first sum runs over the centre's own pairs through pair_transpose:
// each atom adds its terms in a fixed order, with no atomics.
#include "chunk.hpp"

namespace soap {
namespace {

using namespace dev;

template <typename T>
__global__ void __launch_bounds__(kThreads) k_ps_backward(FeatureArgs a, const T* grad_p, T* grad_c, bool all)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const Dims d = make_dims(a.S, a.nmax, a.lmax);
    const int KL2 = d.K * d.L2;
    T* c = sm;            // [K][L2]
    T* w = c + KL2;       // packed W_l: of every l at once when `all`, else of one l at a time
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    const int PL = (d.lmax + 1) * d.KK;
    const T* gp = grad_p + i * int64_t(PL);
    copy_in(c, static_cast<const T*>(a.coeffs) + i * KL2, KL2);
    T* g_out = grad_c + i * KL2;
    const int K = d.K;
    if (all) {
        copy_in(w, gp, PL);
        __syncthreads();
        // one lane per (k, lm), lm over every l
        for (int t = tid; t < K * d.L2; t += kThreads) {
            const int k = t / d.L2, lm = t - k * d.L2;
            const T* wl = w + l_of(lm) * d.KK;
            T acc = T(0);
            for (int kp = 0; kp < K; ++kp) {
                int lo = k < kp ? k : kp, hi = k < kp ? kp : k;
                T wv = wl[lo * K - lo * (lo - 1) / 2 + (hi - lo)];
                if (kp == k) wv += wv;
                acc += wv * c[kp * d.L2 + lm];
            }
            g_out[t] = acc;
        }
        return;
    }
    for (int l = 0; l <= d.lmax; ++l) {
        __syncthreads();
        copy_in(w, gp + l * d.KK, d.KK);
        __syncthreads();
        const int nm = 2 * l + 1;
        for (int t = tid; t < K * nm; t += kThreads) {
            int k = t / nm, m = t - k * nm;
            T acc = T(0);
            for (int kp = 0; kp < K; ++kp) {
                int lo = k < kp ? k : kp, hi = k < kp ? kp : k;
                T wv = w[lo * K - lo * (lo - 1) / 2 + (hi - lo)];
                if (kp == k) wv += wv;
                acc += wv * c[kp * d.L2 + l * l + m];
            }
            g_out[k * d.L2 + l * l + m] = acc;
        }
    }
}

// The same product with W_l unpacked once into a full symmetric K x K
// block per l (diagonal doubled) and each lane forming four channels
// k..k+3 of one lm: per k' one 4-wide read of row k' of W_l (the rows are
// the columns: W_l is symmetric) and one read of c, four FMAs.  K is a
// multiple of 4; c, the packed gradient and the blocks fit 64 KB.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_ps_backward_full(FeatureArgs a, const T* grad_p, T* grad_c)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Dims d = make_dims(a.S, a.nmax, a.lmax);
    const int K = d.K, L2 = d.L2, lm1 = d.lm1, KK = d.KK, KL2 = K * L2, PL = lm1 * KK;
    T* wf = reinterpret_cast<T*>(smem_raw);        // [lm1][K][K]
    T* c = wf + lm1 * K * K;                        // [K][L2]
    T* wp = c + KL2;                                // packed [lm1][KK]
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    copy_in(c, static_cast<const T*>(a.coeffs) + i * KL2, KL2);
    copy_in(wp, grad_p + i * int64_t(PL), PL);
    __syncthreads();
    // one thread per row (l, k1) of the full blocks
    for (int row = tid; row < lm1 * K; row += kThreads) {
        const int l = row / K, k1 = row - l * K;
        const T* src = wp + l * KK;
        T* dst = wf + row * K;
        for (int k2 = 0; k2 < K; ++k2) {
            const int lo = k1 < k2 ? k1 : k2, hi = k1 < k2 ? k2 : k1;
            const T v = src[lo * K - lo * (lo - 1) / 2 + (hi - lo)];
            dst[k2] = k2 == k1 ? v + v : v;
        }
    }
    __syncthreads();
    T* g_out = grad_c + i * KL2;
    const int KB = K / 4;
    for (int t = tid; t < KB * L2; t += kThreads) {
        const int kb = t / L2, lm = t - kb * L2, k = 4 * kb;
        const T* Wl = wf + l_of(lm) * K * K + k;
        T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
        for (int kp = 0; kp < K; ++kp) {
            const V4<T> w = *reinterpret_cast<const V4<T>*>(Wl + kp * K);
            const T cv = c[kp * L2 + lm];
            a0 += w.x * cv;
            a1 += w.y * cv;
            a2 += w.z * cv;
            a3 += w.w * cv;
        }
        g_out[k * L2 + lm] = a0;
        g_out[(k + 1) * L2 + lm] = a1;
        g_out[(k + 2) * L2 + lm] = a2;
        g_out[(k + 3) * L2 + lm] = a3;
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_exp_backward_pairs(FeatureArgs a, Layout L, const T* grad_c,
                                                                 T* grad_pair)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* base = reinterpret_cast<T*>(smem_raw);
    Smem<T> s(base, L);
    const Dims d = make_dims(a.S, a.nmax, a.lmax);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t i = blockIdx.x;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (tid == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    const int KL2 = d.K * d.L2, nL2 = d.nmax * d.L2, lm1 = d.lmax + 1;
    const int chunk = L.chunk;
    init_tables<T>(a, d, L, s);
    const T* g_in = grad_c + i * KL2;
    copy_in(s.c, g_in, KL2);   // the c slot holds dL/dc here
    const int64_t q_begin = a.pair_offsets[i], q_end = a.pair_offsets[i + 1];
    const int n_chunks = int((q_end - q_begin + chunk - 1) / chunk);
    for (int ck = 0; ck < n_chunks; ++ck) {
        int64_t q0 = q_begin + int64_t(ck) * chunk;
        int nc = int(q_end - q0 < chunk ? q_end - q0 : chunk);
        stage_chunk<T, true>(a, d, s, q0, nc);
        for (int p = wave; p < nc; p += kWaves) {
            // g = u sum_lm Y_lm A_lm + sum_lm grad Y_lm B_lm with
            // {A, B}_lm = sum_n G_{n,lm} {(f I~)'_nl, f I~_nl}: one lane per lm
            const T* G = s.c + s.spc[p] * nL2;
            const T* Rp = s.R + p * d.nl;
            const T* dRp = s.dR + p * d.nl;
            T gx = T(0), gy = T(0), gz = T(0);
            for (int lm = lane; lm < d.L2; lm += 64) {
                const int l = s.lof[lm];
                T A = T(0), B = T(0);
                for (int n = 0; n < d.nmax; ++n) {
                    const T Gv = G[n * d.L2 + lm];
                    A += Gv * dRp[n * lm1 + l];
                    B += Gv * Rp[n * lm1 + l];
                }
                const V4<T> yd = s.YD[p * d.L2 + lm];
                const T t = A * yd.x;
                gx += t * s.ux[p] + B * yd.y;
                gy += t * s.uy[p] + B * yd.z;
                gz += t * s.uz[p] + B * yd.w;
            }
            gx = wave_sum(gx);
            gy = wave_sum(gy);
            gz = wave_sum(gz);
            if (lane == 0) {
                int64_t q = q0 + p;
                grad_pair[3 * q] = gx;
                grad_pair[3 * q + 1] = gy;
                grad_pair[3 * q + 2] = gz;
            }
        }
        __syncthreads();
    }
}

// one wave per atom k: lanes over its pairs, then a fixed reduction tree
// (deterministic; no atomics)
template <typename T>
__global__ void __launch_bounds__(256) k_exp_backward_gather(FeatureArgs a, const int32_t* transpose,
                                                             const T* grad_pair, T* grad_pos)
{
    const int lane = threadIdx.x & 63;
    const int64_t k = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (k >= a.n_atoms) return;
    T gx = T(0), gy = T(0), gz = T(0);
    if (a.pair_offsets[a.n_atoms] <= a.pair_capacity) {
        const int64_t q0 = a.pair_offsets[k], q1 = a.pair_offsets[k + 1];
        for (int64_t q = q0 + lane; q < q1; q += 64) {
            const int32_t t = transpose[q];
            const T ox = grad_pair[3 * q], oy = grad_pair[3 * q + 1], oz = grad_pair[3 * q + 2];
            if (t < 0 || t >= a.pair_capacity) { put_status(a.status, SOAP_EGEOMETRY); continue; }
            gx += grad_pair[3 * int64_t(t)] - ox;
            gy += grad_pair[3 * int64_t(t) + 1] - oy;
            gz += grad_pair[3 * int64_t(t) + 2] - oz;
        }
    }
    gx = wave_sum(gx);
    gy = wave_sum(gy);
    gz = wave_sum(gz);
    if (lane == 0) {
        grad_pos[3 * k] = gx;
        grad_pos[3 * k + 1] = gy;
        grad_pos[3 * k + 2] = gz;
    }
}

// Virial: per centre (one wave, lanes over its pairs) the nine sums
// g_a r_b, then per structure (one work-group, lanes over its centres) a
// fixed-order reduction of the centre sums.
template <typename T>
__global__ void __launch_bounds__(256) k_virial_centres(int64_t n_atoms, const int64_t* pair_offsets,
                                                        int64_t capacity, const T* vec, const T* g, T* part,
                                                        int32_t* status)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (i >= n_atoms) return;
    T acc[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) acc[e] = T(0);
    if (pair_offsets[n_atoms] <= capacity) {
        for (int64_t q = pair_offsets[i] + lane; q < pair_offsets[i + 1]; q += 64) {
            const T g0 = g[3 * q], g1 = g[3 * q + 1], g2 = g[3 * q + 2];
            const T r0 = vec[3 * q], r1 = vec[3 * q + 1], r2 = vec[3 * q + 2];
            acc[0] += g0 * r0; acc[1] += g0 * r1; acc[2] += g0 * r2;
            acc[3] += g1 * r0; acc[4] += g1 * r1; acc[5] += g1 * r2;
            acc[6] += g2 * r0; acc[7] += g2 * r1; acc[8] += g2 * r2;
        }
    } else if (lane == 0 && i == 0) {
        put_status(status, SOAP_ECAPACITY);
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const T v = wave_sum(acc[e]);
        if (lane == 0) part[9 * i + e] = v;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_virial_structures(const int64_t* atom_offsets, const T* part, T* out)
{
    __shared__ T red[9][256];
    const int s = blockIdx.x, t = threadIdx.x;
    const int64_t lo = atom_offsets[s], hi = atom_offsets[s + 1];
    T acc[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) acc[e] = T(0);
    for (int64_t i = lo + t; i < hi; i += 256)
#pragma unroll
        for (int e = 0; e < 9; ++e) acc[e] += part[9 * i + e];
#pragma unroll
    for (int e = 0; e < 9; ++e) red[e][t] = acc[e];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int e = 0; e < 9; ++e) red[e][t] += red[e][t + w];
        __syncthreads();
    }
    if (t < 9) out[9 * int64_t(s) + t] = red[t][0];
}

template <typename T>
hipError_t virial_t(int32_t n_structures, const int64_t* atom_offsets, int64_t n_atoms, const int64_t* pair_offsets,
                    const void* vec, const void* g, int64_t capacity, void* part, void* out, int32_t* status,
                    hipStream_t stream)
{
    if (n_atoms > 0)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_virial_centres<T>), dim3(unsigned((n_atoms + 3) / 4)), dim3(256), 0,
                           stream, n_atoms, pair_offsets, capacity, static_cast<const T*>(vec),
                           static_cast<const T*>(g), static_cast<T*>(part), status);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_virial_structures<T>), dim3(unsigned(n_structures)), dim3(256), 0, stream,
                       atom_offsets, static_cast<const T*>(part), static_cast<T*>(out));
    return hipGetLastError();
}

template <typename T>
hipError_t ps_backward_t(const FeatureArgs& a, const void* grad_p, void* grad_c, hipStream_t stream)
{
    Dims d = make_dims(a.S, a.nmax, a.lmax);
    const size_t full_lds =
        (size_t(d.lm1) * d.K * d.K + size_t(d.K) * d.L2 + size_t(d.lm1) * d.KK) * sizeof(T);
    if (d.K % 4 == 0 && full_lds <= 64 * 1024) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ps_backward_full<T>), dim3(unsigned(a.n_atoms)), dim3(kThreads),
                           full_lds, stream, a, static_cast<const T*>(grad_p), static_cast<T*>(grad_c));
        return hipGetLastError();
    }
    // the upstream gradient of every l in LDS at once when that fits 64 KB
    const size_t all_lds = (size_t(d.K) * d.L2 + size_t(d.lmax + 1) * d.KK) * sizeof(T);
    const bool all = all_lds <= 64 * 1024;
    size_t lds = all ? all_lds : (size_t(d.K) * d.L2 + size_t(d.KK)) * sizeof(T);
    if (lds > 160 * 1024) return hipErrorNotSupported;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ps_backward<T>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ps_backward<T>), dim3(unsigned(a.n_atoms)), dim3(kThreads), lds, stream, a,
                       static_cast<const T*>(grad_p), static_cast<T*>(grad_c), all);
    return hipGetLastError();
}

template <typename T>
hipError_t exp_backward_t(const FeatureArgs& a, const int32_t* transpose, const void* grad_c, void* grad_pair,
                          void* grad_pos, hipStream_t stream)
{
    Dims d = make_dims(a.S, a.nmax, a.lmax);
    const bool f64 = std::is_same<T, double>::value;
    // one lane per pair when dL/dc of a centre fits the wave's LDS, else the
    // LDS-staged kernel
    const bool lanes = expansion_backward_lanes_fits(a, f64);
    if (a.pair_capacity > 0 && lanes) {
        hipError_t e = launch_expansion_backward_lanes(a, f64, grad_c, grad_pair, stream);
        if (e != hipSuccess) return e;
    } else if (a.pair_capacity > 0) {
        Layout L = choose_layout<T>(d, true, false, false);
        if (L.total == 0) return hipErrorNotSupported;
        size_t lds = size_t(L.total) * sizeof(T);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_exp_backward_pairs<T>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_exp_backward_pairs<T>), dim3(unsigned(a.n_atoms)), dim3(kThreads), lds,
                           stream, a, L, static_cast<const T*>(grad_c), static_cast<T*>(grad_pair));
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_exp_backward_gather<T>), dim3(unsigned((a.n_atoms + 3) / 4)), dim3(256),
                       0, stream, a, transpose, static_cast<const T*>(grad_pair), static_cast<T*>(grad_pos));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_power_spectrum_backward(const FeatureArgs& a, bool f64, const void* grad_p, void* grad_coeffs,
                                          hipStream_t stream)
{
    return f64 ? ps_backward_t<double>(a, grad_p, grad_coeffs, stream)
               : ps_backward_t<float>(a, grad_p, grad_coeffs, stream);
}

hipError_t launch_virial(bool f64, int32_t n_structures, const int64_t* atom_offsets, int64_t n_atoms,
                         const int64_t* pair_offsets, const void* pair_vec, const void* grad_pair_vec,
                         int64_t capacity, void* partials, void* virial, int32_t* status, hipStream_t stream)
{
    return f64 ? virial_t<double>(n_structures, atom_offsets, n_atoms, pair_offsets, pair_vec, grad_pair_vec,
                                  capacity, partials, virial, status, stream)
               : virial_t<float>(n_structures, atom_offsets, n_atoms, pair_offsets, pair_vec, grad_pair_vec,
                                 capacity, partials, virial, status, stream);
}

hipError_t launch_expansion_backward(const FeatureArgs& a, bool f64, const int32_t* pair_transpose,
                                     const void* grad_coeffs, void* grad_pair_vec, void* grad_positions,
                                     hipStream_t stream)
{
    return f64 ? exp_backward_t<double>(a, pair_transpose, grad_coeffs, grad_pair_vec, grad_positions, stream)
               : exp_backward_t<float>(a, pair_transpose, grad_coeffs, grad_pair_vec, grad_positions, stream);
}

}  // namespace soap
