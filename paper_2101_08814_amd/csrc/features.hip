// Spherical expansion, power spectrum and forward-mode gradient rows.
//
// One work-group of 256 lanes owns one centre i.  Its pairs are staged in
// chunks of up to kChunk pairs through LDS:
//   stage   - per pair: unit vector, 1/r, f_cut, f'_cut, species of j
//             (one lane per pair); the Qt table and (x + i y)^m (one lane per
//             (pair, m)); Y_lm and its gradient (one lane per (pair, lm)) and
//             the splined radial integral f I~_nl and (f I~_nl)' (one lane per
//             (pair, n, l)).  Nothing per pair touches HBM except pair_vec
//             and the species of j; the spline table is L2-resident.
//   combine - c_{a,n,lm} += sum over the chunk's pairs of species a of
//             R_nl Y_lm (Sec. 4.A, 4.F); each output element is owned by one
//             lane, so no atomics, and pairs sorted by species make the loop
//             run only over the pairs that contribute.
// With gradients the same loop accumulates the self row
//   d c_i / d r_i = -sum_q [(f I~)' Y u + f I~ grad Y]
// (App. B: d r_ji / d r_i = -1).  After the last chunk c, p and the self
// rows are written with consecutive lanes on consecutive addresses.
//
// Gradient rows (Sec. 4.G) then take one wave per pair.  The product rule
//   dp_{x,l,k1 k2} = sum_m dc_{x,k1,lm} c_{k2,lm} + c_{k1,lm} dc_{x,k2,lm}
// is summed in the reordered form
//   sum_m dc_{x,(a_j,n),lm} c_{k,lm} = (f I~)'_nl u_x y_{l,k} + f I~_nl z_{x,l,k},
//   y_{l,k} = sum_m Y_lm c_{k,lm},  z_{x,l,k} = sum_m dY_{x,lm} c_{k,lm},
// so a row costs O(K L2) instead of O(K^2 L2) and the dc row is written to
// memory but never read back.
#include "chunk.hpp"

namespace soap {
namespace {

using namespace dev;

template <typename T, bool GRAD, bool WANT_P>
__global__ void __launch_bounds__(kThreads) k_features(FeatureArgs a, int chunk, Layout L)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* base = reinterpret_cast<T*>(smem_raw);
    Smem<T> s(base, L);
    const Dims d = make_dims(a.S, a.nmax, a.lmax);
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (tid == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    const int64_t q_begin = a.pair_offsets[i], q_end = a.pair_offsets[i + 1];
    const int n_pairs = int(q_end - q_begin);
    const int n_chunks = (n_pairs + chunk - 1) / chunk;
    const int KL2 = d.K * d.L2;
    const int nL2 = d.nmax * d.L2;
    for (int e = tid; e < KL2; e += kThreads) {
        s.c[e] = T(0);
        if (GRAD) { s.dcs[e] = T(0); s.dcs[KL2 + e] = T(0); s.dcs[2 * KL2 + e] = T(0); }
    }
    // ---------------------------------------------------- expansion
    for (int ck = 0; ck < n_chunks; ++ck) {
        int64_t q0 = q_begin + int64_t(ck) * chunk;
        int nc = int(q_end - q0 < chunk ? q_end - q0 : chunk);
        stage_chunk<T, GRAD>(a, d, s, q0, nc);
        for (int e = tid; e < KL2; e += kThreads) {
            int sp = e / nL2, rem = e - sp * nL2, n = rem / d.L2, lm = rem - n * d.L2;
            int l = dev::l_of(lm);
            int rl = n * (d.lmax + 1) + l;
            T acc = s.c[e];
            T g0 = T(0), g1 = T(0), g2 = T(0);
            int p0 = s.seg[2 * sp], p1 = s.seg[2 * sp + 1];
            for (int p = p0; p < p1; ++p) {
                if (s.spc[p] != sp) continue;
                T Rv = s.R[p * d.nl + rl], Yv = s.Y[p * d.L2 + lm];
                acc += Rv * Yv;
                if (GRAD) {
                    T t = s.dR[p * d.nl + rl] * Yv;
                    g0 += t * s.ux[p] + Rv * s.dY[(p * 3 + 0) * d.L2 + lm];
                    g1 += t * s.uy[p] + Rv * s.dY[(p * 3 + 1) * d.L2 + lm];
                    g2 += t * s.uz[p] + Rv * s.dY[(p * 3 + 2) * d.L2 + lm];
                }
            }
            s.c[e] = acc;
            if (GRAD) { s.dcs[e] -= g0; s.dcs[KL2 + e] -= g1; s.dcs[2 * KL2 + e] -= g2; }
        }
        if (ck + 1 < n_chunks) __syncthreads();
    }
    __syncthreads();
    if (a.include_center && tid < d.nmax) {
        int sp = a.species[i];
        if (sp >= 0 && sp < d.S) s.c[(sp * d.nmax + tid) * d.L2] += static_cast<const T*>(a.center)[tid];
        else put_status(a.status, SOAP_ESPECIES);
    }
    __syncthreads();
    T* c_out = static_cast<T*>(a.coeffs) + i * KL2;
    for (int e = tid; e < KL2; e += kThreads) c_out[e] = s.c[e];
    if (GRAD) {
        T* dcs_out = static_cast<T*>(a.dcoeffs_self) + i * 3 * KL2;
        for (int e = tid; e < 3 * KL2; e += kThreads) dcs_out[e] = s.dcs[e];
    }
    // ---------------------------------------------------- power spectrum
    const int lm1 = d.lmax + 1;
    const int64_t PL = int64_t(lm1) * d.KK;
    if (WANT_P) {
        T* p_out = static_cast<T*>(a.p) + i * PL;
        for (int64_t o = tid; o < PL; o += kThreads) {
            int l = int(o / d.KK);
            int kk = int(o - int64_t(l) * d.KK);
            int k1, k2;
            dev::tri_decode(d.K, kk, k1, k2);
            const T* c1 = s.c + k1 * d.L2 + l * l;
            const T* c2 = s.c + k2 * d.L2 + l * l;
            T acc = T(0);
            for (int m = 0; m < 2 * l + 1; ++m) acc += c1[m] * c2[m];
            p_out[o] = acc;
        }
        if (GRAD) {
            T* dps_out = static_cast<T*>(a.dp_self) + i * 3 * PL;
            for (int64_t o = tid; o < 3 * PL; o += kThreads) {
                int x = int(o / PL);
                int64_t r0 = o - x * PL;
                int l = int(r0 / d.KK);
                int kk = int(r0 - int64_t(l) * d.KK);
                int k1, k2;
                dev::tri_decode(d.K, kk, k1, k2);
                const T* c1 = s.c + k1 * d.L2 + l * l;
                const T* c2 = s.c + k2 * d.L2 + l * l;
                const T* g1 = s.dcs + x * KL2 + k1 * d.L2 + l * l;
                const T* g2 = s.dcs + x * KL2 + k2 * d.L2 + l * l;
                T acc = T(0);
                for (int m = 0; m < 2 * l + 1; ++m) acc += g1[m] * c2[m] + c1[m] * g2[m];
                dps_out[o] = acc;
            }
        }
    }
    if (!GRAD) return;
    // ---------------------------------------------------- gradient rows
    const int wave = tid >> 6, lane = tid & 63;
    T* yz = s.yz + wave * 4 * lm1 * d.K;
    const int yzn = lm1 * d.K;
    for (int ck = n_chunks - 1; ck >= 0; --ck) {
        int64_t q0 = q_begin + int64_t(ck) * chunk;
        int nc = int(q_end - q0 < chunk ? q_end - q0 : chunk);
        if (ck != n_chunks - 1) {
            __syncthreads();
            stage_chunk<T, GRAD>(a, d, s, q0, nc);
        }
        for (int p = wave; p < nc; p += kWaves) {
            const int64_t q = q0 + p;
            const T ux = s.ux[p], uy = s.uy[p], uz = s.uz[p];
            const int blk = s.spc[p] * d.nmax;
            if (WANT_P) {
                for (int t = lane; t < 4 * yzn; t += 64) {
                    int comp = t / yzn, rem = t - comp * yzn, l = rem / d.K, k = rem - l * d.K;
                    const T* src = comp == 0 ? s.Y + p * d.L2 : s.dY + (p * 3 + comp - 1) * d.L2;
                    const T* ck_ = s.c + k * d.L2 + l * l;
                    src += l * l;
                    T acc = T(0);
                    for (int m = 0; m < 2 * l + 1; ++m) acc += src[m] * ck_[m];
                    yz[t] = acc;
                }
                wave_sync();
            }
            T* dc_row = static_cast<T*>(a.dcoeffs) + q * 3 * nL2;
            for (int e = lane; e < 3 * nL2; e += 64) {
                int x = e / nL2, rem = e - x * nL2, n = rem / d.L2, lm = rem - n * d.L2;
                int rl = n * lm1 + dev::l_of(lm);
                T u = x == 0 ? ux : (x == 1 ? uy : uz);
                dc_row[e] = s.dR[p * d.nl + rl] * u * s.Y[p * d.L2 + lm] + s.R[p * d.nl + rl] * s.dY[(p * 3 + x) * d.L2 + lm];
            }
            if (WANT_P) {
                T* dp_row = static_cast<T*>(a.dp) + q * 3 * PL;
                for (int64_t o = lane; o < 3 * PL; o += 64) {
                    int x = int(o / PL);
                    int64_t r0 = o - x * PL;
                    int l = int(r0 / d.KK);
                    int kk = int(r0 - int64_t(l) * d.KK);
                    int k1, k2;
                    dev::tri_decode(d.K, kk, k1, k2);
                    T u = x == 0 ? ux : (x == 1 ? uy : uz);
                    const T* y = yz + l * d.K;
                    const T* z = yz + (1 + x) * yzn + l * d.K;
                    T v = T(0);
                    int n1 = k1 - blk, n2 = k2 - blk;
                    if (n1 >= 0 && n1 < d.nmax)
                        v += s.dR[p * d.nl + n1 * lm1 + l] * u * y[k2] + s.R[p * d.nl + n1 * lm1 + l] * z[k2];
                    if (n2 >= 0 && n2 < d.nmax)
                        v += s.dR[p * d.nl + n2 * lm1 + l] * u * y[k1] + s.R[p * d.nl + n2 * lm1 + l] * z[k1];
                    dp_row[o] = v;
                }
                wave_sync();
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Power spectrum (and forward-mode rows) from coefficients in memory.
// ---------------------------------------------------------------------------
template <typename T, bool GRAD>
__global__ void __launch_bounds__(kThreads) k_power_spectrum(FeatureArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const Dims d = make_dims(a.S, a.nmax, a.lmax);
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    const int KL2 = d.K * d.L2, nL2 = d.nmax * d.L2, lm1 = d.lmax + 1;
    const int64_t PL = int64_t(lm1) * d.KK;
    T* c = sm;                 // [K][L2]
    T* g = c + KL2;            // [3][K][L2] self row, then per-wave row buffers
    const T* c_in = static_cast<const T*>(a.coeffs) + i * KL2;
    for (int e = tid; e < KL2; e += kThreads) c[e] = c_in[e];
    if (GRAD) {
        const T* g_in = static_cast<const T*>(a.dcoeffs_self) + i * 3 * KL2;
        for (int e = tid; e < 3 * KL2; e += kThreads) g[e] = g_in[e];
    }
    __syncthreads();
    T* p_out = static_cast<T*>(a.p) + i * PL;
    for (int64_t o = tid; o < PL; o += kThreads) {
        int l = int(o / d.KK);
        int kk = int(o - int64_t(l) * d.KK);
        int k1, k2;
        dev::tri_decode(d.K, kk, k1, k2);
        const T* c1 = c + k1 * d.L2 + l * l;
        const T* c2 = c + k2 * d.L2 + l * l;
        T acc = T(0);
        for (int m = 0; m < 2 * l + 1; ++m) acc += c1[m] * c2[m];
        p_out[o] = acc;
    }
    if (!GRAD) return;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (tid == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    T* dps_out = static_cast<T*>(a.dp_self) + i * 3 * PL;
    for (int64_t o = tid; o < 3 * PL; o += kThreads) {
        int x = int(o / PL);
        int64_t r0 = o - x * PL;
        int l = int(r0 / d.KK);
        int kk = int(r0 - int64_t(l) * d.KK);
        int k1, k2;
        dev::tri_decode(d.K, kk, k1, k2);
        const T* c1 = c + k1 * d.L2 + l * l;
        const T* c2 = c + k2 * d.L2 + l * l;
        const T* g1 = g + x * KL2 + k1 * d.L2 + l * l;
        const T* g2 = g + x * KL2 + k2 * d.L2 + l * l;
        T acc = T(0);
        for (int m = 0; m < 2 * l + 1; ++m) acc += g1[m] * c2[m] + c1[m] * g2[m];
        dps_out[o] = acc;
    }
    __syncthreads();
    // rows: one wave per pair; w[x][l][n][k] = sum_m dc_{x,n,lm} c_{k,lm}
    const int wave = tid >> 6, lane = tid & 63;
    const int wn = 3 * lm1 * d.nmax * d.K;
    T* row = g + wave * (3 * nL2 + wn);
    T* w = row + 3 * nL2;
    const int64_t q_begin = a.pair_offsets[i], q_end = a.pair_offsets[i + 1];
    for (int64_t q = q_begin + wave; q < q_end; q += kWaves) {
        const T* dc_in = static_cast<const T*>(a.dcoeffs) + q * 3 * nL2;
        for (int e = lane; e < 3 * nL2; e += 64) row[e] = dc_in[e];
        int jq = a.pair_j[q];
        int sp = (jq >= 0 && jq < a.n_atoms) ? a.species[jq] : -1;
        if (sp < 0 || sp >= d.S) { put_status(a.status, SOAP_ESPECIES); sp = 0; }
        const int blk = sp * d.nmax;
        wave_sync();
        for (int t = lane; t < wn; t += 64) {
            int x = t / (lm1 * d.nmax * d.K);
            int rem = t - x * lm1 * d.nmax * d.K;
            int l = rem / (d.nmax * d.K);
            rem -= l * d.nmax * d.K;
            int n = rem / d.K, k = rem - n * d.K;
            const T* r1 = row + x * nL2 + n * d.L2 + l * l;
            const T* c2 = c + k * d.L2 + l * l;
            T acc = T(0);
            for (int m = 0; m < 2 * l + 1; ++m) acc += r1[m] * c2[m];
            w[t] = acc;
        }
        wave_sync();
        T* dp_row = static_cast<T*>(a.dp) + q * 3 * PL;
        for (int64_t o = lane; o < 3 * PL; o += 64) {
            int x = int(o / PL);
            int64_t r0 = o - x * PL;
            int l = int(r0 / d.KK);
            int kk = int(r0 - int64_t(l) * d.KK);
            int k1, k2;
            dev::tri_decode(d.K, kk, k1, k2);
            const T* wl = w + (x * lm1 + l) * d.nmax * d.K;
            T v = T(0);
            int n1 = k1 - blk, n2 = k2 - blk;
            if (n1 >= 0 && n1 < d.nmax) v += wl[n1 * d.K + k2];
            if (n2 >= 0 && n2 < d.nmax) v += wl[n2 * d.K + k1];
            dp_row[o] = v;
        }
        wave_sync();
    }
}

template <typename K>
hipError_t launch_dyn(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t stream, const FeatureArgs& a)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, a);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_feat(K kernel, size_t lds, hipStream_t stream, const FeatureArgs& a, int chunk, const Layout& L)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, dim3(unsigned(a.n_atoms)), dim3(kThreads), lds, stream, a, chunk, L);
    return hipGetLastError();
}

constexpr size_t kMaxLds = 160 * 1024;

template <typename T>
hipError_t features_t(const FeatureArgs& a, hipStream_t stream)
{
    Dims d = make_dims(a.S, a.nmax, a.lmax);
    bool grad = a.dcoeffs_self != nullptr;
    bool want_p = a.p != nullptr;
    // largest chunk (<= 32 pairs) whose layout fits 64 KB, else 160 KB
    int chunk = 32;
    Layout L = make_layout(d, chunk, grad, want_p);
    while (chunk > 4 && L.total * sizeof(T) > 65536) {
        chunk /= 2;
        L = make_layout(d, chunk, grad, want_p);
    }
    size_t lds = size_t(L.total) * sizeof(T);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    if (grad) {
        if (want_p) return launch_feat(k_features<T, true, true>, lds, stream, a, chunk, L);
        return launch_feat(k_features<T, true, false>, lds, stream, a, chunk, L);
    }
    if (want_p) return launch_feat(k_features<T, false, true>, lds, stream, a, chunk, L);
    return launch_feat(k_features<T, false, false>, lds, stream, a, chunk, L);
}

template <typename T>
hipError_t power_spectrum_t(const FeatureArgs& a, hipStream_t stream)
{
    Dims d = make_dims(a.S, a.nmax, a.lmax);
    bool grad = a.dp != nullptr;
    size_t n = size_t(d.K) * d.L2;
    size_t self_row = 3 * size_t(d.K) * d.L2;
    size_t row_bufs = size_t(kWaves) * (3 * d.nmax * d.L2 + 3 * (d.lmax + 1) * d.nmax * d.K);
    if (grad) n += self_row > row_bufs ? self_row : row_bufs;
    size_t lds = n * sizeof(T);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    dim3 grid(unsigned(a.n_atoms)), block(kThreads);
    if (grad) return launch_dyn(k_power_spectrum<T, true>, grid, block, lds, stream, a);
    return launch_dyn(k_power_spectrum<T, false>, grid, block, lds, stream, a);
}

}  // namespace

size_t features_lds_bytes(int S, int nmax, int lmax, bool f64, bool grad, bool want_p)
{
    Dims d = make_dims(S, nmax, lmax);
    int chunk = 32;
    size_t es = f64 ? 8 : 4;
    Layout L = make_layout(d, chunk, grad, want_p);
    while (chunk > 4 && L.total * es > 65536) {
        chunk /= 2;
        L = make_layout(d, chunk, grad, want_p);
    }
    return size_t(L.total) * es;
}

hipError_t launch_features(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    return f64 ? features_t<double>(a, stream) : features_t<float>(a, stream);
}

hipError_t launch_power_spectrum_valu(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    return f64 ? power_spectrum_t<double>(a, stream) : power_spectrum_t<float>(a, stream);
}

}  // namespace soap
