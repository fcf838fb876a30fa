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
// The pair rows d c / d r_ji and d p / d r_ji are written by a second
// kernel (gradient_rows.hip) once c of every centre is in memory.
#include <type_traits>

#include "chunk.hpp"

namespace soap {
namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// Per-centre pass: c, p and (with gradients) the self rows of c and p.
// One thread owns a species channel and an lm and accumulates every n of it
// over the centre's pairs of that species.
// ---------------------------------------------------------------------------
template <typename T, int LM, bool GRAD, bool WANT_P>
__global__ void __launch_bounds__(kThreads) k_centres(FeatureArgs a, Layout L)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* base = reinterpret_cast<T*>(smem_raw);
    Smem<T> s(base, L);
    const Dims d = make_dims(a.S, a.nmax, lmax_of(a, LM));
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (tid == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    const int chunk = L.chunk;
    init_tables<T>(a, d, L, s);
    const int64_t q_begin = a.pair_offsets[i], q_end = a.pair_offsets[i + 1];
    const int n_chunks = int((q_end - q_begin + chunk - 1) / chunk);
    const int KL2 = d.K * d.L2, nL2 = d.nmax * d.L2, lm1 = d.lm1;
    for (int e = tid; e < KL2; e += kThreads) {
        s.c[e] = T(0);
        if (GRAD) { s.dcs[e] = T(0); s.dcs[KL2 + e] = T(0); s.dcs[2 * KL2 + e] = T(0); }
    }
    // items (species, n pair, lm): two n per thread share the Y and dY loads
    const int ng = (d.nmax + 1) / 2;
    const int items = d.S * ng * d.L2;
    for (int ck = 0; ck < n_chunks; ++ck) {
        int64_t q0 = q_begin + int64_t(ck) * chunk;
        int nc = int(q_end - q0 < chunk ? q_end - q0 : chunk);
        stage_chunk<T, GRAD>(a, d, s, q0, nc);
        for (int t = tid; t < items; t += kThreads) {
            const int sp = t / (ng * d.L2), rem = t - sp * (ng * d.L2), g = rem / d.L2, lm = rem - g * d.L2;
            const int n0 = 2 * g, two = n0 + 1 < d.nmax;
            const int l = s.lof[lm];
            const int e0 = (sp * d.nmax + n0) * d.L2 + lm;
            T c0 = T(0), c1 = T(0);
            T a0 = T(0), a1 = T(0), a2 = T(0), b0 = T(0), b1 = T(0), b2 = T(0);
            const int p0 = s.seg[2 * sp], p1 = s.seg[2 * sp + 1];
            for (int p = p0; p < p1; ++p) {
                if (s.spc[p] != sp) continue;
                const T Yv = s.Y[p * d.L2 + lm];
                const T* Rp = s.R + p * d.nl + n0 * lm1 + l;
                const T R0 = Rp[0], R1 = two ? Rp[lm1] : T(0);
                c0 += R0 * Yv;
                c1 += R1 * Yv;
                if (GRAD) {
                    // d c_i / d r_i = -sum over pairs of [(f I~)' Y u + f I~ grad Y]
                    const T* dRp = s.dR + p * d.nl + n0 * lm1 + l;
                    const T* D = s.dY + p * 3 * d.L2 + lm;
                    const T D0 = D[0], D1 = D[d.L2], D2 = D[2 * d.L2];
                    const T ux = s.ux[p], uy = s.uy[p], uz = s.uz[p];
                    const T t0 = dRp[0] * Yv, t1 = (two ? dRp[lm1] : T(0)) * Yv;
                    a0 += t0 * ux + R0 * D0;
                    a1 += t0 * uy + R0 * D1;
                    a2 += t0 * uz + R0 * D2;
                    b0 += t1 * ux + R1 * D0;
                    b1 += t1 * uy + R1 * D1;
                    b2 += t1 * uz + R1 * D2;
                }
            }
            s.c[e0] += c0;
            if (two) s.c[e0 + d.L2] += c1;
            if (GRAD) {
                s.dcs[e0] -= a0;
                s.dcs[KL2 + e0] -= a1;
                s.dcs[2 * KL2 + e0] -= a2;
                if (two) {
                    s.dcs[e0 + d.L2] -= b0;
                    s.dcs[KL2 + e0 + d.L2] -= b1;
                    s.dcs[2 * KL2 + e0 + d.L2] -= b2;
                }
            }
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
    if (!WANT_P) return;
    const int KK = d.KK, PL = lm1 * KK;
    const bool tri_tab = L.pos != L.tri;
    T* p_out = static_cast<T*>(a.p) + i * int64_t(PL);
    T* dps_out = GRAD ? static_cast<T*>(a.dp_self) + i * int64_t(3 * PL) : nullptr;
    int l = tid / KK, kk = tid - (tid / KK) * KK;
    for (int o = tid; o < PL; o += kThreads) {
        int k1, k2;
        tri_pair(d, s, tri_tab, kk, k1, k2);
        const T* c1 = s.c + k1 * d.L2 + l * l;
        const T* c2 = s.c + k2 * d.L2 + l * l;
        T acc = T(0);
        for (int m = 0; m < 2 * l + 1; ++m) acc += c1[m] * c2[m];
        p_out[o] = acc;
        if (GRAD) {
            // self rows of p: the product rule on the self rows of c
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const T* g1 = s.dcs + x * KL2 + k1 * d.L2 + l * l;
                const T* g2 = s.dcs + x * KL2 + k2 * d.L2 + l * l;
                T acc2 = T(0);
                for (int m = 0; m < 2 * l + 1; ++m) acc2 += g1[m] * c2[m] + c1[m] * g2[m];
                dps_out[x * PL + o] = acc2;
            }
        }
        kk += kThreads;
        while (kk >= KK) { kk -= KK; ++l; }
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
hipError_t launch_feat(K kernel, size_t lds, hipStream_t stream, const FeatureArgs& a, const Layout& L)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, dim3(unsigned(a.n_atoms)), dim3(kThreads), lds, stream, a, L);
    return hipGetLastError();
}

constexpr size_t kMaxLds = 160 * 1024;

template <typename T, int LM>
hipError_t centres_launch(const FeatureArgs& a, const Layout& L, size_t lds, hipStream_t stream)
{
    const bool grad = a.dcoeffs_self != nullptr, want_p = a.p != nullptr;
    if (grad)
        return want_p ? launch_feat(k_centres<T, LM, true, true>, lds, stream, a, L)
                      : launch_feat(k_centres<T, LM, true, false>, lds, stream, a, L);
    return want_p ? launch_feat(k_centres<T, LM, false, true>, lds, stream, a, L)
                  : launch_feat(k_centres<T, LM, false, false>, lds, stream, a, L);
}

template <typename T, int LM>
struct CentresFn {
    static hipError_t run(const FeatureArgs& a, const Layout& L, size_t lds, hipStream_t st)
    {
        return centres_launch<T, LM>(a, L, lds, st);
    }
};

// per-centre pass (c, p, self rows) then, if asked for, the pair rows
template <typename T>
hipError_t features_t(const FeatureArgs& a, hipStream_t stream)
{
    Dims d = make_dims(a.S, a.nmax, a.lmax);
    bool grad = a.dcoeffs_self != nullptr;
    bool want_p = a.p != nullptr;
    Layout L = choose_layout<T>(d, grad, false, true, want_p);
    if (L.total == 0) return hipErrorNotSupported;
    size_t lds = size_t(L.total) * sizeof(T);
    FeatureArgs c = a;
    c.dp_self = want_p ? a.dp_self : nullptr;
    hipError_t e = by_lmax<T, CentresFn>(a.lmax, c, L, lds, stream);
    if (e != hipSuccess) return e;
    return launch_gradient_rows(a, std::is_same<T, double>::value, stream);
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
    if (lds > kMaxLds) return hipErrorNotSupported;
    dim3 grid(unsigned(a.n_atoms)), block(kThreads);
    if (grad) return launch_dyn(k_power_spectrum<T, true>, grid, block, lds, stream, a);
    return launch_dyn(k_power_spectrum<T, false>, grid, block, lds, stream, a);
}

}  // namespace

hipError_t launch_features(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    return f64 ? features_t<double>(a, stream) : features_t<float>(a, stream);
}

hipError_t launch_power_spectrum_valu(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    return f64 ? power_spectrum_t<double>(a, stream) : power_spectrum_t<float>(a, stream);
}

}  // namespace soap
