// Power spectrum on the matrix cores (gfx950 MFMA), bfloat16 operands with
// float accumulation, and the same kernel with FP32 operands
// (v_mfma_f32_16x16x4_f32, four of the 2l+1 values per step) for the FP32
// path of many centres.
//
// For a centre and a degree l the power spectrum is the Gram matrix
//   P_l = C_l C_l^T,   C_l = [c_{k, l^2 .. l^2+2l}]  (K x (2l+1)),
// of which the packed upper triangle k1 <= k2 is kept (Sec. 2 Eq.
// nu2-basis-coupled with real coefficients).  bfloat16 keeps 8 significant
// bits, too few for a 2e-3 relative error on p, so C is split into
// H = bf16(C) and L = bf16(C - H) and
//   P_l ~= H H^T + H L^T + L H^T,
// three products of inner dimension 2l+1 (one 32-wide MFMA step each for
// lmax <= 12); the dropped L L^T term and the rounding of L leave a
// relative error of order 2^-16.
//
// W waves own one centre (W = 1, four centres per work-group, when C is
// small and K <= 48; W = 4, one centre per work-group, otherwise): the
// centre's waves split C into their LDS region as {H, L} pairs, then for
// each l run the 16 x 16 output tiles (I <= J) as three
// v_mfma_f32_16x16x32_bf16 each (a lane reads 8 consecutive {H, L} words
// of each of its two rows; one wave per centre reads every row block's
// words into registers once per l, four waves take contiguous runs of
// tiles in row-major order and read a row block once per row they touch),
// put the packed upper triangle in LDS and store it as contiguous float4
// rows (the accumulators alone give 64-byte pieces).
// One wave per centre needs no work-group barrier; four take two per l.
#include "soap_internal.hpp"

namespace soap {

hipError_t launch_power_spectrum_valu(const FeatureArgs& a, bool f64, hipStream_t stream);

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kLoadBatch = 16;   // coefficient loads a lane keeps in flight
constexpr int kRows1 = 3;        // row blocks of 16 (K <= 48) a one-wave centre holds in registers
constexpr int kStepsF32 = 7;     // 4-wide MFMA steps of a row of 2l+1 <= 25 values (lmax <= 12)
constexpr int64_t kF32MfmaAtoms = 8192;   // FP32 spectra of at least this many centres use the matrix cores

// round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short to_bf16(float f)
{
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A lane's operand values of row k of C_l (hl_l points at m = 8 kg of row
// 0): {H, L} words m = 8 kg + j, zero for j >= nj (past 2l+1) or k >= K.
// Rows past K read row 0, and every read stays inside the {H, L} region
// (padded by 32 words past C).
__device__ __forceinline__ void row_operands(const unsigned int* hl_l, int k, int K, int L2, int nj, u16x8& h,
                                             u16x8& lo)
{
    const unsigned int* r = hl_l + (k < K ? k : 0) * L2;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const unsigned int x = j < nj && k < K ? r[j] : 0u;
        h[j] = (unsigned short)(x & 0xFFFFu);
        lo[j] = (unsigned short)(x >> 16);
    }
}

// The 16 x 16 tile (I, J) of P_l ~= H H^T + H L^T + L H^T into the packed
// upper triangle ob, given the operand values of rows I (ha, la) and J
// (hb, lb).
__device__ __forceinline__ void tile(float* ob, int I, int J, int row, int kg, int K, const u16x8& ha,
                                     const u16x8& la, const u16x8& hb, const u16x8& lb)
{
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ha), __builtin_bit_cast(bf16x8, hb), acc,
                                                  0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ha), __builtin_bit_cast(bf16x8, lb), acc,
                                                  0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, la), __builtin_bit_cast(bf16x8, hb), acc,
                                                  0, 0, 0);
    // lane holds D[4 kg + v][row] = P[k1][k2] with k1 = 16 I + 4 kg + v,
    // k2 = 16 J + row; the packed index k1 K - k1 (k1 - 1) / 2 + k2 - k1
    // grows by K - k1 - 1 from k1 to k1 + 1
    const int k2 = J * 16 + row;
    int k1 = I * 16 + 4 * kg;
    int idx = k1 * K - k1 * (k1 - 1) / 2 + (k2 - k1);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        if (k1 <= k2 && k2 < K) ob[idx] = acc[v];
        idx += K - k1 - 1;
        ++k1;
    }
}

// FP32 operands (v_mfma_f32_16x16x4_f32, one step per 4 of the 2l+1
// values): lane (row, kg) supplies the values m = kg NS + s, s < NS =
// ceil((2l+1) / 4), of row k of C_l (c_l points at m = 0 of row 0), so that
// its NS reads are consecutive; A and B take the same order of m, which
// leaves the product unchanged.  Zero past 2l+1 or K; rows past K read row
// 0, and every read stays inside the region (padded by 32 words past C).
__device__ __forceinline__ void row_operands_f32(const float* c_l, int k, int K, int L2, int w, int NS, int kg,
                                                 float (&x)[kStepsF32])
{
    const float* r = c_l + (k < K ? k : 0) * L2 + kg * NS;
#pragma unroll
    for (int s = 0; s < kStepsF32; ++s) x[s] = s < NS && kg * NS + s < w && k < K ? r[s] : 0.f;
}

// The tile (I, J) of P_l = C_l C_l^T from FP32 operands, into the packed
// upper triangle ob (the same output layout as the bfloat16 tile)
__device__ __forceinline__ void tile_f32(float* ob, int I, int J, int row, int kg, int K, int NS,
                                         const float (&xa)[kStepsF32], const float (&xb)[kStepsF32])
{
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < kStepsF32; ++s)
        if (s < NS) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[s], xb[s], acc, 0, 0, 0);
    const int k2 = J * 16 + row;
    int k1 = I * 16 + 4 * kg;
    int idx = k1 * K - k1 * (k1 - 1) / 2 + (k2 - k1);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        if (k1 <= k2 && k2 < K) ob[idx] = acc[v];
        idx += K - k1 - 1;
        ++k1;
    }
}

// One body for both operand forms: F32 keeps C in FP32 (the FP32 path),
// otherwise the {H, L} bfloat16 split.
template <int W, bool F32>
__device__ __forceinline__ void spectrum_body(const FeatureArgs& a)
{
    constexpr int CPG = kThreads / 64 / W;   // centres per work-group
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int S = a.S, nmax = a.nmax, lmax = a.lmax;
    const int K = S * nmax, L2 = (lmax + 1) * (lmax + 1);
    const int KK = K * (K + 1) / 2;
    const int KL2 = K * L2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = wave / W, wc = wave - slot * W;   // centre slot in the work-group, wave within the centre
    const int64_t i = int64_t(blockIdx.x) * CPG + slot;
    if (i >= a.n_atoms) return;
    // {H, L} of every element of C: H in the low half, L in the high half;
    // then the packed P_l of the current l
    const int HLS = (KL2 + 32 + 3) & ~3, OBS = (KK + 3) & ~3;   // 16-byte aligned regions
    unsigned int* hl = reinterpret_cast<unsigned int*>(smem_raw) + size_t(slot) * (HLS + OBS);
    float* ob = reinterpret_cast<float*>(hl + HLS);
    const float* c_in = static_cast<const float*>(a.coeffs) + i * KL2;
    // kLoadBatch loads in flight per lane before any is used
    for (int e0 = wc * 64 + lane; e0 < KL2; e0 += kLoadBatch * W * 64) {
        float v[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int e = e0 + u * W * 64;
            v[u] = e < KL2 ? c_in[e] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int e = e0 + u * W * 64;
            if (e < KL2) {
                if constexpr (F32) {
                    hl[e] = __float_as_uint(v[u]);
                } else {
                    const unsigned short h = to_bf16(v[u]);
                    hl[e] = (unsigned int)h | ((unsigned int)to_bf16(v[u] - from_bf16(h)) << 16);
                }
            }
        }
    }
    if (W == 1) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();   // one centre per work-group
    }
    const int T = (K + 15) / 16;
    const int row = lane & 15, kg = lane >> 4;
    float* p_out = static_cast<float*>(a.p) + i * int64_t(lmax + 1) * KK;
    for (int l = 0; l <= lmax; ++l) {
        const int w = 2 * l + 1;   // <= 25 for lmax <= 12: one 32-wide step per product
        const int nj = w - 8 * kg;  // this lane's operand values m = 8 kg + j with j < nj are inside the row
        const unsigned int* hl_l = hl + l * l + kg * 8;
        float* dst = p_out + int64_t(l) * KK;
        // tiles (I, J), I <= J, row-major over the upper triangle
        const int NS = (w + 3) / 4;   // FP32: 4-wide steps per product
        const float* c_l = reinterpret_cast<const float*>(hl) + l * l;
        if constexpr (W == 1) {
            // one wave: the operand values of every row block read once
            // (T <= kRows1), all reads issued before the first product
            if constexpr (F32) {
                float rx[kRows1][kStepsF32];
#pragma unroll
                for (int I = 0; I < kRows1; ++I)
                    if (I < T) row_operands_f32(c_l, I * 16 + row, K, L2, w, NS, kg, rx[I]);
#pragma unroll
                for (int I = 0; I < kRows1; ++I)
#pragma unroll
                    for (int J = I; J < kRows1; ++J)
                        if (J < T) tile_f32(ob, I, J, row, kg, K, NS, rx[I], rx[J]);
            } else {
                u16x8 rh[kRows1], rl[kRows1];
#pragma unroll
                for (int I = 0; I < kRows1; ++I)
                    if (I < T) row_operands(hl_l, I * 16 + row, K, L2, nj, rh[I], rl[I]);
#pragma unroll
                for (int I = 0; I < kRows1; ++I)
#pragma unroll
                    for (int J = I; J < kRows1; ++J)
                        if (J < T) tile(ob, I, J, row, kg, K, rh[I], rl[I], rh[J], rl[J]);
            }
        } else {
            // each wave a contiguous run of tiles in row-major order, so
            // that row I's operand values are read once per row it touches
            const int n_tiles = T * (T + 1) / 2;
            const int per = (n_tiles + W - 1) / W;
            const int t0 = wc * per, t1 = t0 + per < n_tiles ? t0 + per : n_tiles;
            int I = 0, rem = t0;
            while (I < T && rem >= T - I) { rem -= T - I; ++I; }
            int J = I + rem;
            if constexpr (F32) {
                float xa[kStepsF32];
                if (t0 < t1) row_operands_f32(c_l, I * 16 + row, K, L2, w, NS, kg, xa);
                for (int t = t0; t < t1; ++t) {
                    float xb[kStepsF32];
                    row_operands_f32(c_l, J * 16 + row, K, L2, w, NS, kg, xb);
                    tile_f32(ob, I, J, row, kg, K, NS, xa, xb);
                    if (++J == T && t + 1 < t1) {
                        ++I;
                        J = I;
                        row_operands_f32(c_l, I * 16 + row, K, L2, w, NS, kg, xa);
                    }
                }
            } else {
                u16x8 ha, la;
                if (t0 < t1) row_operands(hl_l, I * 16 + row, K, L2, nj, ha, la);
                for (int t = t0; t < t1; ++t) {
                    u16x8 hb, lb;
                    row_operands(hl_l, J * 16 + row, K, L2, nj, hb, lb);
                    tile(ob, I, J, row, kg, K, ha, la, hb, lb);
                    if (++J == T && t + 1 < t1) {
                        ++I;
                        J = I;
                        row_operands(hl_l, I * 16 + row, K, L2, nj, ha, la);
                    }
                }
            }
        }
        {
            // the packed P_l leaves as contiguous rows: float4 stores when
            // aligned, else one float per lane
            if (W == 1) wave_sync(); else __syncthreads();
            if ((KK & 3) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
                for (int e = wc * 64 + lane; e < KK / 4; e += W * 64)
                    reinterpret_cast<float4*>(dst)[e] = reinterpret_cast<const float4*>(ob)[e];
            } else {
                for (int e = wc * 64 + lane; e < KK; e += W * 64) dst[e] = ob[e];
            }
            if (W == 1) wave_sync(); else __syncthreads();
        }
    }
}

template <int W>
__global__ void __launch_bounds__(kThreads) k_power_spectrum_bf16(FeatureArgs a)
{
    spectrum_body<W, false>(a);
}

template <int W>
__global__ void __launch_bounds__(kThreads) k_power_spectrum_f32mfma(FeatureArgs a)
{
    spectrum_body<W, true>(a);
}

// LDS words of one centre's slot: {H, L} of C (or C), then the packed P_l
size_t bf16_slot_words(int S, int nmax, int lmax, int W)
{
    const size_t K = size_t(S) * nmax, KL2 = K * (lmax + 1) * (lmax + 1), KK = K * (K + 1) / 2;
    return ((KL2 + 32 + 3) & ~size_t(3)) + ((KK + 3) & ~size_t(3));
}

// waves per centre: one when four centres' slots fit 40 KB of LDS (and
// K <= 16 kRows1)
int bf16_waves_per_centre(int S, int nmax, int lmax)
{
    return 4 * 4 * bf16_slot_words(S, nmax, lmax, 1) <= 40 * 1024 && S * nmax <= 16 * kRows1 ? 1 : 4;
}

}  // namespace

size_t power_spectrum_bf16_lds(int S, int nmax, int lmax)
{
    const int W = bf16_waves_per_centre(S, nmax, lmax);
    return size_t(kThreads / 64 / W) * 4 * bf16_slot_words(S, nmax, lmax, W);
}

template <int W, bool F32>
hipError_t launch_mfma(const FeatureArgs& a, size_t lds, hipStream_t stream)
{
    const void* fn = F32 ? reinterpret_cast<const void*>(k_power_spectrum_f32mfma<W>)
                         : reinterpret_cast<const void*>(k_power_spectrum_bf16<W>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    constexpr int cpg = kThreads / 64 / W;
    const unsigned groups = unsigned((a.n_atoms + cpg - 1) / cpg);
    if constexpr (F32)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_power_spectrum_f32mfma<W>), dim3(groups), dim3(kThreads), lds, stream, a);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_power_spectrum_bf16<W>), dim3(groups), dim3(kThreads), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_power_spectrum_f32mfma(const FeatureArgs& a, hipStream_t stream)
{
    const size_t lds = power_spectrum_bf16_lds(a.S, a.nmax, a.lmax);
    if (lds > 160 * 1024 || a.lmax > 12) return hipErrorNotSupported;
    if (a.n_atoms == 0) return hipSuccess;
    return bf16_waves_per_centre(a.S, a.nmax, a.lmax) == 1 ? launch_mfma<1, true>(a, lds, stream)
                                                             : launch_mfma<4, true>(a, lds, stream);
}

hipError_t launch_power_spectrum(const FeatureArgs& a, soap_precision prec, hipStream_t stream)
{
    // FP32 without gradient rows from kF32MfmaAtoms centres on: FP32
    // operands on the matrix cores (28,924 centres at K = 32: 165 -> 124 us,
    // 131k at K = 96: 9.0 -> 6.9 ms); below, the VALU kernel (4096 centres
    // at K = 20: 20 us against 24)
    if (prec == SOAP_F32 && a.dp == nullptr && a.n_atoms >= kF32MfmaAtoms) {
        const hipError_t e = launch_power_spectrum_f32mfma(a, stream);
        if (e != hipErrorNotSupported) return e;
    }
    if (prec != SOAP_BF16_F32ACC) return launch_power_spectrum_valu(a, prec == SOAP_F64, stream);
    const size_t lds = power_spectrum_bf16_lds(a.S, a.nmax, a.lmax);
    if (lds > 160 * 1024) return hipErrorNotSupported;
    if (a.n_atoms == 0) return hipSuccess;
    return bf16_waves_per_centre(a.S, a.nmax, a.lmax) == 1 ? launch_mfma<1, false>(a, lds, stream)
                                                             : launch_mfma<4, false>(a, lds, stream);
}

}  // namespace soap
