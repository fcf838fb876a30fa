// Power spectrum on the matrix cores (gfx950 MFMA), bfloat16 operands with
// float accumulation.
//
// For a centre and a degree l the power spectrum is the Gram matrix
//   P_l = C_l C_l^T,   C_l = [c_{k, l^2 .. l^2+2l}]  (K x (2l+1)),
// of which the packed upper triangle k1 <= k2 is kept (Sec. 2 Eq.
// nu2-basis-coupled with real coefficients).  bfloat16 keeps 8 significant
// bits, too few for a 2e-3 relative error on p, so C is split into
// H = bf16(C) and L = bf16(C - H) and
//   P_l ~= H H^T + H L^T + L H^T = [H | L | H] [H | H | L]^T,
// one product whose inner dimension is 3(2l+1); the dropped L L^T term and
// the rounding of L leave a relative error of order 2^-16.
//
// One work-group of four waves owns one centre.  C is split once into LDS;
// for each l the 16 x 16 output tiles (I <= J) are spread over the waves,
// each a chain of v_mfma_f32_16x16x32_bf16 over the padded inner dimension.
// The tile lands in an LDS copy of the packed row p_{i,l,.}, which is then
// written to memory with consecutive lanes on consecutive addresses.
#include "soap_internal.hpp"

namespace soap {

hipError_t launch_power_spectrum_valu(const FeatureArgs& a, bool f64, hipStream_t stream);

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

// round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short to_bf16(float f)
{
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

__global__ void __launch_bounds__(kThreads) k_power_spectrum_bf16(FeatureArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int S = a.S, nmax = a.nmax, lmax = a.lmax;
    const int K = S * nmax, L2 = (lmax + 1) * (lmax + 1);
    const int KK = K * (K + 1) / 2;
    const int KL2 = K * L2;
    unsigned short* hi = reinterpret_cast<unsigned short*>(smem_raw);
    unsigned short* lo = hi + KL2;
    float* prow = reinterpret_cast<float*>(smem_raw + ((4 * size_t(KL2) + 15) & ~size_t(15)));
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t i = blockIdx.x;
    const float* c_in = static_cast<const float*>(a.coeffs) + i * KL2;
    for (int e = tid; e < KL2; e += kThreads) {
        float v = c_in[e];
        unsigned short h = to_bf16(v);
        hi[e] = h;
        lo[e] = to_bf16(v - from_bf16(h));
    }
    __syncthreads();
    const int T = (K + 15) / 16;
    const int n_tiles = T * (T + 1) / 2;
    const int row = lane & 15, kg = lane >> 4;
    float* p_out = static_cast<float*>(a.p) + i * int64_t(lmax + 1) * KK;
    for (int l = 0; l <= lmax; ++l) {
        const int w = 2 * l + 1, inner = 3 * w, steps = (inner + 31) / 32;
        for (int t = wave; t < n_tiles; t += kThreads / 64) {
            // tile t -> (I, J), I <= J, row-major over the upper triangle
            int I = 0, rem = t;
            while (rem >= T - I) { rem -= T - I; ++I; }
            int J = I + rem;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const int ka = I * 16 + row, kb = J * 16 + row;
            for (int st = 0; st < steps; ++st) {
                u16x8 av, bv;
                for (int j = 0; j < 8; ++j) {
                    int q = st * 32 + kg * 8 + j;
                    int seg = q / w, m = q - seg * w;
                    unsigned short va = 0, vb = 0;
                    if (seg < 3) {
                        if (ka < K) va = (seg == 1 ? lo : hi)[ka * L2 + l * l + m];
                        if (kb < K) vb = (seg == 2 ? lo : hi)[kb * L2 + l * l + m];
                    }
                    av[j] = va;
                    bv[j] = vb;
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                              __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
            }
            // lane holds D[4*kg + v][row]
            const int k2 = J * 16 + row;
            for (int v = 0; v < 4; ++v) {
                int k1 = I * 16 + 4 * kg + v;
                if (k1 <= k2 && k2 < K) prow[k1 * K - k1 * (k1 - 1) / 2 + (k2 - k1)] = acc[v];
            }
        }
        __syncthreads();
        float* dst = p_out + int64_t(l) * KK;
        for (int e = tid; e < KK; e += kThreads) dst[e] = prow[e];
        __syncthreads();
    }
}

}  // namespace

size_t power_spectrum_bf16_lds(int S, int nmax, int lmax)
{
    size_t K = size_t(S) * nmax, L2 = size_t(lmax + 1) * (lmax + 1);
    return ((4 * K * L2 + 15) & ~size_t(15)) + 4 * (K * (K + 1) / 2);
}

hipError_t launch_power_spectrum(const FeatureArgs& a, soap_precision prec, hipStream_t stream)
{
    if (prec != SOAP_BF16_F32ACC) return launch_power_spectrum_valu(a, prec == SOAP_F64, stream);
    size_t lds = power_spectrum_bf16_lds(a.S, a.nmax, a.lmax);
    if (lds > 160 * 1024) return hipErrorNotSupported;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_power_spectrum_bf16),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_power_spectrum_bf16, dim3(unsigned(a.n_atoms)), dim3(kThreads), lds, stream, a);
    return hipGetLastError();
}

}  // namespace soap
