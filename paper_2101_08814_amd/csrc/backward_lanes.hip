// Adjoint of the expansion with respect to positions with one lane per pair.
//
// Adjoint (App. B Eq. energy-derivative), k_exp_backward_lanes: one wave per
// centre i, one lane per pair q = (i, j, s).  With G = dL/dc_i (the
// neighbour's species block, staged once per wave in LDS) the lane forms
//   A_lm = sum_n G_{n,lm} (f I~)'_nl,   B_lm = sum_n G_{n,lm} f I~_nl
// degree by degree while the harmonics of that degree come out of the
// recurrence, and
//   g_q = dL/dr_ji = u sum_lm A_lm Y_lm + sum_lm B_lm grad Y_lm
//       = u (sA - sL / r) + t / r,
//   sA = sum A Y, sL = sum l B Y, t = sum B grad Z
// (grad Y_lm = (grad Z_lm - l Y_lm u) / r).  Nothing per pair is staged and
// no lane decodes an index; the per-atom sums stay in the gather kernel of
// backward.hip.
#include "lane_pair.hpp"

namespace soap {
namespace {

using namespace dev;

template <typename T, int LMAX>
__global__ void __launch_bounds__(64) k_exp_backward_lanes(FeatureArgs a, const T* __restrict__ grad_c,
                                                           T* __restrict__ grad_pair)
{
    constexpr int LM1 = LMAX + 1, L2 = LM1 * LM1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* G = reinterpret_cast<T*>(smem_raw);
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (lane == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    const int nmax = a.nmax;
    const int nL2 = nmax * L2, KL2 = a.S * nL2;
    {
        const T* gi = grad_c + i * int64_t(KL2);
        for (int e0 = lane; e0 < KL2; e0 += 4 * 64) {
            T v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = e0 + 64 * u < KL2 ? gi[e0 + 64 * u] : T(0);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (e0 + 64 * u < KL2) G[e0 + 64 * u] = v[u];
        }
    }
    wave_sync();
    const int64_t qb = a.pair_offsets[i], qe = a.pair_offsets[i + 1];
    const V4<T>* __restrict__ coef = static_cast<const V4<T>*>(a.coef_ln);
    const T* __restrict__ vec = static_cast<const T*>(a.pair_vec);
    const T inv_delta = T(a.inv_delta);
    for (int64_t q0 = qb; q0 < qe; q0 += 64) {
        const int64_t q = q0 + lane;
        if (q >= qe) continue;
        const PairGeom<T> g = pair_geometry<T>(a, vec[3 * q], vec[3 * q + 1], vec[3 * q + 2]);
        const int sp = pair_species(a, q);
        const T* Gs = G + sp * nL2;
        const V4<T>* cf = coef + int64_t(g.k) * (LM1 * nmax);
        YlmStream<T, LMAX> ys(g.ux, g.uy, g.uz);
        T sA = T(0), sL = T(0), tx = T(0), ty = T(0), tz = T(0);
        // the interval's cubics are contiguous ([l][n]); they stream two
        // ahead of their use, across degrees (the table has zero entries past
        // its end for the last ones)
        V4<T> c0 = cf[0], c1 = cf[1];
        const V4<T>* cnext = cf + 2;
        static_for<0, LM1>([&](auto Lc) __attribute__((always_inline)) {
            constexpr int L = decltype(Lc)::value;
            constexpr int NM = 2 * L + 1;
            T A[NM], B[NM];
#pragma unroll
            for (int m = 0; m < NM; ++m) A[m] = B[m] = T(0);
            const T* gr = Gs + L * L;
            for (int n = 0; n < nmax; ++n) {
                const V4<T> c = c0;
                c0 = c1;
                c1 = *cnext++;
                T v, dv;
                spline_poly<T>(c.x, c.y, c.z, c.w, g.t, inv_delta, v, dv);
                const T R = g.f * v, dR = g.df * v + g.f * dv;
#pragma unroll
                for (int m = 0; m < NM; ++m) {
                    const T gv = gr[m];
                    A[m] += gv * dR;
                    B[m] += gv * R;
                }
                gr += L2;
            }
            T sB = T(0);
            ys.template degree<L, true>([&](int mi, T Y, T zx, T zy, T zz) __attribute__((always_inline)) {
                sA += A[mi] * Y;
                sB += B[mi] * Y;
                tx += B[mi] * zx;
                ty += B[mi] * zy;
                tz += B[mi] * zz;
            });
            sL += T(L) * sB;
        });
        const T radial = sA - sL * g.rinv;
        grad_pair[3 * q] = g.ux * radial + tx * g.rinv;
        grad_pair[3 * q + 1] = g.uy * radial + ty * g.rinv;
        grad_pair[3 * q + 2] = g.uz * radial + tz * g.rinv;
    }
}

template <typename T, int LM>
struct BackLanesFn {
    static hipError_t run(const FeatureArgs& a, const void* grad_c, void* grad_pair, hipStream_t st)
    {
        if constexpr (LM < 0) {
            return hipErrorNotSupported;
        } else {
            const size_t lds = size_t(a.S) * a.nmax * (LM + 1) * (LM + 1) * sizeof(T);
            if (lds > 65536) {
                hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_exp_backward_lanes<T, LM>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_exp_backward_lanes<T, LM>), dim3(unsigned(a.n_atoms)), dim3(64),
                               lds, st, a, static_cast<const T*>(grad_c), static_cast<T*>(grad_pair));
            return hipGetLastError();
        }
    }
};

}  // namespace

bool expansion_backward_lanes_fits(const FeatureArgs& a, bool f64)
{
    const size_t lds = size_t(a.S) * a.nmax * (a.lmax + 1) * (a.lmax + 1) * (f64 ? 8 : 4);
    return lds <= 64 * 1024;
}

hipError_t launch_expansion_backward_lanes(const FeatureArgs& a, bool f64, const void* grad_c, void* grad_pair,
                                           hipStream_t stream)
{
    if (!expansion_backward_lanes_fits(a, f64)) return hipErrorNotSupported;
    if (a.n_atoms == 0) return hipSuccess;
    return f64 ? by_degree<double, BackLanesFn>(a.lmax, a, grad_c, grad_pair, stream)
               : by_degree<float, BackLanesFn>(a.lmax, a, grad_c, grad_pair, stream);
}

}  // namespace soap
