// Sparse kernel model on the features (Sec. 5.B): per centre i of species a_i
//   E_i     = sum over active points I with a_I = a_i of w_I (M_I . p_i)^zeta
//   dE_i/dp = sum over the same I of w_I zeta (M_I . p_i)^(zeta-1) M_I
// (Eq. sparse-gp with the polynomial kernel; the active-set sum is taken
// before the features' gradients are touched, Eq. gpr-force-order, so forces
// and virial are one adjoint pass over dE/dp).
//
// Both contractions are dense products, done as 64 x 64 output tiles per
// 256-lane work-group with a 16-deep LDS slab of each operand (the next slab
// is fetched into registers while the current one is used):
//   k_gpr_dots:   D = P M^T ([N, F] x [F, n_active]); the epilogue forms the
//                 species-masked energy terms w (M.p)^zeta and the gradient
//                 coefficients w zeta (M.p)^(zeta-1) into the workspace;
//   k_gpr_energy: one wave per centre sums its row of energy terms in a
//                 fixed order;
//   k_gpr_grad:   dE/dp = G M ([N, n_active] x [n_active, F]).
// Every sum runs in a fixed order, so results are bitwise reproducible.
#include "soap_internal.hpp"

namespace soap {
namespace {

constexpr int kTile = 64;    // output rows and columns of a work-group
constexpr int kDepth = 16;   // contraction slab staged in LDS
constexpr int kPad = 4;

template <typename T>
__device__ __forceinline__ T ipow(T x, int n)
{
    T r = T(1);
    for (int k = 0; k < n; ++k) r *= x;
    return r;
}

// C(row0 + ty + 16u, col0 + tx + 16v) for u, v < 4 of
//   C = A B,  A(i, k) = a[i * lda + k]  (rows < n_rows),
//             B(k, j) = TRANS_B ? b[j * ldb + k] : b[k * ldb + j]  (cols < n_cols),
// over k < depth; out-of-range operand elements read as zero.
template <typename T, bool TRANS_B>
__device__ __forceinline__ void tile_product(const T* __restrict__ a, int64_t lda, int64_t n_rows,
                                             const T* __restrict__ b, int64_t ldb, int64_t n_cols, int64_t depth,
                                             int64_t row0, int64_t col0, T (&acc)[4][4])
{
    __shared__ T As[kDepth][kTile + kPad];
    __shared__ T Bs[kDepth][kTile + kPad];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
    // element r of this lane's share of a slab: A as (row = e >> 4, k = e & 15);
    // B as (col = e >> 4, k = e & 15) when transposed, else (k = e >> 6, col = e & 63)
    T ra[4], rb[4];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            const int64_t i = row0 + (e >> 4), k = k0 + (e & 15);
            ra[r] = (i < n_rows && k < depth) ? a[i * lda + k] : T(0);
            if (TRANS_B) {
                const int64_t j = col0 + (e >> 4);
                rb[r] = (j < n_cols && k < depth) ? b[j * ldb + k] : T(0);
            } else {
                const int64_t kb = k0 + (e >> 6), j = col0 + (e & 63);
                rb[r] = (j < n_cols && kb < depth) ? b[kb * ldb + j] : T(0);
            }
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            As[e & 15][e >> 4] = ra[r];
            if (TRANS_B) Bs[e & 15][e >> 4] = rb[r];
            else Bs[e >> 6][e & 63] = rb[r];
        }
    };
    fetch(0);
    for (int64_t k0 = 0; k0 < depth; k0 += kDepth) {
        put();
        __syncthreads();
        if (k0 + kDepth < depth) fetch(k0 + kDepth);   // in flight during the slab's products
#pragma unroll
        for (int kk = 0; kk < kDepth; ++kk) {
            T x[4], y[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = As[kk][ty + 16 * u];
#pragma unroll
            for (int v = 0; v < 4; ++v) y[v] = Bs[kk][tx + 16 * v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += x[u] * y[v];
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gpr_dots(int64_t n, int64_t n_feat, const int32_t* __restrict__ species,
                                                  const T* __restrict__ p, int64_t n_active,
                                                  const int32_t* __restrict__ active_species,
                                                  const T* __restrict__ m, const T* __restrict__ w, int zeta,
                                                  T* __restrict__ e_terms, T* __restrict__ g_coef)
{
    const int64_t row0 = int64_t(blockIdx.x) * kTile, col0 = int64_t(blockIdx.y) * kTile;
    T acc[4][4];
    tile_product<T, true>(p, n_feat, n, m, n_feat, n_active, n_feat, row0, col0, acc);
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = row0 + ty + 16 * u;
        if (i >= n) continue;
        const int si = species[i];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t I = col0 + tx + 16 * v;
            if (I >= n_active) continue;
            const bool same = active_species[I] == si;
            const T d = acc[u][v], wi = w[I];
            const T km1 = ipow(d, zeta - 1);
            e_terms[i * n_active + I] = same ? wi * (km1 * d) : T(0);
            if (g_coef) g_coef[i * n_active + I] = same ? wi * T(zeta) * km1 : T(0);
        }
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <typename T>
__global__ void __launch_bounds__(256) k_gpr_energy(int64_t n, int64_t n_active, const T* __restrict__ e_terms,
                                                    T* __restrict__ energies)
{
    const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    T s = T(0);
    for (int64_t I = lane; I < n_active; I += 64) s += e_terms[i * n_active + I];
    s = wave_sum(s);
    if (lane == 0) energies[i] = s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_gpr_grad(int64_t n, int64_t n_feat, int64_t n_active,
                                                  const T* __restrict__ g_coef, const T* __restrict__ m,
                                                  T* __restrict__ grad)
{
    const int64_t row0 = int64_t(blockIdx.x) * kTile, col0 = int64_t(blockIdx.y) * kTile;
    T acc[4][4];
    tile_product<T, false>(g_coef, n_active, n, m, n_feat, n_feat, n_active, row0, col0, acc);
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = row0 + ty + 16 * u;
        if (i >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t j = col0 + tx + 16 * v;
            if (j < n_feat) grad[i * n_feat + j] = acc[u][v];
        }
    }
}

template <typename T>
hipError_t gpr_t(int64_t n, int64_t n_feat, const int32_t* species, const void* p, int64_t n_active,
                 const int32_t* active_species, const void* m, const void* w, int zeta, void* workspace,
                 void* energies, void* grad, hipStream_t stream)
{
    T* e_terms = static_cast<T*>(workspace);
    T* g_coef = grad ? e_terms + n * n_active : nullptr;
    // row tiles along x (up to 2^31 - 1 work-groups), column tiles along y
    const dim3 tiles_a(unsigned((n + kTile - 1) / kTile), unsigned((n_active + kTile - 1) / kTile));
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gpr_dots<T>), tiles_a, dim3(256), 0, stream, n, n_feat, species,
                       static_cast<const T*>(p), n_active, active_species, static_cast<const T*>(m),
                       static_cast<const T*>(w), zeta, e_terms, g_coef);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gpr_energy<T>), dim3(unsigned((n + 3) / 4)), dim3(256), 0, stream, n,
                       n_active, static_cast<const T*>(e_terms), static_cast<T*>(energies));
    if (grad) {
        const dim3 tiles_g(unsigned((n + kTile - 1) / kTile), unsigned((n_feat + kTile - 1) / kTile));
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gpr_grad<T>), tiles_g, dim3(256), 0, stream, n, n_feat, n_active,
                           static_cast<const T*>(g_coef), static_cast<const T*>(m), static_cast<T*>(grad));
    }
    return hipGetLastError();
}

}  // namespace

size_t gpr_workspace_bytes(bool f64, int64_t n, int64_t n_active)
{
    return size_t(2) * size_t(n) * size_t(n_active) * (f64 ? 8 : 4);
}

hipError_t launch_gpr_predict(bool f64, int64_t n, int64_t n_feat, const int32_t* species, const void* p,
                              int64_t n_active, const int32_t* active_species, const void* m, const void* w,
                              int zeta, void* workspace, void* energies, void* grad, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    return f64 ? gpr_t<double>(n, n_feat, species, p, n_active, active_species, m, w, zeta, workspace, energies, grad,
                               stream)
               : gpr_t<float>(n, n_feat, species, p, n_active, active_species, m, w, zeta, workspace, energies, grad,
                              stream);
}

}  // namespace soap
