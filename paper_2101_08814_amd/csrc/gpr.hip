// Sparse kernel model on the features (Sec. 5.B): per centre i of species a_i
//   E_i     = sum over active points I with a_I = a_i of w_I (M_I . p_i)^zeta
//   dE_i/dp = sum over the same I of w_I zeta (M_I . p_i)^(zeta-1) M_I
// (Eq. sparse-gp with the polynomial kernel; the active-set sum is taken
// before the features' gradients are touched, Eq. gpr-force-order, so forces
// and virial are one adjoint pass over dE/dp).
//
// Both contractions are dense products, done as 64 x 64 output tiles per
// 256-lane work-group with a 16-deep LDS slab of each operand (the next slab
// is fetched into registers while the current one is used).  In float each
// wave owns a 32 x 32 quarter of the tile as four v_mfma_f32_16x16x4_f32
// accumulators (a lane holds A[r][g] and B[g][r] of a 16 x 4 x 16 step and
// D[4g + v][r], r = lane & 15, g = lane >> 4); in double every lane
// accumulates a 4 x 4 set of outputs on the vector units.
//   k_gpr_dots:   D = P M^T ([N, F] x [F, n_active]); the epilogue forms the
//                 species-masked energy terms w (M.p)^zeta, sums each row's
//                 64 of them in LDS in column order into one partial per
//                 (centre, column tile), and writes the gradient
//                 coefficients w zeta (M.p)^(zeta-1) to the workspace;
//   k_gpr_energy: one wave per centre adds its column-tile partials in a
//                 fixed order;
//   k_gpr_grad:   dE/dp = G M ([N, n_active] x [n_active, F]); when the
//                 output has too few tiles to fill the chip, the n_active
//                 range is split over the grid's z dimension into fixed
//                 slices whose partial products k_gpr_reduce adds in slice
//                 order.
// Every sum runs in a fixed order, so results are bitwise reproducible.
#include "soap_internal.hpp"

#include <type_traits>

namespace soap {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;    // output rows and columns of a work-group
constexpr int kDepth = 16;   // contraction slab staged in LDS
constexpr int kPad = 4;
constexpr int kFillGroups = 2048;   // work-groups that keep every CU busy

template <typename T>
__device__ __forceinline__ T ipow(T x, int n)
{
    T r = T(1);
    for (int k = 0; k < n; ++k) r *= x;
    return r;
}

// Output element (u, v) of a lane, u, v < 4, sits at tile row tile_row and
// column tile_col: in float, accumulator u = 2 bi + bj of wave w holds rows
// 32 (w >> 1) + 16 bi + 4 g + v and column 32 (w & 1) + 16 bj + r; in double,
// row ty + 16 u and column tx + 16 v (ty = lane index >> 4, tx = & 15).
template <typename T>
__device__ __forceinline__ int tile_row(int u, int v)
{
    if (std::is_same<T, float>::value) {
        const int w = threadIdx.x >> 6, g = (threadIdx.x >> 4) & 3;
        return 32 * (w >> 1) + 16 * (u >> 1) + 4 * g + v;
    }
    return int(threadIdx.x >> 4) + 16 * u;
}

template <typename T>
__device__ __forceinline__ int tile_col(int u, int v)
{
    if (std::is_same<T, float>::value) {
        const int w = threadIdx.x >> 6, r = threadIdx.x & 15;
        return 32 * (w & 1) + 16 * (u & 1) + r;
    }
    return int(threadIdx.x & 15) + 16 * v;
}

// acc[v] += the 16 x 16 x 4 product of this wave's A and B lane values
__device__ __forceinline__ void mfma_acc(float (&acc)[4], float a, float b)
{
    f32x4 c = {acc[0], acc[1], acc[2], acc[3]};
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    acc[0] = c[0];
    acc[1] = c[1];
    acc[2] = c[2];
    acc[3] = c[3];
}
__device__ __forceinline__ void mfma_acc(double (&)[4], double, double) {}

// the 64 x 64 tile at (row0, col0) of
//   C = A B,  A(i, k) = a[i * lda + k]  (rows < n_rows),
//             B(k, j) = TRANS_B ? b[j * ldb + k] : b[k * ldb + j]  (cols < n_cols),
// over k_begin <= k < depth; out-of-range operand elements read as zero
// (as guarded loads: clamped unconditional loads were measured twice as slow
// here).
template <typename T, bool TRANS_B>
__device__ __forceinline__ void tile_product(const T* __restrict__ a, int64_t lda, int64_t n_rows,
                                             const T* __restrict__ b, int64_t ldb, int64_t n_cols, int64_t k_begin,
                                             int64_t depth, int64_t row0, int64_t col0, T (&acc)[4][4])
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
    fetch(k_begin);
    for (int64_t k0 = k_begin; k0 < depth; k0 += kDepth) {
        put();
        __syncthreads();
        if (k0 + kDepth < depth) fetch(k0 + kDepth);   // in flight during the slab's products
        if constexpr (std::is_same<T, float>::value) {
            const int w = tid >> 6, r = tid & 15, g = (tid >> 4) & 3;
            const int ar = 32 * (w >> 1) + r, bc = 32 * (w & 1) + r;
#pragma unroll
            for (int kk = 0; kk < kDepth; kk += 4) {
                const float a0 = As[kk + g][ar], a1 = As[kk + g][ar + 16];
                const float b0 = Bs[kk + g][bc], b1 = Bs[kk + g][bc + 16];
                mfma_acc(acc[0], a0, b0);
                mfma_acc(acc[1], a0, b1);
                mfma_acc(acc[2], a1, b0);
                mfma_acc(acc[3], a1, b1);
            }
        } else {
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
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gpr_dots(int64_t n, int64_t n_feat, const int32_t* __restrict__ species,
                                                  const T* __restrict__ p, int64_t n_active,
                                                  const int32_t* __restrict__ active_species,
                                                  const T* __restrict__ m, const T* __restrict__ w, int zeta,
                                                  T* __restrict__ e_part, T* __restrict__ g_coef)
{
    __shared__ T es[kTile][kTile + 1];   // energy terms of the tile, [row][column]
    const int64_t row0 = int64_t(blockIdx.x) * kTile, col0 = int64_t(blockIdx.y) * kTile;
    T acc[4][4];
    tile_product<T, true>(p, n_feat, n, m, n_feat, n_active, 0, n_feat, row0, col0, acc);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int tr = tile_row<T>(u, v), tc = tile_col<T>(u, v);
            const int64_t i = row0 + tr, I = col0 + tc;
            T e = T(0);
            if (i < n && I < n_active) {
                const bool same = active_species[I] == species[i];
                const T d = acc[u][v], wi = w[I];
                const T km1 = ipow(d, zeta - 1);
                e = same ? wi * (km1 * d) : T(0);
                if (g_coef) g_coef[i * n_active + I] = same ? wi * T(zeta) * km1 : T(0);
            }
            es[tr][tc] = e;
        }
    }
    __syncthreads();
    if (threadIdx.x < kTile && row0 + threadIdx.x < n) {
        T s = T(0);
        for (int c = 0; c < kTile; ++c) s += es[threadIdx.x][c];
        e_part[int64_t(blockIdx.y) * n + row0 + threadIdx.x] = s;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gpr_energy(int64_t n, int col_tiles, const T* __restrict__ e_part,
                                                    T* __restrict__ energies)
{
    const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    // lane t holds tiles t, t + 64, ... in order, then a fixed butterfly
    T s = T(0);
    for (int t = lane; t < col_tiles; t += 64) s += e_part[int64_t(t) * n + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) energies[i] = s;
}

// slice z of the active points: [z * slice, min(n_active, (z + 1) * slice));
// the product of slice z goes to out + z * n * n_feat
template <typename T>
__global__ void __launch_bounds__(256) k_gpr_grad(int64_t n, int64_t n_feat, int64_t n_active, int64_t slice,
                                                  const T* __restrict__ g_coef, const T* __restrict__ m,
                                                  T* __restrict__ out)
{
    const int64_t row0 = int64_t(blockIdx.x) * kTile, col0 = int64_t(blockIdx.y) * kTile;
    const int64_t k0 = int64_t(blockIdx.z) * slice, k1 = k0 + slice < n_active ? k0 + slice : n_active;
    T* grad = out + int64_t(blockIdx.z) * n * n_feat;
    T acc[4][4];
    tile_product<T, false>(g_coef, n_active, n, m, n_feat, n_feat, k0, k1, row0, col0, acc);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = row0 + tile_row<T>(u, v), j = col0 + tile_col<T>(u, v);
            if (i < n && j < n_feat) grad[i * n_feat + j] = acc[u][v];
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gpr_reduce(int64_t count, int slices, const T* __restrict__ part,
                                                    T* __restrict__ grad)
{
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= count) return;
    T s = part[e];
    for (int z = 1; z < slices; ++z) s += part[int64_t(z) * count + e];
    grad[e] = s;
}

// slices of the active points for the gradient product (1 = no split):
// enough to fill the chip, each at least 128 deep
int grad_slices(int64_t n, int64_t n_feat, int64_t n_active)
{
    const int64_t tiles = ((n + kTile - 1) / kTile) * ((n_feat + kTile - 1) / kTile);
    int64_t z = (kFillGroups + tiles - 1) / tiles;
    const int64_t deep = (n_active + 127) / 128;
    if (z > deep) z = deep;
    if (z > 64) z = 64;
    return z < 1 ? 1 : int(z);
}

int64_t slice_depth(int64_t n_active, int slices)
{
    const int64_t d = (n_active + slices - 1) / slices;
    return (d + kDepth - 1) / kDepth * kDepth;
}

template <typename T>
hipError_t gpr_t(int64_t n, int64_t n_feat, const int32_t* species, const void* p, int64_t n_active,
                 const int32_t* active_species, const void* m, const void* w, int zeta, void* workspace,
                 void* energies, void* grad, hipStream_t stream)
{
    // workspace: energy partials [col_tiles][n], gradient coefficients
    // [n][n_active], partial gradients [slices][n][n_feat]
    const int col_tiles = int((n_active + kTile - 1) / kTile);
    T* e_part = static_cast<T*>(workspace);
    T* g_coef = grad ? e_part + int64_t(col_tiles) * n : nullptr;
    // row tiles along x (up to 2^31 - 1 work-groups), column tiles along y
    const dim3 tiles_a(unsigned((n + kTile - 1) / kTile), unsigned(col_tiles));
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gpr_dots<T>), tiles_a, dim3(256), 0, stream, n, n_feat, species,
                       static_cast<const T*>(p), n_active, active_species, static_cast<const T*>(m),
                       static_cast<const T*>(w), zeta, e_part, g_coef);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gpr_energy<T>), dim3(unsigned((n + 3) / 4)), dim3(256), 0, stream, n,
                       col_tiles, static_cast<const T*>(e_part), static_cast<T*>(energies));
    if (grad) {
        const int z = grad_slices(n, n_feat, n_active);
        const int64_t slice = slice_depth(n_active, z);
        const int zs = int((n_active + slice - 1) / slice);   // non-empty slices
        T* part = zs > 1 ? g_coef + n * n_active : static_cast<T*>(grad);
        const dim3 tiles_g(unsigned((n + kTile - 1) / kTile), unsigned((n_feat + kTile - 1) / kTile), unsigned(zs));
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gpr_grad<T>), tiles_g, dim3(256), 0, stream, n, n_feat, n_active, slice,
                           static_cast<const T*>(g_coef), static_cast<const T*>(m), part);
        if (zs > 1) {
            const int64_t count = n * n_feat;
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gpr_reduce<T>), dim3(unsigned((count + 255) / 256)), dim3(256), 0,
                               stream, count, zs, static_cast<const T*>(part), static_cast<T*>(grad));
        }
    }
    return hipGetLastError();
}

}  // namespace

size_t gpr_workspace_bytes(bool f64, int64_t n, int64_t n_feat, int64_t n_active)
{
    const int z = grad_slices(n, n_feat, n_active);
    const int64_t zs = (n_active + slice_depth(n_active, z) - 1) / slice_depth(n_active, z);
    const size_t part = zs > 1 ? size_t(zs) * size_t(n) * size_t(n_feat) : 0;
    const size_t col_tiles = size_t((n_active + kTile - 1) / kTile);
    return (col_tiles * size_t(n) + size_t(n) * size_t(n_active) + part) * (f64 ? 8 : 4);
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
