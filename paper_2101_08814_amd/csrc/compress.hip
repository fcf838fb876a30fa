// Learned equivariant channel compression of the expansion coefficients,
// its training gradients, the kernel-matrix loss and the optimiser step.
//
// The compression is the learned counterpart of the paper's data-driven
// reduction of the feature space (Sec. 4.H; the lossy strategy of Sec. 7),
// built so that the symmetry of the features is kept: for every degree l
// one two-layer network acts on the channel index k = (species, n) of each
// m-column of c, shared over m,
//   h_l = W1_l c_l,  g_{l,q} = h_{l,q} 2 sigma(alpha_{l,q} |h_{l,q}| + beta_{l,q}),
//   c~_l = W2_l g_l,  p~_{l,q1<=q2} = sum_m c~_{q1,lm} c~_{q2,lm},
// with |.| the norm over m (a rotation of the structure rotates the m of
// each l, which commutes with every step).  alpha = beta = 0 is the
// identity gate.  Weights are one float array, per l: W1_l [H][K],
// W2_l [Q][H], alpha_l [H], beta_l [H].
//
// Training compares the linear kernel of the compressed spectrum with that
// of the full one over a batch of centres, K_ij = sum_{l,k1,k2} p p over the
// full symmetric spectrum (packed off-diagonal entries weighted 2):
//   L = |K~ - K|_F^2 / |K|_F^2.
#include <cmath>

#include "chunk.hpp"

namespace soap {
namespace {

using namespace dev;

__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

// weight of packed position t of a Q(Q+1)/2 triangle in the full-spectrum
// inner product: 1 on the diagonal, 2 off it
__device__ __forceinline__ float full_weight(int Q, int t)
{
    int q1, q2;
    tri_decode(Q, t, q1, q2);
    return q1 == q2 ? 1.0f : 2.0f;
}

// ------------------------------------------------------------ forward (FP32)
// One work-group per centre: c in LDS; per l the hidden layer (one lane per
// (q, m)), the gate (one lane per q), the output layer (one lane per (p, m))
// and the compressed spectrum (one lane per packed (q1, q2)).
template <bool WANT_CT, bool WANT_PT>
__global__ void __launch_bounds__(kThreads) k_cmp_fwd(CompressArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* sm = reinterpret_cast<float*>(smem_raw);
    const int K = a.K, Q = a.Q, H = a.H, lmax = a.lmax, L2 = (lmax + 1) * (lmax + 1), MX = 2 * lmax + 1;
    const int QQ = Q * (Q + 1) / 2, tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    float* c = sm;                  // [K][L2]
    float* h = c + K * L2;          // [H][MX]
    float* gs = h + H * MX;         // [H] gate factor
    float* ct = gs + H;             // [Q][MX]
    const float* ci = a.c + i * int64_t(K) * L2;
    for (int e = tid; e < K * L2; e += kThreads) c[e] = ci[e];
    __syncthreads();
    const float* w = a.w;
    for (int l = 0; l <= lmax; ++l) {
        const int M = 2 * l + 1, b = l * l;
        const float* W1 = w;
        const float* W2 = W1 + H * K;
        const float* al = W2 + Q * H;
        const float* be = al + H;
        w = be + H;
        for (int t = tid; t < H * M; t += kThreads) {
            const int q = t / M, m = t - q * M;
            const float* wr = W1 + q * K;
            float acc = 0.0f;
            for (int k = 0; k < K; ++k) acc += wr[k] * c[k * L2 + b + m];
            h[q * MX + m] = acc;
        }
        __syncthreads();
        for (int q = tid; q < H; q += kThreads) {
            float s = 0.0f;
            for (int m = 0; m < M; ++m) s += h[q * MX + m] * h[q * MX + m];
            gs[q] = 2.0f * sigm(al[q] * sqrtf(s) + be[q]);
        }
        __syncthreads();
        for (int t = tid; t < Q * M; t += kThreads) {
            const int p = t / M, m = t - p * M;
            const float* wr = W2 + p * H;
            float acc = 0.0f;
            for (int q = 0; q < H; ++q) acc += wr[q] * (gs[q] * h[q * MX + m]);
            ct[p * MX + m] = acc;
            if (WANT_CT) a.ct[(i * Q + p) * L2 + b + m] = acc;
        }
        __syncthreads();
        if (WANT_PT) {
            float* out = a.pt + (i * (lmax + 1) + l) * int64_t(QQ);
            for (int t = tid; t < QQ; t += kThreads) {
                int q1, q2;
                tri_decode(Q, t, q1, q2);
                float acc = 0.0f;
                for (int m = 0; m < M; ++m) acc += ct[q1 * MX + m] * ct[q2 * MX + m];
                out[t] = acc;
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------- backward (FP32)
// Grid (lmax + 1, slices): work-group (l, s) takes the centres s, s + S, ...
// recomputes the forward pass of degree l for each and accumulates the
// gradients of W1_l, W2_l, alpha_l, beta_l in LDS; partial sums per slice go
// to gpart[s][...] in the layout of the weights (summed by k_reduce).
__global__ void __launch_bounds__(kThreads) k_cmp_bwd(CompressArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* sm = reinterpret_cast<float*>(smem_raw);
    const int K = a.K, Q = a.Q, H = a.H, lmax = a.lmax, L2 = (lmax + 1) * (lmax + 1);
    const int QQ = Q * (Q + 1) / 2, tid = threadIdx.x;
    const int l = blockIdx.x, S = gridDim.y, s = blockIdx.y;
    const int M = 2 * l + 1, b = l * l;
    const int64_t lsize = int64_t(H) * K + Q * H + 2 * H;
    const float* W1 = a.w + l * lsize;
    const float* W2 = W1 + H * K;
    const float* al = W2 + Q * H;
    const float* be = al + H;
    float* gW1 = sm;                 // [H][K]
    float* gW2 = gW1 + H * K;        // [Q][H]
    float* gal = gW2 + Q * H;        // [H]
    float* gbe = gal + H;            // [H]
    float* x = gbe + H;              // [K][M]
    float* h = x + K * M;            // [H][M]
    float* g = h + H * M;            // [H][M]
    float* dh = g + H * M;           // [H][M]
    float* ct = dh + H * M;          // [Q][M]
    float* dct = ct + Q * M;         // [Q][M]
    float* nrm = dct + Q * M;        // [H]
    float* sg = nrm + H;             // [H] sigma
    float* gsv = sg + H;             // [H] gate factor 2 sigma
    float* cf = gsv + H;             // [H] d|h| coefficient
    float* gp = cf + H;              // [QQ] upstream gradient of this centre and l
    for (int e = tid; e < lsize; e += kThreads) gW1[e] = 0.0f;
    __syncthreads();
    for (int64_t i = s; i < a.n; i += S) {
        const float* ci = a.c + i * int64_t(K) * L2 + b;
        for (int t = tid; t < K * M; t += kThreads) {
            const int k = t / M, m = t - k * M;
            x[t] = ci[k * L2 + m];
        }
        const float* gpi = a.gpt + (i * (lmax + 1) + l) * int64_t(QQ);
        for (int t = tid; t < QQ; t += kThreads) gp[t] = gpi[t];
        __syncthreads();
        for (int t = tid; t < H * M; t += kThreads) {
            const int q = t / M, m = t - q * M;
            const float* wr = W1 + q * K;
            float acc = 0.0f;
            for (int k = 0; k < K; ++k) acc += wr[k] * x[k * M + m];
            h[t] = acc;
        }
        __syncthreads();
        for (int q = tid; q < H; q += kThreads) {
            float ss = 0.0f;
            for (int m = 0; m < M; ++m) ss += h[q * M + m] * h[q * M + m];
            const float n_ = sqrtf(ss), sgm = sigm(al[q] * n_ + be[q]);
            nrm[q] = n_;
            sg[q] = sgm;
            gsv[q] = 2.0f * sgm;
        }
        __syncthreads();
        for (int t = tid; t < H * M; t += kThreads) g[t] = gsv[t / M] * h[t];
        __syncthreads();
        for (int t = tid; t < Q * M; t += kThreads) {
            const int p = t / M, m = t - p * M;
            const float* wr = W2 + p * H;
            float acc = 0.0f;
            for (int q = 0; q < H; ++q) acc += wr[q] * g[q * M + m];
            ct[t] = acc;
        }
        __syncthreads();
        // dL/dc~_{p,m} = sum_q G_{pq} c~_{q,m}, G the symmetric unpacking of
        // the upstream gradient with a doubled diagonal
        for (int t = tid; t < Q * M; t += kThreads) {
            const int p = t / M, m = t - p * M;
            float acc = 0.0f;
            for (int q = 0; q < Q; ++q) {
                const int lo = p < q ? p : q, hi = p < q ? q : p;
                const float gv = gp[lo * Q - lo * (lo - 1) / 2 + (hi - lo)];
                acc += (p == q ? 2.0f * gv : gv) * ct[q * M + m];
            }
            dct[t] = acc;
        }
        __syncthreads();
        for (int t = tid; t < Q * H; t += kThreads) {
            const int p = t / H, q = t - p * H;
            float acc = 0.0f;
            for (int m = 0; m < M; ++m) acc += dct[p * M + m] * g[q * M + m];
            gW2[t] += acc;
        }
        for (int t = tid; t < H * M; t += kThreads) {
            const int q = t / M, m = t - q * M;
            float acc = 0.0f;
            for (int p = 0; p < Q; ++p) acc += W2[p * H + q] * dct[p * M + m];
            dh[t] = acc;                                  // dL/dg for now
        }
        __syncthreads();
        for (int q = tid; q < H; q += kThreads) {
            float dG = 0.0f;
            for (int m = 0; m < M; ++m) dG += dh[q * M + m] * h[q * M + m];
            const float dz = dG * 2.0f * sg[q] * (1.0f - sg[q]);
            gal[q] += dz * nrm[q];
            gbe[q] += dz;
            cf[q] = nrm[q] > 0.0f ? dz * al[q] / nrm[q] : 0.0f;
        }
        __syncthreads();
        for (int t = tid; t < H * M; t += kThreads) {
            const int q = t / M;
            dh[t] = dh[t] * gsv[q] + cf[q] * h[t];
        }
        __syncthreads();
        for (int t = tid; t < H * K; t += kThreads) {
            const int q = t / K, k = t - q * K;
            float acc = 0.0f;
            for (int m = 0; m < M; ++m) acc += dh[q * M + m] * x[k * M + m];
            gW1[t] += acc;
        }
        __syncthreads();
    }
    float* out = a.gpart + int64_t(s) * a.n_params + l * lsize;
    for (int e = tid; e < lsize; e += kThreads) out[e] = gW1[e];
}

__global__ void k_reduce(const float* part, int slices, int64_t n, float* out)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float acc = 0.0f;
    for (int s = 0; s < slices; ++s) acc += part[int64_t(s) * n + e];
    out[e] = acc;
}

// Per-l channel covariance sum_{i, m} c_{i,k1,lm} c_{i,k2,lm}, partial sums
// over slices of the centres.  Wide channel counts (K > 128): one
// work-group per (l, k1, slice), lanes over k2, centres s, s + S, ...
__global__ void __launch_bounds__(kThreads) k_channel_cov_wide(CompressArgs a, float* part)
{
    const int K = a.K, lmax = a.lmax, L2 = (lmax + 1) * (lmax + 1);
    const int l = blockIdx.x, k1 = blockIdx.y, S = gridDim.z, s = blockIdx.z;
    const int M = 2 * l + 1, b = l * l;
    for (int k2 = threadIdx.x; k2 < K; k2 += kThreads) {
        float acc = 0.0f;
        for (int64_t i = s; i < a.n; i += S) {
            const float* ci = a.c + i * int64_t(K) * L2 + b;
            for (int m = 0; m < M; ++m) acc += ci[k1 * L2 + m] * ci[k2 * L2 + m];
        }
        part[((int64_t(s) * (lmax + 1) + l) * K + k1) * K + k2] = acc;
    }
}

constexpr int kCovBatch = 4;
constexpr int kCovR = 8;

// Per-l channel covariance sum_{i, m} c_{i,k1,lm} c_{i,k2,lm} over a
// contiguous slice of the centres (grid (lmax + 1, slices)): kCovBatch
// centres' X_l at a time go to LDS (loads in flight together), and lane
// (a, b) of the 16 x 16 lanes accumulates the k1 = a + 16 u, k2 = b + 16 v
// entries in registers (K <= 16 kCovR).
__global__ void __launch_bounds__(kThreads) k_channel_cov(CompressArgs a, float* part)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* X = reinterpret_cast<float*>(smem_raw);   // [kCovBatch][K][M]
    const int K = a.K, lmax = a.lmax, L2 = (lmax + 1) * (lmax + 1);
    const int l = blockIdx.x, S = gridDim.y, s = blockIdx.y;
    const int M = 2 * l + 1, b = l * l, KM = K * M;
    const int64_t lo = a.n * s / S, hi = a.n * (s + 1) / S;
    const int ta = threadIdx.x >> 4, tb = threadIdx.x & 15;
    float acc[kCovR][kCovR];
#pragma unroll
    for (int u = 0; u < kCovR; ++u)
#pragma unroll
        for (int v = 0; v < kCovR; ++v) acc[u][v] = 0.0f;
    for (int64_t i0 = lo; i0 < hi; i0 += kCovBatch) {
        const int nb = hi - i0 < kCovBatch ? int(hi - i0) : kCovBatch;
        __syncthreads();
        for (int e0 = threadIdx.x; e0 < nb * KM; e0 += 8 * kThreads) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * kThreads;
                if (e < nb * KM) {
                    const int c = e / KM, r = e - c * KM, k = r / M, m = r - k * M;
                    v[u] = a.c[((i0 + c) * K + k) * int64_t(L2) + b + m];
                } else {
                    v[u] = 0.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e0 + u * kThreads < nb * KM) X[e0 + u * kThreads] = v[u];
        }
        __syncthreads();
        for (int c = 0; c < nb; ++c) {
            const float* Xc = X + c * KM;
            for (int m = 0; m < M; ++m) {
                float xa[kCovR], xb[kCovR];
#pragma unroll
                for (int u = 0; u < kCovR; ++u) {
                    const int k1 = ta + 16 * u, k2 = tb + 16 * u;
                    xa[u] = k1 < K ? Xc[k1 * M + m] : 0.0f;
                    xb[u] = k2 < K ? Xc[k2 * M + m] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kCovR; ++u)
#pragma unroll
                    for (int v = 0; v < kCovR; ++v) acc[u][v] += xa[u] * xb[v];
            }
        }
    }
    float* out = part + (int64_t(s) * (lmax + 1) + l) * K * K;
#pragma unroll
    for (int u = 0; u < kCovR; ++u)
#pragma unroll
        for (int v = 0; v < kCovR; ++v) {
            const int k1 = ta + 16 * u, k2 = tb + 16 * v;
            if (k1 < K && k2 < K) out[k1 * K + k2] = acc[u][v];
        }
}


// ------------------------------------------------ kernel matrix and loss
// Tiled products of the feature matrix X [n][F] (F = (lmax+1) Q(Q+1)/2):
// gram C = X diag(w) X^T, and C = D X (D [n][n]) scaled by w and a device
// scalar.  64 x 64 output tiles, 16-wide slices of the inner dimension in
// LDS, 4 x 4 outputs per lane.
constexpr int kT = 64, kKd = 16;

__global__ void __launch_bounds__(256) k_gram(int n, int F, int Q, const float* X, float* C)
{
    __shared__ float As[kKd][kT + 1], Bs[kKd][kT + 1];
    const int QQ = Q * (Q + 1) / 2;
    const int i0 = blockIdx.y * kT, j0 = blockIdx.x * kT;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    float acc[4][4] = {};
    for (int f0 = 0; f0 < F; f0 += kKd) {
        for (int e = threadIdx.x; e < kT * kKd; e += 256) {
            const int r = e / kKd, f = e - r * kKd, ff = f0 + f;
            const bool inf = ff < F;
            const float wf = inf ? full_weight(Q, ff % QQ) : 0.0f;
            As[f][r] = (inf && i0 + r < n) ? X[int64_t(i0 + r) * F + ff] * wf : 0.0f;
            Bs[f][r] = (inf && j0 + r < n) ? X[int64_t(j0 + r) * F + ff] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < kKd; ++f) {
            float av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) { av[u] = As[f][ty + 16 * u]; bv[u] = Bs[f][tx + 16 * u]; }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ty + 16 * u, j = j0 + tx + 16 * v;
            if (i < n && j < n) C[int64_t(i) * n + j] = acc[u][v];
        }
}

// loss = sum (Kt - Kref)^2 / sum Kref^2 (one work-group); D <- (Kt - Kref)
// in place of Kt and scale[0] = 4 / sum Kref^2 (the factor of dL/dX)
__global__ void __launch_bounds__(1024) k_kernel_loss(int64_t nn, float* Kt, const float* Kref, float* loss,
                                                      float* scale)
{
    __shared__ double s1[1024], s2[1024];
    double a1 = 0.0, a2 = 0.0;
    for (int64_t e = threadIdx.x; e < nn; e += 1024) {
        const double d = double(Kt[e]) - double(Kref[e]);
        Kt[e] = float(d);
        a1 += d * d;
        a2 += double(Kref[e]) * double(Kref[e]);
    }
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double norm2 = s2[0] > 0.0 ? s2[0] : 1.0;
        loss[0] = float(s1[0] / norm2);
        scale[0] = float(4.0 / norm2);
    }
}

// dX[i][f] = scale * w_f * sum_j D[i][j] X[j][f]  (D symmetric)
__global__ void __launch_bounds__(256) k_loss_grad(int n, int F, int Q, const float* D, const float* X,
                                                   const float* scale, float* dX)
{
    __shared__ float As[kKd][kT + 1], Bs[kKd][kT + 1];
    const int QQ = Q * (Q + 1) / 2;
    const int i0 = blockIdx.y * kT, f0 = blockIdx.x * kT;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    float acc[4][4] = {};
    for (int j0 = 0; j0 < n; j0 += kKd) {
        for (int e = threadIdx.x; e < kT * kKd; e += 256) {
            const int r = e / kKd, j = e - r * kKd;
            As[j][r] = (i0 + r < n && j0 + j < n) ? D[int64_t(i0 + r) * n + j0 + j] : 0.0f;
        }
        for (int e = threadIdx.x; e < kT * kKd; e += 256) {
            const int j = e / kT, f = e - j * kT;
            Bs[j][f] = (j0 + j < n && f0 + f < F) ? X[int64_t(j0 + j) * F + f0 + f] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kKd; ++j) {
            float av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) { av[u] = As[j][ty + 16 * u]; bv[u] = Bs[j][tx + 16 * u]; }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
        }
        __syncthreads();
    }
    const float sc = scale[0];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ty + 16 * u, f = f0 + tx + 16 * v;
            if (i < n && f < F) dX[int64_t(i) * F + f] = sc * full_weight(Q, f % QQ) * acc[u][v];
        }
}

// -------------------------------------------------------------- optimiser
// Adam (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// p <- p - lr mhat / (sqrt(vhat) + eps) with the bias corrections of step t.
__global__ void k_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gv = g[e];
    const float mv = b1 * m[e] + (1.0f - b1) * gv;
    const float vv = b2 * v[e] + (1.0f - b2) * gv * gv;
    m[e] = mv;
    v[e] = vv;
    p[e] -= lr * (mv / c1) / (sqrtf(vv / c2) + eps);
}

// ---------------------------------------------------- forward on MFMA
// Inference with bfloat16 operands and float accumulation
// (v_mfma_f32_16x16x32_bf16; lane (r = lane & 15, g = lane >> 4) holds
// A[r][8g + j], B[8g + j][r] and D[4g + v][r]).  A work-group of four
// waves owns 16 centres, the 16 columns of every product.  Per l:
//   X_l     c_{k, l^2 + m} of the 16 centres -> LDS, bfloat16, [m][centre][k];
//   pass 1  H_m = W1_l X_m (16-row tiles of hidden units spread over the
//           waves, W1 fragments held in registers for the whole l), summing
//           |h|^2 over m in registers; the gate factor per (q, centre);
//   pass 2  H_m again, times the gate, -> LDS bfloat16 [centre][q]; the
//           waves that own a 16-row tile of outputs form c~_m = W2_l G_m;
//   then    p~_{q1 q2} = sum_m c~ c~ per centre, written packed.
constexpr int kCC = 16;        // centres per work-group
constexpr int kMT = 4;         // hidden tiles per wave (H <= 256)
constexpr int kKS1 = 4;        // k-steps of the first layer (K <= 128)
constexpr int kKS2 = 8;        // k-steps of the second layer (H <= 256)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float f)
{
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

struct Bf16Dims {
    int Kp, XS, Hp, HS, QT, HT, KS1, KS2;
};

__host__ __device__ inline Bf16Dims bf16_dims(int K, int Q, int H)
{
    Bf16Dims d;
    d.Kp = (K + 31) / 32 * 32;
    d.XS = d.Kp + 8;            // row stride of X (bf16), padded against bank conflicts
    d.Hp = (H + 31) / 32 * 32;
    d.HS = d.Hp + 8;
    d.QT = (Q + 15) / 16;
    d.HT = (H + 15) / 16;
    d.KS1 = d.Kp / 32;
    d.KS2 = d.Hp / 32;
    return d;
}

template <bool WANT_CT, bool WANT_PT>
__global__ void __launch_bounds__(kThreads) k_cmp_fwd_bf16(CompressArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int K = a.K, Q = a.Q, H = a.H, lmax = a.lmax, L2 = (lmax + 1) * (lmax + 1), MX = 2 * lmax + 1;
    const int QQ = Q * (Q + 1) / 2;
    const Bf16Dims D = bf16_dims(K, Q, H);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
    const int64_t i0 = int64_t(blockIdx.x) * kCC;
    const int nc = a.n - i0 < kCC ? int(a.n - i0) : kCC;
    unsigned short* Xs = reinterpret_cast<unsigned short*>(smem_raw);      // [MX][kCC][XS]
    unsigned short* Hs = Xs + MX * kCC * D.XS;                              // [kCC][HS]
    float* CT = reinterpret_cast<float*>(smem_raw + ((2 * size_t(MX * kCC * D.XS + kCC * D.HS) + 15) & ~size_t(15)));
    const float* w = a.w;
    for (int l = 0; l <= lmax; ++l) {
        const int M = 2 * l + 1, b = l * l;
        const float* W1 = w;
        const float* W2 = W1 + H * K;
        const float* al = W2 + Q * H;
        const float* be = al + H;
        w = be + H;
        // X_l of the 16 centres, bfloat16, zero beyond K and beyond the last centre
        for (int e = tid; e < kCC * D.Kp * M; e += kThreads) {
            const int m = e % M, k = (e / M) % D.Kp, c = e / (M * D.Kp);
            float v = 0.0f;
            if (k < K && c < nc) v = a.c[((i0 + c) * K + k) * L2 + b + m];
            Xs[(m * kCC + c) * D.XS + k] = to_bf16(v);
        }
        // first-layer fragments of this wave's hidden tiles (tile = wave + 4 t)
        u16x8 A1[kMT][kKS1];
#pragma unroll
        for (int t = 0; t < kMT; ++t)
#pragma unroll
            for (int ks = 0; ks < kKS1; ++ks) {
                const int q = (wave + 4 * t) * 16 + r;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = ks * 32 + 8 * g + j;
                    A1[t][ks][j] = (q < H && k < K && ks < D.KS1) ? to_bf16(W1[q * K + k]) : (unsigned short)0;
                }
            }
        __syncthreads();
        // pass 1: |h_q|^2 over m for the (q, centre) this lane holds
        float n2[kMT][4] = {};
        for (int m = 0; m < M; ++m) {
            u16x8 B[kKS1];
#pragma unroll
            for (int ks = 0; ks < kKS1; ++ks)
                if (ks < D.KS1) B[ks] = *reinterpret_cast<const u16x8*>(&Xs[(m * kCC + r) * D.XS + ks * 32 + 8 * g]);
#pragma unroll
            for (int t = 0; t < kMT; ++t) {
                if (wave + 4 * t >= D.HT) break;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < kKS1; ++ks)
                    if (ks < D.KS1)
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A1[t][ks]),
                                                                      __builtin_bit_cast(bf16x8, B[ks]), acc, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) n2[t][v] += acc[v] * acc[v];
            }
        }
        // gate factor 2 sigma(alpha |h| + beta) of (q = tile 16 + 4g + v, centre r)
        float G[kMT][4];
#pragma unroll
        for (int t = 0; t < kMT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q = (wave + 4 * t) * 16 + 4 * g + v;
                G[t][v] = q < H ? 2.0f * sigm(al[q] * sqrtf(n2[t][v]) + be[q]) : 0.0f;
            }
        // second-layer fragments: wave w owns output tile w
        u16x8 A2[kKS2];
#pragma unroll
        for (int ks = 0; ks < kKS2; ++ks) {
            const int p = wave * 16 + r;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int q = ks * 32 + 8 * g + j;
                A2[ks][j] = (wave < D.QT && p < Q && q < H && ks < D.KS2) ? to_bf16(W2[p * H + q]) : (unsigned short)0;
            }
        }
        // pass 2: gated hidden layer -> LDS, then c~_m
        for (int m = 0; m < M; ++m) {
            u16x8 B[kKS1];
#pragma unroll
            for (int ks = 0; ks < kKS1; ++ks)
                if (ks < D.KS1) B[ks] = *reinterpret_cast<const u16x8*>(&Xs[(m * kCC + r) * D.XS + ks * 32 + 8 * g]);
#pragma unroll
            for (int t = 0; t < kMT; ++t) {
                if (wave + 4 * t >= D.HT) break;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < kKS1; ++ks)
                    if (ks < D.KS1)
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A1[t][ks]),
                                                                      __builtin_bit_cast(bf16x8, B[ks]), acc, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = (wave + 4 * t) * 16 + 4 * g + v;
                    Hs[r * D.HS + q] = to_bf16(acc[v] * G[t][v]);
                }
            }
            // hidden units in [HT 16, Hp) stay zero
            for (int e = tid; e < kCC * (D.Hp - D.HT * 16); e += kThreads) {
                const int c = e / (D.Hp - D.HT * 16), q = D.HT * 16 + e % (D.Hp - D.HT * 16);
                Hs[c * D.HS + q] = 0;
            }
            __syncthreads();
            if (wave < D.QT) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < kKS2; ++ks)
                    if (ks < D.KS2) {
                        const u16x8 Bv = *reinterpret_cast<const u16x8*>(&Hs[r * D.HS + ks * 32 + 8 * g]);
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A2[ks]),
                                                                      __builtin_bit_cast(bf16x8, Bv), acc, 0, 0, 0);
                    }
#pragma unroll
                for (int v = 0; v < 4; ++v) CT[(m * (D.QT * 16) + wave * 16 + 4 * g + v) * kCC + r] = acc[v];
            }
            __syncthreads();
        }
        // p~ of the 16 centres; c~ if asked for
        if (WANT_PT)
            for (int e = tid; e < nc * QQ; e += kThreads) {
                const int c = e / QQ, t = e - c * QQ;
                int q1, q2;
                tri_decode(Q, t, q1, q2);
                float acc = 0.0f;
                for (int m = 0; m < M; ++m)
                    acc += CT[(m * (D.QT * 16) + q1) * kCC + c] * CT[(m * (D.QT * 16) + q2) * kCC + c];
                a.pt[((i0 + c) * (lmax + 1) + l) * int64_t(QQ) + t] = acc;
            }
        if (WANT_CT)
            for (int e = tid; e < nc * Q * M; e += kThreads) {
                const int m = e % M, q = (e / M) % Q, c = e / (M * Q);
                a.ct[((i0 + c) * Q + q) * L2 + b + m] = CT[(m * (D.QT * 16) + q) * kCC + c];
            }
        __syncthreads();
    }
}

size_t compress_bf16_lds(const CompressArgs& a)
{
    const Bf16Dims D = bf16_dims(a.K, a.Q, a.H);
    const int MX = 2 * a.lmax + 1;
    const size_t ct_slices = a.Q <= 32 ? 1 : size_t(MX);   // one m slice of c~ when p~ sums in registers
    return ((2 * size_t(MX * kCC * D.XS + kCC * D.HS) + 15) & ~size_t(15)) + 4 * ct_slices * D.QT * 16 * kCC;
}

// The same product for Q <= 32 with the packed p~ of the 16 centres kept
// in registers and summed over m as each c~_m appears (one m slice of c~
// in LDS instead of all of them): about half the LDS of the form above, so
// two work-groups share a CU.  Lane j < ceil(Q/2) of centre c (16 lanes
// per centre) owns rows q1 = j and Q-1-j of its packed triangle, Q + 1
// entries, so no index is decoded.  X_l is read row by row, the M values
// of a (centre, k) row in flight together.
constexpr int kMMax = 25;   // 2 lmax + 1 for lmax <= 12

template <bool WANT_CT, bool WANT_PT, int QMAX>
__global__ void __launch_bounds__(kThreads, 2) k_cmp_fwd_bf16_r(CompressArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int K = a.K, Q = a.Q, H = a.H, lmax = a.lmax, L2 = (lmax + 1) * (lmax + 1), MX = 2 * lmax + 1;
    const int QQ = Q * (Q + 1) / 2;
    const Bf16Dims D = bf16_dims(K, Q, H);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
    const int64_t i0 = int64_t(blockIdx.x) * kCC;
    const int nc = a.n - i0 < kCC ? int(a.n - i0) : kCC;
    unsigned short* Xs = reinterpret_cast<unsigned short*>(smem_raw);      // [MX][kCC][XS]
    unsigned short* Hs = Xs + MX * kCC * D.XS;                              // [kCC][HS]
    float* CTm = reinterpret_cast<float*>(smem_raw + ((2 * size_t(MX * kCC * D.XS + kCC * D.HS) + 15) & ~size_t(15)));
    // p~ rows of this lane: centre pc, rows q1 = pj and Q-1-pj (once if equal)
    const int pc = tid >> 4, pj = tid & 15;
    const int rowA = pj, rowB = Q - 1 - pj;
    const bool p_on = WANT_PT && pc < nc && rowA <= rowB;
    const int nA = Q - rowA, nB = rowB > rowA ? Q - rowB : 0;   // entries of the two rows
    float acc_p[QMAX + 1];
#pragma unroll
    for (int u = 0; u <= QMAX; ++u) acc_p[u] = 0.0f;
    const float* w = a.w;
    for (int l = 0; l <= lmax; ++l) {
        const int M = 2 * l + 1, b = l * l;
        const float* W1 = w;
        const float* W2 = W1 + H * K;
        const float* al = W2 + Q * H;
        const float* be = al + H;
        w = be + H;
        // X_l of the 16 centres, bfloat16, zero beyond K and beyond the last centre
        for (int row = tid; row < kCC * D.Kp; row += kThreads) {
            const int c = row / D.Kp, k = row - c * D.Kp;
            const bool ok = k < K && c < nc;
            const float* src = a.c + ((i0 + (ok ? c : 0)) * K + (ok ? k : 0)) * L2 + b;
            float v[kMMax];
#pragma unroll
            for (int m = 0; m < kMMax; ++m) v[m] = (ok && m < M) ? src[m] : 0.0f;
#pragma unroll
            for (int m = 0; m < kMMax; ++m)
                if (m < M) Xs[(m * kCC + c) * D.XS + k] = to_bf16(v[m]);
        }
        u16x8 A1[kMT][kKS1];
#pragma unroll
        for (int t = 0; t < kMT; ++t)
#pragma unroll
            for (int ks = 0; ks < kKS1; ++ks) {
                const int q = (wave + 4 * t) * 16 + r;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = ks * 32 + 8 * g + j;
                    A1[t][ks][j] = (q < H && k < K && ks < D.KS1) ? to_bf16(W1[q * K + k]) : (unsigned short)0;
                }
            }
        __syncthreads();
        float n2[kMT][4] = {};
        for (int m = 0; m < M; ++m) {
            u16x8 B[kKS1];
#pragma unroll
            for (int ks = 0; ks < kKS1; ++ks)
                if (ks < D.KS1) B[ks] = *reinterpret_cast<const u16x8*>(&Xs[(m * kCC + r) * D.XS + ks * 32 + 8 * g]);
#pragma unroll
            for (int t = 0; t < kMT; ++t) {
                if (wave + 4 * t >= D.HT) break;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < kKS1; ++ks)
                    if (ks < D.KS1)
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A1[t][ks]),
                                                                      __builtin_bit_cast(bf16x8, B[ks]), acc, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) n2[t][v] += acc[v] * acc[v];
            }
        }
        float G[kMT][4];
#pragma unroll
        for (int t = 0; t < kMT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q = (wave + 4 * t) * 16 + 4 * g + v;
                G[t][v] = q < H ? 2.0f * sigm(al[q] * sqrtf(n2[t][v]) + be[q]) : 0.0f;
            }
        u16x8 A2[kKS2];
#pragma unroll
        for (int ks = 0; ks < kKS2; ++ks) {
            const int p = wave * 16 + r;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int q = ks * 32 + 8 * g + j;
                A2[ks][j] = (wave < D.QT && p < Q && q < H && ks < D.KS2) ? to_bf16(W2[p * H + q]) : (unsigned short)0;
            }
        }
        for (int m = 0; m < M; ++m) {
            u16x8 B[kKS1];
#pragma unroll
            for (int ks = 0; ks < kKS1; ++ks)
                if (ks < D.KS1) B[ks] = *reinterpret_cast<const u16x8*>(&Xs[(m * kCC + r) * D.XS + ks * 32 + 8 * g]);
#pragma unroll
            for (int t = 0; t < kMT; ++t) {
                if (wave + 4 * t >= D.HT) break;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < kKS1; ++ks)
                    if (ks < D.KS1)
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A1[t][ks]),
                                                                      __builtin_bit_cast(bf16x8, B[ks]), acc, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = (wave + 4 * t) * 16 + 4 * g + v;
                    Hs[r * D.HS + q] = to_bf16(acc[v] * G[t][v]);
                }
            }
            for (int e = tid; e < kCC * (D.Hp - D.HT * 16); e += kThreads) {
                const int c = e / (D.Hp - D.HT * 16), q = D.HT * 16 + e % (D.Hp - D.HT * 16);
                Hs[c * D.HS + q] = 0;
            }
            __syncthreads();
            if (wave < D.QT) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < kKS2; ++ks)
                    if (ks < D.KS2) {
                        const u16x8 Bv = *reinterpret_cast<const u16x8*>(&Hs[r * D.HS + ks * 32 + 8 * g]);
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A2[ks]),
                                                                      __builtin_bit_cast(bf16x8, Bv), acc, 0, 0, 0);
                    }
                // c~_m[q][centre]
#pragma unroll
                for (int v = 0; v < 4; ++v) CTm[(wave * 16 + 4 * g + v) * kCC + r] = acc[v];
            }
            __syncthreads();
            if (p_on) {
                const float a1 = CTm[rowA * kCC + pc], b1 = CTm[rowB * kCC + pc];
#pragma unroll
                for (int u = 0; u <= QMAX; ++u) {
                    // entry u: (rowA, rowA + u) for u < nA, then (rowB, rowB + u - nA)
                    if (u < nA) acc_p[u] += a1 * CTm[(rowA + u) * kCC + pc];
                    else if (u < nA + nB) acc_p[u] += b1 * CTm[(rowB + u - nA) * kCC + pc];
                }
            }
            if (WANT_CT)
                for (int e = tid; e < nc * Q; e += kThreads) {
                    const int q = e % Q, c = e / Q;
                    a.ct[((i0 + c) * Q + q) * L2 + b + m] = CTm[q * kCC + c];
                }
        }
        if (p_on) {
            float* dst = a.pt + ((i0 + pc) * (lmax + 1) + l) * int64_t(QQ);
            const int sA = rowA * Q - rowA * (rowA - 1) / 2, sB = rowB * Q - rowB * (rowB - 1) / 2;
#pragma unroll
            for (int u = 0; u <= QMAX; ++u) {
                if (u < nA) dst[sA + u] = acc_p[u];
                else if (u < nA + nB) dst[sB + u - nA] = acc_p[u];
                acc_p[u] = 0.0f;
            }
        }
        __syncthreads();
    }
}

inline unsigned blocks_of(int64_t n, int t) { return unsigned((n + t - 1) / t); }

}  // namespace

size_t compress_fwd_lds(const CompressArgs& a)
{
    const int L2 = (a.lmax + 1) * (a.lmax + 1), MX = 2 * a.lmax + 1;
    return sizeof(float) * (size_t(a.K) * L2 + size_t(a.H) * MX + a.H + size_t(a.Q) * MX);
}

size_t compress_bwd_lds(const CompressArgs& a)
{
    const int MX = 2 * a.lmax + 1, QQ = a.Q * (a.Q + 1) / 2;
    const size_t lsize = size_t(a.H) * a.K + size_t(a.Q) * a.H + 2 * size_t(a.H);
    return sizeof(float) * (lsize + size_t(a.K) * MX + 3 * size_t(a.H) * MX + 2 * size_t(a.Q) * MX +
                            4 * size_t(a.H) + QQ);
}

hipError_t launch_compress_forward(const CompressArgs& a, hipStream_t stream)
{
    if (a.n == 0) return hipSuccess;
    const size_t lds = compress_fwd_lds(a);
    if (lds > 160 * 1024) return hipErrorNotSupported;
    auto kernel = a.ct ? (a.pt ? k_cmp_fwd<true, true> : k_cmp_fwd<true, false>) : k_cmp_fwd<false, true>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, dim3(unsigned(a.n)), dim3(kThreads), lds, stream, a);
    return hipGetLastError();
}


hipError_t launch_compress_forward_bf16(const CompressArgs& a, hipStream_t stream)
{
    if (a.n == 0) return hipSuccess;
    if (a.K > 32 * kKS1 || a.H > 16 * 4 * kMT || a.Q > 64) return hipErrorNotSupported;
    const size_t lds = compress_bf16_lds(a);
    if (lds > 160 * 1024) return hipErrorNotSupported;
    auto kernel = a.Q <= 16 ? (a.ct ? (a.pt ? k_cmp_fwd_bf16_r<true, true, 16> : k_cmp_fwd_bf16_r<true, false, 16>)
                                    : k_cmp_fwd_bf16_r<false, true, 16>)
                : a.Q <= 32 ? (a.ct ? (a.pt ? k_cmp_fwd_bf16_r<true, true, 32> : k_cmp_fwd_bf16_r<true, false, 32>)
                                    : k_cmp_fwd_bf16_r<false, true, 32>)
                            : (a.ct ? (a.pt ? k_cmp_fwd_bf16<true, true> : k_cmp_fwd_bf16<true, false>)
                                    : k_cmp_fwd_bf16<false, true>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, dim3(blocks_of(a.n, kCC)), dim3(kThreads), lds, stream, a);
    return hipGetLastError();
}

hipError_t launch_compress_backward(const CompressArgs& a, float* grad, hipStream_t stream)
{
    const size_t lds = compress_bwd_lds(a);
    if (lds > 160 * 1024) return hipErrorNotSupported;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_cmp_bwd),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_cmp_bwd, dim3(unsigned(a.lmax + 1), unsigned(a.slices)), dim3(kThreads), lds, stream, a);
    hipLaunchKernelGGL(k_reduce, dim3(blocks_of(a.n_params, 256)), dim3(256), 0, stream, a.gpart, a.slices,
                       a.n_params, grad);
    return hipGetLastError();
}

hipError_t launch_channel_cov(const CompressArgs& a, float* part, int slices, hipStream_t stream)
{
    if (a.K > 16 * kCovR) {
        hipLaunchKernelGGL(k_channel_cov_wide, dim3(unsigned(a.lmax + 1), unsigned(a.K), unsigned(slices)),
                           dim3(kThreads), 0, stream, a, part);
        return hipGetLastError();
    }
    const size_t lds = sizeof(float) * kCovBatch * size_t(a.K) * (2 * a.lmax + 1);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_channel_cov),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_channel_cov, dim3(unsigned(a.lmax + 1), unsigned(slices)), dim3(kThreads), lds, stream, a,
                       part);
    return hipGetLastError();
}

hipError_t launch_spectrum_gram(int n, int Q, int lmax, const float* X, float* C, hipStream_t stream)
{
    const int F = (lmax + 1) * Q * (Q + 1) / 2;
    hipLaunchKernelGGL(k_gram, dim3(blocks_of(n, kT), blocks_of(n, kT)), dim3(256), 0, stream, n, F, Q, X, C);
    return hipGetLastError();
}

hipError_t launch_spectrum_kernel_loss(int n, int Q, int lmax, const float* X, const float* Kref, float* Kt,
                                       float* loss, float* scale, float* dX, hipStream_t stream)
{
    const int F = (lmax + 1) * Q * (Q + 1) / 2;
    hipLaunchKernelGGL(k_gram, dim3(blocks_of(n, kT), blocks_of(n, kT)), dim3(256), 0, stream, n, F, Q, X, Kt);
    hipLaunchKernelGGL(k_kernel_loss, dim3(1), dim3(1024), 0, stream, int64_t(n) * n, Kt, Kref, loss, scale);
    hipLaunchKernelGGL(k_loss_grad, dim3(blocks_of(F, kT), blocks_of(n, kT)), dim3(256), 0, stream, n, F, Q, Kt, X,
                       scale, dX);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                       float eps, int step, hipStream_t stream)
{
    const float c1 = 1.0f - std::pow(b1, float(step)), c2 = 1.0f - std::pow(b2, float(step));
    hipLaunchKernelGGL(k_adam, dim3(blocks_of(n, 256)), dim3(256), 0, stream, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace soap
