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

// One wave per centre, cpw centres per work-group sharing the weights of
// the current l in LDS.  The centre's c of degree l goes to the wave's LDS
// as FP32 rows [k][2l+1], copied straight from global memory to LDS while
// the previous l computes (after its layer 1 has read its own), and is
// rounded to bfloat16 as the layer-1 operands are read; holding one l
// rather than every lm lets twice as many centres share a work-group.  Per
// l the columns of every product are the m of the centre (one 16-wide
// tile, two when 2l + 1 > 16):
//   layer 1  h = W1_l X_m, 16-row tiles of hidden units, 32-wide k-steps;
//            h stays in registers for the whole l;
//   gate     |h_q|^2 over m, summed across the 16 column lanes of a row
//            with DPP rotations;
//   layer 2  c~ = W2_l (G h).  W1_l is staged in LDS with its rows in the
//            order that makes a lane's layer-1 accumulators its operand of
//            the layer-2 product: row 4g + v of tile t holds hidden unit
//            32 (t >> 1) + 8 g + 4 (t & 1) + v, so the two tiles of k-step
//            ks give lane g exactly units 32 ks + 8 g + j, j < 8;
//   p~       the Gram matrix of c~ over m on the matrix cores, c~ split into
//            bfloat16 high and low parts (H H^T + H L^T + L H^T, as for the
//            full spectrum), from c~ staged in the wave's own LDS.
// Two work-group barriers per l (the shared weights); none per m.
constexpr int kWaveCentres = 8;   // most centres (waves) per work-group
constexpr int kCB = 36;           // row stride of the c~ staging (floats, 16-byte rows)
constexpr int kWQuads = 12;       // weight float4s a lane stages per l from kept offsets

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// two floats to packed bfloat16 (round to nearest even), low half first
__device__ __forceinline__ unsigned int pack_bf16(float lo, float hi)
{
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(unsigned int, __builtin_convertvector(v, bf16x2));
}

// sum over the 16 lanes of a DPP row (every lane receives the sum)
__device__ __forceinline__ float row_sum16(float s)
{
    s += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), 0x128, 0xF, 0xF, false));
    s += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), 0x124, 0xF, 0xF, false));
    s += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), 0x122, 0xF, 0xF, false));
    s += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), 0x121, 0xF, 0xF, false));
    return s;
}

struct WaveLayout {
    int Kp, XS, Hp, HS, HT, KS, KS2, QT, cpw;
    int E1, E2, E;           // weight float4s per l: W1 rows, W2 rows, then {alpha, beta}
    int x_bytes, cb_bytes;   // per centre
    int w1, w2, ab, x, cb, total;   // byte offsets, 16-byte aligned
    int wbytes;              // bytes of one l's weights in LDS
    int wstride;             // with the image: one l's image rounded up to whole 1 KB pieces (two LDS buffers)
};

__host__ __device__ inline int up16(int b) { return (b + 15) & ~15; }

__host__ __device__ inline WaveLayout wave_layout(int K, int Q, int H, int lmax, int cpw, bool img = false)
{
    WaveLayout W;
    W.Kp = (K + 31) / 32 * 32;
    W.XS = W.Kp + 8;   // row stride (bf16) of W1: 16 consecutive rows hit distinct banks
    W.Hp = (H + 31) / 32 * 32;
    W.HS = W.Hp + 8;
    W.HT = W.Hp / 16;
    W.KS = W.Kp / 32;
    W.KS2 = W.Hp / 32;
    W.QT = (Q + 15) / 16;
    W.cpw = cpw;
    W.E1 = W.HT * 16 * (W.Kp / 4);
    W.E2 = W.QT * 16 * (W.Hp / 4);
    W.E = W.E1 + W.E2 + W.Hp / 2;
    const int L2 = (lmax + 1) * (lmax + 1);
    // c of one l in FP32, [k][2l+1] rows, whole 64-element pieces
    W.x_bytes = up16(((K * (2 * lmax + 1) + 63) / 64) * 64 * 4);
    W.cb_bytes = up16(W.QT * 16 * kCB * 4);
    int o = 0;
    W.w1 = o; o += up16(W.HT * 16 * W.XS * 2);
    W.w2 = o; o += up16(W.QT * 16 * W.HS * 2);
    W.ab = o; o += up16(2 * W.Hp * 4);
    W.wbytes = o;
    W.wstride = (o + 1023) & ~1023;
    if (img) o = 2 * W.wstride;
    W.x = o; o += cpw * W.x_bytes;
    W.cb = o; o += cpw * W.cb_bytes;
    W.total = o;
    return W;
}

// hidden unit held by LDS row `row` of the staged W1
__device__ __forceinline__ int wave_unit(int row)
{
    const int t = row >> 4, rho = row & 15;
    return 32 * (t >> 1) + 8 * (rho >> 2) + 4 * (t & 1) + (rho & 3);
}

// Weight float4 e of one l: its offset in the l's weights (-1: outside
// them, staged as zeros) and its byte offset in LDS.  W1 rows (bfloat16, in
// the unit order above), W2 rows (bfloat16), then {alpha_l, beta_l} (float).
__device__ __forceinline__ void wave_weight_slot(const CompressArgs& a, const WaveLayout& W, int e, int& src, int& dst)
{
    const int K = a.K, H = a.H, Q = a.Q;
    if (e < W.E1) {
        const int kq = W.Kp / 4, row = e / kq, k = 4 * (e - row * kq), q = wave_unit(row);
        src = (q < H && k < K) ? q * K + k : -1;
        dst = W.w1 + 2 * (row * W.XS + k);
    } else if (e < W.E1 + W.E2) {
        const int hq = W.Hp / 4, f = e - W.E1, p = f / hq, q = 4 * (f - p * hq);
        src = (p < Q && q < H) ? H * K + p * H + q : -1;
        dst = W.w2 + 2 * (p * W.HS + q);
    } else {
        const int j = 4 * (e - W.E1 - W.E2), q = j < W.Hp ? j : j - W.Hp;
        src = q < H ? H * K + Q * H + (j < W.Hp ? 0 : H) + q : -1;
        dst = W.ab + 4 * j;
    }
}

__device__ __forceinline__ void wave_weight_put(unsigned char* smem, const WaveLayout& W, int dst, float4 v)
{
    if (dst < W.ab) {
        uint2 pk;
        pk.x = pack_bf16(v.x, v.y);
        pk.y = pack_bf16(v.z, v.w);
        *reinterpret_cast<uint2*>(smem + dst) = pk;
    } else {
        *reinterpret_cast<float4*>(smem + dst) = v;
    }
}

// The weights of every l as they sit in LDS (bfloat16 rows of W1 in the
// unit order, W2 rows, then {alpha, beta} in float, zeros elsewhere): one
// work-group per l writes bytes [0, W.x) of image l.
__global__ void __launch_bounds__(256) k_cmp_image(CompressArgs a, WaveLayout W)
{
    const int l = blockIdx.x;
    unsigned char* img = static_cast<unsigned char*>(a.img) + size_t(l) * W.wstride;
    const float* wl = a.w + size_t(l) * (a.H * a.K + a.Q * a.H + 2 * a.H);
    for (int e = threadIdx.x; e < W.wstride / 16; e += blockDim.x)
        reinterpret_cast<uint4*>(img)[e] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    for (int e = threadIdx.x; e < W.E; e += blockDim.x) {
        int src, dst;
        wave_weight_slot(a, W, e, src, dst);
        wave_weight_put(img, W, dst, src >= 0 ? *reinterpret_cast<const float4*>(wl + src) : make_float4(0.f, 0.f, 0.f, 0.f));
    }
}


// the layer-1 operand of column m: X[k0 + j][m], j < 8, as bfloat16 (zero
// for k >= K), from the FP32 rows [k][w] of one l
__device__ __forceinline__ u16x8 x_operand(const float* Xf, int w, int m, int k0, int K)
{
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = k0 + j < K ? Xf[(k0 + j) * w + m] : 0.0f;
    u32x4 p;
#pragma unroll
    for (int j = 0; j < 4; ++j) p[j] = pack_bf16(x[2 * j], x[2 * j + 1]);
    return __builtin_bit_cast(u16x8, p);
}

template <bool WANT_CT, bool WANT_PT, int QT, bool IMG>
__global__ void __launch_bounds__(kWaveCentres * 64) k_cmp_fwd_wave(CompressArgs a, WaveLayout W)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int K = a.K, Q = a.Q, H = a.H, lmax = a.lmax, L2 = (lmax + 1) * (lmax + 1);
    const int QQ = Q * (Q + 1) / 2;
    const int tid = threadIdx.x, nthr = blockDim.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
    const int64_t i = int64_t(blockIdx.x) * W.cpw + wave;
    const bool live = i < a.n;
    const unsigned short* W1s = reinterpret_cast<const unsigned short*>(smem_raw + W.w1);
    const unsigned short* W2s = reinterpret_cast<const unsigned short*>(smem_raw + W.w2);
    const float* ab = reinterpret_cast<const float*>(smem_raw + W.ab);   // (buffer l % 2 with the image)
    float* Xf = reinterpret_cast<float*>(smem_raw + W.x + wave * W.x_bytes);
    float* cb = reinterpret_cast<float*>(smem_raw + W.cb + wave * W.cb_bytes);
    const int lsize = H * K + Q * H + 2 * H;

    // this lane's weight float4s (the same offsets for every l)
    int wsrc[IMG ? 1 : kWQuads], wdst[IMG ? 1 : kWQuads];
    if constexpr (!IMG) {
#pragma unroll
        for (int u = 0; u < kWQuads; ++u) {
            const int e = tid + nthr * u;
            wsrc[u] = -1;
            wdst[u] = -1;
            if (e < W.E) wave_weight_slot(a, W, e, wsrc[u], wdst[u]);
        }
    }
    // with the image: l's weights go straight from global memory to LDS
    // buffer l % 2 (16 bytes per lane, 1 KB per wave and instruction), the
    // next l's while the current one is computed
    const int nwaves = nthr >> 6;
    auto fetch_image = [&](int l) __attribute__((always_inline)) {
        const unsigned char* src = static_cast<const unsigned char*>(a.img) + size_t(l) * W.wstride;
        unsigned char* dst = smem_raw + (l & 1) * W.wstride;
        for (int piece = wave; piece < W.wstride / 1024; piece += nwaves)
            __builtin_amdgcn_global_load_lds(src + piece * 1024 + lane * 16,
                                             (__attribute__((address_space(3))) void*)(dst + piece * 1024),
                                             16, 0, 0);
    };
    if constexpr (IMG) fetch_image(0);

    // c of degree l of this centre into the wave's X, FP32 rows [k][2l+1],
    // straight from global memory to LDS (64 elements per instruction; the
    // lanes past the end of the last piece read the first element and write
    // the piece's tail, which nothing reads), issued one l ahead
    const float* cc = a.c + (live ? i : 0) * int64_t(K) * L2;
    auto fetch_x = [&](int l) __attribute__((always_inline)) {
        const int w = 2 * l + 1, n = K * w;
        const float inv = 1.0f / float(w);
        for (int e0 = 0; e0 < n; e0 += 64) {
            const int e = e0 + lane < n ? e0 + lane : 0;
            const int k = int((float(e) + 0.5f) * inv), m = e - k * w;
            __builtin_amdgcn_global_load_lds(cc + k * L2 + l * l + m,
                                             (__attribute__((address_space(3))) void*)(Xf + e0), 4, 0, 0);
        }
    };
    if (live) fetch_x(0);

    const float* wl = a.w;
    for (int l = 0; l <= lmax; ++l, wl += lsize) {
        __syncthreads();   // the weights of l - 1 are no longer read
        if constexpr (IMG) {
            // l's image is in buffer l % 2 once every wave's loads are done;
            // buffer (l + 1) % 2 held l - 1, which no wave reads any more
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (l < lmax) fetch_image(l + 1);
            const unsigned char* wb = smem_raw + (l & 1) * W.wstride;
            W1s = reinterpret_cast<const unsigned short*>(wb + W.w1);
            W2s = reinterpret_cast<const unsigned short*>(wb + W.w2);
            ab = reinterpret_cast<const float*>(wb + W.ab);
        } else {
            __builtin_amdgcn_s_waitcnt(0);   // this wave's X of l
            float4 wv[kWQuads];
#pragma unroll
            for (int u = 0; u < kWQuads; ++u)   // every load issued before any is used
                wv[u] = *reinterpret_cast<const float4*>(wl + (wsrc[u] >= 0 ? wsrc[u] : 0));
#pragma unroll
            for (int u = 0; u < kWQuads; ++u)
                if (wdst[u] >= 0)
                    wave_weight_put(smem_raw, W, wdst[u], wsrc[u] >= 0 ? wv[u] : make_float4(0.f, 0.f, 0.f, 0.f));
            for (int e = tid + nthr * kWQuads; e < W.E; e += nthr) {   // beyond the kept offsets
                int s0, d0;
                wave_weight_slot(a, W, e, s0, d0);
                wave_weight_put(smem_raw, W, d0,
                                s0 >= 0 ? *reinterpret_cast<const float4*>(wl + s0) : make_float4(0.f, 0.f, 0.f, 0.f));
            }
            __syncthreads();
        }
        if (!live) continue;
        const int M = 2 * l + 1, b = l * l, MT = (M + 15) >> 4;
        // layer 1: k-steps outside, the hidden tiles' accumulators inside;
        // each W1 fragment serves both column tiles as it is read
        f32x4 h[2][8];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int t = 0; t < 8; ++t) h[ct][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            if (kk < W.KS) {
                u16x8 B0 = u16x8{0, 0, 0, 0, 0, 0, 0, 0}, B1 = B0;
                if (r < M) B0 = x_operand(Xf, M, r, 32 * kk + 8 * g, K);
                if (16 + r < M) B1 = x_operand(Xf, M, 16 + r, 32 * kk + 8 * g, K);
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    if (t < W.HT) {
                        const u16x8 A = *reinterpret_cast<const u16x8*>(&W1s[(16 * t + r) * W.XS + 32 * kk + 8 * g]);
                        h[0][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, A), __builtin_bit_cast(bf16x8, B0), h[0][t], 0, 0, 0);
                        if (MT > 1)
                            h[1][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf16x8, A), __builtin_bit_cast(bf16x8, B1), h[1][t], 0, 0, 0);
                    }
                }
            }
        }
        wave_sync();   // every read of X of l is done
        if (l < lmax) fetch_x(l + 1);
        // gate factor 2 sigma(alpha |h| + beta) of unit q (row 4g + v of
        // tile t), |h_q|^2 summed over the m columns (zero where not
        // computed); h is scaled in place
        for (int t = 0; t < 8; ++t) {
            const int q0 = 32 * (t >> 1) + 8 * g + 4 * (t & 1);
            const float4 al = *reinterpret_cast<const float4*>(ab + q0);
            const float4 be = *reinterpret_cast<const float4*>(ab + W.Hp + q0);
            const float alv[4] = {al.x, al.y, al.z, al.w}, bev[4] = {be.x, be.y, be.z, be.w};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float s = row_sum16(h[0][t][v] * h[0][t][v] + h[1][t][v] * h[1][t][v]);
                const float x = alv[v] * __builtin_amdgcn_sqrtf(s) + bev[v];
                const float G = (t < W.HT && q0 + v < H)
                                    ? 2.0f * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * x))
                                    : 0.0f;
                h[0][t][v] *= G;
                h[1][t][v] *= G;
            }
        }
        // layer 2: c~ of the m columns -> the wave's staging (and c~ out)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            if (ct >= MT) continue;
            f32x4 acc2[QT];
#pragma unroll
            for (int pt = 0; pt < QT; ++pt) acc2[pt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                if (ks >= W.KS2) continue;
                u32x4 Bw;
                Bw[0] = pack_bf16(h[ct][2 * ks][0], h[ct][2 * ks][1]);
                Bw[1] = pack_bf16(h[ct][2 * ks][2], h[ct][2 * ks][3]);
                Bw[2] = pack_bf16(h[ct][2 * ks + 1][0], h[ct][2 * ks + 1][1]);
                Bw[3] = pack_bf16(h[ct][2 * ks + 1][2], h[ct][2 * ks + 1][3]);
#pragma unroll
                for (int pt = 0; pt < QT; ++pt) {
                    const u16x8 A2 = *reinterpret_cast<const u16x8*>(&W2s[(16 * pt + r) * W.HS + 32 * ks + 8 * g]);
                    acc2[pt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A2),
                                                                       __builtin_bit_cast(bf16x8, Bw), acc2[pt], 0, 0, 0);
                }
            }
            const int m = 16 * ct + r;
#pragma unroll
            for (int pt = 0; pt < QT; ++pt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int p = 16 * pt + 4 * g + v;
                    cb[p * kCB + m] = acc2[pt][v];
                    if (WANT_CT && p < Q && m < M) a.ct[(i * Q + p) * int64_t(L2) + b + m] = acc2[pt][v];
                }
        }
        if (WANT_PT) {
            wave_sync();
            // rows 16 P + r of c~ as the lane's operand: m = 8 g + j, zero past
            // the columns written for this l; high and low bfloat16 parts
            u32x4 hi[QT], lo[QT];
#pragma unroll
            for (int P = 0; P < QT; ++P) {
                float x[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (8 * g < 16 * MT) {
                    const float4 x0 = *reinterpret_cast<const float4*>(cb + (16 * P + r) * kCB + 8 * g);
                    const float4 x1 = *reinterpret_cast<const float4*>(cb + (16 * P + r) * kCB + 8 * g + 4);
                    x[0] = x0.x; x[1] = x0.y; x[2] = x0.z; x[3] = x0.w;
                    x[4] = x1.x; x[5] = x1.y; x[6] = x1.z; x[7] = x1.w;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const unsigned int hp = pack_bf16(x[2 * j], x[2 * j + 1]);
                    hi[P][j] = hp;
                    lo[P][j] = pack_bf16(x[2 * j] - __uint_as_float(hp << 16), x[2 * j + 1] - __uint_as_float(hp & 0xFFFF0000u));
                }
            }
            float* dst = a.pt + (i * (lmax + 1) + l) * int64_t(QQ);
#pragma unroll
            for (int P1 = 0; P1 < QT; ++P1)
#pragma unroll
                for (int P2 = P1; P2 < QT; ++P2) {
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, hi[P1]),
                                                                  __builtin_bit_cast(bf16x8, hi[P2]), acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, hi[P1]),
                                                                  __builtin_bit_cast(bf16x8, lo[P2]), acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, lo[P1]),
                                                                  __builtin_bit_cast(bf16x8, hi[P2]), acc, 0, 0, 0);
                    // lane holds p~[p1][p2], p1 = 16 P1 + 4 g + v, p2 = 16 P2 + r
                    const int p2 = 16 * P2 + r;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int p1 = 16 * P1 + 4 * g + v;
                        if (p1 <= p2 && p2 < Q) dst[p1 * Q - p1 * (p1 - 1) / 2 + (p2 - p1)] = acc[v];
                    }
                }
            wave_sync();
        }
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


template <int QT, bool IMG>
hipError_t launch_cmp_wave_q(const CompressArgs& a, const WaveLayout& W, hipStream_t stream)
{
    if (IMG) {
        hipLaunchKernelGGL(k_cmp_image, dim3(unsigned(a.lmax + 1)), dim3(256), 0, stream, a, W);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    auto kernel = a.ct ? (a.pt ? k_cmp_fwd_wave<true, true, QT, IMG> : k_cmp_fwd_wave<true, false, QT, IMG>)
                       : k_cmp_fwd_wave<false, true, QT, IMG>;
    if (W.total > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, W.total);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, dim3(blocks_of(a.n, W.cpw)), dim3(64 * W.cpw), size_t(W.total), stream, a, W);
    return hipGetLastError();
}

// the one-wave-per-centre form when the shapes fit it: K, H <= 128 and
// multiples of 4 (weights and c read as float4), Q <= 32, 1 <= lmax <= 12
// (a float4 of c then spans at most two lm rows), 16-byte aligned c and
// weights, at least two centres per work-group
bool cmp_wave_fits(const CompressArgs& a, WaveLayout& W, bool img = false)
{
    if (a.K > 128 || a.H > 128 || a.Q > 32 || a.lmax < 1 || a.lmax > 12) return false;
    if (a.K % 4 != 0 || a.H % 4 != 0) return false;
    if ((reinterpret_cast<uintptr_t>(a.c) & 15) != 0 || (reinterpret_cast<uintptr_t>(a.w) & 15) != 0) return false;
    for (int cpw = kWaveCentres; cpw >= 2; --cpw) {
        W = wave_layout(a.K, a.Q, a.H, a.lmax, cpw, img);
        if (W.total <= 160 * 1024) return true;
    }
    return false;
}

size_t compress_image_bytes(int K, int Q, int H, int lmax)
{
    if (K > 128 || H > 128 || Q > 32 || lmax < 1 || lmax > 12 || K % 4 != 0 || H % 4 != 0) return 0;
    const WaveLayout W = wave_layout(K, Q, H, lmax, 2, true);
    return size_t(lmax + 1) * W.wstride;
}

hipError_t launch_compress_forward_bf16(const CompressArgs& a, hipStream_t stream)
{
    if (a.n == 0) return hipSuccess;
    WaveLayout W;
    if (a.img && (reinterpret_cast<uintptr_t>(a.img) & 15) == 0 && cmp_wave_fits(a, W, true))
        return a.Q <= 16 ? launch_cmp_wave_q<1, true>(a, W, stream) : launch_cmp_wave_q<2, true>(a, W, stream);
    if (cmp_wave_fits(a, W))
        return a.Q <= 16 ? launch_cmp_wave_q<1, false>(a, W, stream) : launch_cmp_wave_q<2, false>(a, W, stream);
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
