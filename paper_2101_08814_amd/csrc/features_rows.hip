// Spherical expansion, power spectrum and every forward-mode gradient row in
// one kernel, with each pair staged once.
//
// One work-group of 256 lanes owns one centre i (the same outputs as
// k_centres with rows: c, p, the self rows dc_i/dr_i, dp_i/dr_i and the pair
// rows dc/dr_ji, dp/dr_ji of Sec. 4.A, 4.F, 4.G and App. B).
//
// Staging keeps per pair only what cannot be rebuilt cheaply: the harmonics
// Y_lm (not their gradients), R_nl = f I~_nl and
// D_nl = (f I~_nl)' - l R_nl / r, the unit vector and 1/r.  The gradient
// with respect to the pair vector follows from the harmonics of one degree
// lower: with Z_lm the solid harmonic,
//   grad Y_lm = (grad Z_lm - l Y_lm u) / r,
// and grad Z_lm is a combination of at most two Y_{l-1,m'} per component
// (kHarmonicGrad), so that
//   dc_{x,n,lm} = (f I~)'_nl u_x Y_lm + f I~_nl d_x Y_lm
//               = D_nl u_x Y_lm + (R_nl / r) d_x Z_lm.
// A pair then takes about a third of the LDS of a {Y, grad Y} record, and a
// centre of up to 32 pairs (FP32) is staged in one round: no second staging
// and no restaging for the pair rows of p.
//
// Staging: one lane per pair computes the geometry and every Y_lm with the
// degree recurrence in registers (lane_pair.hpp); one lane per (pair, n)
// loads the lmax+1 contiguous cubics of its interval and forms R and D.
// Combination: one lane per (species, n pair, lm) sums c and the self rows
// over the pairs of that species and stores each pair's dc values as it
// forms them (consecutive lanes, consecutive addresses).  Pair rows of p:
// each wave takes whole pairs, expands the pair's {Y, grad Y} into its own
// LDS buffer, forms
//   y_{l,k} = sum_m Y_lm c_{k,lm},   z_{x,l,k} = sum_m d_x Y_lm c_{k,lm},
// and writes, one lane per packed position (l, k1, k2),
//   dp_{x,l,k1k2} = u_x (A_{k1} y_{k2} + A_{k2} y_{k1}) + B_{k1} z_{x,k2}
//                   + B_{k2} z_{x,k1},
//   {A, B}_{l,k} = {(f I~)'_nl, f I~_nl} in the neighbour's species block.
// A centre with more pairs than one chunk holds is staged in chunks (the
// partial one first) and the earlier chunks are staged again for the pair
// rows of p.
#include "lane_pair.hpp"

namespace soap {
namespace {

using namespace dev;

constexpr int kRowsThreads = 256;
constexpr int kRowsWaves = kRowsThreads / 64;
constexpr int kNB = 4;   // radial channels n summed by one lane

// LDS layout in elements of T (ints in T-sized slots).  R and D hold npad
// = nmax rounded up to kNB channels per pair, the padding zero, so a lane
// reads its kNB channels without a bounds test.
struct RowsLayout {
    int ch;                 // pairs per chunk
    int npad;
    int c, dcs, ux, uy, uz, rinv, f, df, t, k, spc, Y, R, D, seg, flag, pos, pyz, lk, yd, yz, ab, total;
};

inline RowsLayout rows_layout(int S, int nmax, int lmax, int ch)
{
    const int L2 = (lmax + 1) * (lmax + 1), lm1 = lmax + 1, K = S * nmax;
    const int KK = K * (K + 1) / 2;
    RowsLayout L{};
    L.ch = ch;
    L.npad = (nmax + kNB - 1) / kNB * kNB;
    int o = 0;
    L.c = o; o += K * L2;
    L.dcs = o; o += 3 * K * L2;
    L.ux = o; o += ch;
    L.uy = o; o += ch;
    L.uz = o; o += ch;
    L.rinv = o; o += ch;
    L.f = o; o += ch;
    L.df = o; o += ch;
    L.t = o; o += ch;
    L.k = o; o += ch;
    L.spc = o; o += ch;
    L.Y = o; o += ch * L2;
    L.R = o; o += ch * L.npad * lm1;
    L.D = o; o += ch * L.npad * lm1;
    L.seg = o; o += 2 * S;
    L.flag = o; o += 2;
    L.pos = o; o += lm1 * KK;
    L.pyz = o; o += lm1 * KK;
    L.lk = o; o += lm1 * K;
    o = (o + 3) & ~3;
    L.yd = o; o += kRowsWaves * 4 * L2;
    L.yz = o; o += kRowsWaves * 4 * lm1 * K;
    L.ab = o; o += kRowsWaves * 2 * lm1 * K;
    L.total = o;
    return L;
}

template <typename T>
struct RowsSmem {
    T *c, *dcs, *ux, *uy, *uz, *rinv, *f, *df, *t, *Y, *R, *D;
    V4<T>*yd, *yz;
    V2<T>* ab;
    int *k, *spc, *seg, *flag, *pos, *pyz, *lk;
    __device__ RowsSmem(T* b, const RowsLayout& L)
        : c(b + L.c), dcs(b + L.dcs), ux(b + L.ux), uy(b + L.uy), uz(b + L.uz), rinv(b + L.rinv), f(b + L.f),
          df(b + L.df), t(b + L.t), Y(b + L.Y), R(b + L.R), D(b + L.D), yd(reinterpret_cast<V4<T>*>(b + L.yd)),
          yz(reinterpret_cast<V4<T>*>(b + L.yz)), ab(reinterpret_cast<V2<T>*>(b + L.ab)),
          k(reinterpret_cast<int*>(b + L.k)), spc(reinterpret_cast<int*>(b + L.spc)),
          seg(reinterpret_cast<int*>(b + L.seg)), flag(reinterpret_cast<int*>(b + L.flag)),
          pos(reinterpret_cast<int*>(b + L.pos)), pyz(reinterpret_cast<int*>(b + L.pyz)),
          lk(reinterpret_cast<int*>(b + L.lk))
    {
    }
};

// Stage pairs [q0, q0 + nc) (nc <= ch <= 64); every lane of the block takes
// part and the caller synchronises afterwards.  The species segments must
// have been reset to (nc, 0) before, by the caller, behind a barrier.
// The first wave forms each pair's geometry (one lane per pair) and, after
// the block barrier, its harmonics from the registers it still holds; the
// other waves read the geometry back and evaluate the radial integrals one
// lane per (pair, n).  *flag becomes 1 when the pairs come grouped by
// species in ascending order (then the combination needs no species test).
template <typename T, int LMAX>
__device__ __forceinline__ void stage_rows(const FeatureArgs& a, RowsSmem<T>& s, const RowsLayout& LY, int64_t q0,
                                           int nc)
{
    constexpr int LM1 = LMAX + 1, L2 = LM1 * LM1;
    const int tid = threadIdx.x;
    const T* __restrict__ vec = static_cast<const T*>(a.pair_vec);
    const int nmax = a.nmax, npad = LY.npad, nl = npad * LM1;
    PairGeom<T> g{};
    const bool mine = tid < nc;
    if (tid < 64) {
        int sp = 0;
        if (mine) {
            const int64_t q = q0 + tid;
            g = pair_geometry<T>(a, vec[3 * q], vec[3 * q + 1], vec[3 * q + 2]);
            sp = pair_species(a, q);
            s.ux[tid] = g.ux;
            s.uy[tid] = g.uy;
            s.uz[tid] = g.uz;
            s.rinv[tid] = g.rinv;
            s.f[tid] = g.f;
            s.df[tid] = g.df;
            s.t[tid] = g.t;
            s.k[tid] = g.k;
            s.spc[tid] = sp;
            atomicMin(&s.seg[2 * sp], tid);
            atomicMax(&s.seg[2 * sp + 1], tid + 1);
        }
        const int prev = __shfl_up(sp, 1);
        const bool ordered = !mine || tid == 0 || prev <= sp;
        if (tid == 0) s.flag[0] = __ballot(!ordered) == 0ull ? 1 : 0;
    }
    __syncthreads();
    if (tid < 64) {
        if (mine) {
            YlmStream<T, LMAX> ys(g.ux, g.uy, g.uz);
            T* Yp = s.Y + tid * L2;
            static_for<0, LM1>([&](auto Lc) __attribute__((always_inline)) {
                constexpr int L = decltype(Lc)::value;
                ys.template degree<L, false>(
                    [&](int mi, T Y, T, T, T) __attribute__((always_inline)) { Yp[L * L + mi] = Y; });
            });
        }
        return;
    }
    const V4<T>* __restrict__ coef = static_cast<const V4<T>*>(a.coef);
    const T inv_delta = T(a.inv_delta);
    const int items = nc * npad;
    for (int it = tid - 64; it < items; it += kRowsThreads - 64) {
        const int p = it / npad, n = it - p * npad;
        T* Rp = s.R + p * nl + n * LM1;
        T* Dp = s.D + p * nl + n * LM1;
        if (n >= nmax) {
#pragma unroll
            for (int l = 0; l < LM1; ++l) Rp[l] = Dp[l] = T(0);
            continue;
        }
        const T f = s.f[p], df = s.df[p], t = s.t[p], ri = s.rinv[p];
        const V4<T>* cf = coef + int64_t(s.k[p]) * (nmax * LM1) + n * LM1;
        V4<T> c4[LM1];
#pragma unroll
        for (int l = 0; l < LM1; ++l) c4[l] = cf[l];
#pragma unroll
        for (int l = 0; l < LM1; ++l) {
            T v, dv;
            spline_poly<T>(c4[l].x, c4[l].y, c4[l].z, c4[l].w, t, inv_delta, v, dv);
            const T R = f * v;
            Rp[l] = R;
            Dp[l] = df * v + f * dv - T(l) * R * ri;
        }
    }
}

// c of kNB channels n0.. of one (species, lm) and the self rows, summed over
// the pairs [p0, p1); each pair's dc values are stored as they are formed.
// CHECK: skip pairs of another species (lists not grouped by species).
template <typename T, int LMAX, bool CHECK>
__device__ __forceinline__ void combine_item(const RowsSmem<T>& s, int nl, int nmax, int sp, int n0, int lm, int p0,
                                             int p1, T* __restrict__ dq0, int64_t row_stride, T (&cs)[kNB],
                                             T (&gs)[kNB][3])
{
    constexpr int LM1 = LMAX + 1, L2 = LM1 * LM1;
    const int l = l_of(lm);
    const int nL2 = nmax * L2;
    const int ix0 = kHarmonicGrad.ix[lm][0], ix1 = kHarmonicGrad.ix[lm][1];
    const int iy0 = kHarmonicGrad.iy[lm][0], iy1 = kHarmonicGrad.iy[lm][1], iz = kHarmonicGrad.iz[lm];
    const T gx0 = T(kHarmonicGrad.gx[lm][0]), gx1 = T(kHarmonicGrad.gx[lm][1]);
    const T gy0 = T(kHarmonicGrad.gy[lm][0]), gy1 = T(kHarmonicGrad.gy[lm][1]);
    const T gz = T(kHarmonicGrad.gz[lm]);
    const int roff = n0 * LM1 + l;
    for (int p = p0; p < p1; ++p) {
        if (CHECK && s.spc[p] != sp) continue;
        const T* Yp = s.Y + p * L2;
        const T Yv = Yp[lm];
        const T zx = gx0 * Yp[ix0] + gx1 * Yp[ix1];
        const T zy = gy0 * Yp[iy0] + gy1 * Yp[iy1];
        const T zz = gz * Yp[iz];
        const T ri = s.rinv[p];
        const T al0 = s.ux[p] * Yv, al1 = s.uy[p] * Yv, al2 = s.uz[p] * Yv;
        const T* Rp = s.R + p * nl + roff;
        const T* Dp = s.D + p * nl + roff;
        T* dq = dq0 + int64_t(p) * row_stride;
#pragma unroll
        for (int u = 0; u < kNB; ++u) {
            const T R = Rp[u * LM1], D = Dp[u * LM1];
            const T P = R * ri;
            const T r0 = D * al0 + P * zx, r1 = D * al1 + P * zy, r2 = D * al2 + P * zz;
            cs[u] += R * Yv;
            gs[u][0] += r0;
            gs[u][1] += r1;
            gs[u][2] += r2;
            if (n0 + u < nmax) {
                dq[u * L2] = r0;
                dq[nL2 + u * L2] = r1;
                dq[2 * nL2 + u * L2] = r2;
            }
        }
    }
}

template <typename T, int LMAX>
__global__ void __launch_bounds__(kRowsThreads, sizeof(T) == 4 ? 4 : 2) k_features_rows(FeatureArgs a, RowsLayout LY)
{
    constexpr int LM1 = LMAX + 1, L2 = LM1 * LM1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    RowsSmem<T> s(reinterpret_cast<T*>(smem_raw), LY);
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (tid == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    const int64_t q_begin = a.pair_offsets[i], q_end = a.pair_offsets[i + 1];
    const int S = a.S, nmax = a.nmax, K = S * nmax, npad = LY.npad, nl = npad * LM1;
    const int KL2 = K * L2, nL2 = nmax * L2, KK = K * (K + 1) / 2, PL = LM1 * KK;
    const int ch = LY.ch;
    const int n_chunks = int((q_end - q_begin + ch - 1) / ch);
    const int pad = int(int64_t(n_chunks) * ch - (q_end - q_begin));
    for (int e = tid; e < KL2; e += kRowsThreads) {
        s.c[e] = T(0);
        s.dcs[e] = T(0);
        s.dcs[KL2 + e] = T(0);
        s.dcs[2 * KL2 + e] = T(0);
    }
    // dp positions (l, k1, k2): the first two per lane are loaded now and
    // reach LDS after the combination, so their round trip overlaps the
    // staging
    int posr[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int o = tid + j * kRowsThreads;
        posr[j] = o < PL ? a.dp_pos[o] : 0;
    }
    for (int t = tid; t < LM1 * K; t += kRowsThreads) s.lk[t] = (t / K) | ((t % K) << 8);
    // items (species, block of kNB channels, lm)
    const int nb = npad / kNB;
    const int items = S * nb * L2;
    T* __restrict__ dc_out = static_cast<T*>(a.dcoeffs);
    const int64_t row_stride = 3 * int64_t(nL2);
    for (int ck = 0; ck < n_chunks; ++ck) {
        const int64_t q0 = q_begin + (ck == 0 ? 0 : int64_t(ck) * ch - pad);
        const int nc = ck == 0 ? ch - pad : ch;
        for (int sp = tid; sp < S; sp += kRowsThreads) {
            s.seg[2 * sp] = nc;
            s.seg[2 * sp + 1] = 0;
        }
        __syncthreads();
        stage_rows<T, LMAX>(a, s, LY, q0, nc);
        __syncthreads();
        const bool grouped = s.flag[0] != 0;
        for (int t = tid; t < items; t += kRowsThreads) {
            const int sp = t / (nb * L2), rem = t - sp * (nb * L2), b = rem / L2, lm = rem - b * L2;
            const int n0 = b * kNB;
            T cs[kNB], gs[kNB][3];
#pragma unroll
            for (int u = 0; u < kNB; ++u) cs[u] = gs[u][0] = gs[u][1] = gs[u][2] = T(0);
            const int p0 = s.seg[2 * sp], p1 = s.seg[2 * sp + 1];
            T* dq0 = dc_out + q0 * row_stride + (n0 * L2 + lm);
            if (grouped)
                combine_item<T, LMAX, false>(s, nl, nmax, sp, n0, lm, p0, p1, dq0, row_stride, cs, gs);
            else
                combine_item<T, LMAX, true>(s, nl, nmax, sp, n0, lm, p0, p1, dq0, row_stride, cs, gs);
#pragma unroll
            for (int u = 0; u < kNB; ++u) {
                if (n0 + u >= nmax) break;
                const int e = (sp * nmax + n0 + u) * L2 + lm;
                s.c[e] += cs[u];
                s.dcs[e] -= gs[u][0];
                s.dcs[KL2 + e] -= gs[u][1];
                s.dcs[2 * KL2 + e] -= gs[u][2];
            }
        }
        __syncthreads();
    }
    // the position tables: (l, k1, k2) for p and its self rows, and the
    // {y, z} slots l K + k1 | (l K + k2) << 16 for the pair rows
    for (int o = tid; o < PL; o += kRowsThreads) {
        const int j = (o - tid) / kRowsThreads;
        const int v = j == 0 ? posr[0] : (j == 1 ? posr[1] : a.dp_pos[o]);
        const int l = v & 15, k1 = (v >> 4) & 1023, k2 = v >> 14;
        s.pos[o] = v;
        s.pyz[o] = (l * K + k1) | ((l * K + k2) << 16);
    }
    if (tid == 0) s.flag[1] = 0;
    if (a.include_center && tid < nmax) {
        const int sp = a.species[i];
        if (sp >= 0 && sp < S) s.c[(sp * nmax + tid) * L2] += static_cast<const T*>(a.center)[tid];
        else put_status(a.status, SOAP_ESPECIES);
    }
    __syncthreads();
    T* c_out = static_cast<T*>(a.coeffs) + i * KL2;
    for (int e = tid; e < KL2; e += kRowsThreads) c_out[e] = s.c[e];
    T* dcs_out = static_cast<T*>(a.dcoeffs_self) + i * 3 * KL2;
    for (int e = tid; e < 3 * KL2; e += kRowsThreads) dcs_out[e] = s.dcs[e];
    // p and its self rows (the product rule on the self rows of c); the m
    // loop runs to 2 lmax + 1 for every lane with the terms past 2l + 1 zero
    // (their reads clamped), so all reads of a lane are issued together
    T* p_out = static_cast<T*>(a.p) + i * int64_t(PL);
    T* dps_out = static_cast<T*>(a.dp_self) + i * int64_t(3 * PL);
    // the last wave forms p and its self rows while the others start on the
    // pair rows; waves take pairs from a counter in LDS as they come free
    const int wave = tid >> 6, lane = tid & 63;
    for (int o = wave == kRowsWaves - 1 ? lane : PL; o < PL; o += 64) {
        const int v = s.pos[o];
        const int l = v & 15, k1 = (v >> 4) & 1023, k2 = v >> 14;
        const int b1 = k1 * L2 + l * l, b2 = k2 * L2 + l * l;
        T acc = T(0), d0 = T(0), d1 = T(0), d2 = T(0);
#pragma unroll
        for (int m = 0; m < 2 * LMAX + 1; ++m) {
            const bool in = m <= 2 * l;
            const int mm = in ? m : 0;
            const T c1 = in ? s.c[b1 + mm] : T(0), c2 = in ? s.c[b2 + mm] : T(0);
            acc += c1 * c2;
            d0 += s.dcs[b1 + mm] * c2 + c1 * s.dcs[b2 + mm];
            d1 += s.dcs[KL2 + b1 + mm] * c2 + c1 * s.dcs[KL2 + b2 + mm];
            d2 += s.dcs[2 * KL2 + b1 + mm] * c2 + c1 * s.dcs[2 * KL2 + b2 + mm];
        }
        p_out[o] = acc;
        dps_out[o] = d0;
        dps_out[PL + o] = d1;
        dps_out[2 * PL + o] = d2;
    }
    // pair rows of p: the last chunk is still staged, earlier ones are
    // staged again; waves synchronise only with themselves in between
    const int nlk = LM1 * K;
    V4<T>* ydw = s.yd + wave * L2;
    V4<T>* yzw = s.yz + wave * nlk;
    V2<T>* abw = s.ab + wave * nlk;
    T* __restrict__ dp_out = static_cast<T*>(a.dp);
    for (int ck = n_chunks - 1; ck >= 0; --ck) {
        const int64_t q0 = q_begin + (ck == 0 ? 0 : int64_t(ck) * ch - pad);
        const int nc = ck == 0 ? ch - pad : ch;
        if (ck != n_chunks - 1) {
            __syncthreads();
            for (int sp = tid; sp < S; sp += kRowsThreads) {
                s.seg[2 * sp] = nc;
                s.seg[2 * sp + 1] = 0;
            }
            __syncthreads();
            if (tid == 0) s.flag[1] = 0;
            stage_rows<T, LMAX>(a, s, LY, q0, nc);
            __syncthreads();
        }
        for (;;) {
            int p = 0;
            if (lane == 0) p = atomicAdd(&s.flag[1], 1);
            p = __builtin_amdgcn_readfirstlane(p);
            if (p >= nc) break;
            const T ux = s.ux[p], uy = s.uy[p], uz = s.uz[p], ri = s.rinv[p];
            const T* Yp = s.Y + p * L2;
            for (int lm = lane; lm < L2; lm += 64) {
                const T Yv = Yp[lm];
                const T zx = T(kHarmonicGrad.gx[lm][0]) * Yp[kHarmonicGrad.ix[lm][0]] +
                             T(kHarmonicGrad.gx[lm][1]) * Yp[kHarmonicGrad.ix[lm][1]];
                const T zy = T(kHarmonicGrad.gy[lm][0]) * Yp[kHarmonicGrad.iy[lm][0]] +
                             T(kHarmonicGrad.gy[lm][1]) * Yp[kHarmonicGrad.iy[lm][1]];
                const T zz = T(kHarmonicGrad.gz[lm]) * Yp[kHarmonicGrad.iz[lm]];
                const T lY = T(l_of(lm)) * Yv;
                ydw[lm] = V4<T>{Yv, (zx - lY * ux) * ri, (zy - lY * uy) * ri, (zz - lY * uz) * ri};
            }
            wave_sync();
            // {y, z} and {A, B} of every (l, k); the m loop as for p above
            const int blk = s.spc[p] * nmax;
            const T* Rp = s.R + p * nl;
            const T* Dp = s.D + p * nl;
            for (int t = lane; t < nlk; t += 64) {
                const int v = s.lk[t];
                const int l2 = v & 255, k = v >> 8;
                const T* ck_ = s.c + k * L2 + l2 * l2;
                const V4<T>* yl = ydw + l2 * l2;
                T y = T(0), z0 = T(0), z1 = T(0), z2 = T(0);
#pragma unroll
                for (int m = 0; m < 2 * LMAX + 1; ++m) {
                    const bool in = m <= 2 * l2;
                    const int mm = in ? m : 0;
                    const T cv = in ? ck_[mm] : T(0);
                    const V4<T> yd = yl[mm];
                    y += yd.x * cv;
                    z0 += yd.y * cv;
                    z1 += yd.z * cv;
                    z2 += yd.w * cv;
                }
                yzw[t] = V4<T>{y, z0, z1, z2};
                const int n = k - blk;
                const bool inb = n >= 0 && n < nmax;
                const int rn = inb ? n * LM1 + l2 : 0;
                const T B = inb ? Rp[rn] : T(0);
                // (f I~)' = D + l R / r
                const T A = inb ? Dp[rn] + T(l2) * B * ri : T(0);
                abw[t] = V2<T>{A, B};
            }
            wave_sync();
            T* row = dp_out + (q0 + p) * int64_t(3 * PL);
            for (int o = lane; o < PL; o += 64) {
                const int v = s.pyz[o];
                const int i1 = v & 0xFFFF, i2 = v >> 16;
                const V4<T> q1 = yzw[i1], q2 = yzw[i2];
                const V2<T> e1 = abw[i1], e2 = abw[i2];
                const T a0 = e1.x * q2.x + e2.x * q1.x;
                row[o] = ux * a0 + e1.y * q2.y + e2.y * q1.y;
                row[PL + o] = uy * a0 + e1.y * q2.z + e2.y * q1.z;
                row[2 * PL + o] = uz * a0 + e1.y * q2.w + e2.y * q1.w;
            }
            wave_sync();
        }
    }
}

template <typename T, int LM>
struct RowsFn {
    static hipError_t run(const FeatureArgs& a, const RowsLayout& L, hipStream_t st)
    {
        if constexpr (LM < 0) {
            return hipErrorNotSupported;
        } else {
            const size_t lds = size_t(L.total) * sizeof(T);
            if (lds > 65536) {
                hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_features_rows<T, LM>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_features_rows<T, LM>), dim3(unsigned(a.n_atoms)),
                               dim3(kRowsThreads), lds, st, a, L);
            return hipGetLastError();
        }
    }
};

}  // namespace

// The largest chunk (at most 64 pairs) whose layout fits 40 KB (four
// work-groups per CU), else 64 KB; ch = 0 if none does or the dp position
// table is missing.
bool features_rows_layout(int S, int nmax, int lmax, size_t elem, int& ch, size_t& bytes)
{
    const size_t limits[2] = {40 * 1024, 64 * 1024};
    for (size_t lim : limits)
        for (int c = 64; c >= 8; c -= 8) {
            const RowsLayout L = rows_layout(S, nmax, lmax, c);
            if (size_t(L.total) * elem <= lim) {
                ch = c;
                bytes = size_t(L.total) * elem;
                return true;
            }
        }
    ch = 0;
    bytes = 0;
    return false;
}

hipError_t launch_features_rows(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    if (!a.dp_pos || a.lmax > 12) return hipErrorNotSupported;
    int ch = 0;
    size_t bytes = 0;
    if (!features_rows_layout(a.S, a.nmax, a.lmax, f64 ? 8 : 4, ch, bytes)) return hipErrorNotSupported;
    if (a.n_atoms == 0) return hipSuccess;
    const RowsLayout L = rows_layout(a.S, a.nmax, a.lmax, ch);
    return f64 ? by_degree<double, RowsFn>(a.lmax, a, L, stream) : by_degree<float, RowsFn>(a.lmax, a, L, stream);
}

}  // namespace soap
