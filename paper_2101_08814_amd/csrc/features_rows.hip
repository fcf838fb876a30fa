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

// LDS layout in elements of T (ints in T-sized slots).
struct RowsLayout {
    int ch;                 // pairs per chunk
    int c, dcs, ux, uy, uz, rinv, spc, Y, R, D, seg, pos, yd, yz, total;
};

inline RowsLayout rows_layout(int S, int nmax, int lmax, int ch)
{
    const int L2 = (lmax + 1) * (lmax + 1), lm1 = lmax + 1, K = S * nmax;
    const int KK = K * (K + 1) / 2;
    RowsLayout L{};
    L.ch = ch;
    int o = 0;
    L.c = o; o += K * L2;
    L.dcs = o; o += 3 * K * L2;
    L.ux = o; o += ch;
    L.uy = o; o += ch;
    L.uz = o; o += ch;
    L.rinv = o; o += ch;
    L.spc = o; o += ch;
    L.Y = o; o += ch * L2;
    L.R = o; o += ch * nmax * lm1;
    L.D = o; o += ch * nmax * lm1;
    L.seg = o; o += 2 * S;
    L.pos = o; o += lm1 * KK;
    o = (o + 3) & ~3;
    L.yd = o; o += kRowsWaves * 4 * L2;
    L.yz = o; o += kRowsWaves * 4 * lm1 * K;
    L.total = o;
    return L;
}

template <typename T>
struct RowsSmem {
    T *c, *dcs, *ux, *uy, *uz, *rinv, *Y, *R, *D;
    V4<T>*yd, *yz;
    int *spc, *seg, *pos;
    __device__ RowsSmem(T* b, const RowsLayout& L)
        : c(b + L.c), dcs(b + L.dcs), ux(b + L.ux), uy(b + L.uy), uz(b + L.uz), rinv(b + L.rinv), Y(b + L.Y),
          R(b + L.R), D(b + L.D), yd(reinterpret_cast<V4<T>*>(b + L.yd)), yz(reinterpret_cast<V4<T>*>(b + L.yz)),
          spc(reinterpret_cast<int*>(b + L.spc)), seg(reinterpret_cast<int*>(b + L.seg)),
          pos(reinterpret_cast<int*>(b + L.pos))
    {
    }
};

// Stage pairs [q0, q0 + nc) (nc <= ch); every lane of the block takes part
// and the caller synchronises afterwards.  The species segments must have
// been reset to (nc, 0) before, by the caller, behind a barrier.
template <typename T, int LMAX>
__device__ __forceinline__ void stage_rows(const FeatureArgs& a, RowsSmem<T>& s, int64_t q0, int nc)
{
    constexpr int LM1 = LMAX + 1, L2 = LM1 * LM1;
    const int tid = threadIdx.x;
    const T* __restrict__ vec = static_cast<const T*>(a.pair_vec);
    const int nmax = a.nmax, nl = nmax * LM1;
    // harmonics: one lane per pair in the first wave
    for (int p = tid; tid < 64 && p < nc; p += 64) {
        const int64_t q = q0 + p;
        const PairGeom<T> g = pair_geometry<T>(a, vec[3 * q], vec[3 * q + 1], vec[3 * q + 2]);
        const int sp = pair_species(a, q);
        s.ux[p] = g.ux;
        s.uy[p] = g.uy;
        s.uz[p] = g.uz;
        s.rinv[p] = g.rinv;
        s.spc[p] = sp;
        atomicMin(&s.seg[2 * sp], p);
        atomicMax(&s.seg[2 * sp + 1], p + 1);
        YlmStream<T, LMAX> ys(g.ux, g.uy, g.uz);
        T* Yp = s.Y + p * L2;
        static_for<0, LM1>([&](auto Lc) __attribute__((always_inline)) {
            constexpr int L = decltype(Lc)::value;
            ys.template degree<L, false>(
                [&](int mi, T Y, T, T, T) __attribute__((always_inline)) { Yp[L * L + mi] = Y; });
        });
    }
    // radial integrals: one lane per (pair, n) in the other waves (in every
    // lane when the block has no other wave to spare)
    const V4<T>* __restrict__ coef = static_cast<const V4<T>*>(a.coef);
    const T inv_delta = T(a.inv_delta);
    const int first = nc <= 64 * (kRowsWaves - 1) / 2 ? 64 : 0;
    const int items = nc * nmax;
    for (int t = tid - first; t < items; t += kRowsThreads - first) {
        if (t < 0) break;
        const int p = t / nmax, n = t - p * nmax;
        const int64_t q = q0 + p;
        const PairGeom<T> g = pair_geometry<T>(a, vec[3 * q], vec[3 * q + 1], vec[3 * q + 2]);
        const V4<T>* cf = coef + int64_t(g.k) * nl + n * LM1;
        V4<T> c4[LM1];
#pragma unroll
        for (int l = 0; l < LM1; ++l) c4[l] = cf[l];
        T* Rp = s.R + p * nl + n * LM1;
        T* Dp = s.D + p * nl + n * LM1;
#pragma unroll
        for (int l = 0; l < LM1; ++l) {
            T v, dv;
            spline_poly<T>(c4[l].x, c4[l].y, c4[l].z, c4[l].w, g.t, inv_delta, v, dv);
            const T R = g.f * v;
            Rp[l] = R;
            Dp[l] = g.df * v + g.f * dv - T(l) * R * g.rinv;
        }
    }
}

template <typename T, int LMAX>
__global__ void __launch_bounds__(kRowsThreads) k_features_rows(FeatureArgs a, RowsLayout LY)
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
    const int S = a.S, nmax = a.nmax, K = S * nmax, nl = nmax * LM1;
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
    for (int o = tid; o < PL; o += kRowsThreads) s.pos[o] = a.dp_pos[o];
    // items (species, n pair, lm): two n per lane share the harmonic loads
    const int ng = (nmax + 1) / 2;
    const int items = S * ng * L2;
    T* __restrict__ dc_out = static_cast<T*>(a.dcoeffs);
    for (int ck = 0; ck < n_chunks; ++ck) {
        const int64_t q0 = q_begin + (ck == 0 ? 0 : int64_t(ck) * ch - pad);
        const int nc = ck == 0 ? ch - pad : ch;
        for (int sp = tid; sp < S; sp += kRowsThreads) {
            s.seg[2 * sp] = nc;
            s.seg[2 * sp + 1] = 0;
        }
        __syncthreads();
        stage_rows<T, LMAX>(a, s, q0, nc);
        __syncthreads();
        for (int t = tid; t < items; t += kRowsThreads) {
            const int sp = t / (ng * L2), rem = t - sp * (ng * L2), g = rem / L2, lm = rem - g * L2;
            const int n0 = 2 * g;
            const bool two = n0 + 1 < nmax;
            const int l = l_of(lm);
            const int e0 = (sp * nmax + n0) * L2 + lm;
            const int ix0 = kHarmonicGrad.ix[lm][0], ix1 = kHarmonicGrad.ix[lm][1];
            const int iy0 = kHarmonicGrad.iy[lm][0], iy1 = kHarmonicGrad.iy[lm][1], iz = kHarmonicGrad.iz[lm];
            const T gx0 = T(kHarmonicGrad.gx[lm][0]), gx1 = T(kHarmonicGrad.gx[lm][1]);
            const T gy0 = T(kHarmonicGrad.gy[lm][0]), gy1 = T(kHarmonicGrad.gy[lm][1]);
            const T gz = T(kHarmonicGrad.gz[lm]);
            T c0 = T(0), c1 = T(0);
            T a0 = T(0), a1 = T(0), a2 = T(0), b0 = T(0), b1 = T(0), b2 = T(0);
            const int p0 = s.seg[2 * sp], p1 = s.seg[2 * sp + 1];
            for (int p = p0; p < p1; ++p) {
                if (s.spc[p] != sp) continue;
                const T* Yp = s.Y + p * L2;
                const T Yv = Yp[lm];
                const T zx = gx0 * Yp[ix0] + gx1 * Yp[ix1];
                const T zy = gy0 * Yp[iy0] + gy1 * Yp[iy1];
                const T zz = gz * Yp[iz];
                const T* Rp = s.R + p * nl + n0 * LM1 + l;
                const T* Dp = s.D + p * nl + n0 * LM1 + l;
                const T R0 = Rp[0], R1 = two ? Rp[LM1] : T(0);
                const T D0 = Dp[0], D1 = two ? Dp[LM1] : T(0);
                const T ri = s.rinv[p];
                const T al0 = s.ux[p] * Yv, al1 = s.uy[p] * Yv, al2 = s.uz[p] * Yv;
                const T P0 = R0 * ri, P1 = R1 * ri;
                const T r00 = D0 * al0 + P0 * zx, r01 = D0 * al1 + P0 * zy, r02 = D0 * al2 + P0 * zz;
                const T r10 = D1 * al0 + P1 * zx, r11 = D1 * al1 + P1 * zy, r12 = D1 * al2 + P1 * zz;
                c0 += R0 * Yv;
                c1 += R1 * Yv;
                a0 += r00;
                a1 += r01;
                a2 += r02;
                b0 += r10;
                b1 += r11;
                b2 += r12;
                T* dq = dc_out + (q0 + p) * int64_t(3 * nL2) + (n0 * L2 + lm);
                dq[0] = r00;
                dq[nL2] = r01;
                dq[2 * nL2] = r02;
                if (two) {
                    dq[L2] = r10;
                    dq[nL2 + L2] = r11;
                    dq[2 * nL2 + L2] = r12;
                }
            }
            s.c[e0] += c0;
            s.dcs[e0] -= a0;
            s.dcs[KL2 + e0] -= a1;
            s.dcs[2 * KL2 + e0] -= a2;
            if (two) {
                s.c[e0 + L2] += c1;
                s.dcs[e0 + L2] -= b0;
                s.dcs[KL2 + e0 + L2] -= b1;
                s.dcs[2 * KL2 + e0 + L2] -= b2;
            }
        }
        __syncthreads();
    }
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
    // p and its self rows (the product rule on the self rows of c)
    T* p_out = static_cast<T*>(a.p) + i * int64_t(PL);
    T* dps_out = static_cast<T*>(a.dp_self) + i * int64_t(3 * PL);
    for (int o = tid; o < PL; o += kRowsThreads) {
        const int v = s.pos[o];
        const int l = v & 15, k1 = (v >> 4) & 1023, k2 = v >> 14;
        const T* c1 = s.c + k1 * L2 + l * l;
        const T* c2 = s.c + k2 * L2 + l * l;
        T acc = T(0);
        for (int m = 0; m < 2 * l + 1; ++m) acc += c1[m] * c2[m];
        p_out[o] = acc;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const T* g1 = s.dcs + x * KL2 + k1 * L2 + l * l;
            const T* g2 = s.dcs + x * KL2 + k2 * L2 + l * l;
            T acc2 = T(0);
            for (int m = 0; m < 2 * l + 1; ++m) acc2 += g1[m] * c2[m] + c1[m] * g2[m];
            dps_out[x * PL + o] = acc2;
        }
    }
    // pair rows of p: the last chunk is still staged, earlier ones are
    // staged again; waves synchronise only with themselves in between
    const int wave = tid >> 6, lane = tid & 63;
    const int nlk = LM1 * K;
    V4<T>* ydw = s.yd + wave * L2;
    V4<T>* yzw = s.yz + wave * nlk;
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
            stage_rows<T, LMAX>(a, s, q0, nc);
            __syncthreads();
        }
        for (int p = wave; p < nc; p += kRowsWaves) {
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
            for (int t = lane; t < nlk; t += 64) {
                const int l2 = t / K, k = t - l2 * K;
                const int m0 = l2 * l2;
                const T* ck_ = s.c + k * L2;
                T y = T(0), z0 = T(0), z1 = T(0), z2 = T(0);
                for (int m = m0; m < m0 + 2 * l2 + 1; ++m) {
                    const T cv = ck_[m];
                    const V4<T> yd = ydw[m];
                    y += yd.x * cv;
                    z0 += yd.y * cv;
                    z1 += yd.z * cv;
                    z2 += yd.w * cv;
                }
                yzw[t] = V4<T>{y, z0, z1, z2};
            }
            wave_sync();
            const int blk = s.spc[p] * nmax;
            const T* Rp = s.R + p * nl;
            const T* Dp = s.D + p * nl;
            T* row = dp_out + (q0 + p) * int64_t(3 * PL);
            for (int o = lane; o < PL; o += 64) {
                const int v = s.pos[o];
                const int l2 = v & 15, k1 = (v >> 4) & 1023, k2 = v >> 14;
                const V4<T> q1 = yzw[l2 * K + k1], q2 = yzw[l2 * K + k2];
                const int n1 = k1 - blk, n2 = k2 - blk;
                const bool in1 = n1 >= 0 && n1 < nmax, in2 = n2 >= 0 && n2 < nmax;
                const T B1 = in1 ? Rp[n1 * LM1 + l2] : T(0), B2 = in2 ? Rp[n2 * LM1 + l2] : T(0);
                // (f I~)' = D + l R / r
                const T A1 = in1 ? Dp[n1 * LM1 + l2] + T(l2) * B1 * ri : T(0);
                const T A2 = in2 ? Dp[n2 * LM1 + l2] + T(l2) * B2 * ri : T(0);
                const T a0 = A1 * q2.x + A2 * q1.x;
                row[o] = ux * a0 + B1 * q2.y + B2 * q1.y;
                row[PL + o] = uy * a0 + B1 * q2.z + B2 * q1.z;
                row[2 * PL + o] = uz * a0 + B1 * q2.w + B2 * q1.w;
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
