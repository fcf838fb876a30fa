// Spherical expansion (and power spectrum) with one lane per pair.
//
// Expansion (Sec. 4.A Eq. spherical_expansion_coefficients_gaussians, Sec.
// 4.F), k_expansion_lanes: one wave per centre.  For a chunk of up to 64 of
// its pairs, lane p forms pair p's harmonics Y_lm and radial values
// R_nl = f I~_nl in registers and puts them in the wave's LDS rows; then
// each lane owns items (four n, one lm) of a species block and sums
// R_{n..n+3,l} Y_lm over the pairs of that species (one 16-byte and one
// 4-byte LDS read per four FMAs).  Pairs arrive grouped by neighbour species
// (the order soap_compute_neighbors writes), so a block is complete when the
// species changes and is written then; a list that is not grouped is
// detected and the centre is redone one species at a time.  With WANT_P the
// blocks also go to an LDS copy of c_i and the power spectrum
// p_{l,k1<=k2} = sum_m c_{k1,lm} c_{k2,lm} (Sec. 2 Eq. nu2-basis-coupled up
// to the factor of reading R4) is formed from it, one lane per (k1, k2).
// Each output element has one owner: no atomics.
#include "lane_pair.hpp"

namespace soap {
namespace {

using namespace dev;

// ------------------------------------------------------------- expansion
template <typename T, int LMAX, bool WANT_P>
__global__ void __launch_bounds__(64) k_expansion_lanes(FeatureArgs a, LaneLayout W)
{
    constexpr int LM1 = LMAX + 1, L2 = LM1 * LM1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* base = reinterpret_cast<T*>(smem_raw);
    T* Rs = base + W.rs;
    T* Ys = base + W.ys;
    T* Cs = base + W.cs;
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (lane == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    const int nmax = a.nmax, S = a.S;
    const int nL2 = nmax * L2, KL2 = S * nL2;
    const int NI = ((nmax + 3) >> 2) * L2;
    const int nl = LM1 * nmax;
    const int64_t qb = a.pair_offsets[i], qe = a.pair_offsets[i + 1];
    const int n_chunks = int((qe - qb + W.ch - 1) / W.ch);
    const T* __restrict__ centre_term = static_cast<const T*>(a.center);
    const V4<T>* __restrict__ coef = static_cast<const V4<T>*>(a.coef_ln);
    const T* __restrict__ vec = static_cast<const T*>(a.pair_vec);
    int sp_i = -1;
    if (a.include_center) {
        sp_i = a.species[i];
        if (sp_i < 0 || sp_i >= S) {
            if (lane == 0) put_status(a.status, SOAP_ESPECIES);
            sp_i = -1;
        }
    }
    T* c_out = static_cast<T*>(a.coeffs) + i * int64_t(KL2);

    // Items (n group ng, lm), v = ng L2 + lm < NI: the four sums over n =
    // 4 ng..4 ng+3 of one lm, held in the block buffer blk4[v] (LDS) of the
    // species being summed; a lane takes items lane, lane + 64, ...
    V4<T>* const cs4 = reinterpret_cast<V4<T>*>(Cs);
    auto block = [&](int sp) __attribute__((always_inline)) { return cs4 + (WANT_P ? sp * NI : 0); };
    auto zero_block = [&](V4<T>* blk) __attribute__((always_inline)) {
        for (int v = lane; v < NI; v += 64) blk[v] = V4<T>{T(0), T(0), T(0), T(0)};
    };
    // species block sp of c to HBM with consecutive lanes on consecutive
    // addresses; the central atom adds its term to lm = 0 of its own species
    // on the way (and, with WANT_P, to the LDS copy)
    auto flush = [&](int sp) __attribute__((always_inline)) {
        V4<T>* blk = block(sp);
        T* b1 = reinterpret_cast<T*>(blk);
        wave_sync();
        T* dst = c_out + sp * nL2;
        const bool own = sp == sp_i;
        for (int e = lane; e < nL2; e += 64) {
            const int n = e / L2, lm = e - n * L2;
            T* src = b1 + ((n >> 2) * L2 + lm) * 4 + (n & 3);
            T v = *src;
            if (own && lm == 0) {
                v += centre_term[n];
                if (WANT_P) *src = v;
            }
            dst[e] = v;
        }
        wave_sync();
        if (!WANT_P) {
            zero_block(blk);
            wave_sync();
        }
    };
    // the chunk's pairs [lo, hi) of species sp added to its block: per item
    // and pair one 4-byte and one 16-byte LDS read and four FMAs
    auto accumulate = [&](int sp, int lo, int hi) __attribute__((always_inline)) {
        V4<T>* blk = block(sp);
        for (int v = lane; v < NI; v += 64) {
            const int ng = v / L2, lm = v - ng * L2;
            V4<T> s4 = blk[v];
            const T* yp = Ys + lo * W.l2s + lm;
            const T* rp = Rs + lo * W.nls + l_of(lm) * W.np + 4 * ng;
#pragma unroll 4
            for (int p = lo; p < hi; ++p) {
                const T Y = yp[0];
                const V4<T> R = *reinterpret_cast<const V4<T>*>(rp);
                s4.x += R.x * Y;
                s4.y += R.y * Y;
                s4.z += R.z * Y;
                s4.w += R.w * Y;
                yp += W.l2s;
                rp += W.nls;
            }
            blk[v] = s4;
        }
    };
    if (WANT_P) {
        for (int v = lane; v < S * NI; v += 64) cs4[v] = V4<T>{T(0), T(0), T(0), T(0)};
    } else {
        zero_block(cs4);
    }

    // lane p < nc stages pair q0 + p (harmonics and radial values in its
    // LDS rows) and returns its neighbour's species (-1 past the chunk).
    // The radial values j = l nmax + n of the pair's interval are
    // contiguous in the table: they stream in batches of eight with two
    // batches in flight, one batch consumed after each degree of harmonics.
    // The table has 32 zero entries past its end and each LDS row spare
    // elements for the rest of the last batch, so the last batches read and
    // write past the pair's values without a bounds check.
    // LDS offset of radial value j = l nmax + n in the rows [l][np]:
    // j + l (np - nmax), l = floor(j / nmax) = (j * ceil(2^16 / nmax)) >> 16
    // (exact for j < 2^12)
    const int rpad = W.np - nmax, rmul = (65536 + nmax - 1) / nmax;
    auto stage = [&](int64_t q0, int nc) __attribute__((always_inline)) -> int {
        int my_sp = -1;
        if (lane < nc) {
            const int64_t q = q0 + lane;
            const PairGeom<T> g = pair_geometry<T>(a, vec[3 * q], vec[3 * q + 1], vec[3 * q + 2]);
            my_sp = pair_species(a, q);
            const V4<T>* cf = coef + int64_t(g.k) * nl;
            T* yrow = Ys + lane * W.l2s;
            T* rrow = Rs + lane * W.nls;
            const T tt = g.t, f = g.f;
            V4<T> A[8], B[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                A[u] = cf[u];
                B[u] = cf[8 + u];
            }
            int jb = 0;
            auto consume = [&]() __attribute__((always_inline)) {
                // jb opaque here: the offsets of each batch are formed where
                // they are used instead of all at once at the kernel start
                asm volatile("" : "+s"(jb));
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const T v = f * (A[u].x + tt * (A[u].y + tt * (A[u].z + tt * A[u].w)));
                    const int j = jb + u;
                    rrow[j + rpad * ((j * rmul) >> 16)] = v;
                    A[u] = B[u];
                    B[u] = cf[jb + 16 + u];
                }
                jb += 8;
            };
            YlmStream<T, LMAX> ys(g.ux, g.uy, g.uz);
            static_for<0, LM1>([&](auto Lc) __attribute__((always_inline)) {
                constexpr int L = decltype(Lc)::value;
                ys.template degree<L, false>([&](int mi, T Y, T, T, T) __attribute__((always_inline)) {
                    yrow[L * L + mi] = Y;
                });
                if (jb < nl) consume();
            });
            while (jb < nl) consume();
        }
        wave_sync();
        return my_sp;
    };

    // Grouped pass: blocks written as the species changes.  A chunk whose
    // species decrease anywhere (or start below the current block) marks
    // the centre as not grouped.
    int cur = 0;
    bool grouped = true;
    for (int ck = 0; ck < n_chunks && grouped; ++ck) {
        const int64_t q0 = qb + int64_t(ck) * W.ch;
        const int nc = int(qe - q0 < W.ch ? qe - q0 : W.ch);
        const int my_sp = stage(q0, nc);
        const int prev = __shfl_up(my_sp, 1, 64);
        const bool bad = lane < nc && my_sp < (lane == 0 ? cur : prev);
        if (__ballot(bad)) {
            grouped = false;
            break;
        }
        for (int lo = 0; lo < nc;) {
            const int sp = __builtin_amdgcn_readlane(my_sp, lo);
            const int cnt = __popcll(__ballot(lane < nc && my_sp == sp));
            while (cur < sp) {
                flush(cur);
                ++cur;
            }
            accumulate(sp, lo, lo + cnt);
            lo += cnt;
        }
        wave_sync();
    }
    if (grouped) {
        for (int sp = cur; sp < S; ++sp) flush(sp);
    } else {
        // pairs not grouped by species: every block, one species per pass
        if (WANT_P) {
            for (int v = lane; v < S * NI; v += 64) cs4[v] = V4<T>{T(0), T(0), T(0), T(0)};
        } else {
            zero_block(cs4);
        }
        for (int sp = 0; sp < S; ++sp) {
            for (int ck = 0; ck < n_chunks; ++ck) {
                const int64_t q0 = qb + int64_t(ck) * W.ch;
                const int nc = int(qe - q0 < W.ch ? qe - q0 : W.ch);
                const int my_sp = stage(q0, nc);
                for (int p = 0; p < nc; ++p)
                    if (__builtin_amdgcn_readlane(my_sp, p) == sp) accumulate(sp, p, p + 1);
                wave_sync();
            }
            flush(sp);
        }
    }
    if constexpr (WANT_P) {
        wave_sync();
        const int K = S * nmax, KK = K * (K + 1) / 2;
        T* p_out = static_cast<T*>(a.p) + i * int64_t(LM1 * KK);
        for (int kk = lane; kk < KK; kk += 64) {
            int k1, k2;
            tri_decode(K, kk, k1, k2);
            // c_{k, lm} sits at ((ng L2 + lm) 4 + n % 4) of species a's block
            const int s1 = k1 / nmax, n1 = k1 - s1 * nmax, s2 = k2 / nmax, n2 = k2 - s2 * nmax;
            const T* c1 = Cs + (s1 * NI + (n1 >> 2) * L2) * 4 + (n1 & 3);
            const T* c2 = Cs + (s2 * NI + (n2 >> 2) * L2) * 4 + (n2 & 3);
            static_for<0, LM1>([&](auto Lc) __attribute__((always_inline)) {
                constexpr int L = decltype(Lc)::value;
                T s = T(0);
#pragma unroll
                for (int m = L * L; m < (L + 1) * (L + 1); ++m) s += c1[4 * m] * c2[4 * m];
                p_out[L * KK + kk] = s;
            });
        }
    }
}

template <typename T, int LM>
struct LanesFn {
    static hipError_t run(const FeatureArgs& a, const LaneLayout& W, bool want_p, hipStream_t st)
    {
        if constexpr (LM < 0) {
            return hipErrorNotSupported;
        } else {
            const size_t lds = size_t(W.total) * sizeof(T);
            const void* fn = want_p ? reinterpret_cast<const void*>(k_expansion_lanes<T, LM, true>)
                                    : reinterpret_cast<const void*>(k_expansion_lanes<T, LM, false>);
            if (lds > 65536) {
                hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
                if (e != hipSuccess) return e;
            }
            if (want_p)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_expansion_lanes<T, LM, true>), dim3(unsigned(a.n_atoms)),
                                   dim3(64), lds, st, a, W);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_expansion_lanes<T, LM, false>), dim3(unsigned(a.n_atoms)),
                                   dim3(64), lds, st, a, W);
            return hipGetLastError();
        }
    }
};

}  // namespace

LaneLayout lane_layout(int S, int nmax, int lmax, bool want_p, int ch)
{
    LaneLayout W{};
    const int lm1 = lmax + 1, L2 = lm1 * lm1;
    W.ch = ch;
    W.np = (nmax + 3) & ~3;
    // the last batch of eight radial values may run past nl: room for its
    // offsets j + (np - nmax) floor(j / nmax)
    int end = lm1 * W.np;
    const int nl = lm1 * nmax;
    for (int j = nl; j < ((nl + 7) & ~7); ++j) {
        const int o = j + (W.np - nmax) * (j / nmax) + 1;
        end = o > end ? o : end;
    }
    W.nls = (end + 3) & ~3;
    W.l2s = L2 | 1;
    int o = 0;
    W.rs = o; o += ch * W.nls;
    W.ys = o; o += ch * W.l2s;
    W.sp = o; o += ch;
    o = (o + 3) & ~3;
    W.cb = W.np * L2;
    W.cs = o; o += (want_p ? S : 1) * W.cb;
    W.total = o;
    return W;
}

// Largest chunk (64, 32 or 16 pairs) whose per-wave LDS keeps at least six
// waves per CU, else the smallest that fits 64 KB; total = 0 if none fits.
LaneLayout choose_lane_layout(int S, int nmax, int lmax, bool want_p, size_t elem)
{
    for (int ch = 64; ch >= 16; ch /= 2) {
        LaneLayout W = lane_layout(S, nmax, lmax, want_p, ch);
        if (size_t(W.total) * elem <= 24 * 1024) return W;
    }
    LaneLayout W = lane_layout(S, nmax, lmax, want_p, 16);
    if (size_t(W.total) * elem > 64 * 1024) W.total = 0;
    return W;
}

constexpr int64_t kSplitAtoms = 4096;   // c and p in two kernels from this many centres

hipError_t launch_expansion_lanes(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    const bool want_p = a.p != nullptr;
    if (!want_p) {
        hipError_t e = launch_expansion_packed(a, f64, stream);
        if (e != hipErrorNotSupported) return e;
    } else if (a.n_atoms >= kSplitAtoms) {
        // c with the pairs packed across centres, then p from c in HBM
        // (4096-atom liquid: 86 us against 113 for c and p in one kernel;
        // smaller systems are faster in one launch)
        FeatureArgs c = a;
        c.p = nullptr;
        hipError_t e = launch_expansion_packed(c, f64, stream);
        if (e == hipSuccess) {
            FeatureArgs q = a;
            q.dcoeffs = q.dcoeffs_self = q.dp = q.dp_self = nullptr;
            e = launch_power_spectrum(q, f64 ? SOAP_F64 : SOAP_F32, stream);
            if (e != hipErrorNotSupported) return e;
        } else if (e != hipErrorNotSupported) {
            return e;
        }
    }
    const size_t elem = f64 ? 8 : 4;
    LaneLayout W = choose_lane_layout(a.S, a.nmax, a.lmax, want_p, elem);
    if (W.total == 0 || a.n_atoms == 0) return W.total == 0 ? hipErrorNotSupported : hipSuccess;
    return f64 ? by_degree<double, LanesFn>(a.lmax, a, W, want_p, stream)
               : by_degree<float, LanesFn>(a.lmax, a, W, want_p, stream);
}

}  // namespace soap
