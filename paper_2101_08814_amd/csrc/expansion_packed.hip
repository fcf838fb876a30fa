// Spherical expansion c alone (Sec. 4.A Eq.
// spherical_expansion_coefficients_gaussians, Sec. 4.F) with the pairs of
// several centres packed into one wave's chunks.
//
// A wave takes a few consecutive centres and walks their pairs, which are
// stored contiguously and grouped by centre and then by neighbour species,
// in chunks of 32: a chunk may hold the end of one centre and the start of
// the next, so the lanes stay busy when centres have few pairs.  Both
// halves of the wave stage the same 32 pairs: each lane forms its pair's
// geometry and harmonics Y_lm (both halves write the same values to the
// wave's LDS rows) and half of its radial values R_nl = f I~_nl, four n at
// a time with one 16-byte LDS store.  Each lane then owns up to
// pack_slots items (four n, one lm) of c and sums R_{n..n+3,l} Y_lm over
// the pairs of the current (centre, species) segment in registers; when
// the segment ends the sums go straight to HBM (consecutive lanes on
// consecutive lm) with the central atom's term added, and species without
// pairs are written as zeros.  Every output element has one owner.  A list
// whose species are not grouped within a centre is detected, and the
// wave's centres are then redone one species at a time.
#include "lane_pair.hpp"

namespace soap {
namespace {

using namespace dev;

constexpr int kPackCh = 32;      // pairs per chunk, two lanes per pair
constexpr int kPackMaxCpw = 4;   // centres per wave
constexpr int kPackMaxN = 16;    // nmax covered by the register items

// items per lane with at most GMAX groups of four n (nmax <= 4 GMAX)
template <int LMAX, int GMAX>
constexpr int pack_slots()
{
    return (GMAX * (LMAX + 1) * (LMAX + 1) + 63) / 64;
}

// waves per SIMD the register allocation aims at (where it fits without
// spilling: three at nmax <= 8, lmax <= 6 in FP32, where the LDS allows
// eleven waves per CU; two up to lmax 8)
template <typename T, int LMAX, int GMAX>
constexpr int pack_waves()
{
    return sizeof(T) != 4 ? 1 : (GMAX <= 2 && LMAX <= 6) ? 3 : LMAX <= 8 ? 2 : 1;
}

template <typename T, int LMAX, int GMAX>
__global__ void __launch_bounds__(64, (pack_waves<T, LMAX, GMAX>())) k_expansion_packed(FeatureArgs a, PackLayout W)
{
    constexpr int LM1 = LMAX + 1, L2 = LM1 * LM1, NS = pack_slots<LMAX, GMAX>();
    constexpr int kNB = GMAX <= 2 ? 3 : 2;   // radial quads in flight
    // LDS rows of a pair: radial values [l][4 GMAX] and a spare quad, and
    // the harmonics (odd stride)
    constexpr int NP = 4 * GMAX, NLS = LM1 * NP + 4, L2S = L2 | 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Rs = reinterpret_cast<T*>(smem_raw);   // [pair][NLS] radial values
    T* Ys = Rs + kPackCh * NLS;                // [pair][L2S] harmonics
    const int lane = threadIdx.x;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (lane == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    const int nmax = a.nmax, S = a.S, G = W.G;
    const int nL2 = nmax * L2, NI = G * L2, nq = LM1 * G;
    const int nl = LM1 * nmax;
    const int pad = 4 * G - nmax, gmul = (65536 + G - 1) / G;   // l of quad u: (u * gmul) >> 16
    const int64_t c0 = int64_t(blockIdx.x) * W.cpw;
    const int ncw = int(a.n_atoms - c0 < W.cpw ? a.n_atoms - c0 : W.cpw);
    int64_t bnd[kPackMaxCpw + 1];   // pair range of each of the wave's centres
#pragma unroll
    for (int k = 0; k <= kPackMaxCpw; ++k) bnd[k] = a.pair_offsets[c0 + (k < ncw ? k : ncw)];
    const T* __restrict__ centre_term = static_cast<const T*>(a.center);
    const V4<T>* __restrict__ coef = static_cast<const V4<T>*>(a.coef_ln);
    const T* __restrict__ vec = static_cast<const T*>(a.pair_vec);
    T* c_out = static_cast<T*>(a.coeffs) + c0 * S * int64_t(nL2);

    // items v = lane + 64 u (u < NS, v < NI): n = 4 ng .. 4 ng + 3 of one lm;
    // lanes past NI in the last slot read row 0 and write nothing
    int yoff[NS], roff[NS];
    V4<T> acc[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int v = lane + 64 * u;
        const int ng = v / L2, lm = v - ng * L2;
        const bool in = v < NI;
        yoff[u] = in ? lm : 0;
        roff[u] = in ? l_of(lm) * NP + 4 * ng : 0;
        acc[u] = V4<T>{T(0), T(0), T(0), T(0)};
    }
    // the central atom's terms in LDS, so that writing a block waits on no
    // global load
    T* Cs = Ys + kPackCh * L2S;
    if (lane < kPackMaxN) Cs[lane] = lane < nmax ? centre_term[lane] : T(0);
    // species of the wave's centres, 16 bits each (0xFFFF: no central term)
    uint64_t cspc = ~uint64_t(0);
#pragma unroll
    for (int k = 0; k < kPackMaxCpw; ++k) {
        if (a.include_center && k < ncw) {
            const int si = a.species[c0 + k];
            if (si < 0 || si >= S) {
                if (lane == 0) put_status(a.status, SOAP_ESPECIES);
            } else {
                cspc = (cspc & ~(uint64_t(0xFFFF) << (16 * k))) | (uint64_t(si) << (16 * k));
            }
        }
    }
    const int nsl = (NI + 63) >> 6;   // slots with items

    // the inputs of pair q0 + p (p = lane mod 32, p < nc): vector and
    // neighbour index, loaded a chunk ahead; the neighbour's species once
    // the index has arrived
    struct PairIn {
        T x, y, z;
        int j;
    };
    auto load_in = [&](int64_t q0, int nc) __attribute__((always_inline)) -> PairIn {
        PairIn r{T(0), T(0), T(1), 0};
        const int p = lane & (kPackCh - 1);
        if (p < nc) {
            const int64_t q = q0 + p;
            r.x = vec[3 * q];
            r.y = vec[3 * q + 1];
            r.z = vec[3 * q + 2];
            r.j = a.pair_j[q];
        }
        return r;
    };
    // species of neighbour j, checked (an invalid j stores SOAP_EINVAL, an
    // invalid species SOAP_ESPECIES; both count as species 0)
    auto species_of = [&](int j, bool valid) __attribute__((always_inline)) -> int {
        if (!valid) return 0;
        if (j < 0 || j >= a.n_atoms) {
            put_status(a.status, SOAP_EINVAL);
            return 0;
        }
        const int sp = a.species[j];
        if (sp < 0 || sp >= S) {
            put_status(a.status, SOAP_ESPECIES);
            return 0;
        }
        return sp;
    };
    // Pair q0 + p staged by both halves; returns its key (centre of the
    // wave) S + (neighbour species), -1 past the chunk.
    auto stage = [&](int64_t q0, int nc, const PairIn& in, int spq) __attribute__((always_inline)) -> int {
        const int p = lane & (kPackCh - 1), h = lane >> 5;
        int key = -1;
        if (p < nc) {
            const int64_t q = q0 + p;
            const PairGeom<T> g = pair_geometry<T>(a, in.x, in.y, in.z);
            int cl = 0;
#pragma unroll
            for (int k = 1; k < kPackMaxCpw; ++k) cl += q >= bnd[k] ? 1 : 0;
            key = cl * S + spq;
            const V4<T>* cf = coef + int64_t(g.k) * nl;
            T* rrow = Rs + p * NLS;
            const T tt = g.t, f = g.f;
            // radial quads u = h + 2 i: four n of one l, coefficient
            // j = l nmax + 4 (u - l G) = 4 u - l pad, LDS l NP + 4 (u - l G)
            // = 4 u + 4 l (GMAX - G).
            // The last quad of a degree may read up to three values past it
            // (the next interval's, or the table's zero tail), which land in
            // the row's padding.  Every lane takes QH quads: those past nq
            // read the last quad's coefficients and write the row's spare
            // quad, so that each load is used on every path.
            constexpr int QH = (LM1 * GMAX + 1) / 2;
            auto coefs = [&](int u, V4<T>* A) __attribute__((always_inline)) {
                u = u < nq ? u : nq - 1;
                const int j = 4 * u - ((u * gmul) >> 16) * pad;
#pragma unroll
                for (int k = 0; k < 4; ++k) A[k] = cf[j + k];
            };
            auto put = [&](int u, const V4<T>* A) __attribute__((always_inline)) {
                const int o = u < nq ? 4 * u + 4 * ((u * gmul) >> 16) * (GMAX - G) : LM1 * NP;
                V4<T> r;
                r.x = f * (A[0].x + tt * (A[0].y + tt * (A[0].z + tt * A[0].w)));
                r.y = f * (A[1].x + tt * (A[1].y + tt * (A[1].z + tt * A[1].w)));
                r.z = f * (A[2].x + tt * (A[2].y + tt * (A[2].z + tt * A[2].w)));
                r.w = f * (A[3].x + tt * (A[3].y + tt * (A[3].z + tt * A[3].w)));
                *reinterpret_cast<V4<T>*>(rrow + o) = r;
            };
            // the first three quads in flight during the harmonics, then each
            // buffer refilled with the quad three ahead
            constexpr int NB = QH < kNB ? QH : kNB;
            V4<T> Bf[NB][4];
            static_for<0, NB>([&](auto I) __attribute__((always_inline)) {
                constexpr int i = decltype(I)::value;
                coefs(h + 2 * i, Bf[i]);
            });
            T* yrow = Ys + p * L2S;
            YlmStream<T, LMAX> ys(g.ux, g.uy, g.uz);
            static_for<0, LM1>([&](auto Lc) __attribute__((always_inline)) {
                constexpr int L = decltype(Lc)::value;
                ys.template degree<L, false>([&](int mi, T Y, T, T, T) __attribute__((always_inline)) {
                    yrow[L * L + mi] = Y;
                });
            });
            static_for<0, QH>([&](auto I) __attribute__((always_inline)) {
                constexpr int i = decltype(I)::value;
                put(h + 2 * i, Bf[i % NB]);
                if constexpr (i + NB < QH) coefs(h + 2 * (i + NB), Bf[i % NB]);
            });
        }
        wave_sync();
        return key;
    };
    // pairs [lo, hi) of the chunk added to the lane's items
    // (per pair, the lane's slots together: their LDS reads in flight at once)
    auto accumulate = [&](int lo, int hi) __attribute__((always_inline)) {
        static_for<1, NS + 1>([&](auto Nc) __attribute__((always_inline)) {
            constexpr int NU = decltype(Nc)::value;
            if (nsl == NU) {
                const T* yb = Ys + lo * L2S;
                const T* rb = Rs + lo * NLS;
                auto pair = [&](int k) __attribute__((always_inline)) {
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        const T Y = yb[k * L2S + yoff[u]];
                        const V4<T> R = *reinterpret_cast<const V4<T>*>(rb + k * NLS + roff[u]);
                        acc[u].x += R.x * Y;
                        acc[u].y += R.y * Y;
                        acc[u].z += R.z * Y;
                        acc[u].w += R.w * Y;
                    }
                };
                // four pairs per step at fixed offsets from one address per slot
                int p = lo;
                for (; p + 4 <= hi; p += 4) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) pair(k);
                    yb += 4 * L2S;
                    rb += 4 * NLS;
                }
                for (; p < hi; ++p) {
                    pair(0);
                    yb += L2S;
                    rb += NLS;
                }
            }
        });
    };
    // block key = cl S + sp of c to HBM and the sums cleared; the central
    // atom adds its term to lm = 0 of its own species
    auto flush = [&](int cl, int sp) __attribute__((always_inline)) {
        const int key = cl * S + sp;
        const bool own = int((cspc >> (16 * cl)) & 0xFFFF) == sp;
        T* out = c_out + int64_t(key) * nL2;
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int v = lane + 64 * u;
            const int ng = v / L2, lm = v - ng * L2;
            const int nn = v < NI ? min(4, nmax - 4 * ng) : 0;   // n of the item that exist
            T x4[4] = {acc[u].x, acc[u].y, acc[u].z, acc[u].w};
            if (own) {   // the same for the whole wave
                const bool cen = lm == 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const T ck = Cs[min(4 * ng + k, kPackMaxN - 1)];
                    x4[k] += cen ? ck : T(0);
                }
            }
            T* o = out + 4 * ng * L2 + lm;
            if (nn == 4) {
#pragma unroll
                for (int k = 0; k < 4; ++k) o[k * L2] = x4[k];
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < nn) o[k * L2] = x4[k];
            }
            acc[u] = V4<T>{T(0), T(0), T(0), T(0)};
        }
    };

    const int nkeys = ncw * S;
    int cur = 0, ccl = 0, csp = 0;   // blocks below cur = ccl S + csp are written
    auto flush_cur = [&]() __attribute__((always_inline)) {
        flush(ccl, csp);
        ++cur;
        if (++csp == S) {
            csp = 0;
            ++ccl;
        }
    };
    bool grouped = true;
    const int64_t pe = bnd[kPackMaxCpw];
    auto chunk_n = [&](int64_t q0) __attribute__((always_inline)) {
        return int(pe - q0 < kPackCh ? pe - q0 : kPackCh);
    };
    // The next chunk's inputs are loaded after this chunk's coefficient
    // loads have been used (vector loads complete in order, so loads issued
    // before them would hold them up) and arrive during the sums.
    PairIn nxt = load_in(bnd[0], chunk_n(bnd[0]));
    int nsp = species_of(nxt.j, (lane & (kPackCh - 1)) < chunk_n(bnd[0]));
    for (int64_t q0 = bnd[0]; q0 < pe; q0 += kPackCh) {
        const int nc = chunk_n(q0);
        const PairIn in = nxt;
        const int spq = nsp;
        const bool more = q0 + kPackCh < pe;
        const int nc1 = more ? chunk_n(q0 + kPackCh) : 0;
        const int key = stage(q0, nc, in, spq);
        if (more) nxt = load_in(q0 + kPackCh, nc1);
        const int prev = __shfl_up(key, 1, 64);
        if (__ballot(lane < nc && key < (lane == 0 ? cur : prev))) {
            grouped = false;
            break;
        }
        for (int lo = 0; lo < nc;) {
            const int k = __builtin_amdgcn_readlane(key, lo);
            const int cnt = __popcll(__ballot(lane < nc && key == k));
            while (cur < k) flush_cur();
            accumulate(lo, lo + cnt);
            lo += cnt;
        }
        if (more) nsp = species_of(nxt.j, (lane & (kPackCh - 1)) < nc1);
        wave_sync();   // the rows are read before the next chunk overwrites them
    }
    if (grouped) {
        while (cur < nkeys) flush_cur();
        return;
    }
    // species not grouped within a centre: each centre again, one species
    // per pass over its pairs
#pragma unroll
    for (int u = 0; u < NS; ++u) acc[u] = V4<T>{T(0), T(0), T(0), T(0)};
    for (int cl = 0; cl < ncw; ++cl) {
        for (int sp = 0; sp < S; ++sp) {
            for (int64_t q0 = bnd[cl]; q0 < bnd[cl + 1]; q0 += kPackCh) {
                const int nc = int(bnd[cl + 1] - q0 < kPackCh ? bnd[cl + 1] - q0 : kPackCh);
                const PairIn in = load_in(q0, nc);
                const int key = stage(q0, nc, in, species_of(in.j, (lane & (kPackCh - 1)) < nc));
                for (int p = 0; p < nc; ++p)
                    if (__builtin_amdgcn_readlane(key, p) == cl * S + sp) accumulate(p, p + 1);
                wave_sync();
            }
            flush(cl, sp);
        }
    }
}

template <typename T, int LM>
struct PackedFn {
    template <int GMAX>
    static hipError_t launch(const FeatureArgs& a, const PackLayout& W, hipStream_t st)
    {
        const size_t lds = size_t(W.total) * sizeof(T);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_expansion_packed<T, LM, GMAX>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
            if (e != hipSuccess) return e;
        }
        const int64_t waves = (a.n_atoms + W.cpw - 1) / W.cpw;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_expansion_packed<T, LM, GMAX>), dim3(unsigned(waves)), dim3(64), lds, st,
                           a, W);
        return hipGetLastError();
    }
    static hipError_t run(const FeatureArgs& a, const PackLayout& W, hipStream_t st)
    {
        if constexpr (LM < 0) {
            return hipErrorNotSupported;
        } else {
            if (W.gmax == 2) return launch<2>(a, W, st);
            if (W.gmax == 3) return launch<3>(a, W, st);
            return launch<4>(a, W, st);
        }
    }
};

}  // namespace

PackLayout pack_layout(int nmax, int lmax, int64_t n_atoms, int64_t pair_capacity)
{
    PackLayout W{};
    const int lm1 = lmax + 1;
    W.G = (nmax + 3) / 4;
    W.gmax = W.G < 2 ? 2 : W.G;   // the kernel's radial rows hold 4 gmax n per l
    const int nls = lm1 * 4 * W.gmax + 4, l2s = (lm1 * lm1) | 1;   // a spare quad per row
    W.total = kPackCh * (nls + l2s) + kPackMaxN;
    // enough waves to fill the chip before centres are packed; centres with
    // a chunk of pairs or more each gain little from sharing a wave
    // (4096-atom liquid, 45 pairs per centre: 86 us at one centre per wave,
    // 96 at two or four)
    const bool long_envs = pair_capacity >= int64_t(kPackCh) * n_atoms;
    W.cpw = long_envs ? 1 : n_atoms >= 8192 ? 4 : n_atoms >= 2048 ? 2 : 1;
    return W;
}

hipError_t launch_expansion_packed(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    if (a.p != nullptr || a.nmax > kPackMaxN) return hipErrorNotSupported;
    if (a.n_atoms == 0) return hipSuccess;
    const PackLayout W = pack_layout(a.nmax, a.lmax, a.n_atoms, a.pair_capacity);
    if (size_t(W.total) * (f64 ? 8 : 4) > 64 * 1024) return hipErrorNotSupported;
    return f64 ? by_degree<double, PackedFn>(a.lmax, a, W, stream) : by_degree<float, PackedFn>(a.lmax, a, W, stream);
}

}  // namespace soap
