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

template <typename T, int LMAX, int GMAX>
__global__ void __launch_bounds__(64) k_expansion_packed(FeatureArgs a, PackLayout W)
{
    constexpr int LM1 = LMAX + 1, L2 = LM1 * LM1, NS = pack_slots<LMAX, GMAX>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Rs = reinterpret_cast<T*>(smem_raw);   // [pair][l][np] radial values
    T* Ys = Rs + W.ys;                         // [pair][l2s] harmonics
    const int lane = threadIdx.x;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (lane == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    const int nmax = a.nmax, S = a.S, G = W.G, np = W.np;
    const int nL2 = nmax * L2, NI = G * L2, nq = LM1 * G;
    const int nl = LM1 * nmax;
    const int pad = np - nmax, gmul = (65536 + G - 1) / G;   // l of quad u: (u * gmul) >> 16
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
        roff[u] = in ? l_of(lm) * np + 4 * ng : 0;
        acc[u] = V4<T>{T(0), T(0), T(0), T(0)};
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
            T* rrow = Rs + p * W.nls;
            const T tt = g.t, f = g.f;
            // radial quads u = h, h + 2, ...: four n of one l, coefficient
            // j = l nmax + 4 (u - l G) = 4 u - l pad, LDS l np + 4 (u - l G) = 4 u.
            // The last quad of a degree may read up to three values past it
            // (the next interval's, or the table's zero tail), which land in
            // the row's padding.
            auto coefs = [&](int u, V4<T>* A) __attribute__((always_inline)) {
                const int j = 4 * u - ((u * gmul) >> 16) * pad;
#pragma unroll
                for (int k = 0; k < 4; ++k) A[k] = cf[j + k];
            };
            auto put = [&](int u, const V4<T>* A) __attribute__((always_inline)) {
                V4<T> r;
                r.x = f * (A[0].x + tt * (A[0].y + tt * (A[0].z + tt * A[0].w)));
                r.y = f * (A[1].x + tt * (A[1].y + tt * (A[1].z + tt * A[1].w)));
                r.z = f * (A[2].x + tt * (A[2].y + tt * (A[2].z + tt * A[2].w)));
                r.w = f * (A[3].x + tt * (A[3].y + tt * (A[3].z + tt * A[3].w)));
                *reinterpret_cast<V4<T>*>(rrow + 4 * u) = r;
            };
            V4<T> A[4], B[4];
            int u = h;
            if (u < nq) coefs(u, A);   // in flight during the harmonics
            T* yrow = Ys + p * W.l2s;
            YlmStream<T, LMAX> ys(g.ux, g.uy, g.uz);
            static_for<0, LM1>([&](auto Lc) __attribute__((always_inline)) {
                constexpr int L = decltype(Lc)::value;
                ys.template degree<L, false>([&](int mi, T Y, T, T, T) __attribute__((always_inline)) {
                    yrow[L * L + mi] = Y;
                });
            });
            for (; u < nq; u += 4) {
                if (u + 2 < nq) coefs(u + 2, B);
                put(u, A);
                if (u + 2 >= nq) break;
                if (u + 4 < nq) coefs(u + 4, A);
                put(u + 2, B);
            }
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
                const T* yb = Ys + lo * W.l2s;
                const T* rb = Rs + lo * W.nls;
#pragma unroll 2
                for (int p = lo; p < hi; ++p) {
#pragma unroll
                    for (int u = 0; u < NU; ++u) {
                        const T Y = yb[yoff[u]];
                        const V4<T> R = *reinterpret_cast<const V4<T>*>(rb + roff[u]);
                        acc[u].x += R.x * Y;
                        acc[u].y += R.y * Y;
                        acc[u].z += R.z * Y;
                        acc[u].w += R.w * Y;
                    }
                    yb += W.l2s;
                    rb += W.nls;
                }
            }
        });
    };
    // block key = cl S + sp of c to HBM and the sums cleared; the central
    // atom adds its term to lm = 0 of its own species
    auto flush = [&](int cl, int sp) __attribute__((always_inline)) {
        const int key = cl * S + sp;
        bool own = false;
        if (a.include_center) {
            const int si = a.species[c0 + cl];
            if (si < 0 || si >= S) {
                if (lane == 0) put_status(a.status, SOAP_ESPECIES);
            } else {
                own = si == sp;
            }
        }
        T* out = c_out + int64_t(key) * nL2;
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const T x4[4] = {acc[u].x, acc[u].y, acc[u].z, acc[u].w};
            const int v = lane + 64 * u;
            const int ng = v / L2, lm = v - ng * L2;
            const int nn = v < NI ? min(4, nmax - 4 * ng) : 0;   // n of the item that exist
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < nn) {
                    T x = x4[k];
                    if (own && lm == 0) x += centre_term[4 * ng + k];
                    out[(4 * ng + k) * L2 + lm] = x;
                }
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
    PairIn nxt = load_in(bnd[0], chunk_n(bnd[0]));
    int nsp = species_of(nxt.j, (lane & (kPackCh - 1)) < chunk_n(bnd[0]));
    for (int64_t q0 = bnd[0]; q0 < pe; q0 += kPackCh) {
        const int nc = chunk_n(q0);
        const PairIn in = nxt;
        const int spq = nsp;
        const bool more = q0 + kPackCh < pe;
        const int nc1 = more ? chunk_n(q0 + kPackCh) : 0;
        if (more) nxt = load_in(q0 + kPackCh, nc1);
        const int key = stage(q0, nc, in, spq);
        if (more) nsp = species_of(nxt.j, (lane & (kPackCh - 1)) < nc1);
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
    static hipError_t run(const FeatureArgs& a, const PackLayout& W, hipStream_t st)
    {
        if constexpr (LM < 0) {
            return hipErrorNotSupported;
        } else {
            const size_t lds = size_t(W.total) * sizeof(T);
            const void* fn = W.G <= 2 ? reinterpret_cast<const void*>(k_expansion_packed<T, LM, 2>)
                                      : reinterpret_cast<const void*>(k_expansion_packed<T, LM, 4>);
            if (lds > 65536) {
                hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
                if (e != hipSuccess) return e;
            }
            const int64_t waves = (a.n_atoms + W.cpw - 1) / W.cpw;
            if (W.G <= 2)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_expansion_packed<T, LM, 2>), dim3(unsigned(waves)), dim3(64), lds,
                                   st, a, W);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_expansion_packed<T, LM, 4>), dim3(unsigned(waves)), dim3(64), lds,
                                   st, a, W);
            return hipGetLastError();
        }
    }
};

}  // namespace

PackLayout pack_layout(int nmax, int lmax, int64_t n_atoms)
{
    PackLayout W{};
    const int lm1 = lmax + 1;
    W.G = (nmax + 3) / 4;
    W.np = 4 * W.G;
    W.nls = lm1 * W.np;
    W.l2s = (lm1 * lm1) | 1;
    W.ys = kPackCh * W.nls;
    W.total = W.ys + kPackCh * W.l2s;
    // enough waves to fill the chip before centres are packed
    W.cpw = n_atoms >= 8192 ? 4 : n_atoms >= 2048 ? 2 : 1;
    return W;
}

hipError_t launch_expansion_packed(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    if (a.p != nullptr || a.nmax > kPackMaxN) return hipErrorNotSupported;
    if (a.n_atoms == 0) return hipSuccess;
    const PackLayout W = pack_layout(a.nmax, a.lmax, a.n_atoms);
    if (size_t(W.total) * (f64 ? 8 : 4) > 64 * 1024) return hipErrorNotSupported;
    return f64 ? by_degree<double, PackedFn>(a.lmax, a, W, stream) : by_degree<float, PackedFn>(a.lmax, a, W, stream);
}

}  // namespace soap
