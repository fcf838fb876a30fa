// Per-centre LDS staging of a chunk of pairs, shared by the forward
// (expansion, power spectrum, gradient rows) and reverse-mode kernels.
//
// A work-group of kThreads lanes owns one centre.  For a chunk of its pairs
// the staging step leaves in LDS, per pair p: the unit vector u, r, 1/r,
// f_cut and f'_cut, the species of j, the splined radial integral times the
// cutoff R_nl = f I~_nl and (with gradients) its r-derivative dR_nl, the real
// harmonics Y_lm and (with gradients) their gradients with respect to the
// pair vector, dY_{x,lm}.  One lane per pair computes the geometry, one lane
// per (pair, m) a column of the Legendre table, one lane per (pair, n, l)
// evaluates the spline, one lane per (pair, lm) the harmonics.
//
// Small per-block tables (filled once by init_tables): the degree l of each
// packed lm, the harmonic normalisation K_lm (built on the host), and the
// (k1, k2) of each packed
// upper-triangle index, so no lane divides or takes a square root to decode
// an index.
#pragma once

#include <type_traits>

#include "soap_internal.hpp"
#include "sph.hpp"

namespace soap {
namespace dev {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kTriMax = 8192;    // largest K (K+1)/2 kept as an LDS table
constexpr int kSplineBatch = 4;  // spline coefficient loads a lane keeps in flight
constexpr int kCopyBatch = 8;    // loads a lane keeps in flight when copying to LDS

// Kernels are instantiated with the degree lmax as a template parameter LM
// (0..12) for float; LM = -1 takes lmax at run time.
__device__ __forceinline__ int lmax_of(const FeatureArgs& a, int LM) { return LM >= 0 ? LM : a.lmax; }

__device__ __forceinline__ void put_status(int32_t* st, int v)
{
    if (st) *st = v;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Dims {
    int S, nmax, lmax, L2, nl, K, nq, lm1;
    int KK;
};

__host__ __device__ inline Dims make_dims(int S, int nmax, int lmax)
{
    Dims d;
    d.S = S;
    d.nmax = nmax;
    d.lmax = lmax;
    d.lm1 = lmax + 1;
    d.L2 = (lmax + 1) * (lmax + 1);
    d.nl = nmax * (lmax + 1);
    d.K = S * nmax;
    d.nq = (lmax + 1) * (lmax + 2) / 2;
    d.KK = d.K * (d.K + 1) / 2;
    return d;
}

// LDS layout in elements of T (ints occupy T-sized slots).
struct Layout {
    int chunk;                          // pairs per staged chunk
    int c, dcs, ux, uy, uz, r, rinv, f, df, R, dR, Y, qt, cre, cim, yz, spc, seg, ynorm, lof, tri, pos, total;
};

// yz: elements of the region for the per-(pair, l, k) operands of the
// gradient rows (it reuses the Legendre table's space); pos: entries of the
// table of dp row positions.
// with_c = false leaves out the c accumulator (kept in registers instead).
__host__ __device__ inline Layout make_layout(const Dims& d, int ch, bool grad, int yz = 0, bool self_rows = true,
                                              bool want_tri = false, int pos = 0, bool with_c = true)
{
    Layout L;
    L.chunk = ch;
    int o = 0;
    L.c = o; o += with_c ? d.K * d.L2 : 0;
    L.dcs = o; o += (grad && self_rows) ? 3 * d.K * d.L2 : 0;
    L.ux = o; o += ch;
    L.uy = o; o += ch;
    L.uz = o; o += ch;
    L.r = o; o += ch;
    L.rinv = o; o += ch;
    L.f = o; o += ch;
    L.df = o; o += ch;
    L.R = o; o += ch * d.nl;
    L.dR = o; o += grad ? ch * d.nl : 0;
    // harmonics: Y alone, or {Y, dY_x, dY_y, dY_z} records (4-element
    // aligned) with gradients
    o = (o + 3) & ~3;
    L.Y = o; o += (grad ? 4 : 1) * ch * d.L2;
    // the Legendre table is dead once the harmonics are staged; the
    // operands of the gradient rows reuse its space, 4-element aligned for
    // vector loads
    o = (o + 3) & ~3;
    int scratch = ch * (d.nq + 2 * d.lm1);
    L.qt = o;
    L.cre = o + ch * d.nq;
    L.cim = L.cre + ch * d.lm1;
    L.yz = o;
    o += scratch > yz ? scratch : yz;
    L.spc = o; o += ch;
    L.seg = o; o += 2 * d.S;
    L.ynorm = o; o += d.L2;
    L.lof = o; o += d.L2;
    L.tri = o; o += (want_tri && d.KK <= kTriMax) ? d.KK : 0;
    L.pos = o; o += pos;
    L.total = o;
    return L;
}

// Largest chunk (<= 32 pairs, at least 4) whose layout fits 40 KB of LDS
// (four work-groups of 256 lanes per CU), else 64 KB, else 160 KB;
// total = 0 if nothing fits.
template <typename T>
inline Layout choose_layout(const Dims& d, bool grad, bool self_rows, bool want_tri, bool with_c = true)
{
    const size_t limits[3] = {40 * 1024, 64 * 1024, 160 * 1024};
    for (size_t lim : limits)
        for (int ch = 32; ch >= 4; ch /= 2) {
            Layout L = make_layout(d, ch, grad, 0, self_rows, want_tri, 0, with_c);
            if (size_t(L.total) * sizeof(T) <= lim) return L;
        }
    Layout L = make_layout(d, 2, grad, 0, self_rows, want_tri, 0, with_c);
    if (size_t(L.total) * sizeof(T) > 160 * 1024) L.total = 0;
    return L;
}

// Layout of the expansion kernel that also writes the pair rows: one
// buffer of {y, z_x, z_y, z_z} operands per wave and the dp position table.
// Largest chunk first under the same LDS limits; total = 0 if nothing fits.
template <typename T>
inline Layout choose_rows_layout(const Dims& d)
{
    const size_t limits[3] = {40 * 1024, 64 * 1024, 160 * 1024};
    const int yz = kWaves * 4 * d.lm1 * d.K;
    for (size_t lim : limits)
        for (int ch = 32; ch >= 4; ch /= 2) {
            Layout L = make_layout(d, ch, true, yz, true, false, d.lm1 * d.KK);
            if (size_t(L.total) * sizeof(T) <= lim) return L;
        }
    Layout L = make_layout(d, 2, true, 0, true, false, 0);
    L.total = 0;
    return L;
}

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
    T x, y, z, w;
};

template <typename T>
struct alignas(2 * sizeof(T)) V2 {
    T x, y;
};

template <typename T>
struct Smem {
    T *c, *dcs, *ux, *uy, *uz, *r, *rinv, *f, *df, *R, *dR, *Y, *qt, *cre, *cim, *yz, *ynorm;
    V4<T>* YD;   // {Y, dY_x, dY_y, dY_z} of each (pair, lm) when staged with gradients
    int *spc, *seg, *lof, *tri, *pos;
    __device__ Smem(T* base, const Layout& L)
        : c(base + L.c), dcs(base + L.dcs), ux(base + L.ux), uy(base + L.uy), uz(base + L.uz), r(base + L.r),
          rinv(base + L.rinv), f(base + L.f), df(base + L.df), R(base + L.R), dR(base + L.dR), Y(base + L.Y),
          qt(base + L.qt), cre(base + L.cre), cim(base + L.cim), yz(base + L.yz),
          YD(reinterpret_cast<V4<T>*>(base + L.Y)),
          ynorm(base + L.ynorm), spc(reinterpret_cast<int*>(base + L.spc)),
          seg(reinterpret_cast<int*>(base + L.seg)), lof(reinterpret_cast<int*>(base + L.lof)),
          tri(reinterpret_cast<int*>(base + L.tri)), pos(reinterpret_cast<int*>(base + L.pos))
    {
    }
};

// Copy n elements from global memory to LDS with all lanes of the block,
// each lane keeping up to kCopyBatch loads in flight before it stores any
// (a plain strided loop waits for every load in turn).
template <typename T>
__device__ __forceinline__ void copy_in(T* dst, const T* src, int n)
{
    for (int e0 = threadIdx.x; e0 < n; e0 += kCopyBatch * kThreads) {
        T v[kCopyBatch];
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u) {
            const int e = e0 + u * kThreads;
            v[u] = e < n ? src[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u) {
            const int e = e0 + u * kThreads;
            if (e < n) dst[e] = v[u];
        }
    }
}

// l of each lm, K_lm, and (when present) the packed-triangle decode table
// tri[kk] = k1 | k2 << 16.  Caller synchronises afterwards.
template <typename T>
__device__ void init_tables(const FeatureArgs& a, const Dims& d, const Layout& L, Smem<T>& s)
{
    const int tid = threadIdx.x;
    const T* knorm = static_cast<const T*>(a.center) + d.nmax;
    for (int lm = tid; lm < d.L2; lm += kThreads) {
        s.lof[lm] = l_of(lm);
        s.ynorm[lm] = knorm[lm];
    }
    if (L.pos != L.tri)
        for (int k1 = tid; k1 < d.K; k1 += kThreads) {
            int start = k1 * d.K - k1 * (k1 - 1) / 2;
            for (int k2 = k1; k2 < d.K; ++k2) s.tri[start + k2 - k1] = k1 | (k2 << 16);
        }
}

template <typename T>
__device__ __forceinline__ void tri_pair(const Dims& d, const Smem<T>& s, bool table, int kk, int& k1, int& k2)
{
    if (table) {
        int v = s.tri[kk];
        k1 = v & 0xFFFF;
        k2 = v >> 16;
    } else {
        tri_decode(d.K, kk, k1, k2);
    }
}

// Stage nc pairs starting at q0 (all lanes of the block take part; the
// tables must be initialised).
template <typename T, bool GRAD>
__device__ void stage_chunk(const FeatureArgs& a, const Dims& d, Smem<T>& s, int64_t q0, int nc)
{
    const int tid = threadIdx.x;
    const T* vec = static_cast<const T*>(a.pair_vec);
    // Geometry of pair tid.  The species of j (a load that depends on j) is
    // only needed for the segments, so its value is taken after the spline
    // loads of the next phase are issued and its round trip overlaps theirs.
    // A pair whose j or species is invalid stores a status and counts as
    // species 0 (the outputs of such a call are not meaningful).
    int sp_j = 0;
    bool bad_j = false;
    if (tid < nc) {
        int64_t q = q0 + tid;
        T vx = vec[3 * q], vy = vec[3 * q + 1], vz = vec[3 * q + 2];
        T r = sqrt(vx * vx + vy * vy + vz * vz);
        int j = a.pair_j[q];
        bad_j = j < 0 || j >= a.n_atoms;
        if (bad_j) put_status(a.status, SOAP_EINVAL);
        sp_j = a.species[bad_j ? 0 : j];
        T f = T(0), df = T(0);
        if (!(r > T(1e-8))) {
            put_status(a.status, SOAP_EGEOMETRY);
            s.ux[tid] = T(0); s.uy[tid] = T(0); s.uz[tid] = T(1); s.rinv[tid] = T(0);
        } else {
            T ri = T(1) / r;
            s.ux[tid] = vx * ri; s.uy[tid] = vy * ri; s.uz[tid] = vz * ri; s.rinv[tid] = ri;
            f = fcut<T>(r, T(a.rcut), T(a.width), df);
        }
        s.f[tid] = f;
        s.df[tid] = df;
        s.r[tid] = r;
    }
    __syncthreads();
    // Qt columns and (x + i y)^m: one lane per (pair, m)
    const int lm1 = d.lm1;
    for (int t = tid; t < nc * lm1; t += kThreads) {
        int p = t / lm1, m = t - p * lm1;
        q_column<T>(m, d.lmax, s.ux[p], s.uy[p], s.uz[p], s.qt + p * d.nq, s.cre + p * lm1, s.cim + p * lm1);
    }
    // radial spline: one lane per (pair, n, l); a lane issues the
    // coefficient loads of up to kSplineBatch of its items before using any
    const V4<T>* coef = static_cast<const V4<T>*>(a.coef);
    const T inv_delta = T(a.inv_delta);
    const int n_items = nc * d.nl;
    for (int t0 = tid; t0 < n_items; t0 += kSplineBatch * kThreads) {
        V4<T> cf[kSplineBatch];
        T tt[kSplineBatch];
#pragma unroll
        for (int u = 0; u < kSplineBatch; ++u) {
            const int t = t0 + u * kThreads;
            if (t < n_items) {
                const int p = t / d.nl, j = t - p * d.nl;
                int64_t k;
                spline_locate<T>(a.M, inv_delta, s.r[p], k, tt[u]);
                cf[u] = coef[k * d.nl + j];
            }
        }
#pragma unroll
        for (int u = 0; u < kSplineBatch; ++u) {
            const int t = t0 + u * kThreads;
            if (t < n_items) {
                const int p = t / d.nl;
                T v, dv;
                spline_poly<T>(cf[u].x, cf[u].y, cf[u].z, cf[u].w, tt[u], inv_delta, v, dv);
                s.R[t] = s.f[p] * v;
                if (GRAD) s.dR[t] = s.df[p] * v + s.f[p] * dv;
            }
        }
    }
    if (tid < nc) {
        int sp = bad_j ? -1 : sp_j;
        if (sp < 0 || sp >= d.S) {
            if (!bad_j) put_status(a.status, SOAP_ESPECIES);
            sp = 0;
        }
        s.spc[tid] = sp;
    }
    __syncthreads();
    // species segments (pairs come sorted by species)
    for (int sp = tid; sp < d.S; sp += kThreads) {
        int lo = nc, hi = 0;
        for (int p = 0; p < nc; ++p)
            if (s.spc[p] == sp) { lo = p < lo ? p : lo; hi = p + 1; }
        s.seg[2 * sp] = lo;
        s.seg[2 * sp + 1] = hi;
    }
    // harmonics and gradients: one lane per (pair, lm)
    for (int t = tid; t < nc * d.L2; t += kThreads) {
        int p = t / d.L2, lm = t - p * d.L2;
        T Y, gx, gy, gz;
        ylm_and_grad<T>(lm, s.lof[lm], s.ynorm[lm], s.qt + p * d.nq, s.cre + p * lm1, s.cim + p * lm1, s.ux[p],
                        s.uy[p], s.uz[p], s.rinv[p], Y, gx, gy, gz);
        if (GRAD) s.YD[p * d.L2 + lm] = V4<T>{Y, gx, gy, gz};
        else s.Y[p * d.L2 + lm] = Y;
    }
    __syncthreads();
}

// Dispatch on lmax: float kernels are specialised on it (LM = 0..12, so
// index decoding and strides fold to constants), everything else takes
// LM = -1 (lmax at run time).
template <typename T, template <typename, int> class Fn, typename... Args>
hipError_t by_lmax(int lmax, Args&&... args)
{
    if constexpr (!std::is_same<T, float>::value) {
        return Fn<T, -1>::run(args...);
    } else {
    switch (lmax) {
    case 0: return Fn<T, 0>::run(args...);
    case 1: return Fn<T, 1>::run(args...);
    case 2: return Fn<T, 2>::run(args...);
    case 3: return Fn<T, 3>::run(args...);
    case 4: return Fn<T, 4>::run(args...);
    case 5: return Fn<T, 5>::run(args...);
    case 6: return Fn<T, 6>::run(args...);
    case 7: return Fn<T, 7>::run(args...);
    case 8: return Fn<T, 8>::run(args...);
    case 9: return Fn<T, 9>::run(args...);
    case 10: return Fn<T, 10>::run(args...);
    case 11: return Fn<T, 11>::run(args...);
    case 12: return Fn<T, 12>::run(args...);
    default: return Fn<T, -1>::run(args...);
    }
    }
}

}  // namespace dev
}  // namespace soap
