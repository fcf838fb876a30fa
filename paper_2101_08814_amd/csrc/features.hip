// Spherical expansion, power spectrum and forward-mode gradient rows.
//
// One work-group of 256 lanes owns one centre i.  Its pairs are staged in
// chunks of up to kChunk pairs through LDS:
//   stage   - per pair: unit vector, 1/r, f_cut, f'_cut, species of j
//             (one lane per pair); the Qt table and (x + i y)^m (one lane per
//             (pair, m)); Y_lm and its gradient (one lane per (pair, lm)) and
//             the splined radial integral f I~_nl and (f I~_nl)' (one lane per
//             (pair, n, l)).  Nothing per pair touches HBM except pair_vec
//             and the species of j; the spline table is L2-resident.
//   combine - c_{a,n,lm} += sum over the chunk's pairs of species a of
//             R_nl Y_lm (Sec. 4.A, 4.F); each output element is owned by one
//             lane, so no atomics, and pairs sorted by species make the loop
//             run only over the pairs that contribute.
// With gradients the same loop accumulates the self row
//   d c_i / d r_i = -sum_q [(f I~)' Y u + f I~ grad Y]
// (App. B: d r_ji / d r_i = -1).  After the last chunk c, p and the self
// rows are written with consecutive lanes on consecutive addresses.
//
// The pair rows d c / d r_ji and d p / d r_ji are written by a second
// kernel (gradient_rows.hip) once c of every centre is in memory.
#include <type_traits>

#include "chunk.hpp"

namespace soap {
namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// Per-centre pass: c, p and (with gradients) the self rows of c and p; with
// ROWS also the pair rows of c and p.
// One thread owns a species channel and an lm and accumulates every n of it
// over the centre's pairs of that species.  REGC (c alone, at most
// kRegItems items per lane): the sums stay in registers, the layout has no c
// region, so the chunk can hold more pairs and a centre takes fewer
// staging rounds.
// ---------------------------------------------------------------------------
constexpr int kRegItems = 16;

// c of one (species, n pair, lm) item summed over the chunk's pairs
// [p0, p1) of that species, in pair order; U pairs' LDS reads are issued
// together (pairs of another species, possible when the list is not
// sorted, are skipped)
template <typename T, int U>
__device__ __forceinline__ void species_sums(const Smem<T>& s, const Dims& d, int sp, int lm, int l, int n0, bool two,
                                             int p0, int p1, T& c0, T& c1)
{
    const int lm1 = d.lm1;
    int p = p0;
    for (; p + U <= p1; p += U) {
        int sc[U];
        T Yv[U], R0[U], R1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sc[u] = s.spc[p + u];
            Yv[u] = s.Y[(p + u) * d.L2 + lm];
            const T* Rp = s.R + (p + u) * d.nl + n0 * lm1 + l;
            R0[u] = Rp[0];
            R1[u] = two ? Rp[lm1] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (sc[u] == sp) {
                c0 += R0[u] * Yv[u];
                c1 += R1[u] * Yv[u];
            }
    }
    for (; p < p1; ++p) {
        if (s.spc[p] != sp) continue;
        const T Yv = s.Y[p * d.L2 + lm];
        const T* Rp = s.R + p * d.nl + n0 * lm1 + l;
        c0 += Rp[0] * Yv;
        c1 += (two ? Rp[lm1] : T(0)) * Yv;
    }
}

template <typename T, int LM, bool GRAD, bool WANT_P, bool ROWS, bool REGC>
__device__ __forceinline__ void centres_body(const FeatureArgs& a, const Layout& L)
{
    static_assert(!ROWS || (GRAD && WANT_P), "pair rows come with the self rows and p");
    static_assert(!REGC || (!GRAD && !WANT_P), "register sums are for c alone");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* base = reinterpret_cast<T*>(smem_raw);
    Smem<T> s(base, L);
    const Dims d = make_dims(a.S, a.nmax, lmax_of(a, LM));
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    const int64_t q_total = a.pair_offsets[a.n_atoms];
    const int64_t q_begin = a.pair_offsets[i], q_end = a.pair_offsets[i + 1];
    if (q_total > a.pair_capacity) {
        if (tid == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    const int chunk = L.chunk;
    init_tables<T>(a, d, L, s);
    const int n_chunks = int((q_end - q_begin + chunk - 1) / chunk);
    // the partial chunk comes first, so the chunk left staged after the
    // accumulation (the last) is a full one and the pair-row phase restages
    // the fewest pairs
    const int pad = int(int64_t(n_chunks) * chunk - (q_end - q_begin));
    const int KL2 = d.K * d.L2, nL2 = d.nmax * d.L2, lm1 = d.lm1;
    const int KK = d.KK, PL = lm1 * KK;
    if (!REGC)
        for (int e = tid; e < KL2; e += kThreads) {
            s.c[e] = T(0);
            if (GRAD) { s.dcs[e] = T(0); s.dcs[KL2 + e] = T(0); s.dcs[2 * KL2 + e] = T(0); }
        }
    // packed (l, k1, k2) of every position of a dp row: l | k1 << 4 | k2 << 14
    if (ROWS)
        for (int o = tid; o < PL; o += kThreads) s.pos[o] = a.dp_pos[o];
    // items (species, n pair, lm): two n per thread share the Y and dY loads
    const int ng = (d.nmax + 1) / 2;
    const int items = d.S * ng * d.L2;
    T rc[REGC ? kRegItems : 1][2];
#pragma unroll
    for (int j = 0; j < (REGC ? kRegItems : 1); ++j) rc[j][0] = rc[j][1] = T(0);
    for (int ck = 0; ck < n_chunks; ++ck) {
        const int64_t q0 = q_begin + (ck == 0 ? 0 : int64_t(ck) * chunk - pad);
        const int nc = ck == 0 ? chunk - pad : chunk;
        stage_chunk<T, GRAD>(a, d, s, q0, nc);
        if constexpr (REGC) {
#pragma unroll
            for (int j = 0; j < kRegItems; ++j) {
                int t = tid + j * kThreads;
                if (t >= items) break;
                // keep the item's decode inside the chunk loop: hoisted
                // for every j it would hold ~100 registers across the staging
                asm volatile("" : "+v"(t));
                const int sp = t / (ng * d.L2), rem = t - sp * (ng * d.L2), g = rem / d.L2, lm = rem - g * d.L2;
                const int n0 = 2 * g, two = n0 + 1 < d.nmax;
                T c0 = T(0), c1 = T(0);
                species_sums<T, 1>(s, d, sp, lm, s.lof[lm], n0, two, s.seg[2 * sp], s.seg[2 * sp + 1], c0, c1);
                rc[j][0] += c0;
                rc[j][1] += c1;
            }
            if (ck + 1 < n_chunks) __syncthreads();
            continue;
        }
        for (int t = tid; t < items; t += kThreads) {
            const int sp = t / (ng * d.L2), rem = t - sp * (ng * d.L2), g = rem / d.L2, lm = rem - g * d.L2;
            const int n0 = 2 * g, two = n0 + 1 < d.nmax;
            const int l = s.lof[lm];
            const int e0 = (sp * d.nmax + n0) * d.L2 + lm;
            T c0 = T(0), c1 = T(0);
            T a0 = T(0), a1 = T(0), a2 = T(0), b0 = T(0), b1 = T(0), b2 = T(0);
            const int p0 = s.seg[2 * sp], p1 = s.seg[2 * sp + 1];
            if (!GRAD) species_sums<T, 4>(s, d, sp, lm, l, n0, two, p0, p1, c0, c1);
            for (int p = p0; p < (GRAD ? p1 : p0); ++p) {
                if (s.spc[p] != sp) continue;
                V4<T> yd;
                if (GRAD) yd = s.YD[p * d.L2 + lm];
                const T Yv = GRAD ? yd.x : s.Y[p * d.L2 + lm];
                const T* Rp = s.R + p * d.nl + n0 * lm1 + l;
                const T R0 = Rp[0], R1 = two ? Rp[lm1] : T(0);
                c0 += R0 * Yv;
                c1 += R1 * Yv;
                if (GRAD) {
                    // pair row d c / d r_ji = (f I~)' u Y + f I~ grad Y; the
                    // self row is minus the sum of the rows (App. B)
                    const T* dRp = s.dR + p * d.nl + n0 * lm1 + l;
                    const T dR0 = dRp[0], dR1 = two ? dRp[lm1] : T(0);
                    const T al0 = s.ux[p] * Yv, al1 = s.uy[p] * Yv, al2 = s.uz[p] * Yv;
                    const T D0 = yd.y, D1 = yd.z, D2 = yd.w;
                    const T r00 = dR0 * al0 + R0 * D0, r01 = dR0 * al1 + R0 * D1, r02 = dR0 * al2 + R0 * D2;
                    const T r10 = dR1 * al0 + R1 * D0, r11 = dR1 * al1 + R1 * D1, r12 = dR1 * al2 + R1 * D2;
                    a0 += r00;
                    a1 += r01;
                    a2 += r02;
                    b0 += r10;
                    b1 += r11;
                    b2 += r12;
                    if (ROWS) {
                        T* dq = static_cast<T*>(a.dcoeffs) + (q0 + p) * int64_t(3 * nL2) + (n0 * d.L2 + lm);
                        dq[0] = r00;
                        dq[nL2] = r01;
                        dq[2 * nL2] = r02;
                        if (two) {
                            dq[d.L2] = r10;
                            dq[nL2 + d.L2] = r11;
                            dq[2 * nL2 + d.L2] = r12;
                        }
                    }
                }
            }
            s.c[e0] += c0;
            if (two) s.c[e0 + d.L2] += c1;
            if (GRAD) {
                s.dcs[e0] -= a0;
                s.dcs[KL2 + e0] -= a1;
                s.dcs[2 * KL2 + e0] -= a2;
                if (two) {
                    s.dcs[e0 + d.L2] -= b0;
                    s.dcs[KL2 + e0 + d.L2] -= b1;
                    s.dcs[2 * KL2 + e0 + d.L2] -= b2;
                }
            }
        }
        if (ck + 1 < n_chunks) __syncthreads();
    }
    if constexpr (REGC) {
        // c straight from the registers, the central atom's term added to
        // the lm = 0 entries of its own species
        const int sp_i = a.include_center ? a.species[i] : -1;
        if (a.include_center && tid == 0 && (sp_i < 0 || sp_i >= d.S)) put_status(a.status, SOAP_ESPECIES);
        const T* centre_term = static_cast<const T*>(a.center);
        T* c_out = static_cast<T*>(a.coeffs) + i * KL2;
#pragma unroll
        for (int j = 0; j < kRegItems; ++j) {
            const int t = tid + j * kThreads;
            if (t >= items) break;
            const int sp = t / (ng * d.L2), rem = t - sp * (ng * d.L2), g = rem / d.L2, lm = rem - g * d.L2;
            const int n0 = 2 * g, two = n0 + 1 < d.nmax;
            T v0 = rc[j][0], v1 = rc[j][1];
            if (lm == 0 && sp == sp_i) {
                v0 += centre_term[n0];
                if (two) v1 += centre_term[n0 + 1];
            }
            const int e0 = (sp * d.nmax + n0) * d.L2 + lm;
            c_out[e0] = v0;
            if (two) c_out[e0 + d.L2] = v1;
        }
        return;
    }
    __syncthreads();
    if (a.include_center && tid < d.nmax) {
        int sp = a.species[i];
        if (sp >= 0 && sp < d.S) s.c[(sp * d.nmax + tid) * d.L2] += static_cast<const T*>(a.center)[tid];
        else put_status(a.status, SOAP_ESPECIES);
    }
    __syncthreads();
    T* c_out = static_cast<T*>(a.coeffs) + i * KL2;
    for (int e = tid; e < KL2; e += kThreads) c_out[e] = s.c[e];
    if (GRAD) {
        T* dcs_out = static_cast<T*>(a.dcoeffs_self) + i * 3 * KL2;
        for (int e = tid; e < 3 * KL2; e += kThreads) dcs_out[e] = s.dcs[e];
    }
    if (!WANT_P) return;
    const bool tri_tab = L.pos != L.tri;
    T* p_out = static_cast<T*>(a.p) + i * int64_t(PL);
    T* dps_out = GRAD ? static_cast<T*>(a.dp_self) + i * int64_t(3 * PL) : nullptr;
    int l = tid / KK, kk = tid - (tid / KK) * KK;
    for (int o = tid; o < PL; o += kThreads) {
        int k1, k2;
        if (ROWS) {
            const int v = s.pos[o];
            l = v & 15;
            k1 = (v >> 4) & 1023;
            k2 = v >> 14;
        } else {
            tri_pair(d, s, tri_tab, kk, k1, k2);
        }
        const T* c1 = s.c + k1 * d.L2 + l * l;
        const T* c2 = s.c + k2 * d.L2 + l * l;
        T acc = T(0);
        for (int m = 0; m < 2 * l + 1; ++m) acc += c1[m] * c2[m];
        p_out[o] = acc;
        if (GRAD) {
            // self rows of p: the product rule on the self rows of c
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const T* g1 = s.dcs + x * KL2 + k1 * d.L2 + l * l;
                const T* g2 = s.dcs + x * KL2 + k2 * d.L2 + l * l;
                T acc2 = T(0);
                for (int m = 0; m < 2 * l + 1; ++m) acc2 += g1[m] * c2[m] + c1[m] * g2[m];
                dps_out[x * PL + o] = acc2;
            }
        }
        if (!ROWS) {
            kk += kThreads;
            while (kk >= KK) { kk -= KK; ++l; }
        }
    }
    if (!ROWS) return;
    // Pair rows of p (Sec. 4.G) in the reordered product rule
    //   dp_{x,l,k1 k2} = u_x (A_{l,k1} y_{l,k2} + A_{l,k2} y_{l,k1})
    //                    + B_{l,k1} z_{x,l,k2} + B_{l,k2} z_{x,l,k1},
    //   y_{l,k} = sum_m Y_lm c_{k,lm},  z_{x,l,k} = sum_m dY_{x,lm} c_{k,lm},
    //   {A, B}_{l,k} = {(f I~)'_nl, f I~_nl} for k = a_j nmax + n, else 0.
    // The last chunk is still staged; earlier chunks are staged again.  Each
    // wave takes whole pairs: its lanes put the {y, z} of every (l, k) of the
    // pair in the wave's own LDS buffer, then one lane per dp position writes
    // its three components; waves synchronise only with themselves.
    const int wave = tid >> 6, lane = tid & 63;
    const int nlk = lm1 * d.K;
    V4<T>* yzw = reinterpret_cast<V4<T>*>(s.yz) + wave * nlk;
    for (int ck = n_chunks - 1; ck >= 0; --ck) {
        const int64_t q0 = q_begin + (ck == 0 ? 0 : int64_t(ck) * chunk - pad);
        const int nc = ck == 0 ? chunk - pad : chunk;
        __syncthreads();
        if (ck != n_chunks - 1) stage_chunk<T, true>(a, d, s, q0, nc);
        for (int p = wave; p < nc; p += kWaves) {
            const V4<T>* YDp = s.YD + p * d.L2;
            for (int t = lane; t < nlk; t += 64) {
                const int l2 = t / d.K, k = t - l2 * d.K;
                const int m0 = l2 * l2;
                const T* ck_ = s.c + k * d.L2;
                T y = T(0), z0 = T(0), z1 = T(0), z2 = T(0);
                for (int m = m0; m < m0 + 2 * l2 + 1; ++m) {
                    const T cv = ck_[m];
                    const V4<T> yd = YDp[m];
                    y += yd.x * cv;
                    z0 += yd.y * cv;
                    z1 += yd.z * cv;
                    z2 += yd.w * cv;
                }
                yzw[t] = V4<T>{y, z0, z1, z2};
            }
            wave_sync();
            const T ux = s.ux[p], uy = s.uy[p], uz = s.uz[p];
            const int blk = s.spc[p] * d.nmax;
            const T* Rp = s.R + p * d.nl;
            const T* dRp = s.dR + p * d.nl;
            T* row = static_cast<T*>(a.dp) + (q0 + p) * int64_t(3 * PL);
            for (int o = lane; o < PL; o += 64) {
                const int v = s.pos[o];
                const int l2 = v & 15, k1 = (v >> 4) & 1023, k2 = v >> 14;
                const V4<T> q1 = yzw[l2 * d.K + k1], q2 = yzw[l2 * d.K + k2];
                const int n1 = k1 - blk, n2 = k2 - blk;
                const bool in1 = n1 >= 0 && n1 < d.nmax, in2 = n2 >= 0 && n2 < d.nmax;
                const T A1 = in1 ? dRp[n1 * lm1 + l2] : T(0), B1 = in1 ? Rp[n1 * lm1 + l2] : T(0);
                const T A2 = in2 ? dRp[n2 * lm1 + l2] : T(0), B2 = in2 ? Rp[n2 * lm1 + l2] : T(0);
                const T a0 = A1 * q2.x + A2 * q1.x;
                row[o] = ux * a0 + B1 * q2.y + B2 * q1.y;
                row[PL + o] = uy * a0 + B1 * q2.z + B2 * q1.z;
                row[2 * PL + o] = uz * a0 + B1 * q2.w + B2 * q1.w;
            }
            wave_sync();
        }
    }
}

template <typename T, int LM, bool GRAD, bool WANT_P, bool ROWS>
__global__ void __launch_bounds__(kThreads) k_centres(FeatureArgs a, Layout L)
{
    centres_body<T, LM, GRAD, WANT_P, ROWS, false>(a, L);
}

// c alone with register sums: four work-groups per CU (at most 128 VGPRs)
template <typename T, int LM>
__global__ void __launch_bounds__(kThreads, 4) k_centres_c(FeatureArgs a, Layout L)
{
    centres_body<T, LM, false, false, false, true>(a, L);
}

// ---------------------------------------------------------------------------
// Power spectrum (and forward-mode rows) from coefficients in memory.
// ---------------------------------------------------------------------------
template <typename T, bool GRAD>
__global__ void __launch_bounds__(kThreads) k_power_spectrum(FeatureArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const Dims d = make_dims(a.S, a.nmax, a.lmax);
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    const int KL2 = d.K * d.L2, nL2 = d.nmax * d.L2, lm1 = d.lmax + 1;
    const int64_t PL = int64_t(lm1) * d.KK;
    T* c = sm;                 // [K][L2]
    T* g = c + KL2;            // [3][K][L2] self row, then per-wave row buffers
    const T* c_in = static_cast<const T*>(a.coeffs) + i * KL2;
    copy_in(c, c_in, KL2);
    if (GRAD) copy_in(g, static_cast<const T*>(a.dcoeffs_self) + i * 3 * KL2, 3 * KL2);
    __syncthreads();
    T* p_out = static_cast<T*>(a.p) + i * PL;
    // one lane per packed (k1, k2), decoded once, every l of it (the lanes
    // of one l store consecutive positions)
    for (int kk = tid; kk < d.KK; kk += kThreads) {
        int k1, k2;
        dev::tri_decode(d.K, kk, k1, k2);
        const T* c1 = c + k1 * d.L2;
        const T* c2 = c + k2 * d.L2;
        for (int l = 0; l < lm1; ++l) {
            T acc = T(0);
            for (int lm = l * l; lm < (l + 1) * (l + 1); ++lm) acc += c1[lm] * c2[lm];
            p_out[int64_t(l) * d.KK + kk] = acc;
        }
    }
    if (!GRAD) return;
    if (a.pair_offsets[a.n_atoms] > a.pair_capacity) {
        if (tid == 0) put_status(a.status, SOAP_ECAPACITY);
        return;
    }
    T* dps_out = static_cast<T*>(a.dp_self) + i * 3 * PL;
    // self rows of p: the product rule on the self rows of c, one lane per
    // packed (k1, k2) over every (x, l)
    for (int kk = tid; kk < d.KK; kk += kThreads) {
        int k1, k2;
        dev::tri_decode(d.K, kk, k1, k2);
        for (int x = 0; x < 3; ++x)
            for (int l = 0; l < lm1; ++l) {
                const T* c1 = c + k1 * d.L2 + l * l;
                const T* c2 = c + k2 * d.L2 + l * l;
                const T* g1 = g + x * KL2 + k1 * d.L2 + l * l;
                const T* g2 = g + x * KL2 + k2 * d.L2 + l * l;
                T acc = T(0);
                for (int m = 0; m < 2 * l + 1; ++m) acc += g1[m] * c2[m] + c1[m] * g2[m];
                dps_out[x * PL + int64_t(l) * d.KK + kk] = acc;
            }
    }
    __syncthreads();
    // rows: one wave per pair; w[x][l][n][k] = sum_m dc_{x,n,lm} c_{k,lm}
    const int wave = tid >> 6, lane = tid & 63;
    const int wn = 3 * lm1 * d.nmax * d.K;
    T* row = g + wave * (3 * nL2 + wn);
    T* w = row + 3 * nL2;
    const int64_t q_begin = a.pair_offsets[i], q_end = a.pair_offsets[i + 1];
    for (int64_t q = q_begin + wave; q < q_end; q += kWaves) {
        const T* dc_in = static_cast<const T*>(a.dcoeffs) + q * 3 * nL2;
        for (int e = lane; e < 3 * nL2; e += 64) row[e] = dc_in[e];
        int jq = a.pair_j[q];
        int sp = (jq >= 0 && jq < a.n_atoms) ? a.species[jq] : -1;
        if (sp < 0 || sp >= d.S) { put_status(a.status, SOAP_ESPECIES); sp = 0; }
        const int blk = sp * d.nmax;
        wave_sync();
        for (int t = lane; t < wn; t += 64) {
            int x = t / (lm1 * d.nmax * d.K);
            int rem = t - x * lm1 * d.nmax * d.K;
            int l = rem / (d.nmax * d.K);
            rem -= l * d.nmax * d.K;
            int n = rem / d.K, k = rem - n * d.K;
            const T* r1 = row + x * nL2 + n * d.L2 + l * l;
            const T* c2 = c + k * d.L2 + l * l;
            T acc = T(0);
            for (int m = 0; m < 2 * l + 1; ++m) acc += r1[m] * c2[m];
            w[t] = acc;
        }
        wave_sync();
        T* dp_row = static_cast<T*>(a.dp) + q * 3 * PL;
        for (int64_t o = lane; o < 3 * PL; o += 64) {
            int x = int(o / PL);
            int64_t r0 = o - x * PL;
            int l = int(r0 / d.KK);
            int kk = int(r0 - int64_t(l) * d.KK);
            int k1, k2;
            dev::tri_decode(d.K, kk, k1, k2);
            const T* wl = w + (x * lm1 + l) * d.nmax * d.K;
            T v = T(0);
            int n1 = k1 - blk, n2 = k2 - blk;
            if (n1 >= 0 && n1 < d.nmax) v += wl[n1 * d.K + k2];
            if (n2 >= 0 && n2 < d.nmax) v += wl[n2 * d.K + k1];
            dp_row[o] = v;
        }
        wave_sync();
    }
}

template <typename K>
hipError_t launch_dyn(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t stream, const FeatureArgs& a)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, a);
    return hipGetLastError();
}

template <typename K>
hipError_t launch_feat(K kernel, size_t lds, hipStream_t stream, const FeatureArgs& a, const Layout& L)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kernel, dim3(unsigned(a.n_atoms)), dim3(kThreads), lds, stream, a, L);
    return hipGetLastError();
}

constexpr size_t kMaxLds = 160 * 1024;

template <typename T, int LM>
hipError_t centres_launch(const FeatureArgs& a, const Layout& L, size_t lds, bool rows, hipStream_t stream)
{
    const bool grad = a.dcoeffs_self != nullptr, want_p = a.p != nullptr;
    if (rows) return launch_feat(k_centres<T, LM, true, true, true>, lds, stream, a, L);
    if constexpr (std::is_same<T, float>::value)
        if (L.c == L.dcs)   // no c region: register sums
            return launch_feat(k_centres_c<T, LM>, lds, stream, a, L);
    if (grad)
        return want_p ? launch_feat(k_centres<T, LM, true, true, false>, lds, stream, a, L)
                      : launch_feat(k_centres<T, LM, true, false, false>, lds, stream, a, L);
    return want_p ? launch_feat(k_centres<T, LM, false, true, false>, lds, stream, a, L)
                  : launch_feat(k_centres<T, LM, false, false, false>, lds, stream, a, L);
}

template <typename T, int LM>
struct CentresFn {
    static hipError_t run(const FeatureArgs& a, const Layout& L, size_t lds, bool rows, hipStream_t st)
    {
        return centres_launch<T, LM>(a, L, lds, rows, st);
    }
};

// Per-centre pass (c, p, self rows).  The pair rows come from the same
// kernel when both are asked for, the position table exists and its layout
// fits; otherwise from the row kernel once c is in memory.
template <typename T>
hipError_t features_t(const FeatureArgs& a, hipStream_t stream)
{
    Dims d = make_dims(a.S, a.nmax, a.lmax);
    bool grad = a.dcoeffs_self != nullptr;
    bool want_p = a.p != nullptr;
    FeatureArgs c = a;
    c.dp_self = want_p ? a.dp_self : nullptr;
    if (grad && want_p && a.dcoeffs && a.dp && a.dp_pos && a.pair_capacity > 0) {
        // each pair staged once (features_rows.hip); the kernel below when
        // its layout does not fit
        hipError_t e = launch_features_rows(a, std::is_same<T, double>::value, stream);
        if (e != hipErrorNotSupported) return e;
        Layout L = choose_rows_layout<T>(d);
        if (L.total != 0)
            return by_lmax<T, CentresFn>(a.lmax, c, L, size_t(L.total) * sizeof(T), true, stream);
    }
    if (!grad) {
        // c (and p) with one lane per pair; the pair rows, if asked for,
        // from the row kernel
        hipError_t e = launch_expansion_lanes(c, std::is_same<T, double>::value, stream);
        if (e == hipSuccess) return launch_gradient_rows(a, std::is_same<T, double>::value, stream);
        if (e != hipErrorNotSupported) return e;
    }
    Layout L = choose_layout<T>(d, grad, true, want_p);
    // c alone in float, when its LDS accumulator forces chunks below 32
    // pairs: register sums instead (128 VGPRs, four work-groups per CU; in
    // double they would spill).  When the chunk already holds 32 pairs the
    // LDS form keeps more work-groups per CU.
    const bool regc = std::is_same<T, float>::value && !grad && !want_p &&
                      d.S * ((d.nmax + 1) / 2) * d.L2 <= kRegItems * kThreads &&
                      (L.chunk < 32 || size_t(L.total) * sizeof(T) > 40 * 1024);
    if (regc) L = choose_layout<T>(d, false, true, false, false);
    if (L.total == 0) return hipErrorNotSupported;
    size_t lds = size_t(L.total) * sizeof(T);
    hipError_t e = by_lmax<T, CentresFn>(a.lmax, c, L, lds, false, stream);
    if (e != hipSuccess) return e;
    return launch_gradient_rows(a, std::is_same<T, double>::value, stream);
}

template <typename T>
hipError_t power_spectrum_t(const FeatureArgs& a, hipStream_t stream)
{
    Dims d = make_dims(a.S, a.nmax, a.lmax);
    bool grad = a.dp != nullptr;
    size_t n = size_t(d.K) * d.L2;
    size_t self_row = 3 * size_t(d.K) * d.L2;
    size_t row_bufs = size_t(kWaves) * (3 * d.nmax * d.L2 + 3 * (d.lmax + 1) * d.nmax * d.K);
    if (grad) n += self_row > row_bufs ? self_row : row_bufs;
    size_t lds = n * sizeof(T);
    if (lds > kMaxLds) return hipErrorNotSupported;
    dim3 grid(unsigned(a.n_atoms)), block(kThreads);
    if (grad) return launch_dyn(k_power_spectrum<T, true>, grid, block, lds, stream, a);
    return launch_dyn(k_power_spectrum<T, false>, grid, block, lds, stream, a);
}

}  // namespace

hipError_t launch_features(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    return f64 ? features_t<double>(a, stream) : features_t<float>(a, stream);
}

hipError_t launch_power_spectrum_valu(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    return f64 ? power_spectrum_t<double>(a, stream) : power_spectrum_t<float>(a, stream);
}

}  // namespace soap
