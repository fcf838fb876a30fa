// Forward-mode gradient rows of every pair (Sec. 4.G; App. B for the sign
// convention d r_ji / d r_j = +1).  For pair q = (i, j, s) with unit vector
// u = r_ji / r, neighbour species a_j and k = a_j nmax + n:
//   dc_{x,n,lm}(q) = (f I~)'_nl u_x Y_lm + f I~_nl dY_{x,lm}
//   dp_{x,l,k1 k2}(q) = sum_m dc_{x,k1,lm} c_{k2,lm} + c_{k1,lm} dc_{x,k2,lm}
// where dc_{x,k,lm} vanishes outside the species block of a_j.  The product
// rule is summed in the reordered form
//   sum_m dc_{x,(a_j,n),lm} c_{k,lm} = A_{l,k} u_x y_{l,k} + B_{l,k} z_{x,l,k},
//   y_{l,k} = sum_m Y_lm c_{k,lm},   z_{x,l,k} = sum_m dY_{x,lm} c_{k,lm},
//   {A, B}_{l,k} = {(f I~)'_nl, f I~_nl} inside the block of a_j, else 0,
// so a dp row costs O(K L2 + K^2 (lmax+1)) and the dc row is written to
// memory but never read back.
//
// Grid (centres, groups): group g of centre i takes a contiguous share of
// its pairs (about one chunk of kRowChunk pairs), restages them through LDS
// (the per-pair evaluation of the expansion kernel) and streams out
//   dc - one lane per (pair, x, lm) writes the nmax values of that (x, lm);
//   dp - the {y, z} and {A, B} operands of every (pair, l, k) go to LDS, then
//        one lane per packed position (l, k1, k2) of a pair writes its three
//        components.
// c of the centre (written by the expansion kernel) is read back into LDS;
// the packed (l, k1, k2) of the dp positions come from a device table built
// with the spline tables.  The rows of a pair are contiguous in memory (dc:
// [3][nmax][L2], dp: [3][lmax+1][K(K+1)/2]) and consecutive lanes write
// consecutive addresses.
#include "chunk.hpp"

namespace soap {
namespace {

using namespace dev;

constexpr int kRowChunk = 8;   // pairs a row group stages at a time
constexpr size_t kMaxRowLds = 160 * 1024;

template <typename T, int LM, bool WANT_DC, bool WANT_DP>
__global__ void __launch_bounds__(kThreads) k_pair_rows(FeatureArgs a, Layout L)
{
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
    const int n_pairs = int(q_end - q_begin);
    const int G = gridDim.y, g = blockIdx.y;
    const int share = (n_pairs + G - 1) / G;
    const int p_lo = g * share, p_hi = (g + 1) * share < n_pairs ? (g + 1) * share : n_pairs;
    if (p_lo >= p_hi) return;
    const int KL2 = d.K * d.L2, nL2 = d.nmax * d.L2, lm1 = d.lm1;
    const int KK = d.KK, PL = lm1 * KK;
    init_tables<T>(a, d, L, s);
    if (WANT_DP) {
        const T* c_in = static_cast<const T*>(a.coeffs) + i * KL2;
        copy_in(s.c, c_in, KL2);
        // packed positions of a dp row: l | k1 << 4 | k2 << 14
        for (int o = tid; o < PL; o += kThreads) s.pos[o] = a.dp_pos[o];
    }
    const int EDC = 3 * nL2;
    const int yzn = lm1 * d.K;
    for (int c0 = p_lo; c0 < p_hi; c0 += L.chunk) {
        const int nc = p_hi - c0 < L.chunk ? p_hi - c0 : L.chunk;
        const int64_t q0 = q_begin + c0;
        if (c0 != p_lo) __syncthreads();
        stage_chunk<T, true>(a, d, s, q0, nc);
        if (WANT_DC) {
            T* dc_base = static_cast<T*>(a.dcoeffs) + q0 * EDC;
            const int per_pair = 3 * d.L2;
            for (int t = tid; t < nc * per_pair; t += kThreads) {
                const int p = t / per_pair, rem = t - p * per_pair, x = rem / d.L2, lm = rem - x * d.L2;
                const int l = s.lof[lm];
                const T u = x == 0 ? s.ux[p] : (x == 1 ? s.uy[p] : s.uz[p]);
                const V4<T> yd = s.YD[p * d.L2 + lm];
                const T alpha = u * yd.x;
                const T beta = x == 0 ? yd.y : (x == 1 ? yd.z : yd.w);
                const T* dRp = s.dR + p * d.nl + l;
                const T* Rp = s.R + p * d.nl + l;
                T* out = dc_base + (uint32_t(p * EDC) + uint32_t(x * nL2 + lm));
#pragma unroll 4
                for (int n = 0; n < d.nmax; ++n) out[n * d.L2] = dRp[n * lm1] * alpha + Rp[n * lm1] * beta;
            }
        }
        if (WANT_DP) {
            // per pair and (l, k): {y, z_x, z_y, z_z}_{l,k} with
            //   y = sum_m Y_lm c_{k,lm},  z_x = sum_m dY_{x,lm} c_{k,lm},
            // and {A, B}_{l,k} = {(f I~)', f I~}_{n l} for k = a_j nmax + n,
            // zero outside the neighbour's species block
            for (int t = tid; t < nc * yzn; t += kThreads) {
                int p = t / yzn, rem = t - p * yzn, l = rem / d.K, k = rem - l * d.K;
                const T* ck_ = s.c + k * d.L2 + l * l;
                const V4<T>* YDp = s.YD + p * d.L2 + l * l;
                T y = T(0), z0 = T(0), z1 = T(0), z2 = T(0);
                for (int m = 0; m < 2 * l + 1; ++m) {
                    const T cv = ck_[m];
                    const V4<T> yd = YDp[m];
                    y += yd.x * cv;
                    z0 += yd.y * cv;
                    z1 += yd.z * cv;
                    z2 += yd.w * cv;
                }
                reinterpret_cast<V4<T>*>(s.yz)[t] = V4<T>{y, z0, z1, z2};
                const int n = k - s.spc[p] * d.nmax;
                const bool in = n >= 0 && n < d.nmax;
                reinterpret_cast<V2<T>*>(s.yz + 4 * nc * yzn)[t] =
                    V2<T>{in ? s.dR[p * d.nl + n * lm1 + l] : T(0), in ? s.R[p * d.nl + n * lm1 + l] : T(0)};
            }
            __syncthreads();
            T* dp_base = static_cast<T*>(a.dp) + q0 * int64_t(3 * PL);
            for (int p = 0; p < nc; ++p) {
                const T ux = s.ux[p], uy = s.uy[p], uz = s.uz[p];
                const V4<T>* yzp = reinterpret_cast<const V4<T>*>(s.yz) + p * yzn;
                const V2<T>* abp = reinterpret_cast<const V2<T>*>(s.yz + 4 * nc * yzn) + p * yzn;
                T* row = dp_base + uint32_t(p * 3 * PL);
                for (int o = tid; o < PL; o += kThreads) {
                    const int v = s.pos[o];
                    const int l = v & 15, k1 = (v >> 4) & 1023, k2 = v >> 14;
                    const int i1 = l * d.K + k1, i2 = l * d.K + k2;
                    const V4<T> q1 = yzp[i1], q2 = yzp[i2];
                    const V2<T> ab1 = abp[i1], ab2 = abp[i2];
                    const T a0 = ab1.x * q2.x + ab2.x * q1.x;
                    row[o] = ux * a0 + ab1.y * q2.y + ab2.y * q1.y;
                    row[PL + o] = uy * a0 + ab1.y * q2.z + ab2.y * q1.z;
                    row[2 * PL + o] = uz * a0 + ab1.y * q2.w + ab2.y * q1.w;
                }
            }
        }
    }
}

template <typename T, int LM>
struct PairRowsFn {
    static hipError_t run(const FeatureArgs& a, const Layout& L, size_t lds, int groups, hipStream_t stream)
    {
        const bool want_dc = a.dcoeffs != nullptr, want_dp = a.dp != nullptr;
        auto kernel = want_dc ? (want_dp ? k_pair_rows<T, LM, true, true> : k_pair_rows<T, LM, true, false>)
                              : k_pair_rows<T, LM, false, true>;
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kernel, dim3(unsigned(a.n_atoms), unsigned(groups)), dim3(kThreads), lds, stream, a, L);
        return hipGetLastError();
    }
};

template <typename T>
hipError_t rows_t(const FeatureArgs& a, hipStream_t stream)
{
    const Dims d = make_dims(a.S, a.nmax, a.lmax);
    const bool want_dc = a.dcoeffs != nullptr, want_dp = a.dp != nullptr;
    if (a.pair_capacity == 0 || a.n_atoms == 0 || (!want_dc && !want_dp)) return hipSuccess;
    if (want_dp && a.dp_pos == nullptr) return hipErrorNotSupported;   // K > 1023: no position table
    // {y, z} and {A, B} of every (pair, l, k) of a chunk, and the table of
    // the (l, k1, k2) of every position of a dp row
    Layout R = make_layout(d, kRowChunk, true, want_dp ? kRowChunk * 6 * d.lm1 * d.K : 0, false, false,
                           want_dp ? d.lm1 * d.KK : 0);
    const size_t lds = size_t(R.total) * sizeof(T);
    if (lds > kMaxRowLds) return hipErrorNotSupported;
    // about one chunk of pairs per work-group at the mean neighbour count
    const int64_t mean = (a.pair_capacity + a.n_atoms - 1) / a.n_atoms;
    int64_t groups = (mean + kRowChunk - 1) / kRowChunk;
    groups = groups < 1 ? 1 : (groups > 64 ? 64 : groups);
    return by_lmax<T, PairRowsFn>(a.lmax, a, R, lds, int(groups), stream);
}

}  // namespace

hipError_t launch_gradient_rows(const FeatureArgs& a, bool f64, hipStream_t stream)
{
    return f64 ? rows_t<double>(a, stream) : rows_t<float>(a, stream);
}

}  // namespace soap
