// Neighbour list on the device (App. B: environments hold every j, periodic
// images included, with r_ji < rcut).
//
// Each structure is cut into a grid of bins whose perpendicular width is at
// least rcut along every periodic lattice direction (one bin along
// non-periodic directions).  An atom's bin comes from its fractional
// coordinates wrapped into the cell; the wrap count is remembered so that
// the reported image shift refers to the caller's (unwrapped) positions.
// A centre visits the bins whose unwrapped index differs from its own by at
// most `reach` along each periodic direction; every unwrapped bin maps to a
// distinct (bin, cell shift) pair, so each image is seen exactly once even
// in cells thinner than rcut.
//
// Phases (one launch each, all on the caller's stream, no host copies):
//   geometry - per structure: inverse cell, bins per axis, stencil reach and
//              first bin (one work-group, scan over structures)
//   assign  - structure, wrap and bin of every atom, bin occupancy counts
//   scan    - bin starts
//   bins    - atoms scattered into their bins
//   count   - pairs per centre
//   scan    - pair_offsets (the total is checked against the capacity)
//   fill    - (j, s) of each centre's pairs, in visiting order
//   sort    - per centre, rank by (species_j, j, s) and rewrite; pair
//             vectors formed in double from the positions
//   transpose (optional) - index of the reverse pair (j, i, -s)
// Integer atomics are used only for bin occupancy; the final order does not
// depend on them, so the output is deterministic.
#include "soap_internal.hpp"

namespace soap {
namespace {

__device__ __forceinline__ void put_status(int32_t* st, int v)
{
    if (st) *st = v;
}

__device__ __forceinline__ int floordiv(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Per-structure geometry.  Bins per periodic axis: floor(width / rcut),
// capped so that a structure never has more bins than atoms (the workspace
// then holds at most N + n_structures bins); the reach is the number of
// bins that spans rcut.  Any invalid input clears *ok and every later phase
// produces an empty list.
__device__ bool make_geometry(const NeighborArgs& a, int s, StructGeom& g)
{
    int64_t lo = a.atom_offsets[s], hi = a.atom_offsets[s + 1];
    g.atom_lo = lo;
    g.atom_hi = hi;
    bool valid = lo >= 0 && hi >= lo && hi <= a.n_atoms;
    int64_t ns = valid ? hi - lo : 0;
    bool any = false;
    for (int k = 0; k < 3; ++k) {
        g.pbc[k] = a.pbc[3 * s + k] ? 1 : 0;
        any = any || g.pbc[k];
    }
    for (int k = 0; k < 9; ++k) g.H[k] = g.Hinv[k] = (k % 4 == 0) ? 1.0 : 0.0;
    for (int k = 0; k < 3; ++k) { g.nbin[k] = 1; g.reach[k] = 0; }
    if (!any) return valid;
    const double* H = a.cells + 9 * s;
    double scale = 0.0;
    for (int k = 0; k < 9; ++k) {
        g.H[k] = H[k];
        scale = fmax(scale, fabs(H[k]));
    }
    double det = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                 H[2] * (H[3] * H[7] - H[4] * H[6]);
    if (!(fabs(det) > 1e-10 * scale * scale * scale) || !(scale > 0.0) || !isfinite(det)) return false;
    double* Hi = g.Hinv;
    Hi[0] = (H[4] * H[8] - H[5] * H[7]) / det;
    Hi[1] = (H[2] * H[7] - H[1] * H[8]) / det;
    Hi[2] = (H[1] * H[5] - H[2] * H[4]) / det;
    Hi[3] = (H[5] * H[6] - H[3] * H[8]) / det;
    Hi[4] = (H[0] * H[8] - H[2] * H[6]) / det;
    Hi[5] = (H[2] * H[3] - H[0] * H[5]) / det;
    Hi[6] = (H[3] * H[7] - H[4] * H[6]) / det;
    Hi[7] = (H[1] * H[6] - H[0] * H[7]) / det;
    Hi[8] = (H[0] * H[4] - H[1] * H[3]) / det;
    int cap = 1;
    while (int64_t(cap + 1) * (cap + 1) * (cap + 1) <= ns && cap < 128) ++cap;
    for (int k = 0; k < 3; ++k) {
        if (!g.pbc[k]) continue;
        double gk = sqrt(Hi[0 * 3 + k] * Hi[0 * 3 + k] + Hi[1 * 3 + k] * Hi[1 * 3 + k] + Hi[2 * 3 + k] * Hi[2 * 3 + k]);
        double width = 1.0 / gk;
        double nbf = floor(width / a.rcut);
        int nb = nbf < 1.0 ? 1 : (nbf > double(cap) ? cap : int(nbf));
        double need = ceil(a.rcut * nb / width * (1.0 + 1e-12));
        if (!(need <= 1024.0)) return false;
        g.nbin[k] = nb;
        g.reach[k] = need < 1.0 ? 1 : int(need);
    }
    return valid;
}

__global__ void __launch_bounds__(1024) k_geometry(NeighborArgs a)
{
    __shared__ int64_t part[1024];
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t == 0) bad = (a.atom_offsets[0] != 0 || a.atom_offsets[a.n_structures] != a.n_atoms) ? 1 : 0;
    __syncthreads();
    const int64_t n = a.n_structures;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
    int64_t sum = 0;
    for (int64_t s = b; s < e; ++s) {
        StructGeom g;
        if (!make_geometry(a, int(s), g)) bad = 1;
        sum += int64_t(g.nbin[0]) * g.nbin[1] * g.nbin[2];
        a.geom[s] = g;
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int64_t s = b; s < e; ++s) {
        a.geom[s].bin_lo = run;
        run += int64_t(a.geom[s].nbin[0]) * a.geom[s].nbin[1] * a.geom[s].nbin[2];
    }
    __syncthreads();
    if (t == 0) {
        if (part[1023] > a.max_bins) bad = 1;
        *a.ok = bad ? 0 : 1;
        if (bad) put_status(a.status, SOAP_EINVAL);
    }
}

__global__ void k_zero_i32(int32_t* p, int64_t n)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_assign(NeighborArgs a)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_atoms || !*a.ok) return;
    // structure of atom i: first s with atom_hi > i
    int lo = 0, hi = a.n_structures - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a.geom[mid].atom_hi > i) hi = mid; else lo = mid + 1;
    }
    const StructGeom& g = a.geom[lo];
    double r[3] = {a.positions[3 * i], a.positions[3 * i + 1], a.positions[3 * i + 2]};
    int b[3], t[3];
    for (int k = 0; k < 3; ++k) {
        if (!g.pbc[k]) { b[k] = 0; t[k] = 0; continue; }
        double f = r[0] * g.Hinv[0 * 3 + k] + r[1] * g.Hinv[1 * 3 + k] + r[2] * g.Hinv[2 * 3 + k];
        double fl = floor(f);
        double fw = f - fl;
        t[k] = int(fl);
        int bk = int(fw * g.nbin[k]);
        b[k] = bk < 0 ? 0 : (bk >= g.nbin[k] ? g.nbin[k] - 1 : bk);
    }
    int32_t bin = int32_t(g.bin_lo + (int64_t(b[0]) * g.nbin[1] + b[1]) * g.nbin[2] + b[2]);
    a.atom_struct[i] = lo;
    a.atom_bin[i] = bin;
    a.atom_wrap[3 * i + 0] = t[0];
    a.atom_wrap[3 * i + 1] = t[1];
    a.atom_wrap[3 * i + 2] = t[2];
    int sp = a.species[i];
    if (sp < 0 || sp >= a.n_species) put_status(a.status, SOAP_ESPECIES);
    atomicAdd(&a.bin_count[bin], 1);
}

// Exclusive scan of n values into out[0..n], out[n] = total, by one block
// of 1024 threads (each thread owns a contiguous chunk).
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(1024) k_scan(const Tin* in, Tout* out, Tout* out2, int64_t n,
                                               int64_t capacity, int32_t* status)
{
    __shared__ Tout part[1024];
    int t = threadIdx.x;
    int64_t chunk = (n + 1023) / 1024;
    int64_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
    Tout s = 0;
    for (int64_t k = b; k < e; ++k) s += Tout(in[k]);
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        Tout v = t >= off ? part[t - off] : Tout(0);
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    Tout run = part[t] - s;
    for (int64_t k = b; k < e; ++k) {
        out[k] = run;
        if (out2) out2[k] = run;
        run += Tout(in[k]);
    }
    if (t == 1023) {
        out[n] = part[1023];
        if (capacity >= 0 && int64_t(part[1023]) > capacity) put_status(status, SOAP_ECAPACITY);
    }
}

__global__ void k_bins(NeighborArgs a)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_atoms || !*a.ok) return;
    int pos = atomicAdd(&a.bin_cursor[a.atom_bin[i]], 1);
    a.bin_atoms[pos] = int32_t(i);
}

// Visit every (j, s) of centre i with 0 < |r_ji| < rcut.
template <class F>
__device__ void visit(const NeighborArgs& a, int64_t i, F&& emit)
{
    const StructGeom& g = a.geom[a.atom_struct[i]];
    int local = a.atom_bin[i] - int32_t(g.bin_lo);
    int b2 = local % g.nbin[2];
    int b1 = (local / g.nbin[2]) % g.nbin[1];
    int b0 = local / (g.nbin[2] * g.nbin[1]);
    int ti[3] = {a.atom_wrap[3 * i], a.atom_wrap[3 * i + 1], a.atom_wrap[3 * i + 2]};
    double ri[3] = {a.positions[3 * i], a.positions[3 * i + 1], a.positions[3 * i + 2]};
    double rc2 = a.rcut * a.rcut;
    for (int d0 = -g.reach[0]; d0 <= g.reach[0]; ++d0) {
        int u0 = b0 + d0, n0 = g.nbin[0];
        int bb0 = u0 - floordiv(u0, n0) * n0, c0 = floordiv(u0, n0);
        for (int d1 = -g.reach[1]; d1 <= g.reach[1]; ++d1) {
            int u1 = b1 + d1, n1 = g.nbin[1];
            int bb1 = u1 - floordiv(u1, n1) * n1, c1 = floordiv(u1, n1);
            for (int d2 = -g.reach[2]; d2 <= g.reach[2]; ++d2) {
                int u2 = b2 + d2, n2 = g.nbin[2];
                int bb2 = u2 - floordiv(u2, n2) * n2, c2 = floordiv(u2, n2);
                int64_t bin = g.bin_lo + (int64_t(bb0) * n1 + bb1) * n2 + bb2;
                int q0 = a.bin_start[bin], q1 = a.bin_start[bin + 1];
                for (int q = q0; q < q1; ++q) {
                    int j = a.bin_atoms[q];
                    int s0 = g.pbc[0] ? c0 + ti[0] - a.atom_wrap[3 * j + 0] : 0;
                    int s1 = g.pbc[1] ? c1 + ti[1] - a.atom_wrap[3 * j + 1] : 0;
                    int s2 = g.pbc[2] ? c2 + ti[2] - a.atom_wrap[3 * j + 2] : 0;
                    if (j == i && s0 == 0 && s1 == 0 && s2 == 0) continue;
                    double v[3];
                    for (int x = 0; x < 3; ++x)
                        v[x] = (a.positions[3 * j + x] - ri[x]) + s0 * g.H[0 * 3 + x] + s1 * g.H[1 * 3 + x] +
                               s2 * g.H[2 * 3 + x];
                    double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                    if (r2 >= rc2) continue;
                    if (r2 == 0.0) { put_status(a.status, SOAP_EGEOMETRY); continue; }
                    emit(j, s0, s1, s2);
                }
            }
        }
    }
}

__global__ void k_count(NeighborArgs a)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_atoms) return;
    int64_t n = 0;
    if (*a.ok) visit(a, i, [&](int, int, int, int) { ++n; });
    a.centre_count[i] = n;
}

__global__ void k_fill(NeighborArgs a)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_atoms || !*a.ok) return;
    if (a.pair_offsets[a.n_atoms] > a.capacity) return;
    int64_t o = a.pair_offsets[i];
    visit(a, i, [&](int j, int s0, int s1, int s2) {
        a.pair_j[o] = j;
        a.pair_shift[3 * o + 0] = s0;
        a.pair_shift[3 * o + 1] = s1;
        a.pair_shift[3 * o + 2] = s2;
        ++o;
    });
}

// sort key: (species_j, j) in the high word, the three shifts (offset by
// 2^20, 21 bits each) in the low word
__device__ __forceinline__ void make_key(int sp, int j, int s0, int s1, int s2, int64_t& hi, int64_t& lo)
{
    hi = (int64_t(sp) << 32) | int64_t(uint32_t(j));
    lo = (int64_t(s0 + (1 << 20)) << 42) | (int64_t(s1 + (1 << 20)) << 21) | int64_t(s2 + (1 << 20));
}

__device__ __forceinline__ bool key_less(int64_t ah, int64_t al, int64_t bh, int64_t bl)
{
    return ah < bh || (ah == bh && al < bl);
}

constexpr int kSortCap = 1024;

template <bool F64>
__device__ void write_vec(const NeighborArgs& a, int64_t i, int64_t q)
{
    const StructGeom& g = a.geom[a.atom_struct[i]];
    int j = a.pair_j[q];
    int s0 = a.pair_shift[3 * q], s1 = a.pair_shift[3 * q + 1], s2 = a.pair_shift[3 * q + 2];
    for (int x = 0; x < 3; ++x) {
        double v = (a.positions[3 * j + x] - a.positions[3 * i + x]) + s0 * g.H[0 * 3 + x] + s1 * g.H[1 * 3 + x] +
                   s2 * g.H[2 * 3 + x];
        if (F64) static_cast<double*>(a.pair_vec)[3 * q + x] = v;
        else static_cast<float*>(a.pair_vec)[3 * q + x] = float(v);
    }
}

// One wave per centre.
template <bool F64>
__global__ void __launch_bounds__(64) k_sort(NeighborArgs a)
{
    __shared__ int64_t khi[kSortCap], klo[kSortCap];
    __shared__ int32_t kj[kSortCap], ks[3 * kSortCap];
    int64_t i = blockIdx.x;
    if (a.pair_offsets[a.n_atoms] > a.capacity) return;
    int64_t o0 = a.pair_offsets[i], o1 = a.pair_offsets[i + 1];
    int n = int(o1 - o0);
    int t = threadIdx.x;
    if (n <= kSortCap) {
        for (int p = t; p < n; p += 64) {
            int64_t q = o0 + p;
            int j = a.pair_j[q];
            int s0 = a.pair_shift[3 * q], s1 = a.pair_shift[3 * q + 1], s2 = a.pair_shift[3 * q + 2];
            make_key(a.species[j], j, s0, s1, s2, khi[p], klo[p]);
            kj[p] = j;
            ks[3 * p] = s0; ks[3 * p + 1] = s1; ks[3 * p + 2] = s2;
        }
        __syncthreads();
        for (int p = t; p < n; p += 64) {
            int rank = 0;
            int64_t h = khi[p], l = klo[p];
            for (int q = 0; q < n; ++q) rank += key_less(khi[q], klo[q], h, l) ? 1 : 0;
            int64_t dst = o0 + rank;
            a.pair_j[dst] = kj[p];
            a.pair_shift[3 * dst] = ks[3 * p];
            a.pair_shift[3 * dst + 1] = ks[3 * p + 1];
            a.pair_shift[3 * dst + 2] = ks[3 * p + 2];
        }
    } else if (t == 0) {
        // long environments: insertion sort in place in global memory
        for (int64_t p = o0 + 1; p < o1; ++p) {
            int j = a.pair_j[p];
            int s0 = a.pair_shift[3 * p], s1 = a.pair_shift[3 * p + 1], s2 = a.pair_shift[3 * p + 2];
            int64_t h, l;
            make_key(a.species[j], j, s0, s1, s2, h, l);
            int64_t q = p - 1;
            while (q >= o0) {
                int jq = a.pair_j[q];
                int64_t hq, lq;
                make_key(a.species[jq], jq, a.pair_shift[3 * q], a.pair_shift[3 * q + 1], a.pair_shift[3 * q + 2], hq, lq);
                if (!key_less(h, l, hq, lq)) break;
                a.pair_j[q + 1] = jq;
                for (int x = 0; x < 3; ++x) a.pair_shift[3 * (q + 1) + x] = a.pair_shift[3 * q + x];
                --q;
            }
            a.pair_j[q + 1] = j;
            a.pair_shift[3 * (q + 1)] = s0; a.pair_shift[3 * (q + 1) + 1] = s1; a.pair_shift[3 * (q + 1) + 2] = s2;
        }
    }
    __syncthreads();
    for (int p = t; p < n; p += 64) write_vec<F64>(a, i, o0 + p);
}

__global__ void k_transpose(NeighborArgs a)
{
    int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t P = a.pair_offsets[a.n_atoms];
    if (P > a.capacity || q >= P) return;
    // centre of pair q: last i with pair_offsets[i] <= q
    int64_t lo = 0, hi = a.n_atoms - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (a.pair_offsets[mid] <= q) lo = mid; else hi = mid - 1;
    }
    int64_t i = lo;
    int j = a.pair_j[q];
    int64_t th, tl;
    make_key(a.species[i], int(i), -a.pair_shift[3 * q], -a.pair_shift[3 * q + 1], -a.pair_shift[3 * q + 2], th, tl);
    int64_t b = a.pair_offsets[j], e = a.pair_offsets[j + 1];
    while (b < e) {   // first entry with key >= target
        int64_t mid = (b + e) >> 1;
        int jm = a.pair_j[mid];
        int64_t mh, ml;
        make_key(a.species[jm], jm, a.pair_shift[3 * mid], a.pair_shift[3 * mid + 1], a.pair_shift[3 * mid + 2], mh, ml);
        if (key_less(mh, ml, th, tl)) b = mid + 1; else e = mid;
    }
    bool found = false;
    if (b < a.pair_offsets[j + 1]) {
        int jb = a.pair_j[b];
        int64_t bh, bl;
        make_key(a.species[jb], jb, a.pair_shift[3 * b], a.pair_shift[3 * b + 1], a.pair_shift[3 * b + 2], bh, bl);
        found = (bh == th && bl == tl);
    }
    a.pair_transpose[q] = found ? int32_t(b) : -1;
    if (!found) put_status(a.status, SOAP_EGEOMETRY);
}

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

}  // namespace

hipError_t launch_neighbors(const NeighborArgs& a, hipStream_t stream)
{
    const int T = 256;
    int64_t N = a.n_atoms;
    hipLaunchKernelGGL(k_geometry, dim3(1), dim3(1024), 0, stream, a);
    if (N == 0) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan<int64_t, int64_t>), dim3(1), dim3(1024), 0, stream,
                           a.centre_count, a.pair_offsets, (int64_t*)nullptr, int64_t(0), a.capacity, a.status);
        return hipGetLastError();
    }
    int64_t B = a.max_bins;
    hipLaunchKernelGGL(k_zero_i32, dim3(blocks(B + 1, T)), dim3(T), 0, stream, a.bin_count, B + 1);
    hipLaunchKernelGGL(k_assign, dim3(blocks(N, T)), dim3(T), 0, stream, a);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan<int32_t, int32_t>), dim3(1), dim3(1024), 0, stream, a.bin_count,
                       a.bin_start, a.bin_cursor, B, int64_t(-1), a.status);
    hipLaunchKernelGGL(k_bins, dim3(blocks(N, T)), dim3(T), 0, stream, a);
    hipLaunchKernelGGL(k_count, dim3(blocks(N, T)), dim3(T), 0, stream, a);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan<int64_t, int64_t>), dim3(1), dim3(1024), 0, stream, a.centre_count,
                       a.pair_offsets, (int64_t*)nullptr, N, a.capacity, a.status);
    if (a.capacity > 0) {
        hipLaunchKernelGGL(k_fill, dim3(blocks(N, T)), dim3(T), 0, stream, a);
        if (a.vec_f64)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_sort<true>), dim3(unsigned(N)), dim3(64), 0, stream, a);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_sort<false>), dim3(unsigned(N)), dim3(64), 0, stream, a);
        if (a.pair_transpose)
            hipLaunchKernelGGL(k_transpose, dim3(blocks(a.capacity, T)), dim3(T), 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace soap
