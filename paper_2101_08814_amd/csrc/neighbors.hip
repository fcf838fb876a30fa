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
// Bin build: one work-group when the system has at most kSmallBins bins and
// kSmallAtoms atoms (occupancy counted in LDS), otherwise five small launches (geometry,
// clear, assign with integer atomics, scan, scatter).
// Pair list: one wave per centre.  The wave reads the sizes of its stencil
// bins in one round, scans them across lanes, and then tests 64 candidates
// per round; hits are compacted with a ballot.  A counting launch, a scan
// of the counts (pair_offsets), and a filling launch that ranks the
// centre's pairs by (species_j, j, s) in LDS and writes them sorted, with
// pair vectors formed in double from the positions.  Optionally the index
// of the reverse pair (j, i, -s).  The bin contents may be in any order; the
// sorted output does not depend on it, so the list is deterministic.
#include <type_traits>

#include "soap_internal.hpp"

namespace soap {
namespace {

constexpr int kSmallBins = 8192;   // single-work-group bin build up to this many bins
constexpr int kSmallAtoms = 8192;  // ... and this many atoms
constexpr int kPrefixAtoms = 2048; // fill kernel sums the counts itself up to this many atoms
constexpr int kSortCap = 512;      // sort records in LDS per fill work-group (shared by its waves)
constexpr int kFillWaves = 4;      // centres (one wave each) per fill work-group

__device__ __forceinline__ void put_status(int32_t* st, int v)
{
    if (st) *st = v;
}

__device__ __forceinline__ int floordiv(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// ------------------------------------------------------------- geometry
// Bins per periodic axis: floor(width / rcut), capped so that a structure
// never has more bins than atoms (the workspace then holds at most
// N + n_structures bins); the reach is the number of bins that spans rcut.
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
    const double idet = 1.0 / det;
    Hi[0] = (H[4] * H[8] - H[5] * H[7]) * idet;
    Hi[1] = (H[2] * H[7] - H[1] * H[8]) * idet;
    Hi[2] = (H[1] * H[5] - H[2] * H[4]) * idet;
    Hi[3] = (H[5] * H[6] - H[3] * H[8]) * idet;
    Hi[4] = (H[0] * H[8] - H[2] * H[6]) * idet;
    Hi[5] = (H[2] * H[3] - H[0] * H[5]) * idet;
    Hi[6] = (H[3] * H[7] - H[4] * H[6]) * idet;
    Hi[7] = (H[1] * H[6] - H[0] * H[7]) * idet;
    Hi[8] = (H[0] * H[4] - H[1] * H[3]) * idet;
    int cap = 1;
    while (int64_t(cap + 1) * (cap + 1) * (cap + 1) <= ns && cap < 128) ++cap;
    for (int k = 0; k < 3; ++k) {
        if (!g.pbc[k]) continue;
        double gk = sqrt(Hi[0 * 3 + k] * Hi[0 * 3 + k] + Hi[1 * 3 + k] * Hi[1 * 3 + k] + Hi[2 * 3 + k] * Hi[2 * 3 + k]);
        double width = 1.0 / gk;
        double nbf = floor(width / a.rcut);
        int nb = nbf < 1.0 ? 1 : (nbf > double(cap) ? cap : int(nbf));
        double need = ceil(a.rcut * nb / width * (1.0 + 1e-12));
        if (!(need <= 64.0)) return false;
        g.nbin[k] = nb;
        g.reach[k] = need < 1.0 ? 1 : int(need);
    }
    return valid;
}

// Exclusive prefix of v over the 1024 threads of a block (shuffle scan in
// each wave, then over the 16 wave totals); total receives the sum.
template <typename T>
__device__ T block_prefix(T v, T& total)
{
    __shared__ T wsum[17];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    T incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        T u = __shfl_up(incl, off, 64);
        if (lane >= off) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    if (t < 64) {
        T x = t < 16 ? wsum[t] : T(0), y = x;
        for (int off = 1; off < 16; off <<= 1) {
            T u = __shfl_up(y, off, 64);
            if (lane >= off) y += u;
        }
        if (t < 16) wsum[t] = y - x;
        if (t == 15) wsum[16] = y;
    }
    __syncthreads();
    const T r = wsum[wv] + incl - v;
    total = wsum[16];
    __syncthreads();   // wsum may be reused by the next call
    return r;
}

// Exclusive scan of n values by one block of 1024 threads (each owns a
// contiguous chunk); out[n] = total.  Returns the total in every thread.
// Chunks of up to kScanRegs values stay in registers between the two passes
// and all their loads are in flight together; longer chunks are read in
// batches of kScanBatch, twice.
constexpr int kScanRegs = 32;
constexpr int kScanBatch = 8;

template <typename Tin, typename Tout>
__device__ Tout block_scan(const Tin* in, Tout* out, Tout* out2, int64_t n)
{
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
    Tout total;
    if (chunk <= kScanRegs) {
        Tout v[kScanRegs];
        Tout s = 0;
#pragma unroll
        for (int u = 0; u < kScanRegs; ++u) v[u] = b + u < e ? Tout(in[b + u]) : Tout(0);
#pragma unroll
        for (int u = 0; u < kScanRegs; ++u) s += v[u];
        Tout run = block_prefix<Tout>(s, total);
#pragma unroll
        for (int u = 0; u < kScanRegs; ++u) {
            if (b + u < e) {
                out[b + u] = run;
                if (out2) out2[b + u] = run;
                run += v[u];
            }
        }
    } else {
        Tout s = 0;
        for (int64_t k0 = b; k0 < e; k0 += kScanBatch) {
            Tout v[kScanBatch];
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u) v[u] = k0 + u < e ? Tout(in[k0 + u]) : Tout(0);
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u) s += v[u];
        }
        Tout run = block_prefix<Tout>(s, total);
        for (int64_t k0 = b; k0 < e; k0 += kScanBatch) {
            Tout v[kScanBatch];
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u) v[u] = k0 + u < e ? Tout(in[k0 + u]) : Tout(0);
#pragma unroll
            for (int u = 0; u < kScanBatch; ++u) {
                if (k0 + u < e) {
                    out[k0 + u] = run;
                    if (out2) out2[k0 + u] = run;
                    run += v[u];
                }
            }
        }
    }
    if (t == 1023) out[n] = total;
    return total;
}

// Geometry of every structure (one block of 1024 threads).  Returns true in
// every thread when the input is valid; writes *a.ok.  The first cache_n
// structures are also written to the LDS array cache (bin_lo included).
__device__ bool geometry_block(const NeighborArgs& a, StructGeom* cache = nullptr, int cache_n = 0)
{
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    __syncthreads();
    const int64_t n = a.n_structures;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
    int64_t sum = 0;
    bool mine_bad = false;
    for (int64_t s = b; s < e; ++s) {
        StructGeom g;
        if (!make_geometry(a, int(s), g)) mine_bad = true;
        // the structures must tile the atoms from 0 to N
        if (s == 0 && g.atom_lo != 0) mine_bad = true;
        if (s == n - 1 && g.atom_hi != a.n_atoms) mine_bad = true;
        sum += int64_t(g.nbin[0]) * g.nbin[1] * g.nbin[2];
        if (s < cache_n) cache[s] = g;
        else a.geom[s] = g;
    }
    if (mine_bad) bad = 1;
    int64_t total;
    int64_t run = block_prefix<int64_t>(sum, total);
    for (int64_t s = b; s < e; ++s) {
        StructGeom* gp = s < cache_n ? &cache[s] : &a.geom[s];
        gp->bin_lo = run;
        run += int64_t(gp->nbin[0]) * gp->nbin[1] * gp->nbin[2];
        if (s < cache_n) a.geom[s] = *gp;
    }
    if (t == 0 && total > a.max_bins) bad = 1;
    __syncthreads();
    bool ok = bad == 0;
    if (t == 0) {
        *a.ok = ok ? 1 : 0;
        if (!ok) put_status(a.status, SOAP_EINVAL);
    }
    return ok;
}

// wrap t and bin of atom i (position r, species sp) in structure s with
// geometry g (written to the workspace), and its position wrapped into the
// cell, w = r - t.H
__device__ int32_t place_atom(const NeighborArgs& a, int64_t i, int s, const StructGeom& g, const double* r, int sp,
                              double4& w)
{
    int b[3], t[3];
    for (int k = 0; k < 3; ++k) {
        if (!g.pbc[k]) { b[k] = 0; t[k] = 0; continue; }
        double f = r[0] * g.Hinv[0 * 3 + k] + r[1] * g.Hinv[1 * 3 + k] + r[2] * g.Hinv[2 * 3 + k];
        double fl = floor(f);
        t[k] = int(fl);
        int bk = int((f - fl) * g.nbin[k]);
        b[k] = bk < 0 ? 0 : (bk >= g.nbin[k] ? g.nbin[k] - 1 : bk);
    }
    int32_t bin = int32_t(g.bin_lo + (int64_t(b[0]) * g.nbin[1] + b[1]) * g.nbin[2] + b[2]);
    a.atom_struct[i] = s;
    a.atom_bin[i] = bin;
    a.atom_wrap[3 * i + 0] = t[0];
    a.atom_wrap[3 * i + 1] = t[1];
    a.atom_wrap[3 * i + 2] = t[2];
    if (sp < 0 || sp >= a.n_species) put_status(a.status, SOAP_ESPECIES);
    w.x = r[0] - (t[0] * g.H[0] + t[1] * g.H[3] + t[2] * g.H[6]);
    w.y = r[1] - (t[0] * g.H[1] + t[1] * g.H[4] + t[2] * g.H[7]);
    w.z = r[2] - (t[0] * g.H[2] + t[1] * g.H[5] + t[2] * g.H[8]);
    w.w = __longlong_as_double((long long)i);
    return bin;
}

// structure of atom i: last s with atom_lo <= i (geom holds n structures)
__device__ __forceinline__ int structure_of(const StructGeom* geom, int n, int64_t i)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (geom[mid].atom_hi > i) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Whole bin build in one work-group (systems with at most kSmallBins bins
// and kSmallAtoms atoms: at most kAtomsPerLane atoms per lane).  The
// geometry of the first kGeomCache structures is kept in LDS, and each
// lane keeps the bin and wrapped position of its atoms in registers from
// the counting pass to the placing pass.
constexpr int kAtomsPerLane = kSmallAtoms / 1024;
constexpr int kGeomCache = 16;

__global__ void __launch_bounds__(1024) k_bins_small(NeighborArgs a)
{
    __shared__ int cnt[kSmallBins + 1];
    __shared__ StructGeom gc[kGeomCache];
    const int t = threadIdx.x;
    // the first atom of each lane is read before the geometry is built
    double r_first[3] = {0.0, 0.0, 0.0};
    int sp_first = 0;
    if (t < a.n_atoms) {
        r_first[0] = a.positions[3 * t];
        r_first[1] = a.positions[3 * t + 1];
        r_first[2] = a.positions[3 * t + 2];
        sp_first = a.species[t];
    }
    const int ns = a.n_structures;
    const bool cached = ns <= kGeomCache;
    if (!geometry_block(a, gc, cached ? ns : 0)) return;
    const int B = int(a.max_bins);
    for (int b = t; b <= B; b += 1024) cnt[b] = 0;
    __syncthreads();
    const StructGeom* geom = cached ? gc : a.geom;
    int bin_of[kAtomsPerLane];
    double4 w_of[kAtomsPerLane];
#pragma unroll
    for (int u = 0; u < kAtomsPerLane; ++u) {
        const int64_t i = t + 1024 * int64_t(u);
        if (i < a.n_atoms) {
            const int s = structure_of(geom, ns, i);
            if (u == 0) {
                bin_of[u] = place_atom(a, i, s, geom[s], r_first, sp_first, w_of[u]);
            } else {
                const double r[3] = {a.positions[3 * i], a.positions[3 * i + 1], a.positions[3 * i + 2]};
                bin_of[u] = place_atom(a, i, s, geom[s], r, a.species[i], w_of[u]);
            }
            atomicAdd(&cnt[bin_of[u]], 1);
        }
    }
    __syncthreads();
    // bin starts: each thread scans a contiguous chunk of bins in LDS
    const int chunk = (B + 1023) / 1024;
    const int b0 = t * chunk, b1 = b0 + chunk < B ? b0 + chunk : B;
    int sum = 0;
    for (int b = b0; b < b1; ++b) sum += cnt[b];
    int total;
    int run = block_prefix<int>(sum, total);
    for (int b = b0; b < b1; ++b) {
        const int v = cnt[b];
        cnt[b] = run;
        a.bin_start[b] = run;
        run += v;
    }
    if (t == 1023) a.bin_start[B] = total;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kAtomsPerLane; ++u) {
        const int64_t i = t + 1024 * int64_t(u);
        if (i < a.n_atoms) {
            const int pos = atomicAdd(&cnt[bin_of[u]], 1);
            a.bin_atoms[pos] = int32_t(i);
            a.slots[pos] = w_of[u];
        }
    }
}

__global__ void __launch_bounds__(1024) k_geometry(NeighborArgs a) { geometry_block(a); }

__global__ void k_zero_i32(int32_t* p, int64_t n)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Multi-work-group exclusive scan for long arrays: per-tile sums, a
// single-work-group scan of the sums (in place, total at the end), then
// each tile scanned again from its offset through LDS (coalesced loads and
// stores, each lane scanning a contiguous run of kTileRun values).
constexpr int kTileRun = 16;
constexpr int kScanTile = 256 * kTileRun;
constexpr int64_t kMultiScan = 16384;   // arrays longer than this use the multi-work-group scan

template <typename Tout>
__device__ __forceinline__ Tout block256_excl(Tout v, Tout& total)
{
    __shared__ Tout wsum[5];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    Tout incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        Tout u = __shfl_up(incl, off, 64);
        if (lane >= off) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    if (t == 0) {
        Tout r = 0;
        for (int k = 0; k < 4; ++k) { const Tout x = wsum[k]; wsum[k] = r; r += x; }
        wsum[4] = r;
    }
    __syncthreads();
    total = wsum[4];
    return wsum[wv] + incl - v;
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(256) k_tile_sums(const Tin* in, Tout* sums, int64_t n)
{
    const int64_t t0 = int64_t(blockIdx.x) * kScanTile + threadIdx.x;
    Tout v[kTileRun];
#pragma unroll
    for (int u = 0; u < kTileRun; ++u) v[u] = t0 + 256 * u < n ? Tout(in[t0 + 256 * u]) : Tout(0);
    Tout s = 0;
#pragma unroll
    for (int u = 0; u < kTileRun; ++u) s += v[u];
    Tout total;
    block256_excl<Tout>(s, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(256) k_tile_scan(const Tin* in, Tout* out, Tout* out2, const Tout* offs,
                                                   int64_t n, int64_t n_tiles)
{
    __shared__ Tout tile[kScanTile];
    const int t = threadIdx.x;
    const int64_t base = int64_t(blockIdx.x) * kScanTile;
    Tout v[kTileRun];
#pragma unroll
    for (int u = 0; u < kTileRun; ++u) v[u] = base + t + 256 * u < n ? Tout(in[base + t + 256 * u]) : Tout(0);
#pragma unroll
    for (int u = 0; u < kTileRun; ++u) tile[t + 256 * u] = v[u];
    __syncthreads();
    Tout run[kTileRun];
    Tout s = 0;
#pragma unroll
    for (int u = 0; u < kTileRun; ++u) { run[u] = tile[t * kTileRun + u]; s += run[u]; }
    Tout total;
    Tout r = offs[blockIdx.x] + block256_excl<Tout>(s, total);
#pragma unroll
    for (int u = 0; u < kTileRun; ++u) { const Tout x = run[u]; tile[t * kTileRun + u] = r; r += x; }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kTileRun; ++u) {
        const int64_t k = base + t + 256 * u;
        if (k < n) {
            out[k] = tile[t + 256 * u];
            if (out2) out2[k] = tile[t + 256 * u];
        }
    }
    if (blockIdx.x == 0 && t == 0) out[n] = offs[n_tiles];
}

// Large systems, one lane per atom: structure (binary search over the atom
// offsets, kept in LDS for up to kOffsetCache structures), bin, wrap and
// wrapped position (kept for the placing pass), bin occupancy by atomics.
constexpr int kOffsetCache = 2048;

// atomicAdd(&ctr[key], 1) for every active lane of the wave, returning the
// old value, with the lanes that share a key combined into one atomic (a
// molecule's atoms all land in one bin, so plain per-lane atomics on the
// same counter serialise); up to kAggRounds distinct keys per wave this
// way, the rest one atomic per lane.  Lanes of one key take consecutive
// values in lane order.
constexpr int kAggRounds = 4;

__device__ __forceinline__ int wave_counter_inc(int* ctr, int key)
{
    const int lane = threadIdx.x & 63;
    bool pending = true;
    int result = 0;
    for (int round = 0; round < kAggRounds; ++round) {
        const uint64_t pend = __ballot(pending);
        if (pend == 0) break;
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const int lkey = __shfl(key, leader, 64);
        const bool mine = pending && key == lkey;
        const uint64_t m = __ballot(mine);
        int base = 0;
        if (lane == leader) base = atomicAdd(&ctr[lkey], int(__popcll(m)));
        base = __shfl(base, leader, 64);
        if (mine) {
            result = base + int(__popcll(m & ((uint64_t(1) << lane) - 1)));
            pending = false;
        }
    }
    if (pending) result = atomicAdd(&ctr[key], 1);
    return result;
}

__global__ void __launch_bounds__(256) k_assign(NeighborArgs a)
{
    __shared__ int64_t offs[kOffsetCache + 1];
    const int ns = a.n_structures;
    const bool cached = ns <= kOffsetCache;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool in = i < a.n_atoms;
    // position and species first: they do not depend on the structure
    double r[3] = {0.0, 0.0, 0.0};
    int sp = 0;
    if (in) {
        r[0] = a.positions[3 * i];
        r[1] = a.positions[3 * i + 1];
        r[2] = a.positions[3 * i + 2];
        sp = a.species[i];
    }
    const int ok = *a.ok;
    if (cached) {
        for (int k0 = threadIdx.x; k0 <= ns; k0 += 8 * 256) {
            int64_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = k0 + u * 256 <= ns ? a.atom_offsets[k0 + u * 256] : 0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u * 256 <= ns) offs[k0 + u * 256] = v[u];
        }
    }
    __syncthreads();
    if (!in || !ok) return;
    int s;
    if (cached) {
        // first k in [1, ns] with offs[k] > i; the structures tile [0, N) (checked by the geometry pass)
        int lo = 1, hi = ns;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (offs[mid] > i) hi = mid; else lo = mid + 1;
        }
        s = lo - 1;
    } else {
        s = structure_of(a.geom, ns, i);
    }
    double4 w;
    const int32_t bin = place_atom(a, i, s, a.geom[s], r, sp, w);
    a.wrapped[i] = w;
    wave_counter_inc(a.bin_count, bin);
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(1024) k_scan(const Tin* in, Tout* out, Tout* out2, int64_t n, int64_t capacity,
                                               int32_t* status)
{
    Tout total = block_scan<Tin, Tout>(in, out, out2, n);
    if (threadIdx.x == 0 && capacity >= 0 && int64_t(total) > capacity) put_status(status, SOAP_ECAPACITY);
}

__global__ void k_bins(NeighborArgs a)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_atoms || !*a.ok) return;
    const double4 w = a.wrapped[i];
    int pos = wave_counter_inc(a.bin_cursor, a.atom_bin[i]);
    a.bin_atoms[pos] = int32_t(i);
    a.slots[pos] = w;
}

// ------------------------------------------------------- pair enumeration
struct WaveScratch {
    int prefix[65];     // exclusive prefix of the stencil-bin sizes of this round
    int start[64];      // first slot in bin_atoms of each stencil bin
    int cshift[64];     // cell shift of each stencil bin, 3 x 10 bits
};

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// All candidates of centre i, 64 per round, kRounds rounds at a time with
// their slot loads issued together: emit(hit, j, c0, c1, c2, v) is called
// by every lane for every round (hit false for lanes with nothing), with
// the cell shift c of the stencil bin the candidate was found in and, for a
// hit, the pair vector v = (w_j - w_i) + c.H (= r_j - r_i + s.H for the
// image shift s = c + t_i - t_j).
constexpr int kRounds = 4;

// Centre i as the enumeration sees it, loaded before the validity flag is
// looked at: every address read here is in bounds whatever the flag says
// (with one structure the geometry is structure 0; otherwise it is read
// only once the flag is known), so the loads go out together.
struct Centre {
    int ok;
    int32_t bin;
    double4 wi;          // position wrapped into the cell, w = r - t.H
    int t[3];            // integer wrap
    const StructGeom* g;
};

template <bool ONE>
__device__ __forceinline__ Centre load_centre(const NeighborArgs& a, int64_t i)
{
    Centre c;
    c.ok = *a.ok;
    const int32_t s = ONE ? 0 : a.atom_struct[i];
    c.bin = a.atom_bin[i];
    for (int k = 0; k < 3; ++k) c.t[k] = a.atom_wrap[3 * i + k];
    const double r0 = a.positions[3 * i], r1 = a.positions[3 * i + 1], r2 = a.positions[3 * i + 2];
    c.g = a.geom + (ONE ? 0 : (c.ok ? s : 0));
    const StructGeom& g = *c.g;
    c.wi.x = r0 - (c.t[0] * g.H[0] + c.t[1] * g.H[3] + c.t[2] * g.H[6]);
    c.wi.y = r1 - (c.t[0] * g.H[1] + c.t[1] * g.H[4] + c.t[2] * g.H[7]);
    c.wi.z = r2 - (c.t[0] * g.H[2] + c.t[1] * g.H[5] + c.t[2] * g.H[8]);
    c.wi.w = __longlong_as_double((long long)i);
    return c;
}

template <class F>
__device__ void wave_visit(const NeighborArgs& a, int64_t i, const Centre& ce, WaveScratch& w, F&& emit)
{
    const int lane = threadIdx.x & 63;
    const StructGeom& g = *ce.g;
    const int local = ce.bin - int32_t(g.bin_lo);
    const int bz = local % g.nbin[2];
    const int by = (local / g.nbin[2]) % g.nbin[1];
    const int bx = local / (g.nbin[2] * g.nbin[1]);
    const double4 wi = ce.wi;
    const double rc2 = a.rcut * a.rcut;
    const int n0 = 2 * g.reach[0] + 1, n1 = 2 * g.reach[1] + 1, n2 = 2 * g.reach[2] + 1;
    const int nst = ce.ok ? n0 * n1 * n2 : 0;   // nothing is visited on invalid input
    for (int base = 0; base < nst; base += 64) {
        int sb = base + lane;
        int size = 0, start = 0, cs = 0;
        if (sb < nst) {
            int d2 = sb % n2 - g.reach[2], d1 = (sb / n2) % n1 - g.reach[1], d0 = sb / (n1 * n2) - g.reach[0];
            int u0 = bx + d0, u1 = by + d1, u2 = bz + d2;
            int c0 = floordiv(u0, g.nbin[0]), c1 = floordiv(u1, g.nbin[1]), c2 = floordiv(u2, g.nbin[2]);
            int64_t bin = g.bin_lo + (int64_t(u0 - c0 * g.nbin[0]) * g.nbin[1] + (u1 - c1 * g.nbin[1])) * g.nbin[2] +
                          (u2 - c2 * g.nbin[2]);
            start = a.bin_start[bin];
            size = a.bin_start[bin + 1] - start;
            cs = ((c0 + 512) & 1023) | (((c1 + 512) & 1023) << 10) | (((c2 + 512) & 1023) << 20);
        }
        int incl = wave_incl_scan(size);
        w.prefix[lane] = incl - size;
        w.start[lane] = start;
        w.cshift[lane] = cs;
        const int total = __shfl(incl, 63, 64);
        wave_fence();
        const int nb = nst - base < 64 ? nst - base : 64;
        for (int t0 = 0; t0 < total; t0 += 64 * kRounds) {
            double4 rec[kRounds];
            int bin_of[kRounds];
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
                const int t = t0 + 64 * r + lane;
                const int tt = t < total ? t : 0;    // total > 0: slot of candidate 0 is valid
                // last stencil bin whose prefix is <= tt
                int lo = 0, hi = nb - 1;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (w.prefix[mid] <= tt) lo = mid; else hi = mid - 1;
                }
                bin_of[r] = lo;
                rec[r] = a.slots[w.start[lo] + (tt - w.prefix[lo])];
            }
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
                const int t = t0 + 64 * r + lane;
                bool hit = false;
                int j = 0, c0 = 0, c1 = 0, c2 = 0;
                double vx = 0.0, vy = 0.0, vz = 0.0;
                if (t < total) {
                    j = int(__double_as_longlong(rec[r].w));
                    const int cs2 = w.cshift[bin_of[r]];
                    c0 = (cs2 & 1023) - 512;
                    c1 = ((cs2 >> 10) & 1023) - 512;
                    c2 = ((cs2 >> 20) & 1023) - 512;
                    if (!(j == i && c0 == 0 && c1 == 0 && c2 == 0)) {
                        vx = (rec[r].x - wi.x) + c0 * g.H[0] + c1 * g.H[3] + c2 * g.H[6];
                        vy = (rec[r].y - wi.y) + c0 * g.H[1] + c1 * g.H[4] + c2 * g.H[7];
                        vz = (rec[r].z - wi.z) + c0 * g.H[2] + c1 * g.H[5] + c2 * g.H[8];
                        double r2 = vx * vx + vy * vy + vz * vz;
                        if (r2 < rc2) {
                            if (r2 == 0.0) put_status(a.status, SOAP_EGEOMETRY);
                            else hit = true;
                        }
                    }
                }
                emit(hit, j, c0, c1, c2, vx, vy, vz);
            }
        }
        wave_fence();
    }
}

// one wave (block of 64) per centre
template <bool ONE>
__global__ void __launch_bounds__(64) k_count(NeighborArgs a)
{
    __shared__ WaveScratch w;
    const int64_t i = blockIdx.x;
    const Centre ce = load_centre<ONE>(a, i);
    int n = 0;
    wave_visit(a, i, ce, w, [&](bool hit, int, int, int, int, double, double, double) { n += hit ? 1 : 0; });
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
    if (threadIdx.x == 0) a.centre_count[i] = n;
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

template <bool F64>
__device__ __forceinline__ void write_pair(const NeighborArgs& a, const StructGeom& g, int64_t i, int64_t q, int j,
                                           int s0, int s1, int s2)
{
    a.pair_j[q] = j;
    a.pair_shift[3 * q] = s0;
    a.pair_shift[3 * q + 1] = s1;
    a.pair_shift[3 * q + 2] = s2;
    for (int x = 0; x < 3; ++x) {
        double v = (a.positions[3 * j + x] - a.positions[3 * i + x]) + s0 * g.H[0 * 3 + x] + s1 * g.H[1 * 3 + x] +
                   s2 * g.H[2 * 3 + x];
        if (F64) static_cast<double*>(a.pair_vec)[3 * q + x] = v;
        else static_cast<float*>(a.pair_vec)[3 * q + x] = float(v);
    }
}

// image shift of a candidate j of centre i (wrap ti) seen with cell shift c
__device__ __forceinline__ void image_shift(const NeighborArgs& a, const StructGeom& g, const int* ti, int j, int c0,
                                            int c1, int c2, int& s0, int& s1, int& s2)
{
    s0 = g.pbc[0] ? c0 + ti[0] - a.atom_wrap[3 * j] : 0;
    s1 = g.pbc[1] ? c1 + ti[1] - a.atom_wrap[3 * j + 1] : 0;
    s2 = g.pbc[2] ? c2 + ti[2] - a.atom_wrap[3 * j + 2] : 0;
}

// Small systems: one wave per work-group and per centre, with its own
// kSortCap sort records (the few work-groups spread over every CU); this
// form measured faster than k_fill below at one wave per work-group.
// Enumerate again (hits compacted in LDS with their pair vectors), form the
// image shifts and sort keys of all hits at once, rank them by key in LDS
// and write them sorted.  With PREFIX the wave also sums the counts before
// its centre and all counts itself and writes its pair_offsets entry, in
// place of a separate scan.
template <bool ONE, bool F64, bool PREFIX>
__global__ void __launch_bounds__(64) k_fill1(NeighborArgs a)
{
    using VT = typename std::conditional<F64, double, float>::type;
    __shared__ WaveScratch w;
    __shared__ int64_t khi[kSortCap], klo[kSortCap];
    __shared__ int32_t kj[kSortCap], ks[3 * kSortCap];
    __shared__ VT kv[3 * kSortCap];
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    int64_t total, o0;
    int n;
    if (PREFIX) {
        // all loads in flight at once (N <= kPrefixAtoms)
        constexpr int R = kPrefixAtoms / 64;
        int64_t c[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t k = lane + 64 * r;
            c[r] = k < a.n_atoms ? a.centre_count[k] : 0;
        }
        n = int(a.centre_count[i]);
        int64_t before = 0, all = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            all += c[r];
            before += lane + 64 * r < i ? c[r] : 0;
        }
        for (int off = 32; off > 0; off >>= 1) {
            before += __shfl_xor(before, off, 64);
            all += __shfl_xor(all, off, 64);
        }
        o0 = before;
        total = all;
        if (lane == 0) {
            a.pair_offsets[i] = o0;
            if (i == a.n_atoms - 1) {
                a.pair_offsets[a.n_atoms] = total;
                if (total > a.capacity) put_status(a.status, SOAP_ECAPACITY);
            }
        }
    } else {
        total = a.pair_offsets[a.n_atoms];
        o0 = a.pair_offsets[i];
        n = int(a.pair_offsets[i + 1] - o0);
    }
    const Centre ce = load_centre<ONE>(a, i);
    if (!ce.ok || total > a.capacity) return;
    const bool in_lds = n <= kSortCap;
    const StructGeom& g = *ce.g;
    int count = 0;
    wave_visit(a, i, ce, w, [&](bool hit, int j, int c0, int c1, int c2, double vx, double vy, double vz) {
        uint64_t mask = __ballot(hit);
        int idx = count + __popcll(mask & ((uint64_t(1) << lane) - 1));
        if (hit && idx < n) {
            if (in_lds) {
                kj[idx] = j;
                ks[3 * idx] = c0; ks[3 * idx + 1] = c1; ks[3 * idx + 2] = c2;
                kv[3 * idx] = VT(vx); kv[3 * idx + 1] = VT(vy); kv[3 * idx + 2] = VT(vz);
            } else {
                int s0, s1, s2;
                image_shift(a, g, ce.t, j, c0, c1, c2, s0, s1, s2);
                a.pair_j[o0 + idx] = j;
                a.pair_shift[3 * (o0 + idx)] = s0;
                a.pair_shift[3 * (o0 + idx) + 1] = s1;
                a.pair_shift[3 * (o0 + idx) + 2] = s2;
            }
        }
        count += __popcll(mask);
    });
    __syncthreads();
    if (in_lds) {
        for (int p = lane; p < n; p += 64) {
            const int j = kj[p];
            int s0, s1, s2;
            image_shift(a, g, ce.t, j, ks[3 * p], ks[3 * p + 1], ks[3 * p + 2], s0, s1, s2);
            ks[3 * p] = s0; ks[3 * p + 1] = s1; ks[3 * p + 2] = s2;
            make_key(a.species[j], j, s0, s1, s2, khi[p], klo[p]);
        }
        __syncthreads();
        VT* vec = static_cast<VT*>(a.pair_vec);
        for (int p = lane; p < n; p += 64) {
            int64_t h = khi[p], l = klo[p];
            int rank = 0;
            for (int q = 0; q < n; ++q) rank += key_less(khi[q], klo[q], h, l) ? 1 : 0;
            const int64_t q = o0 + rank;
            a.pair_j[q] = kj[p];
            a.pair_shift[3 * q] = ks[3 * p];
            a.pair_shift[3 * q + 1] = ks[3 * p + 1];
            a.pair_shift[3 * q + 2] = ks[3 * p + 2];
            vec[3 * q] = kv[3 * p];
            vec[3 * q + 1] = kv[3 * p + 1];
            vec[3 * q + 2] = kv[3 * p + 2];
        }
        return;
    }
    // long environments: insertion sort in place in global memory
    if (lane == 0) {
        for (int64_t p = o0 + 1; p < o0 + n; ++p) {
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
    for (int p = lane; p < n; p += 64) {
        int64_t q = o0 + p;
        write_pair<F64>(a, g, i, q, a.pair_j[q], a.pair_shift[3 * q], a.pair_shift[3 * q + 1], a.pair_shift[3 * q + 2]);
    }
}

// ------------------------------------------------- small systems, all pairs
// Systems of at most kBruteAtoms atoms in at most 64 structures of on
// average at most kBrutePerStruct atoms: no bins.
// A wave per centre checks the input itself (lane l builds the geometry of
// structure l: the same checks as the bin build) and tests every atom j of
// the centre's structure.  With f = (r_j - r_i) . Hinv the fractional
// difference and w_k the width of the cell across lattice direction k, an
// image s within rcut has |f_k + s_k| <= rcut / w_k, so only the s in that
// box (one image when every width is at least 2 rcut) are tried, in
// lexicographic order; the hit test is |r_j - r_i + s.H|^2 < rcut^2 in
// double, as in the binned enumeration.  Counting and filling are two
// launches; the fill ranks a centre's pairs by (species_j, j, s) in LDS,
// as k_fill1 does, and forms the offsets from the counts itself.
constexpr int kBruteAtoms = 2048;
constexpr int kBruteStructs = 64;
constexpr int kBrutePerStruct = 256;
constexpr int kBruteSortCap = 128;   // sort records per fill wave (more: sorted in global memory)
constexpr int kBruteBatch = 4;   // rounds of 64 candidates whose positions are loaded together

struct BruteCentre {
    bool ok;          // the whole input is valid
    int64_t lo, hi;   // atoms of the centre's structure
    double ri[3];
    double e[3];      // rcut / width per periodic axis (with a margin), 0 otherwise
};

// Validity of the input and the centre's structure geometry (in gs).
// GEOM: from the geometry phase (a.geom, a.ok; the structure found by a
// binary search over the structures' ends, the same address in every
// lane); otherwise built by the wave (at most 64 structures).
template <bool GEOM>
__device__ BruteCentre brute_centre(const NeighborArgs& a, int64_t i, StructGeom& gs)
{
    const int lane = threadIdx.x & 63;
    const int ns = a.n_structures;
    BruteCentre c;
    int s;
    if constexpr (GEOM) {
        c.ok = *a.ok != 0;
        int lo = 0, hi = ns - 1;   // first structure ending after i (the offsets are contiguous and cached)
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a.atom_offsets[mid + 1] > i) hi = mid; else lo = mid + 1;
        }
        s = lo;
        if (lane == 0) gs = a.geom[s];
    } else {
        StructGeom g;
        bool bad = false;
        if (lane < ns) {
            bad = !make_geometry(a, lane, g);
            if (lane == 0 && g.atom_lo != 0) bad = true;
            if (lane == ns - 1 && g.atom_hi != a.n_atoms) bad = true;
        }
        c.ok = __ballot(bad) == 0;
        // structure of i: the structures before it end at or before i
        s = __popcll(__ballot(lane < ns && g.atom_hi <= i));
        if (lane == s && s < ns) gs = g;
    }
    wave_fence();
    c.lo = gs.atom_lo;
    c.hi = gs.atom_hi;
    if (s >= ns || !(c.lo <= i && i < c.hi)) c.ok = false;
    for (int k = 0; k < 3; ++k) {
        c.ri[k] = a.positions[3 * i + k];
        const double bk = sqrt(gs.Hinv[0 * 3 + k] * gs.Hinv[0 * 3 + k] + gs.Hinv[1 * 3 + k] * gs.Hinv[1 * 3 + k] +
                               gs.Hinv[2 * 3 + k] * gs.Hinv[2 * 3 + k]);
        c.e[k] = gs.pbc[k] ? a.rcut * bk * (1.0 + 1e-9) + 1e-12 : 0.0;
    }
    return c;
}

// every candidate j of centre i, kBruteBatch rounds of 64 at a time:
// emit(hit, j, s0, s1, s2, vx, vy, vz) by every lane for every image step
template <class F>
__device__ void brute_visit(const NeighborArgs& a, int64_t i, const BruteCentre& c, const StructGeom& g, F&& emit)
{
    const int lane = threadIdx.x & 63;
    const double rc2 = a.rcut * a.rcut;
    const int64_t lo = c.ok ? c.lo : 0, hi = c.ok ? c.hi : 0;
    for (int64_t j0 = lo; j0 < hi; j0 += 64 * kBruteBatch) {
        double rj[kBruteBatch][3];
#pragma unroll
        for (int r = 0; r < kBruteBatch; ++r) {
            const int64_t j = j0 + 64 * r + lane;
            const int64_t jj = j < hi ? j : lo;
            for (int k = 0; k < 3; ++k) rj[r][k] = a.positions[3 * jj + k];
        }
#pragma unroll
        for (int r = 0; r < kBruteBatch; ++r) {
            const int64_t j = j0 + 64 * r + lane;
            if (__ballot(j < hi) == 0) break;
            const double d0 = rj[r][0] - c.ri[0], d1 = rj[r][1] - c.ri[1], d2 = rj[r][2] - c.ri[2];
            // box of shifts: s_k in [ceil(-f_k - e_k), floor(-f_k + e_k)]
            int smin[3], cnt[3];
            int n_img = j < hi ? 1 : 0;
            for (int k = 0; k < 3; ++k) {
                smin[k] = 0;
                cnt[k] = 1;
                if (g.pbc[k]) {
                    const double f = d0 * g.Hinv[0 * 3 + k] + d1 * g.Hinv[1 * 3 + k] + d2 * g.Hinv[2 * 3 + k];
                    const int a0 = int(ceil(-f - c.e[k])), a1 = int(floor(-f + c.e[k]));
                    smin[k] = a0;
                    cnt[k] = a1 >= a0 ? a1 - a0 + 1 : 0;
                }
                n_img *= cnt[k];
            }
            int n_max = n_img;
            for (int off = 32; off > 0; off >>= 1) n_max = max(n_max, __shfl_xor(n_max, off, 64));
            for (int t = 0; t < n_max; ++t) {
                bool hit = false;
                int s0 = 0, s1 = 0, s2 = 0;
                double vx = 0.0, vy = 0.0, vz = 0.0;
                if (t < n_img) {
                    s2 = smin[2] + t % cnt[2];
                    s1 = smin[1] + (t / cnt[2]) % cnt[1];
                    s0 = smin[0] + t / (cnt[2] * cnt[1]);
                    if (!(j == i && s0 == 0 && s1 == 0 && s2 == 0)) {
                        vx = d0 + s0 * g.H[0] + s1 * g.H[3] + s2 * g.H[6];
                        vy = d1 + s0 * g.H[1] + s1 * g.H[4] + s2 * g.H[7];
                        vz = d2 + s0 * g.H[2] + s1 * g.H[5] + s2 * g.H[8];
                        const double r2 = vx * vx + vy * vy + vz * vz;
                        if (r2 < rc2) {
                            if (r2 == 0.0) put_status(a.status, SOAP_EGEOMETRY);
                            else hit = true;
                        }
                    }
                }
                emit(hit, int(j), s0, s1, s2, vx, vy, vz);
            }
        }
    }
}

template <bool GEOM>
__global__ void __launch_bounds__(64) k_count_bf(NeighborArgs a)
{
    __shared__ StructGeom gs;
    const int64_t i = blockIdx.x;
    const BruteCentre c = brute_centre<GEOM>(a, i, gs);
    if (threadIdx.x == 0) {
        if (!c.ok) put_status(a.status, SOAP_EINVAL);
        const int sp = a.species[i];
        if (sp < 0 || sp >= a.n_species) put_status(a.status, SOAP_ESPECIES);
    }
    int n = 0;
    brute_visit(a, i, c, gs, [&](bool hit, int, int, int, int, double, double, double) { n += hit ? 1 : 0; });
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
    if (threadIdx.x == 0) a.centre_count[i] = n;
}

// Offsets from all counts (without GEOM: N <= kBruteAtoms) or from the
// scan (GEOM); the centre's pairs ranked by key in LDS and written sorted.
template <bool GEOM, bool F64>
__global__ void __launch_bounds__(64) k_fill_bf(NeighborArgs a)
{
    using VT = typename std::conditional<F64, double, float>::type;
    __shared__ StructGeom gs;
    __shared__ int64_t khi[kBruteSortCap], klo[kBruteSortCap];
    __shared__ int32_t kj[kBruteSortCap], ks[3 * kBruteSortCap];
    __shared__ VT kv[3 * kBruteSortCap];
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    int64_t o0, total;
    int n;
    if constexpr (GEOM) {
        o0 = a.pair_offsets[i];
        n = int(a.pair_offsets[i + 1] - o0);
        total = a.pair_offsets[a.n_atoms];
    } else {
        constexpr int R = kBruteAtoms / 64;
        int64_t cv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t k = lane + 64 * r;
            cv[r] = k < a.n_atoms ? a.centre_count[k] : 0;
        }
        n = int(a.centre_count[i]);
        int64_t before = 0, all = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            all += cv[r];
            before += lane + 64 * r < i ? cv[r] : 0;
        }
        for (int off = 32; off > 0; off >>= 1) {
            before += __shfl_xor(before, off, 64);
            all += __shfl_xor(all, off, 64);
        }
        o0 = before;
        total = all;
        if (lane == 0) {
            a.pair_offsets[i] = o0;
            if (i == a.n_atoms - 1) {
                a.pair_offsets[a.n_atoms] = total;
                if (total > a.capacity) put_status(a.status, SOAP_ECAPACITY);
            }
        }
    }
    if (total > a.capacity || n == 0) return;
    const BruteCentre c = brute_centre<GEOM>(a, i, gs);
    const bool in_lds = n <= kBruteSortCap;
    int count = 0;
    brute_visit(a, i, c, gs, [&](bool hit, int j, int s0, int s1, int s2, double vx, double vy, double vz) {
        const uint64_t mask = __ballot(hit);
        const int idx = count + __popcll(mask & ((uint64_t(1) << lane) - 1));
        if (hit && idx < n) {
            if (in_lds) {
                kj[idx] = j;
                ks[3 * idx] = s0; ks[3 * idx + 1] = s1; ks[3 * idx + 2] = s2;
                kv[3 * idx] = VT(vx); kv[3 * idx + 1] = VT(vy); kv[3 * idx + 2] = VT(vz);
            } else {
                a.pair_j[o0 + idx] = j;
                a.pair_shift[3 * (o0 + idx)] = s0;
                a.pair_shift[3 * (o0 + idx) + 1] = s1;
                a.pair_shift[3 * (o0 + idx) + 2] = s2;
            }
        }
        count += __popcll(mask);
    });
    __syncthreads();
    if (in_lds) {
        for (int p = lane; p < n; p += 64) make_key(a.species[kj[p]], kj[p], ks[3 * p], ks[3 * p + 1], ks[3 * p + 2],
                                                    khi[p], klo[p]);
        __syncthreads();
        VT* vec = static_cast<VT*>(a.pair_vec);
        for (int p = lane; p < n; p += 64) {
            const int64_t h = khi[p], l = klo[p];
            int rank = 0;
            for (int q = 0; q < n; ++q) rank += key_less(khi[q], klo[q], h, l) ? 1 : 0;
            const int64_t q = o0 + rank;
            a.pair_j[q] = kj[p];
            a.pair_shift[3 * q] = ks[3 * p];
            a.pair_shift[3 * q + 1] = ks[3 * p + 1];
            a.pair_shift[3 * q + 2] = ks[3 * p + 2];
            vec[3 * q] = kv[3 * p];
            vec[3 * q + 1] = kv[3 * p + 1];
            vec[3 * q + 2] = kv[3 * p + 2];
        }
        return;
    }
    // long environments: insertion sort in place in global memory
    if (lane == 0) {
        for (int64_t p = o0 + 1; p < o0 + n; ++p) {
            const int j = a.pair_j[p];
            const int s0 = a.pair_shift[3 * p], s1 = a.pair_shift[3 * p + 1], s2 = a.pair_shift[3 * p + 2];
            int64_t h, l;
            make_key(a.species[j], j, s0, s1, s2, h, l);
            int64_t q = p - 1;
            while (q >= o0) {
                const int jq = a.pair_j[q];
                int64_t hq, lq;
                make_key(a.species[jq], jq, a.pair_shift[3 * q], a.pair_shift[3 * q + 1], a.pair_shift[3 * q + 2], hq,
                         lq);
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
    for (int p = lane; p < n; p += 64) {
        const int64_t q = o0 + p;
        write_pair<F64>(a, gs, i, q, a.pair_j[q], a.pair_shift[3 * q], a.pair_shift[3 * q + 1], a.pair_shift[3 * q + 2]);
    }
}

// Large systems: kFillWaves centres per work-group (one wave each) that
// draw their sort records from one pool of kSortCap, so that four times as
// many centres are resident as with a pool per wave; a centre whose records
// do not fit sorts in global memory.  Otherwise as k_fill1 (offsets from
// the scan).
template <bool ONE, bool F64>
__global__ void __launch_bounds__(kFillWaves * 64) k_fill(NeighborArgs a)
{
    using VT = typename std::conditional<F64, double, float>::type;
    constexpr int W = kFillWaves;
    __shared__ WaveScratch ws[W];
    // sort records of the work-group's waves, taken from one pool
    __shared__ int64_t khi[kSortCap], klo[kSortCap];
    __shared__ int32_t kj[kSortCap], ks[3 * kSortCap];
    __shared__ VT kv[3 * kSortCap];
    __shared__ int pool_used;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) pool_used = 0;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * W + wave;
    if (i >= a.n_atoms) return;
    WaveScratch& w = ws[wave];
    const int64_t total = a.pair_offsets[a.n_atoms];
    const int64_t o0 = a.pair_offsets[i];
    const int n = int(a.pair_offsets[i + 1] - o0);
    const Centre ce = load_centre<ONE>(a, i);
    if (!ce.ok || total > a.capacity) return;
    // reserve n records of the pool (else sort in global memory)
    int base = -1;
    if (lane == 0) {
        int cur = pool_used;
        while (cur + n <= kSortCap) {
            const int prev = atomicCAS(&pool_used, cur, cur + n);
            if (prev == cur) { base = cur; break; }
            cur = prev;
        }
    }
    base = __shfl(base, 0, 64);
    const bool in_lds = base >= 0;
    const int off = in_lds ? base : 0;
    int64_t* const hh = khi + off;
    int64_t* const hl = klo + off;
    int32_t* const jj = kj + off;
    int32_t* const ss = ks + 3 * off;
    VT* const vv = kv + 3 * off;
    const StructGeom& g = *ce.g;
    int count = 0;
    wave_visit(a, i, ce, w, [&](bool hit, int j, int c0, int c1, int c2, double vx, double vy, double vz) {
        uint64_t mask = __ballot(hit);
        int idx = count + __popcll(mask & ((uint64_t(1) << lane) - 1));
        if (hit && idx < n) {
            if (in_lds) {
                jj[idx] = j;
                ss[3 * idx] = c0; ss[3 * idx + 1] = c1; ss[3 * idx + 2] = c2;
                vv[3 * idx] = VT(vx); vv[3 * idx + 1] = VT(vy); vv[3 * idx + 2] = VT(vz);
            } else {
                int s0, s1, s2;
                image_shift(a, g, ce.t, j, c0, c1, c2, s0, s1, s2);
                a.pair_j[o0 + idx] = j;
                a.pair_shift[3 * (o0 + idx)] = s0;
                a.pair_shift[3 * (o0 + idx) + 1] = s1;
                a.pair_shift[3 * (o0 + idx) + 2] = s2;
            }
        }
        count += __popcll(mask);
    });
    wave_fence();
    if (in_lds) {
        for (int p = lane; p < n; p += 64) {
            const int j = jj[p];
            int s0, s1, s2;
            image_shift(a, g, ce.t, j, ss[3 * p], ss[3 * p + 1], ss[3 * p + 2], s0, s1, s2);
            ss[3 * p] = s0; ss[3 * p + 1] = s1; ss[3 * p + 2] = s2;
            make_key(a.species[j], j, s0, s1, s2, hh[p], hl[p]);
        }
        wave_fence();
        VT* vec = static_cast<VT*>(a.pair_vec);
        for (int p = lane; p < n; p += 64) {
            int64_t h = hh[p], l = hl[p];
            int rank = 0;
            for (int q = 0; q < n; ++q) rank += key_less(hh[q], hl[q], h, l) ? 1 : 0;
            const int64_t q = o0 + rank;
            a.pair_j[q] = jj[p];
            a.pair_shift[3 * q] = ss[3 * p];
            a.pair_shift[3 * q + 1] = ss[3 * p + 1];
            a.pair_shift[3 * q + 2] = ss[3 * p + 2];
            vec[3 * q] = vv[3 * p];
            vec[3 * q + 1] = vv[3 * p + 1];
            vec[3 * q + 2] = vv[3 * p + 2];
        }
        return;
    }
    // long environments: insertion sort in place in global memory
    __threadfence_block();
    if (lane == 0) {
        for (int64_t p = o0 + 1; p < o0 + n; ++p) {
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
    __threadfence_block();
    wave_fence();
    for (int p = lane; p < n; p += 64) {
        int64_t q = o0 + p;
        write_pair<F64>(a, g, i, q, a.pair_j[q], a.pair_shift[3 * q], a.pair_shift[3 * q + 1], a.pair_shift[3 * q + 2]);
    }
}

__device__ void transpose_pair(const NeighborArgs& a, int64_t i, int64_t q)
{
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

// one wave per centre i, lanes over its pairs q = (i, j, s): the reverse
// pair (j, i, -s) is found by binary search in j's sorted list
__global__ void __launch_bounds__(256) k_transpose(NeighborArgs a)
{
    const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (i >= a.n_atoms || a.pair_offsets[a.n_atoms] > a.capacity) return;
    const int64_t q_end = a.pair_offsets[i + 1];
    for (int64_t q = a.pair_offsets[i] + (threadIdx.x & 63); q < q_end; q += 64)
        transpose_pair(a, i, q);
}

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

// exclusive scan of n values (out[n] = total; capacity < 0: no check)
template <typename Tin, typename Tout>
void scan(const Tin* in, Tout* out, Tout* out2, int64_t n, int64_t capacity, int64_t* tmp, int32_t* status,
          hipStream_t stream)
{
    if (n <= kMultiScan) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan<Tin, Tout>), dim3(1), dim3(1024), 0, stream, in, out, out2, n,
                           capacity, status);
        return;
    }
    const int64_t nt = (n + kScanTile - 1) / kScanTile;
    Tout* sums = reinterpret_cast<Tout*>(tmp);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tile_sums<Tin, Tout>), dim3(unsigned(nt)), dim3(256), 0, stream, in, sums, n);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan<Tout, Tout>), dim3(1), dim3(1024), 0, stream, sums, sums,
                       (Tout*)nullptr, nt, capacity, status);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_tile_scan<Tin, Tout>), dim3(unsigned(nt)), dim3(256), 0, stream, in, out, out2,
                       sums, n, nt);
}

}  // namespace

hipError_t launch_neighbors(const NeighborArgs& a, hipStream_t stream)
{
    const int T = 256;
    const int64_t N = a.n_atoms, B = a.max_bins;
    if (N == 0) {
        hipLaunchKernelGGL(k_geometry, dim3(1), dim3(1024), 0, stream, a);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan<int64_t, int64_t>), dim3(1), dim3(1024), 0, stream,
                           a.centre_count, a.pair_offsets, (int64_t*)nullptr, int64_t(0), a.capacity, a.status);
        return hipGetLastError();
    }
    // all pairs when the structures are small (on average at most
    // kBrutePerStruct atoms: a 1024-atom cell is faster with bins)
    if (N <= kBrutePerStruct * int64_t(a.n_structures)) {
        const dim3 grid{unsigned(N)}, wave{64};
        const bool self_check = N <= kBruteAtoms && a.n_structures <= kBruteStructs;
        if (self_check) {
            // each wave checks the input; with pairs to write the fill sums
            // the counts itself
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_count_bf<false>), grid, wave, 0, stream, a);
            if (a.capacity > 0) {
                if (a.vec_f64) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fill_bf<false, true>), grid, wave, 0, stream, a);
                else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fill_bf<false, false>), grid, wave, 0, stream, a);
            }
        } else {
            // many structures: the geometry phase, then the counts
            hipLaunchKernelGGL(k_geometry, dim3(1), dim3(1024), 0, stream, a);
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_count_bf<true>), grid, wave, 0, stream, a);
        }
        if (!self_check || a.capacity <= 0)   // offsets by a scan (which reports the count at capacity 0)
            scan<int64_t, int64_t>(a.centre_count, a.pair_offsets, (int64_t*)nullptr, N, a.capacity, a.scan_tmp,
                                   a.status, stream);
        if (!self_check && a.capacity > 0) {
            if (a.vec_f64) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fill_bf<true, true>), grid, wave, 0, stream, a);
            else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fill_bf<true, false>), grid, wave, 0, stream, a);
        }
        if (a.capacity > 0 && a.pair_transpose)
            hipLaunchKernelGGL(k_transpose, dim3(blocks(a.n_atoms, 4)), dim3(256), 0, stream, a);
        return hipGetLastError();
    }
    const bool small = B <= kSmallBins && N <= kSmallAtoms;
    if (small) {
        hipLaunchKernelGGL(k_bins_small, dim3(1), dim3(1024), 0, stream, a);
    } else {
        hipLaunchKernelGGL(k_geometry, dim3(1), dim3(1024), 0, stream, a);
        hipLaunchKernelGGL(k_zero_i32, dim3(blocks(B + 1, T)), dim3(T), 0, stream, a.bin_count, B + 1);
        hipLaunchKernelGGL(k_assign, dim3(blocks(N, 256)), dim3(256), 0, stream, a);
        scan<int32_t, int32_t>(a.bin_count, a.bin_start, a.bin_cursor, B, int64_t(-1), a.scan_tmp, a.status, stream);
        hipLaunchKernelGGL(k_bins, dim3(blocks(N, T)), dim3(T), 0, stream, a);
    }
    const bool one = a.n_structures == 1;
    const dim3 grid{unsigned(N)}, wave{64};
    if (one) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_count<true>), grid, wave, 0, stream, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_count<false>), grid, wave, 0, stream, a);
    // small systems with pairs to write: the fill kernel forms the offsets;
    // otherwise a scan (which also reports the count when capacity is 0)
    const bool prefix = N <= kPrefixAtoms && a.capacity > 0;
    if (!prefix)
        scan<int64_t, int64_t>(a.centre_count, a.pair_offsets, (int64_t*)nullptr, N, a.capacity, a.scan_tmp, a.status,
                               stream);
    if (a.capacity > 0) {
#define SOAP_FILL(ONE_, F64_)                                                                             \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fill<ONE_, F64_>), dim3(blocks(N, kFillWaves)), dim3(64 * kFillWaves), 0, \
                       stream, a)
        if (prefix) {
#define SOAP_FILL1(ONE_, F64_) \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fill1<ONE_, F64_, true>), grid, wave, 0, stream, a)
            if (a.vec_f64) { if (one) SOAP_FILL1(true, true); else SOAP_FILL1(false, true); }
            else { if (one) SOAP_FILL1(true, false); else SOAP_FILL1(false, false); }
#undef SOAP_FILL1
        } else {
            if (a.vec_f64) { if (one) SOAP_FILL(true, true); else SOAP_FILL(false, true); }
            else { if (one) SOAP_FILL(true, false); else SOAP_FILL(false, false); }
        }
#undef SOAP_FILL
        if (a.pair_transpose && a.n_atoms > 0)
            hipLaunchKernelGGL(k_transpose, dim3(blocks(a.n_atoms, 4)), dim3(256), 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace soap
