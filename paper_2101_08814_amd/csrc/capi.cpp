// C ABI of the library: argument validation, error reporting, spline-table
// upload and kernel dispatch.  Every array argument is checked on the host
// before anything is enqueued; device-detected errors go to exec->dev_status.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "soap_internal.hpp"

namespace soap {

namespace {
thread_local char g_error[512] = "";
}

soap_status fail(soap_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof(g_error), fmt, ap);
    va_end(ap);
    return st;
}

void clear_error() { g_error[0] = '\0'; }

// SOAP_FAIL_ALLOC=1 in the environment makes every allocation the library
// makes or sizes for the caller (calculator, device tables, workspace
// queries) fail with SOAP_ENOMEM, so callers can test that path.
bool alloc_failure_forced()
{
    const char* v = std::getenv("SOAP_FAIL_ALLOC");
    return v && v[0] == '1';
}

soap_status device_tables(const soap_calculator* calc, const DeviceTables** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SOAP_EDEVICE, "no HIP device available");
    std::lock_guard<std::mutex> lock(calc->mu);
    if (int(calc->dev.size()) <= dev) calc->dev.resize(dev + 1);
    DeviceTables& t = calc->dev[dev];
    if (!t.ready) {
        size_t b64 = calc->coef64.size() * sizeof(double), b32 = calc->coef32.size() * sizeof(float);
        size_t c64 = calc->center.size() * sizeof(double), c32 = calc->center.size() * sizeof(float);
        std::vector<float> cf(calc->center.begin(), calc->center.end());
        // degree-major copy: the nmax cubics of one (interval, l) contiguous
        const int lm1t = calc->h.lmax + 1, nmx = calc->h.nmax, nlt = calc->nl;
        // (32 zero cubics past the end, so a lane may read up to 32 entries
        // past its interval's block without a bounds check)
        const size_t pad_ln = 32 * 4;
        std::vector<double> ln64(calc->coef64.size() + pad_ln, 0.0);
        std::vector<float> ln32(calc->coef32.size() + pad_ln, 0.0f);
        for (int64_t k = 0; k < calc->M; ++k)
            for (int n = 0; n < nmx; ++n)
                for (int l = 0; l < lm1t; ++l)
                    for (int e = 0; e < 4; ++e) {
                        const size_t src = ((size_t(k) * nlt + n * lm1t + l) * 4) + e;
                        const size_t dst = ((size_t(k) * lm1t + l) * nmx + n) * 4 + e;
                        ln64[dst] = calc->coef64[src];
                        ln32[dst] = calc->coef32[src];
                    }
        if (alloc_failure_forced() || hipMalloc(&t.coef64, b64) != hipSuccess ||
            hipMalloc(&t.coef32, b32) != hipSuccess || hipMalloc(&t.coef64_ln, ln64.size() * sizeof(double)) != hipSuccess ||
            hipMalloc(&t.coef32_ln, ln32.size() * sizeof(float)) != hipSuccess ||
            hipMalloc(&t.center64, c64) != hipSuccess || hipMalloc(&t.center32, c32) != hipSuccess)
            return fail(SOAP_ENOMEM, "allocation of the spline tables failed on device %d", dev);
        if (hipMemcpy(t.coef64, calc->coef64.data(), b64, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(t.coef32, calc->coef32.data(), b32, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(t.coef64_ln, ln64.data(), ln64.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(t.coef32_ln, ln32.data(), ln32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(t.center64, calc->center.data(), c64, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(t.center32, cf.data(), c32, hipMemcpyHostToDevice) != hipSuccess)
            return fail(SOAP_EDEVICE, "upload of the spline tables failed on device %d", dev);
        // (l, k1, k2) of every position of a packed dp row, for the row kernels
        const int K = calc->K, lm1 = calc->h.lmax + 1;
        if (K <= 1023 && int64_t(lm1) * calc->KK <= (int64_t(1) << 22)) {
            std::vector<int32_t> pos;
            pos.reserve(size_t(lm1) * calc->KK);
            for (int l = 0; l < lm1; ++l)
                for (int k1 = 0; k1 < K; ++k1)
                    for (int k2 = k1; k2 < K; ++k2) pos.push_back(l | (k1 << 4) | (k2 << 14));
            if (hipMalloc(&t.dp_pos, pos.size() * sizeof(int32_t)) != hipSuccess)
                return fail(SOAP_ENOMEM, "allocation of the spline tables failed on device %d", dev);
            if (hipMemcpy(t.dp_pos, pos.data(), pos.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
                return fail(SOAP_EDEVICE, "upload of the spline tables failed on device %d", dev);
        }
        {
            const int nmx = calc->h.nmax, np = (nmx + 3) & ~3, nlt = calc->nl;
            std::vector<int32_t> dst(size_t(nlt) + 16);
            for (int j = 0; j < nlt + 16; ++j) {
                const int jj = j < nlt ? j : nlt - 1;
                dst[j] = (jj / nmx) * np + jj % nmx;
            }
            if (hipMalloc(&t.radial_dst, dst.size() * sizeof(int32_t)) != hipSuccess)
                return fail(SOAP_ENOMEM, "allocation of the spline tables failed on device %d", dev);
            if (hipMemcpy(t.radial_dst, dst.data(), dst.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
                hipSuccess)
                return fail(SOAP_EDEVICE, "upload of the spline tables failed on device %d", dev);
        }
        {
            // constants of the direct radial integral, packed in one array
            const ExactRadial& e = calc->exact;
            const int nmx = e.nmax, lm1e = e.lmax + 1;
            std::vector<double> pack;
            size_t o_alpha = 0, o_pref = 0, o_top = 0, o_X = 0, o_x = 0, o_A = 0;
            if (e.basis == SOAP_RADIAL_DVR) {
                o_x = pack.size(); pack.insert(pack.end(), e.x.begin(), e.x.end());
                o_A = pack.size(); pack.insert(pack.end(), e.A.begin(), e.A.end());
            } else {
                o_alpha = pack.size(); pack.insert(pack.end(), e.alpha.begin(), e.alpha.end());
                o_pref = pack.size(); pack.insert(pack.end(), e.pref.begin(), e.pref.end());
                o_top = pack.size();
                for (const rad::GParams& g : e.top) {
                    pack.push_back(g.a); pack.push_back(g.b); pack.push_back(g.lgr); pack.push_back(g.zswitch);
                }
                o_X = pack.size(); pack.insert(pack.end(), e.X.begin(), e.X.end());
            }
            if (pack.empty()) pack.push_back(0.0);
            if (hipMalloc(&t.exact, pack.size() * sizeof(double)) != hipSuccess)
                return fail(SOAP_ENOMEM, "allocation of the spline tables failed on device %d", dev);
            if (hipMemcpy(t.exact, pack.data(), pack.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
                return fail(SOAP_EDEVICE, "upload of the spline tables failed on device %d", dev);
            t.gto = rad::GtoTables{nmx, e.c, t.exact + o_alpha, t.exact + o_pref,
                                   reinterpret_cast<const rad::GParams*>(t.exact + o_top), t.exact + o_X};
            t.dvr = rad::DvrTables{nmx, e.c, t.exact + o_x, t.exact + o_A};
            (void)lm1e;
        }
        t.ready = true;
    }
    *out = &t;
    return SOAP_OK;
}

}  // namespace soap

using namespace soap;

namespace {

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

#define REQUIRE(cond, ...)                                  \
    do {                                                    \
        if (!(cond)) return fail(SOAP_EINVAL, __VA_ARGS__); \
    } while (0)

soap_status check_ptr(const void* p, size_t align, const char* name, bool nullable = false)
{
    if (!p) return nullable ? SOAP_OK : fail(SOAP_EINVAL, "%s must not be NULL", name);
    if (!aligned(p, align)) return fail(SOAP_EINVAL, "%s is not %zu-byte aligned", name, align);
    return SOAP_OK;
}

#define CHECK(expr)                          \
    do {                                     \
        soap_status st__ = (expr);           \
        if (st__ != SOAP_OK) return st__;    \
    } while (0)

hipStream_t stream_of(const soap_exec* e) { return e ? static_cast<hipStream_t>(e->stream) : nullptr; }
int32_t* status_of(const soap_exec* e) { return e ? e->dev_status : nullptr; }

size_t elem_size(soap_precision p) { return p == SOAP_F64 ? 8 : 4; }

soap_status launched(hipError_t e, const char* what)
{
    if (e == hipErrorNotSupported)
        return fail(SOAP_EUNSUPPORTED, "%s: these sizes exceed what the kernels support (LDS per work-group or index packing)", what);
    if (e != hipSuccess) return fail(SOAP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    hipError_t last = hipGetLastError();
    if (last != hipSuccess) return fail(SOAP_EDEVICE, "%s: %s", what, hipGetErrorString(last));
    return SOAP_OK;
}

soap_status check_calc(const soap_calculator* c)
{
    if (!c) return fail(SOAP_EINVAL, "calculator must not be NULL");
    return SOAP_OK;
}

FeatureArgs base_args(const soap_calculator* calc, const soap_exec* exec, bool f64, const DeviceTables* t)
{
    FeatureArgs a{};
    a.S = calc->h.n_species;
    a.nmax = calc->h.nmax;
    a.lmax = calc->h.lmax;
    a.include_center = calc->h.include_center;
    a.rcut = calc->h.rcut;
    a.width = calc->h.cutoff_width;
    a.M = calc->M;
    a.inv_delta = calc->inv_delta;
    a.coef = f64 ? static_cast<const void*>(t->coef64) : static_cast<const void*>(t->coef32);
    a.coef_ln = f64 ? static_cast<const void*>(t->coef64_ln) : static_cast<const void*>(t->coef32_ln);
    a.center = f64 ? static_cast<const void*>(t->center64) : static_cast<const void*>(t->center32);
    a.dp_pos = t->dp_pos;
    a.radial_dst = t->radial_dst;
    a.status = status_of(exec);
    return a;
}

struct NbLayout {
    size_t geom, ok, atom_struct, atom_bin, atom_wrap, bin_count, bin_start, bin_cursor, bin_atoms, slots, wrapped,
        centre_count, scan_tmp, total;
};

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// at most one bin per atom per structure, and one for an empty structure
int64_t max_bins(int32_t n_struct, int64_t N) { return N + n_struct; }

NbLayout nb_layout(int32_t n_struct, int64_t N)
{
    int64_t B = max_bins(n_struct, N);
    NbLayout L{};
    size_t o = 0;
    L.geom = o; o = up256(o + sizeof(StructGeom) * size_t(n_struct));
    L.ok = o; o = up256(o + 4);
    L.atom_struct = o; o = up256(o + 4 * size_t(N));
    L.atom_bin = o; o = up256(o + 4 * size_t(N));
    L.atom_wrap = o; o = up256(o + 12 * size_t(N));
    L.bin_count = o; o = up256(o + 4 * size_t(B + 1));
    L.bin_start = o; o = up256(o + 4 * size_t(B + 1));
    L.bin_cursor = o; o = up256(o + 4 * size_t(B + 1));
    L.bin_atoms = o; o = up256(o + 4 * size_t(N));
    L.slots = o; o = up256(o + 32 * size_t(N));
    L.wrapped = o; o = up256(o + 32 * size_t(N));
    L.centre_count = o; o = up256(o + 8 * size_t(N + 1));
    L.scan_tmp = o; o = up256(o + 8 * size_t((B + 1) / 4096 + 2));   // one sum per 4096-value tile of the longer scan
    L.total = o;
    return L;
}

}  // namespace

namespace soap {
size_t neighbors_workspace_bytes(int32_t n_structures, int64_t n_atoms) { return nb_layout(n_structures, n_atoms).total; }
}  // namespace soap

namespace {

// ------------------------------------------------------------ compression

constexpr int kCompressSlices = 64;   // partial sums of the backward pass
constexpr int kCovSlices = 32;        // partial sums of the channel covariance

int64_t compress_params(const soap_calculator* calc, int Q, int H)
{
    const int K = calc->K, lm1 = calc->h.lmax + 1;
    return int64_t(lm1) * (int64_t(H) * K + int64_t(Q) * H + 2 * int64_t(H));
}

soap_status check_compress(const soap_calculator* calc, int32_t Q, int32_t H)
{
    CHECK(check_calc(calc));
    REQUIRE(Q >= 1 && Q <= 64, "n_out must be in [1, 64] (got %d)", Q);
    REQUIRE(H >= 1 && H <= 256, "hidden must be in [1, 256] (got %d)", H);
    return SOAP_OK;
}

CompressArgs compress_args(const soap_calculator* calc, const soap_exec* exec, int Q, int H, int64_t n)
{
    CompressArgs a{};
    a.K = calc->K;
    a.Q = Q;
    a.H = H;
    a.lmax = calc->h.lmax;
    a.n = n;
    a.n_params = compress_params(calc, Q, H);
    a.slices = kCompressSlices;
    a.status = status_of(exec);
    return a;
}

size_t compress_workspace(const soap_calculator* calc, int Q, int H)
{
    const size_t grads = size_t(kCompressSlices) * size_t(compress_params(calc, Q, H)) * sizeof(float);
    const size_t cov = size_t(kCovSlices) * (calc->h.lmax + 1) * size_t(calc->K) * calc->K * sizeof(float);
    const size_t img = compress_image_bytes(calc->K, Q, H, calc->h.lmax);
    return std::max(std::max(grads, cov), img);
}

// splitmix64 (Steele, Lea, Flood 2014) and Box-Muller normals
struct SplitMix {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal()
    {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

}  // namespace

extern "C" {

int32_t soap_abi_version(void) { return SOAP_ABI_VERSION; }

const char* soap_last_error(void) { return g_error; }

soap_status soap_calculator_create(const soap_hypers* h, soap_calculator** out)
{
    clear_error();
    REQUIRE(h != nullptr, "hypers must not be NULL");
    REQUIRE(out != nullptr, "out must not be NULL");
    *out = nullptr;
    REQUIRE(h->n_species >= 1 && h->n_species <= 64, "n_species must be in [1, 64] (got %d)", h->n_species);
    REQUIRE(h->nmax >= 1 && h->nmax <= 16, "nmax must be in [1, 16] (got %d)", h->nmax);
    REQUIRE(h->lmax >= 0 && h->lmax <= 12, "lmax must be in [0, 12] (got %d)", h->lmax);
    REQUIRE(std::isfinite(h->rcut) && h->rcut > 0, "rcut must be > 0");
    REQUIRE(std::isfinite(h->cutoff_width) && h->cutoff_width > 0 && h->cutoff_width <= h->rcut,
            "cutoff_width must be in (0, rcut]");
    REQUIRE(std::isfinite(h->sigma) && h->sigma > 0, "sigma must be > 0");
    REQUIRE(h->include_center == 0 || h->include_center == 1, "include_center must be 0 or 1");
    REQUIRE(std::isfinite(h->spline_accuracy) && h->spline_accuracy > 0, "spline_accuracy must be > 0");
    REQUIRE(h->radial_basis == SOAP_RADIAL_GTO || h->radial_basis == SOAP_RADIAL_DVR,
            "radial_basis must be SOAP_RADIAL_GTO or SOAP_RADIAL_DVR (got %d)", h->radial_basis);
    REQUIRE(h->reserved == 0, "reserved must be 0");
    if (alloc_failure_forced()) return fail(SOAP_ENOMEM, "allocation failure forced by SOAP_FAIL_ALLOC");
    soap_calculator* c = new (std::nothrow) soap_calculator();
    if (!c) return fail(SOAP_ENOMEM, "out of host memory");
    c->h = *h;
    c->L2 = (h->lmax + 1) * (h->lmax + 1);
    c->K = h->n_species * h->nmax;
    c->KK = int64_t(c->K) * (c->K + 1) / 2;
    c->nl = h->nmax * (h->lmax + 1);
    soap_status st = build_tables(c);
    if (st != SOAP_OK) {
        delete c;
        return st;
    }
    *out = c;
    return SOAP_OK;
}

soap_status soap_calculator_destroy(soap_calculator* calc)
{
    clear_error();
    if (!calc) return SOAP_OK;
    int cur = 0;
    bool have = hipGetDevice(&cur) == hipSuccess;
    for (size_t d = 0; d < calc->dev.size(); ++d) {
        DeviceTables& t = calc->dev[d];
        if (!t.ready) continue;
        if (have) (void)hipSetDevice(int(d));
        (void)hipFree(t.coef64);
        (void)hipFree(t.coef32);
        (void)hipFree(t.coef64_ln);
        (void)hipFree(t.coef32_ln);
        (void)hipFree(t.center64);
        (void)hipFree(t.center32);
        (void)hipFree(t.dp_pos);
        (void)hipFree(t.radial_dst);
        (void)hipFree(t.exact);
    }
    if (have) (void)hipSetDevice(cur);
    delete calc;
    return SOAP_OK;
}

soap_status soap_calculator_info(const soap_calculator* calc, soap_table_info* info)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(info != nullptr, "info must not be NULL");
    *info = calc->info;
    return SOAP_OK;
}

soap_status soap_calculator_upload(const soap_calculator* calc)
{
    clear_error();
    CHECK(check_calc(calc));
    const DeviceTables* t = nullptr;
    return device_tables(calc, &t);
}

soap_status soap_radial_integral_host(const soap_calculator* calc, int32_t exact, int64_t n_r, const double* r,
                                      double* I, double* dI)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(n_r >= 0, "n_r must be >= 0");
    if (n_r == 0) return SOAP_OK;
    CHECK(check_ptr(r, 8, "r"));
    CHECK(check_ptr(I, 8, "I"));
    CHECK(check_ptr(dI, 8, "dI", true));
    for (int64_t k = 0; k < n_r; ++k)
        REQUIRE(std::isfinite(r[k]) && r[k] >= 0 && r[k] <= calc->h.rcut, "r[%lld] outside [0, rcut]", (long long)k);
    int nl = calc->nl;
    if (exact) {
        radial_exact(calc, n_r, r, I, dI);
    } else {
        for (int64_t k = 0; k < n_r; ++k) radial_spline_host(calc, r[k], I + k * nl, dI ? dI + k * nl : nullptr);
    }
    return SOAP_OK;
}

soap_status soap_radial_integral(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                                 int32_t exact, int64_t n_r, const double* r, void* I, void* dI)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(exact == 0 || exact == 1, "exact must be 0 or 1");
    REQUIRE(!(exact && precision != SOAP_F64), "the direct evaluation is SOAP_F64 only");
    REQUIRE(n_r >= 0 && n_r < (int64_t(1) << 31), "n_r must be in [0, 2^31)");
    if (n_r == 0) return SOAP_OK;
    const size_t es = elem_size(precision);
    CHECK(check_ptr(r, 8, "r"));
    CHECK(check_ptr(I, es, "I"));
    CHECK(check_ptr(dI, es, "dI", true));
    const DeviceTables* t = nullptr;
    CHECK(device_tables(calc, &t));
    RadialArgs a{};
    a.nmax = calc->h.nmax;
    a.lmax = calc->h.lmax;
    a.basis = calc->h.radial_basis;
    a.exact = exact != 0;
    a.M = calc->M;
    a.inv_delta = calc->inv_delta;
    a.coef = precision == SOAP_F64 ? static_cast<const void*>(t->coef64) : static_cast<const void*>(t->coef32);
    a.gto = t->gto;
    a.dvr = t->dvr;
    a.n_r = n_r;
    a.r = r;
    a.I = I;
    a.dI = dI;
    return launched(launch_radial(a, precision == SOAP_F64, stream_of(exec)), "radial integral");
}

soap_status soap_neighbors_workspace_size(const soap_calculator* calc, int32_t n_structures, int64_t n_atoms,
                                          size_t* bytes)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(bytes != nullptr, "bytes must not be NULL");
    REQUIRE(n_structures >= 0, "n_structures must be >= 0 (got %d)", n_structures);
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    if (alloc_failure_forced()) return fail(SOAP_ENOMEM, "allocation failure forced by SOAP_FAIL_ALLOC");
    *bytes = nb_layout(n_structures, n_atoms).total;
    return SOAP_OK;
}

soap_status soap_compute_neighbors(const soap_calculator* calc, const soap_exec* exec, int32_t n_structures,
                                   int64_t n_atoms, const int64_t* atom_offsets, const double* cells,
                                   const uint8_t* pbc, const double* positions, const int32_t* species,
                                   void* workspace, size_t workspace_bytes, int64_t capacity,
                                   soap_precision vec_precision, int64_t* pair_offsets, int32_t* pair_j,
                                   int32_t* pair_shift, void* pair_vec, int32_t* pair_transpose)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(vec_precision == SOAP_F64 || vec_precision == SOAP_F32, "vec_precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(capacity >= 0 && capacity < (int64_t(1) << 31), "capacity must be in [0, 2^31)");
    REQUIRE(n_structures >= 0, "n_structures must be >= 0 (got %d)", n_structures);
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE(n_structures > 0 || n_atoms == 0, "atoms without structures");
    CHECK(check_ptr(atom_offsets, 8, "atom_offsets"));
    CHECK(check_ptr(pair_offsets, 8, "pair_offsets"));
    if (n_structures > 0) {
        CHECK(check_ptr(cells, 8, "cells"));
        CHECK(check_ptr(pbc, 1, "pbc"));
    }
    if (n_atoms > 0) {
        CHECK(check_ptr(positions, 8, "positions"));
        CHECK(check_ptr(species, 4, "species"));
    }
    if (capacity > 0) {
        CHECK(check_ptr(pair_j, 4, "pair_j"));
        CHECK(check_ptr(pair_shift, 4, "pair_shift"));
        CHECK(check_ptr(pair_vec, elem_size(vec_precision), "pair_vec"));
        CHECK(check_ptr(pair_transpose, 4, "pair_transpose", true));
    }
    NbLayout L = nb_layout(n_structures, n_atoms);
    REQUIRE(workspace_bytes >= L.total, "workspace too small: %zu bytes given, %zu needed", workspace_bytes, L.total);
    CHECK(check_ptr(workspace, 256, "workspace"));
    char* ws = static_cast<char*>(workspace);
    NeighborArgs a{};
    a.n_structures = n_structures;
    a.n_atoms = n_atoms;
    a.max_bins = max_bins(n_structures, n_atoms);
    a.rcut = calc->h.rcut;
    a.atom_offsets = atom_offsets;
    a.cells = cells;
    a.pbc = pbc;
    a.positions = positions;
    a.species = species;
    a.n_species = calc->h.n_species;
    a.geom = reinterpret_cast<StructGeom*>(ws + L.geom);
    a.ok = reinterpret_cast<int32_t*>(ws + L.ok);
    a.atom_struct = reinterpret_cast<int32_t*>(ws + L.atom_struct);
    a.atom_bin = reinterpret_cast<int32_t*>(ws + L.atom_bin);
    a.atom_wrap = reinterpret_cast<int32_t*>(ws + L.atom_wrap);
    a.bin_count = reinterpret_cast<int32_t*>(ws + L.bin_count);
    a.bin_start = reinterpret_cast<int32_t*>(ws + L.bin_start);
    a.bin_cursor = reinterpret_cast<int32_t*>(ws + L.bin_cursor);
    a.bin_atoms = reinterpret_cast<int32_t*>(ws + L.bin_atoms);
    a.slots = reinterpret_cast<double4*>(ws + L.slots);
    a.wrapped = reinterpret_cast<double4*>(ws + L.wrapped);
    a.centre_count = reinterpret_cast<int64_t*>(ws + L.centre_count);
    a.scan_tmp = reinterpret_cast<int64_t*>(ws + L.scan_tmp);
    a.capacity = capacity;
    a.pair_offsets = pair_offsets;
    a.pair_j = pair_j;
    a.pair_shift = pair_shift;
    a.pair_vec = pair_vec;
    a.vec_f64 = vec_precision == SOAP_F64;
    a.pair_transpose = pair_transpose;
    a.status = status_of(exec);
    return launched(launch_neighbors(a, stream_of(exec)), "neighbour kernels");
}

static soap_status check_pairs(const int32_t* species, const int64_t* pair_offsets, const int32_t* pair_j,
                               const void* pair_vec, int64_t pair_capacity, size_t es, bool need_vec = true)
{
    CHECK(check_ptr(species, 4, "species"));
    CHECK(check_ptr(pair_offsets, 8, "pair_offsets"));
    REQUIRE(pair_capacity >= 0 && pair_capacity < (int64_t(1) << 31), "pair_capacity must be in [0, 2^31)");
    if (pair_capacity > 0) {
        CHECK(check_ptr(pair_j, 4, "pair_j"));
        if (need_vec) CHECK(check_ptr(pair_vec, es, "pair_vec"));
    }
    return SOAP_OK;
}

soap_status soap_spherical_expansion(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                                     int64_t n_atoms, const int32_t* species, const int64_t* pair_offsets,
                                     const int32_t* pair_j, const void* pair_vec, int64_t pair_capacity,
                                     void* coeffs, void* dcoeffs, void* dcoeffs_self)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE((dcoeffs == nullptr) == (dcoeffs_self == nullptr), "dcoeffs and dcoeffs_self: both or neither");
    if (n_atoms == 0) return SOAP_OK;
    size_t es = elem_size(precision);
    CHECK(check_pairs(species, pair_offsets, pair_j, pair_vec, pair_capacity, es));
    CHECK(check_ptr(coeffs, es, "coeffs"));
    CHECK(check_ptr(dcoeffs, es, "dcoeffs", true));
    CHECK(check_ptr(dcoeffs_self, es, "dcoeffs_self", true));
    const DeviceTables* t = nullptr;
    CHECK(device_tables(calc, &t));
    FeatureArgs a = base_args(calc, exec, precision == SOAP_F64, t);
    a.n_atoms = n_atoms;
    a.species = species;
    a.pair_offsets = pair_offsets;
    a.pair_j = pair_j;
    a.pair_vec = pair_vec;
    a.pair_capacity = pair_capacity;
    a.coeffs = coeffs;
    a.dcoeffs = dcoeffs;
    a.dcoeffs_self = dcoeffs_self;
    return launched(launch_features(a, precision == SOAP_F64, stream_of(exec)), "spherical expansion");
}

soap_status soap_power_spectrum(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                                int64_t n_atoms, const void* coeffs, void* p, const int32_t* species,
                                const int64_t* pair_offsets, const int32_t* pair_j, int64_t pair_capacity,
                                const void* dcoeffs, const void* dcoeffs_self, void* dp, void* dp_self)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32 || precision == SOAP_BF16_F32ACC,
            "precision must be SOAP_F64, SOAP_F32 or SOAP_BF16_F32ACC");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE((dp == nullptr) == (dp_self == nullptr), "dp and dp_self: both or neither");
    REQUIRE(!(precision == SOAP_BF16_F32ACC && dp), "gradient rows are not produced on the bfloat16 path");
    if (n_atoms == 0) return SOAP_OK;
    size_t es = elem_size(precision);
    CHECK(check_ptr(coeffs, es, "coeffs"));
    CHECK(check_ptr(p, es, "p"));
    if (dp) {
        CHECK(check_pairs(species, pair_offsets, pair_j, nullptr, pair_capacity, es, false));
        CHECK(check_ptr(dp, es, "dp"));
        CHECK(check_ptr(dp_self, es, "dp_self"));
        CHECK(check_ptr(dcoeffs_self, es, "dcoeffs_self"));
        if (pair_capacity > 0) CHECK(check_ptr(dcoeffs, es, "dcoeffs"));
    }
    const DeviceTables* t = nullptr;
    CHECK(device_tables(calc, &t));
    FeatureArgs a = base_args(calc, exec, precision == SOAP_F64, t);
    a.n_atoms = n_atoms;
    a.species = species;
    a.pair_offsets = pair_offsets;
    a.pair_j = pair_j;
    a.pair_capacity = pair_capacity;
    a.coeffs = const_cast<void*>(coeffs);
    a.p = p;
    a.dcoeffs = const_cast<void*>(dcoeffs);
    a.dcoeffs_self = const_cast<void*>(dcoeffs_self);
    a.dp = dp;
    a.dp_self = dp_self;
    return launched(launch_power_spectrum(a, precision, stream_of(exec)), "power spectrum");
}

soap_status soap_features(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                          int64_t n_atoms, const int32_t* species, const int64_t* pair_offsets, const int32_t* pair_j,
                          const void* pair_vec, int64_t pair_capacity, void* coeffs, void* p, void* dcoeffs,
                          void* dcoeffs_self, void* dp, void* dp_self)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE((dcoeffs_self == nullptr) == (dp_self == nullptr), "dcoeffs_self and dp_self: both or neither");
    REQUIRE((dcoeffs == nullptr) == (dp == nullptr), "dcoeffs and dp: both or neither");
    if (n_atoms == 0) return SOAP_OK;
    size_t es = elem_size(precision);
    CHECK(check_pairs(species, pair_offsets, pair_j, pair_vec, pair_capacity, es));
    CHECK(check_ptr(coeffs, es, "coeffs"));
    CHECK(check_ptr(p, es, "p"));
    CHECK(check_ptr(dcoeffs, es, "dcoeffs", true));
    CHECK(check_ptr(dcoeffs_self, es, "dcoeffs_self", true));
    CHECK(check_ptr(dp, es, "dp", true));
    CHECK(check_ptr(dp_self, es, "dp_self", true));
    const DeviceTables* t = nullptr;
    CHECK(device_tables(calc, &t));
    FeatureArgs a = base_args(calc, exec, precision == SOAP_F64, t);
    a.n_atoms = n_atoms;
    a.species = species;
    a.pair_offsets = pair_offsets;
    a.pair_j = pair_j;
    a.pair_vec = pair_vec;
    a.pair_capacity = pair_capacity;
    a.coeffs = coeffs;
    a.p = p;
    a.dcoeffs = dcoeffs;
    a.dcoeffs_self = dcoeffs_self;
    a.dp = dp;
    a.dp_self = dp_self;
    return launched(launch_features(a, precision == SOAP_F64, stream_of(exec)), "features");
}

soap_status soap_gradient_rows(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                               int64_t n_atoms, const int32_t* species, const int64_t* pair_offsets,
                               const int32_t* pair_j, const void* pair_vec, int64_t pair_capacity, const void* coeffs,
                               void* dcoeffs, void* dp)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE(dcoeffs != nullptr || dp != nullptr, "dcoeffs and dp must not both be NULL");
    if (n_atoms == 0) return SOAP_OK;
    size_t es = elem_size(precision);
    CHECK(check_pairs(species, pair_offsets, pair_j, pair_vec, pair_capacity, es));
    if (dp) CHECK(check_ptr(coeffs, es, "coeffs"));
    if (pair_capacity > 0) {
        CHECK(check_ptr(dcoeffs, es, "dcoeffs", true));
        CHECK(check_ptr(dp, es, "dp", true));
    }
    const DeviceTables* t = nullptr;
    CHECK(device_tables(calc, &t));
    FeatureArgs a = base_args(calc, exec, precision == SOAP_F64, t);
    a.n_atoms = n_atoms;
    a.species = species;
    a.pair_offsets = pair_offsets;
    a.pair_j = pair_j;
    a.pair_vec = pair_vec;
    a.pair_capacity = pair_capacity;
    a.coeffs = const_cast<void*>(coeffs);
    a.dcoeffs = dcoeffs;
    a.dp = dp;
    return launched(launch_gradient_rows(a, precision == SOAP_F64, stream_of(exec)), "gradient rows");
}

soap_status soap_power_spectrum_backward(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                                         int64_t n_atoms, const void* coeffs, const void* grad_p, void* grad_coeffs)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    if (n_atoms == 0) return SOAP_OK;
    size_t es = elem_size(precision);
    CHECK(check_ptr(coeffs, es, "coeffs"));
    CHECK(check_ptr(grad_p, es, "grad_p"));
    CHECK(check_ptr(grad_coeffs, es, "grad_coeffs"));
    const DeviceTables* t = nullptr;
    CHECK(device_tables(calc, &t));
    FeatureArgs a = base_args(calc, exec, precision == SOAP_F64, t);
    a.n_atoms = n_atoms;
    a.coeffs = const_cast<void*>(coeffs);
    return launched(launch_power_spectrum_backward(a, precision == SOAP_F64, grad_p, grad_coeffs, stream_of(exec)),
                    "power spectrum backward");
}

soap_status soap_spherical_expansion_backward(const soap_calculator* calc, const soap_exec* exec,
                                              soap_precision precision, int64_t n_atoms, const int32_t* species,
                                              const int64_t* pair_offsets, const int32_t* pair_j,
                                              const void* pair_vec, const int32_t* pair_transpose,
                                              int64_t pair_capacity, const void* grad_coeffs, void* grad_pair_vec,
                                              void* grad_positions)
{
    clear_error();
    CHECK(check_calc(calc));
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    if (n_atoms == 0) return SOAP_OK;
    size_t es = elem_size(precision);
    CHECK(check_pairs(species, pair_offsets, pair_j, pair_vec, pair_capacity, es));
    if (pair_capacity > 0) {
        CHECK(check_ptr(pair_transpose, 4, "pair_transpose"));
        CHECK(check_ptr(grad_pair_vec, es, "grad_pair_vec"));
    }
    CHECK(check_ptr(grad_coeffs, es, "grad_coeffs"));
    CHECK(check_ptr(grad_positions, es, "grad_positions"));
    const DeviceTables* t = nullptr;
    CHECK(device_tables(calc, &t));
    FeatureArgs a = base_args(calc, exec, precision == SOAP_F64, t);
    a.n_atoms = n_atoms;
    a.species = species;
    a.pair_offsets = pair_offsets;
    a.pair_j = pair_j;
    a.pair_vec = pair_vec;
    a.pair_capacity = pair_capacity;
    return launched(launch_expansion_backward(a, precision == SOAP_F64, pair_transpose, grad_coeffs, grad_pair_vec,
                                              grad_positions, stream_of(exec)),
                    "expansion backward");
}


soap_status soap_virial(const soap_exec* exec, soap_precision precision, int32_t n_structures,
                        const int64_t* atom_offsets, int64_t n_atoms, const int64_t* pair_offsets,
                        const void* pair_vec, const void* grad_pair_vec, int64_t pair_capacity,
                        void* centre_partials, void* virial)
{
    clear_error();
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_structures >= 0, "n_structures must be >= 0");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE(pair_capacity >= 0, "pair_capacity must be >= 0");
    if (n_structures == 0) return SOAP_OK;
    const size_t es = elem_size(precision);
    CHECK(check_ptr(atom_offsets, 8, "atom_offsets"));
    CHECK(check_ptr(virial, es, "virial"));
    if (n_atoms > 0) {
        CHECK(check_ptr(pair_offsets, 8, "pair_offsets"));
        CHECK(check_ptr(centre_partials, es, "centre_partials"));
        if (pair_capacity > 0) {
            CHECK(check_ptr(pair_vec, es, "pair_vec"));
            CHECK(check_ptr(grad_pair_vec, es, "grad_pair_vec"));
        }
    }
    return launched(launch_virial(precision == SOAP_F64, n_structures, atom_offsets, n_atoms, pair_offsets, pair_vec,
                                  grad_pair_vec, pair_capacity, centre_partials, virial, status_of(exec),
                                  stream_of(exec)),
                    "virial");
}

soap_status soap_power_spectrum_selected(const soap_exec* exec, soap_precision precision, int64_t n_atoms,
                                         int32_t n_channels, int32_t lmax, const void* coeffs, int64_t n_selected,
                                         const int32_t* selected, void* p_selected)
{
    clear_error();
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE(n_channels >= 1, "n_channels must be >= 1");
    REQUIRE(lmax >= 0 && lmax <= 12, "lmax must be in [0, 12]");
    REQUIRE(n_selected >= 0 && n_selected < (int64_t(1) << 31), "n_selected must be in [0, 2^31)");
    const bool f64 = precision == SOAP_F64;
    REQUIRE(power_spectrum_selected_lds(f64, n_channels, lmax) <= 160 * 1024,
            "one centre's coefficients (%zu bytes) must fit 160 KB of LDS",
            power_spectrum_selected_lds(f64, n_channels, lmax));
    if (n_atoms == 0 || n_selected == 0) return SOAP_OK;
    const size_t es = elem_size(precision);
    CHECK(check_ptr(coeffs, es, "coeffs"));
    CHECK(check_ptr(selected, 4, "selected"));
    CHECK(check_ptr(p_selected, es, "p_selected"));
    return launched(launch_power_spectrum_selected(f64, n_atoms, n_channels, lmax, coeffs, n_selected, selected,
                                                   p_selected, status_of(exec), stream_of(exec)),
                    "power_spectrum_selected");
}

soap_status soap_power_spectrum_selected_plan(int32_t n_channels, int32_t lmax, int64_t n_selected,
                                              const int32_t* selected, int32_t* row_offsets, int32_t* entries)
{
    clear_error();
    REQUIRE(n_channels >= 1, "n_channels must be >= 1");
    REQUIRE(lmax >= 0 && lmax <= 12, "lmax must be in [0, 12]");
    REQUIRE(n_selected >= 0 && n_selected < (int64_t(1) << 29), "n_selected must be in [0, 2^29)");
    REQUIRE(row_offsets != nullptr, "row_offsets must not be NULL");
    if (n_selected > 0) {
        REQUIRE(selected != nullptr && entries != nullptr, "selected and entries must not be NULL");
        for (int64_t q = 0; q < n_selected; ++q) {
            const int k1 = selected[3 * q], k2 = selected[3 * q + 1], l = selected[3 * q + 2];
            REQUIRE(k1 >= 0 && k1 < n_channels && k2 >= 0 && k2 < n_channels && l >= 0 && l <= lmax,
                    "selected[%lld] = (%d, %d, %d) is out of range", (long long)q, k1, k2, l);
        }
    }
    selected_backward_plan(n_channels, lmax, n_selected, selected, row_offsets, entries);
    return SOAP_OK;
}

soap_status soap_power_spectrum_selected_backward(const soap_exec* exec, soap_precision precision, int64_t n_atoms,
                                                  int32_t n_channels, int32_t lmax, const void* coeffs,
                                                  int64_t n_selected, const void* grad_p_selected,
                                                  const int32_t* row_offsets, const int32_t* entries,
                                                  void* grad_coeffs)
{
    clear_error();
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE(n_channels >= 1, "n_channels must be >= 1");
    REQUIRE(lmax >= 0 && lmax <= 12, "lmax must be in [0, 12]");
    REQUIRE(n_selected >= 0 && n_selected < (int64_t(1) << 29), "n_selected must be in [0, 2^29)");
    const bool f64 = precision == SOAP_F64;
    const size_t lds = power_spectrum_selected_backward_lds(f64, n_channels, lmax, n_selected);
    REQUIRE(lds <= 160 * 1024, "one centre's coefficients and gradient row (%zu bytes) must fit 160 KB of LDS", lds);
    if (n_atoms == 0) return SOAP_OK;
    const size_t es = elem_size(precision);
    CHECK(check_ptr(coeffs, es, "coeffs"));
    CHECK(check_ptr(grad_coeffs, es, "grad_coeffs"));
    CHECK(check_ptr(row_offsets, 4, "row_offsets"));
    if (n_selected > 0) {
        CHECK(check_ptr(grad_p_selected, es, "grad_p_selected"));
        CHECK(check_ptr(entries, 4, "entries"));
    }
    return launched(launch_power_spectrum_selected_backward(f64, n_atoms, n_channels, lmax, coeffs, n_selected,
                                                            grad_p_selected, row_offsets, entries, grad_coeffs,
                                                            status_of(exec), stream_of(exec)),
                    "power_spectrum_selected_backward");
}

soap_status soap_gpr_workspace_size(soap_precision precision, int64_t n_centres, int64_t n_features,
                                    int64_t n_active, size_t* bytes)
{
    clear_error();
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_centres >= 0 && n_centres < (int64_t(1) << 31), "n_centres must be in [0, 2^31)");
    REQUIRE(n_features >= 1 && n_features <= 64 * int64_t(65535), "n_features must be in [1, 4194240]");
    REQUIRE(n_active >= 1 && n_active <= 64 * int64_t(65535), "n_active must be in [1, 4194240]");
    REQUIRE(bytes != nullptr, "bytes must not be NULL");
    if (alloc_failure_forced()) return fail(SOAP_ENOMEM, "allocation failure forced by SOAP_FAIL_ALLOC");
    *bytes = gpr_workspace_bytes(precision == SOAP_F64, n_centres, n_features, n_active);
    return SOAP_OK;
}

soap_status soap_gpr_predict(const soap_exec* exec, soap_precision precision, int64_t n_centres, int64_t n_features,
                             const int32_t* centre_species, const void* features, int64_t n_active,
                             const int32_t* active_species, const void* active_features, const void* weights,
                             int32_t zeta, void* workspace, size_t workspace_bytes, void* energies,
                             void* grad_features)
{
    clear_error();
    REQUIRE(precision == SOAP_F64 || precision == SOAP_F32, "precision must be SOAP_F64 or SOAP_F32");
    REQUIRE(n_centres >= 0 && n_centres < (int64_t(1) << 31), "n_centres must be in [0, 2^31)");
    // column tiles of 64 run along the grid's y dimension (at most 65535)
    REQUIRE(n_features >= 1 && n_features <= 64 * int64_t(65535), "n_features must be in [1, 4194240]");
    REQUIRE(n_active >= 1 && n_active <= 64 * int64_t(65535), "n_active must be in [1, 4194240]");
    REQUIRE(zeta >= 1 && zeta <= 64, "zeta must be in [1, 64]");
    if (n_centres == 0) return SOAP_OK;
    const bool f64 = precision == SOAP_F64;
    const size_t es = elem_size(precision);
    const size_t need = gpr_workspace_bytes(f64, n_centres, n_features, n_active);
    REQUIRE(workspace_bytes >= need, "workspace_bytes (%zu) is below the %zu bytes needed", workspace_bytes, need);
    CHECK(check_ptr(centre_species, 4, "centre_species"));
    CHECK(check_ptr(features, es, "features"));
    CHECK(check_ptr(active_species, 4, "active_species"));
    CHECK(check_ptr(active_features, es, "active_features"));
    CHECK(check_ptr(weights, es, "weights"));
    CHECK(check_ptr(workspace, es, "workspace"));
    CHECK(check_ptr(energies, es, "energies"));
    CHECK(check_ptr(grad_features, es, "grad_features", true));
    return launched(launch_gpr_predict(f64, n_centres, n_features, centre_species, features, n_active, active_species,
                                       active_features, weights, zeta, workspace, energies, grad_features,
                                       stream_of(exec)),
                    "gpr_predict");
}

soap_status soap_compress_n_params(const soap_calculator* calc, int32_t n_out, int32_t hidden, int64_t* n_params)
{
    clear_error();
    CHECK(check_compress(calc, n_out, hidden));
    REQUIRE(n_params != nullptr, "n_params must not be NULL");
    *n_params = compress_params(calc, n_out, hidden);
    return SOAP_OK;
}

// ------------------------------------------------ compression checkpoint
// File: "SOAPCMP1", then int32 version, n_out, hidden, channels, lmax,
// reserved (0), int64 step, n_params, the three float arrays (weights,
// Adam m, Adam v), and the FNV-1a 64-bit hash of everything before it.
// Little-endian, as the host writes it.
namespace {

constexpr char kCkptMagic[8] = {'S', 'O', 'A', 'P', 'C', 'M', 'P', '1'};
constexpr int32_t kCkptVersion = 1;

struct CkptHeader {
    char magic[8];
    int32_t version, n_out, hidden, channels, lmax, reserved;
    int64_t step, n_params;
};

uint64_t fnv1a(const void* data, size_t n, uint64_t h)
{
    const unsigned char* b = static_cast<const unsigned char*>(data);
    for (size_t k = 0; k < n; ++k) {
        h ^= b[k];
        h *= 1099511628211ull;
    }
    return h;
}

constexpr uint64_t kFnvBasis = 14695981039346656037ull;

}  // namespace

soap_status soap_compress_save(const soap_calculator* calc, int32_t n_out, int32_t hidden, int64_t step,
                               const float* weights, const float* adam_m, const float* adam_v, const char* path)
{
    clear_error();
    CHECK(check_compress(calc, n_out, hidden));
    REQUIRE(path != nullptr && path[0] != '\0', "path must be a file name");
    REQUIRE(step >= 0, "step must be >= 0");
    CHECK(check_ptr(weights, 4, "weights"));
    CHECK(check_ptr(adam_m, 4, "adam_m"));
    CHECK(check_ptr(adam_v, 4, "adam_v"));
    const int64_t n = compress_params(calc, n_out, hidden);
    std::vector<float> host(size_t(3 * n));
    const float* src[3] = {weights, adam_m, adam_v};
    for (int a = 0; a < 3; ++a)
        if (hipMemcpy(host.data() + a * n, src[a], size_t(n) * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(SOAP_EDEVICE, "copy of the compression state to the host failed");
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = kCkptVersion;
    h.n_out = n_out;
    h.hidden = hidden;
    h.channels = calc->K;
    h.lmax = calc->h.lmax;
    h.step = step;
    h.n_params = n;
    uint64_t hash = fnv1a(&h, sizeof(h), kFnvBasis);
    hash = fnv1a(host.data(), host.size() * 4, hash);
    // written to a temporary name, then renamed over the target
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(SOAP_EINVAL, "cannot open %s for writing", tmp.c_str());
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(host.data(), 4, host.size(), f) == host.size() &&
              std::fwrite(&hash, sizeof(hash), 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(SOAP_EINVAL, "writing %s failed", path);
    }
    return SOAP_OK;
}

soap_status soap_compress_load(const soap_calculator* calc, int32_t n_out, int32_t hidden, const char* path,
                               float* weights, float* adam_m, float* adam_v, int64_t* step)
{
    clear_error();
    CHECK(check_compress(calc, n_out, hidden));
    REQUIRE(path != nullptr && path[0] != '\0', "path must be a file name");
    REQUIRE(step != nullptr, "step must not be NULL");
    CHECK(check_ptr(weights, 4, "weights"));
    CHECK(check_ptr(adam_m, 4, "adam_m"));
    CHECK(check_ptr(adam_v, 4, "adam_v"));
    const int64_t n = compress_params(calc, n_out, hidden);
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SOAP_EINVAL, "cannot open %s", path);
    CkptHeader h{};
    std::vector<float> host;
    uint64_t hash = 0;
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1;
    if (ok && std::memcmp(h.magic, kCkptMagic, 8) != 0) {
        std::fclose(f);
        return fail(SOAP_EINVAL, "%s is not a compression checkpoint", path);
    }
    if (ok && (h.version != kCkptVersion || h.n_out != n_out || h.hidden != hidden || h.channels != calc->K ||
               h.lmax != calc->h.lmax || h.n_params != n || h.step < 0 || h.reserved != 0)) {
        std::fclose(f);
        return fail(SOAP_EINVAL,
                    "%s holds version %d, (n_out, hidden, channels, lmax) = (%d, %d, %d, %d); expected version %d, "
                    "(%d, %d, %d, %d)",
                    path, h.version, h.n_out, h.hidden, h.channels, h.lmax, kCkptVersion, n_out, hidden, calc->K,
                    calc->h.lmax);
    }
    if (ok) {
        host.resize(size_t(3 * n));
        ok = std::fread(host.data(), 4, host.size(), f) == host.size() && std::fread(&hash, sizeof(hash), 1, f) == 1;
        char extra;
        ok = ok && std::fread(&extra, 1, 1, f) == 0;   // nothing after the hash
    }
    std::fclose(f);
    if (!ok) return fail(SOAP_EINVAL, "%s is truncated or has trailing data", path);
    uint64_t want = fnv1a(&h, sizeof(h), kFnvBasis);
    want = fnv1a(host.data(), host.size() * 4, want);
    if (want != hash) return fail(SOAP_EINVAL, "%s is corrupted (hash mismatch)", path);
    float* dst[3] = {weights, adam_m, adam_v};
    for (int a = 0; a < 3; ++a)
        if (hipMemcpy(dst[a], host.data() + a * n, size_t(n) * 4, hipMemcpyHostToDevice) != hipSuccess)
            return fail(SOAP_EDEVICE, "copy of the compression state to the device failed");
    *step = h.step;
    return SOAP_OK;
}

soap_status soap_compress_workspace_size(const soap_calculator* calc, int32_t n_out, int32_t hidden, size_t* bytes)
{
    clear_error();
    CHECK(check_compress(calc, n_out, hidden));
    REQUIRE(bytes != nullptr, "bytes must not be NULL");
    if (alloc_failure_forced()) return fail(SOAP_ENOMEM, "allocation failure forced by SOAP_FAIL_ALLOC");
    *bytes = compress_workspace(calc, n_out, hidden);
    return SOAP_OK;
}

soap_status soap_compress_init_pca(const soap_calculator* calc, const soap_exec* exec, int32_t n_out, int32_t hidden,
                                   int64_t n_atoms, const float* coeffs, uint64_t seed, float noise, void* workspace,
                                   size_t workspace_bytes, float* weights)
{
    clear_error();
    CHECK(check_compress(calc, n_out, hidden));
    REQUIRE(n_atoms >= 1 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [1, 2^31)");
    REQUIRE(n_out <= calc->K, "n_out (%d) must not exceed the %d input channels", n_out, calc->K);
    REQUIRE(n_out <= hidden, "n_out (%d) must not exceed hidden (%d)", n_out, hidden);
    REQUIRE(std::isfinite(noise) && noise >= 0.0f, "noise must be finite and >= 0");
    CHECK(check_ptr(coeffs, 4, "coeffs"));
    CHECK(check_ptr(weights, 4, "weights"));
    CHECK(check_ptr(workspace, 256, "workspace"));
    REQUIRE(workspace_bytes >= compress_workspace(calc, n_out, hidden), "workspace too small");
    CompressArgs a = compress_args(calc, exec, n_out, hidden, n_atoms);
    a.c = coeffs;
    float* part = static_cast<float*>(workspace);
    CHECK(launched(launch_channel_cov(a, part, kCovSlices, stream_of(exec)), "channel covariance"));
    const int K = calc->K, lm1 = calc->h.lmax + 1, Q = n_out, H = hidden;
    std::vector<float> hp(size_t(kCovSlices) * lm1 * K * K);
    hipStream_t st = stream_of(exec);
    if (hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(SOAP_EDEVICE, "copy of the channel covariance failed");
    SplitMix rng{seed};
    std::vector<float> w(size_t(compress_params(calc, Q, H)));
    size_t o = 0;
    for (int l = 0; l < lm1; ++l) {
        std::vector<double> C(size_t(K) * K, 0.0), ev, U;
        for (int s = 0; s < kCovSlices; ++s)
            for (int e = 0; e < K * K; ++e) C[e] += hp[(size_t(s) * lm1 + l) * K * K + e];
        for (int r = 0; r < K; ++r)   // symmetrise the float partial sums
            for (int q = r + 1; q < K; ++q) C[r * K + q] = C[q * K + r] = 0.5 * (C[r * K + q] + C[q * K + r]);
        sym_eigen(K, C, ev, U);
        std::vector<int> order(K);
        for (int k = 0; k < K; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ev[x] > ev[y]; });
        for (int q = 0; q < H; ++q)           // W1_l [H][K]
            for (int k = 0; k < K; ++k)
                w[o + size_t(q) * K + k] =
                    q < Q ? float(U[size_t(k) * K + order[q]]) : float(noise * rng.normal() / std::sqrt(double(K)));
        o += size_t(H) * K;
        for (int p = 0; p < Q; ++p)           // W2_l [Q][H]
            for (int q = 0; q < H; ++q)
                w[o + size_t(p) * H + q] =
                    q < Q ? (p == q ? 1.0f : 0.0f) : float(noise * rng.normal() / std::sqrt(double(H)));
        o += size_t(Q) * H;
        for (int q = 0; q < 2 * H; ++q) w[o + q] = 0.0f;   // alpha_l, beta_l
        o += 2 * size_t(H);
    }
    if (hipMemcpyAsync(weights, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(SOAP_EDEVICE, "upload of the initial weights failed");
    return SOAP_OK;
}

soap_status soap_compress_forward(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                                  int32_t n_out, int32_t hidden, int64_t n_atoms, const float* weights,
                                  const float* coeffs, float* coeffs_out, float* p_out)
{
    clear_error();
    CHECK(check_compress(calc, n_out, hidden));
    REQUIRE(precision == SOAP_F32 || precision == SOAP_BF16_F32ACC, "precision must be SOAP_F32 or SOAP_BF16_F32ACC");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE(coeffs_out != nullptr || p_out != nullptr, "coeffs_out and p_out must not both be NULL");
    if (n_atoms == 0) return SOAP_OK;
    CHECK(check_ptr(weights, 4, "weights"));
    CHECK(check_ptr(coeffs, 4, "coeffs"));
    CHECK(check_ptr(coeffs_out, 4, "coeffs_out", true));
    CHECK(check_ptr(p_out, 4, "p_out", true));
    CompressArgs a = compress_args(calc, exec, n_out, hidden, n_atoms);
    a.w = weights;
    a.c = coeffs;
    a.ct = coeffs_out;
    a.pt = p_out;
    if (precision == SOAP_BF16_F32ACC)
        return launched(launch_compress_forward_bf16(a, stream_of(exec)), "compression (bf16)");
    return launched(launch_compress_forward(a, stream_of(exec)), "compression");
}

soap_status soap_compress_forward_ws(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                                     int32_t n_out, int32_t hidden, int64_t n_atoms, const float* weights,
                                     const float* coeffs, float* coeffs_out, float* p_out, void* workspace,
                                     size_t workspace_bytes)
{
    clear_error();
    CHECK(check_compress(calc, n_out, hidden));
    REQUIRE(precision == SOAP_F32 || precision == SOAP_BF16_F32ACC, "precision must be SOAP_F32 or SOAP_BF16_F32ACC");
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    REQUIRE(coeffs_out != nullptr || p_out != nullptr, "coeffs_out and p_out must not both be NULL");
    if (n_atoms == 0) return SOAP_OK;
    CHECK(check_ptr(weights, 4, "weights"));
    CHECK(check_ptr(coeffs, 4, "coeffs"));
    CHECK(check_ptr(coeffs_out, 4, "coeffs_out", true));
    CHECK(check_ptr(p_out, 4, "p_out", true));
    CHECK(check_ptr(workspace, 256, "workspace"));
    REQUIRE(workspace_bytes >= compress_workspace(calc, n_out, hidden), "workspace too small");
    CompressArgs a = compress_args(calc, exec, n_out, hidden, n_atoms);
    a.w = weights;
    a.c = coeffs;
    a.ct = coeffs_out;
    a.pt = p_out;
    if (precision == SOAP_BF16_F32ACC) {
        if (compress_image_bytes(calc->K, n_out, hidden, calc->h.lmax) > 0) a.img = workspace;
        return launched(launch_compress_forward_bf16(a, stream_of(exec)), "compression (bf16)");
    }
    return launched(launch_compress_forward(a, stream_of(exec)), "compression");
}

soap_status soap_compress_backward(const soap_calculator* calc, const soap_exec* exec, int32_t n_out, int32_t hidden,
                                   int64_t n_atoms, const float* weights, const float* coeffs, const float* grad_p,
                                   void* workspace, size_t workspace_bytes, float* grad_weights)
{
    clear_error();
    CHECK(check_compress(calc, n_out, hidden));
    REQUIRE(n_atoms >= 0 && n_atoms < (int64_t(1) << 31), "n_atoms must be in [0, 2^31)");
    CHECK(check_ptr(weights, 4, "weights"));
    CHECK(check_ptr(coeffs, 4, "coeffs", n_atoms == 0));
    CHECK(check_ptr(grad_p, 4, "grad_p", n_atoms == 0));
    CHECK(check_ptr(grad_weights, 4, "grad_weights"));
    CHECK(check_ptr(workspace, 256, "workspace"));
    REQUIRE(workspace_bytes >= compress_workspace(calc, n_out, hidden), "workspace too small");
    CompressArgs a = compress_args(calc, exec, n_out, hidden, n_atoms);
    a.w = weights;
    a.c = coeffs;
    a.gpt = grad_p;
    a.gpart = static_cast<float*>(workspace);
    return launched(launch_compress_backward(a, grad_weights, stream_of(exec)), "compression backward");
}

soap_status soap_spectrum_gram(const soap_exec* exec, int32_t n, int32_t n_channels, int32_t lmax, const float* X,
                               float* K)
{
    clear_error();
    REQUIRE(n >= 0 && n <= 65536, "n must be in [0, 65536]");
    REQUIRE(n_channels >= 1 && n_channels <= 4096, "n_channels must be in [1, 4096]");
    REQUIRE(lmax >= 0 && lmax <= 12, "lmax must be in [0, 12]");
    if (n == 0) return SOAP_OK;
    CHECK(check_ptr(X, 4, "X"));
    CHECK(check_ptr(K, 4, "K"));
    return launched(launch_spectrum_gram(n, n_channels, lmax, X, K, stream_of(exec)), "spectrum gram");
}

soap_status soap_spectrum_kernel_loss(const soap_exec* exec, int32_t n, int32_t n_channels, int32_t lmax,
                                      const float* X, const float* Kref, float* work, float* loss, float* grad_X)
{
    clear_error();
    REQUIRE(n >= 1 && n <= 65536, "n must be in [1, 65536]");
    REQUIRE(n_channels >= 1 && n_channels <= 4096, "n_channels must be in [1, 4096]");
    REQUIRE(lmax >= 0 && lmax <= 12, "lmax must be in [0, 12]");
    CHECK(check_ptr(X, 4, "X"));
    CHECK(check_ptr(Kref, 4, "Kref"));
    CHECK(check_ptr(work, 4, "work"));
    CHECK(check_ptr(loss, 4, "loss"));
    CHECK(check_ptr(grad_X, 4, "grad_X"));
    return launched(launch_spectrum_kernel_loss(n, n_channels, lmax, X, Kref, work, loss, work + int64_t(n) * n,
                                                grad_X, stream_of(exec)),
                    "kernel loss");
}

soap_status soap_adam_step(const soap_exec* exec, int64_t n, float* params, const float* grads, float* m, float* v,
                           float lr, float beta1, float beta2, float eps, int32_t step)
{
    clear_error();
    REQUIRE(n >= 0, "n must be >= 0");
    REQUIRE(step >= 1, "step counts from 1");
    REQUIRE(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f, "betas must be in [0, 1)");
    REQUIRE(std::isfinite(lr) && std::isfinite(eps) && eps > 0.0f, "lr and eps must be finite, eps > 0");
    if (n == 0) return SOAP_OK;
    CHECK(check_ptr(params, 4, "params"));
    CHECK(check_ptr(grads, 4, "grads"));
    CHECK(check_ptr(m, 4, "m"));
    CHECK(check_ptr(v, 4, "v"));
    return launched(launch_adam(n, params, grads, m, v, lr, beta1, beta2, eps, step, stream_of(exec)), "adam");
}

soap_status soap_read_device_status(const soap_exec* exec)
{
    clear_error();
    hipError_t e = hipStreamSynchronize(stream_of(exec));
    if (e != hipSuccess) return fail(SOAP_EDEVICE, "stream synchronisation failed: %s", hipGetErrorString(e));
    if (!exec || !exec->dev_status) return SOAP_OK;
    int32_t v = 0;
    e = hipMemcpy(&v, exec->dev_status, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(SOAP_EDEVICE, "status read failed: %s", hipGetErrorString(e));
    if (v != 0) fail(soap_status(v), "device reported status %d", v);
    return soap_status(v);
}

}  // extern "C"
