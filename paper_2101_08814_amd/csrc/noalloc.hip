// Neighbour list for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// soap_compute_neighbors_noalloc is soap_compute_neighbors with its
// workspace taken from a file-scope device array instead of a caller
// buffer.  The array is resolved once per device, with that device current,
// through hipGetSymbolAddress; the address found there is what the kernels
// receive (the array's name is only a host-side stand-in).  Every call on a
// device shares that device's array, so calls that overlap on one device
// race.  The neighbour kernels write every workspace entry they read within
// the same call (bin counters are cleared by a fill kernel, not a memset),
// so nothing has to be cleared between calls.
#include <mutex>

#include "soap_internal.hpp"

namespace {

constexpr size_t kScratchBytes = SOAP_NEIGHBORS_NOALLOC_BYTES;   // 16 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
soap_status scratch_address(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return soap::fail(SOAP_EDEVICE, "no HIP device available");
    if (dev < 0 || dev >= kMaxDevices) return soap::fail(SOAP_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return soap::fail(SOAP_EDEVICE, "address of the static neighbour scratch on device %d: %s", dev,
                              hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SOAP_OK;
}

}  // namespace

extern "C" {

soap_status soap_compute_neighbors_noalloc(const soap_calculator* calc, const soap_exec* exec, int32_t n_structures,
                                           int64_t n_atoms, const int64_t* atom_offsets, const double* cells,
                                           const uint8_t* pbc, const double* positions, const int32_t* species,
                                           int64_t capacity, soap_precision vec_precision, int64_t* pair_offsets,
                                           int32_t* pair_j, int32_t* pair_shift, void* pair_vec,
                                           int32_t* pair_transpose)
{
    soap::clear_error();
    if (n_structures < 0) return soap::fail(SOAP_EINVAL, "n_structures must be >= 0 (got %d)", n_structures);
    if (n_atoms < 0 || n_atoms >= (int64_t(1) << 31)) return soap::fail(SOAP_EINVAL, "n_atoms must be in [0, 2^31)");
    const size_t need = soap::neighbors_workspace_bytes(n_structures, n_atoms);
    if (need > kScratchBytes)
        return soap::fail(SOAP_EINVAL,
                          "%d structures with %lld atoms need %zu bytes of neighbour scratch; the static scratch "
                          "holds %zu (use soap_compute_neighbors with a caller workspace)",
                          n_structures, (long long)n_atoms, need, kScratchBytes);
    if (!calc) return soap::fail(SOAP_EINVAL, "calculator must not be NULL");
    void* ws = nullptr;
    soap_status st = scratch_address(&ws);
    if (st != SOAP_OK) return st;
    return soap_compute_neighbors(calc, exec, n_structures, n_atoms, atom_offsets, cells, pbc, positions, species, ws,
                                  kScratchBytes, capacity, vec_precision, pair_offsets, pair_j, pair_shift, pair_vec,
                                  pair_transpose);
}

}  // extern "C"
