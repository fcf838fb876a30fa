// Internal declarations shared by the host side of the library and the
// kernel launchers.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "radial_exact.hpp"
#include "soap_mi355x.h"

namespace soap {

// Tables of one calculator on one device.
struct DeviceTables {
    bool ready = false;
    double* coef64 = nullptr;    // [M][nmax][lmax+1][4] local-t cubic coefficients
    float* coef32 = nullptr;
    double* coef64_ln = nullptr; // the same cubics reordered [M][lmax+1][nmax][4], 32 zero cubics past the end
    float* coef32_ln = nullptr;
    double* center64 = nullptr;  // [nmax] I~_n0(0) Y_00, then [L2] harmonic normalisations K_lm
    float* center32 = nullptr;
    int32_t* dp_pos = nullptr;   // [lmax+1][K(K+1)/2]: l | k1 << 4 | k2 << 14 of each dp row position
    int32_t* radial_dst = nullptr; // [nl + 16]: LDS offset l np + n of radial value j = l nmax + n
                                   // (np = nmax rounded up to 4; entries past nl repeat the last)
    double* exact = nullptr;       // constants of the direct radial integral (see ExactRadial)
    rad::GtoTables gto{};          // views into `exact` (device pointers)
    rad::DvrTables dvr{};
};

// Geometry of one structure for the neighbour search (built on the device
// from the caller's cells, pbc flags and atom offsets).
struct StructGeom {
    double H[9];        // rows are lattice vectors h1, h2, h3 (identity if no pbc)
    double Hinv[9];     // inverse of H: fractional f = r . Hinv
    int32_t nbin[3];    // bins per axis (1 on non-periodic axes)
    int32_t reach[3];   // stencil half-width in bins per axis (0 on non-periodic axes)
    int32_t pbc[3];
    int32_t pad0;
    int64_t atom_lo, atom_hi;
    int64_t bin_lo;     // first global bin of this structure
    int64_t pad1;
};

// Constants of the direct (unsplined) radial integral of a calculator: GTO
// (alpha, pref, the four restricted 1F1 of the top degrees per n, S^-1/2)
// or DVR (points x and amplitudes A = 4 pi x sqrt(w)).
struct ExactRadial {
    int basis = 0, nmax = 0, lmax = 0;
    double c = 0.0;
    std::vector<double> alpha, pref, X;
    std::vector<rad::GParams> top;
    std::vector<double> x, A;
};

}  // namespace soap

struct soap_calculator {
    soap_hypers h;
    int L2 = 0, K = 0, nl = 0;
    int64_t KK = 0;
    int64_t M = 0;
    double delta = 0.0, inv_delta = 0.0;
    std::vector<double> coef64;       // host copy of the FP64 table
    std::vector<float> coef32;
    std::vector<double> center;       // [nmax] centre terms, then [L2] K_lm
    std::vector<double> orth;         // S^{-1/2}, [nmax][nmax] (identity for DVR)
    soap::ExactRadial exact;          // constants of the direct radial integral
    soap_table_info info{};
    mutable std::mutex mu;
    mutable std::vector<soap::DeviceTables> dev;
};

namespace soap {

// error reporting (thread-local message)
soap_status fail(soap_status st, const char* fmt, ...);
void clear_error();
bool alloc_failure_forced();   // SOAP_FAIL_ALLOC=1 in the environment

// tables.cpp
soap_status build_tables(soap_calculator* calc);
void radial_exact(const soap_calculator* calc, int64_t n, const double* r, double* I, double* dI);
void build_exact_radial(const soap_hypers& h, const std::vector<double>& orth, ExactRadial& e);
void exact_radial_eval(const ExactRadial& e, double r, double* I, double* dI);
void radial_spline_host(const soap_calculator* calc, double r, double* I, double* dI);
soap_status device_tables(const soap_calculator* calc, const DeviceTables** out);
// symmetric eigen-decomposition A = Q diag(w) Q^T of a small dense matrix
// (row-major n x n; column k of Q is the eigenvector of w[k])
void sym_eigen(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& Q);

// launchers (kernels in the .hip files); each returns a hipError_t
struct FeatureArgs {
    int S, nmax, lmax, include_center;
    double rcut, width;
    int64_t M;
    double inv_delta;
    int64_t n_atoms;
    const int32_t* species;
    const int64_t* pair_offsets;
    const int32_t* pair_j;
    const void* pair_vec;
    int64_t pair_capacity;
    const void* coef;       // table of the working precision
    const void* coef_ln;    // the same table in [M][lmax+1][nmax] order
    const void* center;     // [nmax] centre terms, then [L2] harmonic normalisations
    const int32_t* dp_pos;  // (l, k1, k2) of each position of a dp row, packed; NULL if K > 1023
    const int32_t* radial_dst;  // LDS offset of each radial value in the padded [l][np] rows
    void* coeffs;
    void* p;
    void* dcoeffs;
    void* dcoeffs_self;
    void* dp;
    void* dp_self;
    int32_t* status;
};

hipError_t launch_features(const FeatureArgs& a, bool f64, hipStream_t stream);
// c, p, self rows and pair rows with each pair staged once (hipErrorNotSupported
// when the layout does not fit)
hipError_t launch_features_rows(const FeatureArgs& a, bool f64, hipStream_t stream);

// radial integrals of a batch of radii on the device (spline or direct)
struct RadialArgs {
    int nmax, lmax, basis;
    bool exact;
    int64_t M;
    double inv_delta;
    const void* coef;         // spline table [M][nl][4] of the output precision
    rad::GtoTables gto;
    rad::DvrTables dvr;
    int64_t n_r;
    const double* r;
    void* I;
    void* dI;
};
hipError_t launch_radial(const RadialArgs& a, bool f64, hipStream_t stream);

// Per-wave LDS layout of the one-lane-per-pair expansion (elements of T):
// ch pairs of radial rows [lmax+1][np] and harmonic rows [l2s], and the
// species blocks of c as [np/4][L2][4] (cb elements each): one buffer, or
// with the power spectrum all S of them (an LDS copy of c_i).
struct LaneLayout {
    int ch, np, nls, l2s, rs, ys, sp, cb, cs, total;
};
LaneLayout choose_lane_layout(int S, int nmax, int lmax, bool want_p, size_t elem);
// c (and p when a.p is set) with one lane per pair; hipErrorNotSupported
// when the layout does not fit
hipError_t launch_expansion_lanes(const FeatureArgs& a, bool f64, hipStream_t stream);
// c alone with the pairs of several centres packed into each wave's
// chunks; hipErrorNotSupported when p is asked for or the layout does not fit
struct PackLayout {
    int G, gmax, total, cpw;
};
hipError_t launch_expansion_packed(const FeatureArgs& a, bool f64, hipStream_t stream);
// per-pair dL/dr_ji of the adjoint with one lane per pair
bool expansion_backward_lanes_fits(const FeatureArgs& a, bool f64);
hipError_t launch_expansion_backward_lanes(const FeatureArgs& a, bool f64, const void* grad_c, void* grad_pair,
                                           hipStream_t stream);
hipError_t launch_gradient_rows(const FeatureArgs& a, bool f64, hipStream_t stream);
hipError_t launch_power_spectrum(const FeatureArgs& a, soap_precision prec, hipStream_t stream);
hipError_t launch_power_spectrum_valu(const FeatureArgs& a, bool f64, hipStream_t stream);
hipError_t launch_power_spectrum_backward(const FeatureArgs& a, bool f64, const void* grad_p,
                                          void* grad_coeffs, hipStream_t stream);
size_t power_spectrum_selected_lds(bool f64, int K, int lmax);
hipError_t launch_power_spectrum_selected(bool f64, int64_t n, int K, int lmax, const void* c, int64_t n_sel,
                                          const int32_t* sel, void* out, int32_t* status, hipStream_t stream);
size_t power_spectrum_selected_backward_lds(bool f64, int K, int lmax, int64_t n_sel);
void selected_backward_plan(int K, int lmax, int64_t n_sel, const int32_t* selected, int32_t* row_offsets,
                            int32_t* entries);
hipError_t launch_power_spectrum_selected_backward(bool f64, int64_t n, int K, int lmax, const void* c,
                                                   int64_t n_sel, const void* grad, const int32_t* row_offsets,
                                                   const int32_t* entries, void* grad_c, int32_t* status,
                                                   hipStream_t stream);
size_t gpr_workspace_bytes(bool f64, int64_t n, int64_t n_feat, int64_t n_active);
hipError_t launch_gpr_predict(bool f64, int64_t n, int64_t n_feat, const int32_t* species, const void* p,
                              int64_t n_active, const int32_t* active_species, const void* m, const void* w,
                              int zeta, void* workspace, void* energies, void* grad, hipStream_t stream);
hipError_t launch_virial(bool f64, int32_t n_structures, const int64_t* atom_offsets, int64_t n_atoms,
                         const int64_t* pair_offsets, const void* pair_vec, const void* grad_pair_vec,
                         int64_t capacity, void* partials, void* virial, int32_t* status, hipStream_t stream);
hipError_t launch_expansion_backward(const FeatureArgs& a, bool f64, const int32_t* pair_transpose,
                                     const void* grad_coeffs, void* grad_pair_vec,
                                     void* grad_positions, hipStream_t stream);

struct CompressArgs {
    int K, Q, H, lmax;         // channels in, out, hidden; degree
    int64_t n;                 // centres
    int64_t n_params;          // (lmax+1) (H K + Q H + 2 H)
    const float* w;            // weights: per l W1 [H][K], W2 [Q][H], alpha [H], beta [H]
    const float* c;            // [n][K][L2]
    float* ct;                 // [n][Q][L2] or NULL
    float* pt;                 // [n][lmax+1][Q(Q+1)/2] or NULL
    const float* gpt;          // backward: dL/dpt, same layout as pt
    float* gpart;              // backward: per-slice partial gradients [slices][n_params]
    int slices;
    int32_t* status;
    void* img;                 // bfloat16 forward: LDS image of every l's weights (device workspace) or NULL
};

// bytes of the weight image of the bfloat16 forward (0 when its shapes do
// not take one)
size_t compress_image_bytes(int K, int Q, int H, int lmax);
size_t compress_fwd_lds(const CompressArgs& a);
size_t compress_bwd_lds(const CompressArgs& a);
hipError_t launch_compress_forward(const CompressArgs& a, hipStream_t stream);
hipError_t launch_compress_forward_bf16(const CompressArgs& a, hipStream_t stream);
hipError_t launch_compress_backward(const CompressArgs& a, float* grad, hipStream_t stream);
hipError_t launch_channel_cov(const CompressArgs& a, float* part, int slices, hipStream_t stream);
hipError_t launch_spectrum_gram(int n, int Q, int lmax, const float* X, float* C, hipStream_t stream);
hipError_t launch_spectrum_kernel_loss(int n, int Q, int lmax, const float* X, const float* Kref, float* Kt,
                                       float* loss, float* scale, float* dX, hipStream_t stream);
hipError_t launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                       float eps, int step, hipStream_t stream);

struct NeighborArgs {
    int32_t n_structures;
    int64_t n_atoms;
    int64_t max_bins;             // bound on the total number of bins (workspace size)
    double rcut;
    const int64_t* atom_offsets;  // [n_structures + 1]
    const double* cells;          // [n_structures][3][3]
    const uint8_t* pbc;           // [n_structures][3]
    const double* positions;
    const int32_t* species;
    int32_t n_species;
    // workspace arrays
    StructGeom* geom;             // [n_structures]
    int32_t* atom_struct;         // [N]
    int32_t* atom_bin;            // [N] global bin index
    int32_t* atom_wrap;           // [N][3] integer wrap of the fractional coordinates
    int32_t* bin_count;           // [max_bins + 1]
    int32_t* bin_start;           // [max_bins + 1]
    int32_t* bin_cursor;          // [max_bins + 1]
    int32_t* bin_atoms;           // [N]
    double4* slots;               // [N] atoms in bin order: wrapped position x, y, z and the atom index
    double4* wrapped;             // [N] the same records in atom order (large systems)
    int64_t* centre_count;        // [N + 1]
    int64_t* scan_tmp;            // per-tile sums of the multi-work-group scan
    int32_t* ok;                  // set by the geometry phase: 1 if the input is valid
    int64_t capacity;
    int64_t* pair_offsets;
    int32_t* pair_j;
    int32_t* pair_shift;
    void* pair_vec;
    bool vec_f64;
    int32_t* pair_transpose;
    int32_t* status;
};

hipError_t launch_neighbors(const NeighborArgs& a, hipStream_t stream);
// bytes of neighbour-list workspace for these sizes (as soap_neighbors_workspace_size)
size_t neighbors_workspace_bytes(int32_t n_structures, int64_t n_atoms);

}  // namespace soap
