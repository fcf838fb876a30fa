/*
 * soap_mi355x.h -- C ABI of the MI355X (gfx950) SOAP library.
 *
 * The library computes, on one AMD Instinct MI355X, the hot path of the
 * atom-density representation of Musil et al., "Efficient implementation of
 * atom-density representations" (arXiv 2101.08814):
 *
 *   neighbours   A_i = {(j, s) : 0 < |r_j + s.H - r_i| < rcut}        (App. B)
 *   expansion    c_{i,a,n,lm} = sum_{j in A_i, a_j = a}
 *                  f_cut(r_ji) I~_nl(r_ji) Y_lm(r^_ji)
 *                                   (Sec. 4.A Eq. spherical_expansion_
 *                                    coefficients_gaussians, Sec. 4.B-D)
 *   power spec.  p_{i,l,k1<=k2} = sum_m c_{i,k1,lm} c_{i,k2,lm},
 *                  k = a * nmax + n                (Sec. 2 Eq. nu2-basis-coupled)
 *   gradients    forward-mode rows d c_i / d r_j and d p_i / d r_j (Sec. 4.G)
 *                and the reverse-mode (vector-Jacobian) products
 *                (App. B Eq. energy-derivative).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Radial basis: GTO (Sec. 4.B Eq. GTO), orthogonalised with S^{-1/2};
 *   the radial integral of a Gaussian density exp(-x^2 / 2 sigma^2)
 *   (Eq. rad-int-gto-1) is tabulated as a clamped cubic spline on a uniform
 *   grid over [0, rcut] (Sec. 4.D) with max error <= spline_accuracy.
 * - Cutoff: shifted cosine, 1 below rcut - cutoff_width, 0 at rcut.
 * - Harmonics: real, orthonormal, index lm = l*l + l + m, m = -l..l;
 *   Y_{1,-1}, Y_{1,0}, Y_{1,1} are proportional to y, z, x.
 * - L2 = (lmax+1)^2, K = n_species * nmax, KK = K (K+1) / 2.
 * - Arrays are dense, row-major, and (unless marked [host]) device pointers
 *   on the current HIP device.  The caller owns every array; the library
 *   allocates only its spline tables (once per device, at the first call
 *   on that device or at soap_calculator_upload).
 * - Every device call is asynchronous on exec->stream.  Host-side argument
 *   errors return immediately with nothing enqueued; soap_last_error()
 *   then holds a message.  Errors found on the device (pair capacity
 *   exceeded, coincident atoms, species out of range) are stored as a
 *   nonzero soap_status into *exec->dev_status (caller-zeroed device int32);
 *   soap_read_device_status() synchronises the stream and returns it.
 *   The outputs of a call that stores such a status are not meaningful.
 *   Kernels that read a neighbour list whose total exceeds the capacity
 *   they are given store SOAP_ECAPACITY and write nothing else.
 * - Floating-point type: SOAP_F64 -> double, SOAP_F32 -> float for
 *   pair_vec, coefficients, features and gradients.  SOAP_BF16_F32ACC is
 *   accepted by soap_power_spectrum only: c and p are float in memory and
 *   the contraction runs on MFMA with bfloat16 hi/lo operands and float
 *   accumulation.
 * - A calculator is immutable after creation and may be shared by threads
 *   and streams.  Calls enqueued on the same stream with overlapping
 *   outputs race only if the caller makes them race.
 */
#ifndef SOAP_MI355X_H
#define SOAP_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SOAP_ABI_VERSION 2

typedef enum {
    SOAP_OK = 0,
    SOAP_EINVAL = -1,        /* bad argument (host)                          */
    SOAP_ECAPACITY = -2,     /* neighbour list larger than the given capacity */
    SOAP_EDEVICE = -3,       /* HIP runtime error                             */
    SOAP_ENOMEM = -4,        /* allocation of the spline tables failed        */
    SOAP_EUNSUPPORTED = -5,  /* valid request this build does not implement   */
    SOAP_EGEOMETRY = -6,     /* two distinct atoms (or images) coincide       */
    SOAP_ESPECIES = -7       /* species index outside [0, n_species)          */
} soap_status;

/* The two _RANGE_ members are not precisions: they give the type the range
 * of int32_t, so that an invalid value from a caller is a defined value the
 * library rejects with SOAP_EINVAL. */
typedef enum {
    SOAP_F64 = 0,
    SOAP_F32 = 1,
    SOAP_BF16_F32ACC = 2,
    SOAP_PRECISION_RANGE_MIN_ = -2147483647 - 1,
    SOAP_PRECISION_RANGE_MAX_ = 2147483647
} soap_precision;

/* Radial basis (Sec. 4.B, 4.C). */
typedef enum {
    SOAP_RADIAL_GTO = 0,   /* GTOs orthogonalised with S^{-1/2} (Eq. GTO)   */
    SOAP_RADIAL_DVR = 1    /* DVR on the nmax Gauss-Legendre points of
                              [0, rcut + 3 sigma] (Eq. rad-int-dvr, with the
                              factor 4 pi exp(-c r^2) of the Gaussian-density
                              radial integral; orthonormal)                 */
} soap_radial_basis;

/* Hyper-parameters (Sec. 3 and 4: species, rcut, smoothing, sigma, nmax,
 * lmax, radial basis).  Limits: 1 <= n_species <= 64, 1 <= nmax <= 16,
 * 0 <= lmax <= 12, rcut > 0, 0 < cutoff_width <= rcut, sigma > 0,
 * include_center in {0, 1} (1: the central atom adds its own r = 0 term,
 * l = 0 only, to channel a_i), 0 < spline_accuracy (the paper uses 1e-8,
 * Fig. ri-qm9 caption), radial_basis a soap_radial_basis.  Either basis is
 * tabulated as the same cubic spline, so every kernel runs unchanged. */
typedef struct {
    int32_t n_species;
    int32_t nmax;
    int32_t lmax;
    int32_t include_center;
    double rcut;
    double cutoff_width;
    double sigma;
    double spline_accuracy;
    int32_t radial_basis;
    int32_t reserved;      /* 0 */
} soap_hypers;

/* Facts about a calculator's spline table (host). */
typedef struct {
    int64_t n_intervals;        /* M: grid r_k = k * rcut / M, k = 0..M       */
    double delta;               /* rcut / M                                   */
    double max_error;           /* max |spline - exact| of I~ at 4 interior
                                   points per interval                        */
    double max_error_deriv;     /* same for d I~ / dr                         */
    double overlap_condition;   /* condition number of the GTO overlap S      */
    int64_t table_bytes_f64;    /* device bytes of the double table           */
    int64_t table_bytes_f32;    /* device bytes of the float table            */
} soap_table_info;

typedef struct soap_calculator soap_calculator;

/* Per-call execution context (caller-owned, host struct). */
typedef struct {
    void* stream;          /* hipStream_t; NULL is the null stream           */
    int32_t* dev_status;   /* device int32, zeroed by the caller; may be NULL,
                              then device-side errors are not reported       */
} soap_exec;

int32_t soap_abi_version(void);

/* Thread-local message of the last failed call on this thread. */
const char* soap_last_error(void);

/* Builds the GTO constants, S^{-1/2} and the spline tables in FP64 on the
 * host (Sec. 4.B, 4.D, App. A).  *out receives a new calculator; free it
 * with soap_calculator_destroy.  No device work. */
soap_status soap_calculator_create(const soap_hypers* hypers, soap_calculator** out);
soap_status soap_calculator_destroy(soap_calculator* calc);
soap_status soap_calculator_info(const soap_calculator* calc, soap_table_info* info);

/* Uploads the tables to the current device now (otherwise done at the
 * first call on that device; that call then synchronises once). */
soap_status soap_calculator_upload(const soap_calculator* calc);

/* Host evaluation of the library's radial integral I~_nl(r) and d/dr for
 * n_r radii [host]: exact=1 uses the library's own 1F1 recurrence
 * (App. A), exact=0 the FP64 spline the kernels use.  Outputs
 * [n_r][nmax][lmax+1] [host]; dI may be NULL. */
soap_status soap_radial_integral_host(const soap_calculator* calc, int32_t exact, int64_t n_r,
                                      const double* r, double* I, double* dI);

/* The radial integrals I~_nl(r_k) and d/dr on the device for n_r radii
 * (the per-neighbour step the expansion performs, Sec. 4.B-4.D), either
 * from the spline the kernels use (exact = 0) or evaluated directly per
 * radius (exact = 1): for the GTO basis the restricted 1F1 of App. A
 * (series or asymptotic form at the two largest l, the downward recurrence
 * for the others) and S^{-1/2}; for the DVR basis the closed form with the
 * modified spherical Bessel function.  For comparing the cost of the three
 * evaluations (Sec. 4.D, Fig. ri-qm9) and checking the table.
 * r [n_r] double, device, in [0, rcut].  I and dI (dI may be NULL) are
 * device arrays [nmax][lmax+1][n_r] (radius fastest) of double (SOAP_F64)
 * or float (SOAP_F32; spline only: the direct path is SOAP_F64).        */
soap_status soap_radial_integral(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                                 int32_t exact, int64_t n_r, const double* r, void* I, void* dI);

/* Device bytes of scratch soap_compute_neighbors needs for n_structures
 * structures holding n_atoms atoms in total (independent of positions and
 * cells, so one workspace serves a whole trajectory). */
soap_status soap_neighbors_workspace_size(const soap_calculator* calc, int32_t n_structures, int64_t n_atoms,
                                          size_t* bytes);

/* Full neighbour list with periodic images (App. B; Sec. 3 Fig. 1).
 *
 * For every centre i, every (j, s) with s integer on periodic axes (0 on
 * the others) and 0 < |r_ji| < rcut, r_ji = r_j + s0 h1 + s1 h2 + s2 h3 - r_i.
 * j = i is kept when s != 0 (self-images).  Structures never interact.
 * If any axis of a structure is periodic its cell must be non-singular.
 * Positions may lie outside the cell (any number of cells away).
 *
 * [host] n_structures, n_atoms, capacity, vec_precision, workspace_bytes.
 * [dev]  atom_offsets int64 [n_structures+1] (0 = first, n_atoms = last),
 *        cells double [n_structures][3][3] (rows h1, h2, h3; ignored for
 *        structures without periodic axes), pbc uint8 [n_structures][3],
 *        positions double [N][3], species int32 [N] in [0, n_species),
 *        workspace of >= soap_neighbors_workspace_size bytes (256-aligned).
 * out [dev] pair_offsets int64 [N+1] (CSR over centres; pair_offsets[N] is
 *        the number of pairs P even when P > capacity),
 *        pair_j int32 [capacity], pair_shift int32 [capacity][3],
 *        pair_vec [capacity][3] (double or float per vec_precision,
 *        always formed in double), pair_transpose int32 [capacity] or NULL
 *        (index of the pair (j, i, -s)).
 * Pairs of one centre are ordered by (species_j, j, s0, s1, s2).
 * Nothing is copied between host and device, so the call can be captured
 * in a graph.  Device errors: SOAP_ECAPACITY if P > capacity (the pair
 * arrays then hold nothing usable), SOAP_EGEOMETRY for coincident distinct
 * atoms, SOAP_ESPECIES, SOAP_EINVAL for inconsistent atom_offsets, a
 * singular periodic cell or one thinner than rcut / 1024 (then P = 0).
 * Non-periodic axes are searched without binning (all pairs within the
 * structure along that axis).                                          */
soap_status soap_compute_neighbors(const soap_calculator* calc, const soap_exec* exec,
                                   int32_t n_structures, int64_t n_atoms, const int64_t* atom_offsets,
                                   const double* cells, const uint8_t* pbc,
                                   const double* positions, const int32_t* species,
                                   void* workspace, size_t workspace_bytes, int64_t capacity,
                                   soap_precision vec_precision, int64_t* pair_offsets,
                                   int32_t* pair_j, int32_t* pair_shift, void* pair_vec,
                                   int32_t* pair_transpose);

/* soap_compute_neighbors for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments, outputs and device errors are those of
 * soap_compute_neighbors without workspace / workspace_bytes: the
 * workspace is a static device array of SOAP_NEIGHBORS_NOALLOC_BYTES bytes
 * per device, held until the process ends.  A request whose
 * soap_neighbors_workspace_size exceeds it returns SOAP_EINVAL with
 * nothing enqueued (16 MiB holds about 150,000 atoms).  The call allocates
 * nothing and needs no clearing between calls.  Every call on one device
 * shares that device's array: calls that overlap on one device (other
 * streams, other threads) race, so the caller orders them.              */
#define SOAP_NEIGHBORS_NOALLOC_BYTES ((size_t)16 << 20)
soap_status soap_compute_neighbors_noalloc(const soap_calculator* calc, const soap_exec* exec,
                                           int32_t n_structures, int64_t n_atoms, const int64_t* atom_offsets,
                                           const double* cells, const uint8_t* pbc,
                                           const double* positions, const int32_t* species,
                                           int64_t capacity, soap_precision vec_precision,
                                           int64_t* pair_offsets, int32_t* pair_j, int32_t* pair_shift,
                                           void* pair_vec, int32_t* pair_transpose);

/* Spherical expansion (Sec. 4.A Eq. spherical_expansion_coefficients_
 * gaussians with the splined radial integral of Sec. 4.D and real Y_lm of
 * Sec. 4.E), optionally with forward-mode gradient rows (Sec. 4.G).
 *
 * in  n_atoms, species [N], pair_offsets [N+1], pair_j [P], pair_vec [P][3]
 *     (type per precision), pair_capacity = length of the pair arrays.
 * out coeffs [N][n_species][nmax][L2].
 *     dcoeffs [P][3][nmax][L2] or NULL: row q of centre i is
 *       d c_{i, a_j, n, lm} / d r_ji  (the only nonzero species block);
 *     dcoeffs_self [N][3][n_species][nmax][L2] or NULL: d c_i / d r_i
 *       = - sum of the rows of i (images of i included, App. B).
 *     dcoeffs and dcoeffs_self are both NULL or both given; rows P to
 *     pair_capacity - 1 of dcoeffs are not written.
 * precision: SOAP_F64 or SOAP_F32.                                      */
soap_status soap_spherical_expansion(const soap_calculator* calc, const soap_exec* exec,
                                     soap_precision precision, int64_t n_atoms,
                                     const int32_t* species, const int64_t* pair_offsets,
                                     const int32_t* pair_j, const void* pair_vec,
                                     int64_t pair_capacity, void* coeffs, void* dcoeffs,
                                     void* dcoeffs_self);

/* Power spectrum p [N][lmax+1][KK] from coeffs [N][n_species][nmax][L2]
 * (Sec. 2 Eq. nu2-basis-coupled times sqrt(2l+1); packed k1 <= k2,
 * row-major, no sqrt(2) on off-diagonal entries).
 * Optional forward-mode rows (Sec. 4.G), product rule on the rows of
 * soap_spherical_expansion:
 *   dp [P][3][lmax+1][KK] from dcoeffs, dp_self [N][3][lmax+1][KK] from
 *   dcoeffs_self; both NULL or both given (then species, pair_offsets,
 *   pair_j, dcoeffs, dcoeffs_self are read).
 * precision: SOAP_F64, SOAP_F32, or SOAP_BF16_F32ACC (MFMA, bfloat16 hi/lo
 * split of c with float accumulation; no gradient rows).             */
soap_status soap_power_spectrum(const soap_calculator* calc, const soap_exec* exec,
                                soap_precision precision, int64_t n_atoms, const void* coeffs,
                                void* p, const int32_t* species, const int64_t* pair_offsets,
                                const int32_t* pair_j, int64_t pair_capacity,
                                const void* dcoeffs, const void* dcoeffs_self, void* dp,
                                void* dp_self);

/* Expansion and power spectrum, optionally with forward-mode rows, in one
 * call: a per-centre pass (c, p, and the self rows dcoeffs_self / dp_self)
 * and, if dcoeffs / dp are given, the pair-row pass of
 * soap_gradient_rows.  The coefficient rows are never read back.
 * Arguments as in the calls above; p is required; dcoeffs_self and dp_self
 * are both NULL or both given, and so are dcoeffs and dp.
 * precision: SOAP_F64 or SOAP_F32.                                     */
soap_status soap_features(const soap_calculator* calc, const soap_exec* exec,
                          soap_precision precision, int64_t n_atoms, const int32_t* species,
                          const int64_t* pair_offsets, const int32_t* pair_j,
                          const void* pair_vec, int64_t pair_capacity, void* coeffs, void* p,
                          void* dcoeffs, void* dcoeffs_self, void* dp, void* dp_self);

/* Forward-mode pair rows alone (Sec. 4.G), given the coefficients of every
 * centre (as written by soap_spherical_expansion or soap_features):
 *   dcoeffs [P][3][nmax][L2]        d c_{i,a_j,.} / d r_ji
 *   dp      [P][3][lmax+1][KK]      d p_i / d r_ji, by the product rule
 *           sum_m dc_{x,k1,lm} c_{k2,lm} + c_{k1,lm} dc_{x,k2,lm}
 *           summed as (f I~)'_nl u_x y_{l,k} + f I~_nl z_{x,l,k} with
 *           y = sum_m Y_lm c_{k,lm} and z = sum_m dY_{x,lm} c_{k,lm}.
 * Either output may be NULL (not both).  coeffs is read only for dp.
 * precision: SOAP_F64 or SOAP_F32.                                     */
soap_status soap_gradient_rows(const soap_calculator* calc, const soap_exec* exec,
                               soap_precision precision, int64_t n_atoms, const int32_t* species,
                               const int64_t* pair_offsets, const int32_t* pair_j,
                               const void* pair_vec, int64_t pair_capacity, const void* coeffs,
                               void* dcoeffs, void* dp);

/* Reverse mode of the power spectrum (chain rule of Sec. 4.G):
 *   grad_coeffs_{k,lm} = sum_k' W_{k k'} c_{k',lm},
 *   W_{k k'} = grad_p_{min,max} (k != k'),  W_{k k} = 2 grad_p_{k k},
 * grad_p [N][lmax+1][KK], coeffs and grad_coeffs [N][n_species][nmax][L2].
 * precision: SOAP_F64 or SOAP_F32.                                     */
soap_status soap_power_spectrum_backward(const soap_calculator* calc, const soap_exec* exec,
                                         soap_precision precision, int64_t n_atoms,
                                         const void* coeffs, const void* grad_p,
                                         void* grad_coeffs);

/* Reverse mode of the expansion with respect to positions (App. B Eq.
 * energy-derivative):
 *   g_q = sum_{n,lm} grad_coeffs_{i,a_j,n,lm} d/dr_ji [f I~_nl Y_lm]
 *   grad_positions_k = sum_{q: j_q = k} g_q - sum_{q of centre k} g_q
 * (all images of k move together; an image of i contributes nothing to
 * d/dr_i).  The per-atom sums are taken in a fixed order through
 * pair_transpose (no atomics: results are bitwise reproducible).
 * out grad_pair_vec [P][3] (g_q = dL/dr_ji, input of a virial; required),
 *     grad_positions [N][3] (overwritten).
 * precision: SOAP_F64 or SOAP_F32.                                     */
soap_status soap_spherical_expansion_backward(const soap_calculator* calc, const soap_exec* exec,
                                              soap_precision precision, int64_t n_atoms,
                                              const int32_t* species, const int64_t* pair_offsets,
                                              const int32_t* pair_j, const void* pair_vec,
                                              const int32_t* pair_transpose, int64_t pair_capacity,
                                              const void* grad_coeffs, void* grad_pair_vec,
                                              void* grad_positions);

/* Selected invariants (Sec. 4.H): for each centre i and each triple
 * q = selected[q] = (k1, k2, l) (int32, device, [n_selected][3]),
 *   p_selected[i][q] = sum over m < 2l+1 of c[i][k1][l^2 + m] c[i][k2][l^2 + m],
 * the entry (l, k1, k2) of the full power spectrum (same normalisation as
 * soap_power_spectrum; k1 > k2 is allowed and gives the (k2, k1) value).
 * coeffs [n_atoms][n_channels][(lmax+1)^2] with n_channels = S * nmax
 * (the layout soap_spherical_expansion writes); one centre's coefficients
 * must fit 160 KB.  p_selected [n_atoms][n_selected] is overwritten.  A
 * triple out of range gives 0 and SOAP_EINVAL in the device status word.
 * precision: SOAP_F64 or SOAP_F32.                                     */
soap_status soap_power_spectrum_selected(const soap_exec* exec, soap_precision precision, int64_t n_atoms,
                                         int32_t n_channels, int32_t lmax, const void* coeffs, int64_t n_selected,
                                         const int32_t* selected, void* p_selected);

/* Adjoint of soap_power_spectrum_selected (the chain rule of App. B
 * through the selected invariants):
 *   grad_coeffs[i][k][lm] = sum over selected q = (k1, k2, l) with l(lm) = l of
 *       grad_p_selected[i][q] (c[i][k2][lm] [k == k1] + c[i][k1][lm] [k == k2]).
 * The sums follow a plan built once per selection on the host by
 * soap_power_spectrum_selected_plan from the host copy of `selected`
 * (checked there: an out-of-range triple is SOAP_EINVAL):
 * row_offsets [n_channels * (lmax+1) + 1] and entries [2 * n_selected][2]
 * (q, partner channel), caller-owned host memory; the caller copies both to
 * the device for the backward call.  Per centre the coefficients and the
 * gradient row must fit 160 KB.  grad_coeffs [n_atoms][n_channels][L2] is
 * overwritten; sums run in plan order (bitwise reproducible).  A plan that
 * does not fit n_selected gives 0 and SOAP_EINVAL in the device status.
 * precision: SOAP_F64 or SOAP_F32.                                     */
soap_status soap_power_spectrum_selected_plan(int32_t n_channels, int32_t lmax, int64_t n_selected,
                                              const int32_t* selected, int32_t* row_offsets, int32_t* entries);
soap_status soap_power_spectrum_selected_backward(const soap_exec* exec, soap_precision precision, int64_t n_atoms,
                                                  int32_t n_channels, int32_t lmax, const void* coeffs,
                                                  int64_t n_selected, const void* grad_p_selected,
                                                  const int32_t* row_offsets, const int32_t* entries,
                                                  void* grad_coeffs);

/* Sparse kernel model (Sec. 5.B, Eq. sparse-gp with the polynomial kernel):
 * for each centre i,
 *   energies[i] = sum over active points I with active_species[I] ==
 *                 centre_species[i] of weights[I] (M_I . p_i)^zeta,
 * and, when grad_features is not NULL,
 *   grad_features[i] = sum over the same I of weights[I] zeta
 *                      (M_I . p_i)^(zeta-1) M_I,
 * the active-set sum taken first (Eq. gpr-force-order): passing
 * grad_features as grad_p to soap_power_spectrum_backward and on through
 * soap_spherical_expansion_backward and soap_virial gives the model's
 * energy gradient and virial.  A structure's energy is the sum of its
 * centres' energies (Eq. additive-energy-model).
 * features [n_centres][n_features] (p_i, any per-centre feature vector such
 * as the packed power spectrum), active_features [n_active][n_features]
 * (M_I), weights [n_active], all device memory in the precision's type,
 * row-major; species int32 (device).  zeta in [1, 64]; n_features and
 * n_active at most 4,194,240, n_centres below 2^31 (else SOAP_EINVAL).
 * workspace: device scratch of soap_gpr_workspace_size bytes (energy
 * partials per 64 active points, an [n_centres][n_active] coefficient
 * matrix, and partial gradients when the active set is split to fill the
 * GPU), owned by the caller.
 * energies [n_centres] and grad_features [n_centres][n_features] are
 * overwritten.  Sums run in a fixed order (bitwise reproducible).
 * precision: SOAP_F64 or SOAP_F32.                                     */
soap_status soap_gpr_workspace_size(soap_precision precision, int64_t n_centres, int64_t n_features,
                                    int64_t n_active, size_t* bytes);
soap_status soap_gpr_predict(const soap_exec* exec, soap_precision precision, int64_t n_centres, int64_t n_features,
                             const int32_t* centre_species, const void* features, int64_t n_active,
                             const int32_t* active_species, const void* active_features, const void* weights,
                             int32_t zeta, void* workspace, size_t workspace_bytes, void* energies,
                             void* grad_features);

/* Virial of the loss per structure (App. B, Eq. energy-virial: the
 * stress term of a homogeneous deformation r -> (1 + eps) r of positions
 * and cell):
 *   virial_s[a][b] = sum over the pairs q of the centres of structure s of
 *                    g_{q,a} r_{q,b},
 * with g_q = dL/dr_ji from soap_spherical_expansion_backward (grad_pair_vec)
 * and r_q = pair_vec (images included: a pair to an image carries its
 * shifted vector).  atom_offsets [n_structures+1] (device, int64) tiles
 * the atoms; centre_partials is caller scratch of 9 * n_atoms elements.
 * Sums run in a fixed order (bitwise reproducible).
 * out virial [n_structures][3][3] (overwritten).
 * precision: SOAP_F64 or SOAP_F32 (the type of pair_vec, grad_pair_vec,
 * centre_partials and virial).                                        */
soap_status soap_virial(const soap_exec* exec, soap_precision precision, int32_t n_structures,
                        const int64_t* atom_offsets, int64_t n_atoms, const int64_t* pair_offsets,
                        const void* pair_vec, const void* grad_pair_vec, int64_t pair_capacity,
                        void* centre_partials, void* virial);

/* ------------------------------------------------------------------
 * Learned channel compression (a learned counterpart of the reduction of
 * the feature space of Sec. 4.H and the lossy strategy of Sec. 7, keeping
 * the symmetry of the features).  For every degree l one two-layer network
 * acts on the channel index k = a nmax + n of each m-column of c, shared
 * over m (so it commutes with rotations):
 *   h_l = W1_l c_l,   g_{l,q} = h_{l,q} 2 sigmoid(alpha_{l,q} |h_{l,q}| + beta_{l,q}),
 *   c~_l = W2_l g_l,  p~_{l,q1<=q2} = sum_m c~_{q1,lm} c~_{q2,lm},
 * |.| the norm over m.  K = n_species nmax channels in, n_out out, hidden
 * units.  weights: one float array, per l = 0..lmax in order W1_l
 * [hidden][K], W2_l [n_out][hidden], alpha_l [hidden], beta_l [hidden].
 * All arrays are float and on the device unless stated.
 * Limits: 1 <= n_out <= 64, 1 <= hidden <= 256.
 * ------------------------------------------------------------------ */

/* Number of weights for (n_out, hidden): (lmax+1) (hidden K + n_out hidden + 2 hidden). */
soap_status soap_compress_n_params(const soap_calculator* calc, int32_t n_out, int32_t hidden, int64_t* n_params);

/* Checkpoint of a compression network and its optimiser state (the
 * training of the learned compression, Sec. 4.H and Sec. 7): writes the
 * weights, the Adam moments m and v (device arrays of n_params floats each)
 * and the step count to the host file path, with the shape (n_out, hidden,
 * channels, lmax) and a 64-bit hash of the contents; the file is written
 * under path.tmp and renamed over path.  Synchronous (device-to-host
 * copies).  SOAP_EINVAL when the file cannot be written.               */
soap_status soap_compress_save(const soap_calculator* calc, int32_t n_out, int32_t hidden, int64_t step,
                               const float* weights, const float* adam_m, const float* adam_v, const char* path);

/* Reads a file written by soap_compress_save into the device arrays
 * weights, adam_m, adam_v (n_params floats each) and *step (host).
 * SOAP_EINVAL, with nothing written, when the file is missing, not a
 * checkpoint, of another version or shape (n_out, hidden, the calculator's
 * channels and lmax), truncated, longer than its contents, or fails its
 * hash.                                                                 */
soap_status soap_compress_load(const soap_calculator* calc, int32_t n_out, int32_t hidden, const char* path,
                               float* weights, float* adam_m, float* adam_v, int64_t* step);

/* Bytes of device workspace that soap_compress_init_pca,
 * soap_compress_forward_ws and soap_compress_backward need.             */
soap_status soap_compress_workspace_size(const soap_calculator* calc, int32_t n_out, int32_t hidden,
                                         size_t* bytes);

/* Closed-form start (and baseline): per l the top n_out eigenvectors U_l of
 * the channel covariance sum_{i,m} c_{i,:,lm} c_{i,:,lm}^T over the n_atoms
 * centres of coeffs [N][K][L2]: W1_l = [U_l^T; e R1], W2_l = [I e R2],
 * alpha = beta = 0, where R1, R2 are standard normal draws of a splitmix64
 * stream seeded with seed (hidden units beyond n_out) and e = noise.
 * Synchronises exec->stream (the eigen-decomposition runs on the host).
 * Writes weights (device, n_params floats).                            */
soap_status soap_compress_init_pca(const soap_calculator* calc, const soap_exec* exec, int32_t n_out,
                                   int32_t hidden, int64_t n_atoms, const float* coeffs, uint64_t seed,
                                   float noise, void* workspace, size_t workspace_bytes, float* weights);

/* Forward pass: coeffs [N][K][L2] -> coeffs_out [N][n_out][L2] and/or
 * p_out [N][lmax+1][n_out (n_out+1)/2] (either may be NULL, not both).
 * precision SOAP_F32: float arithmetic throughout.  SOAP_BF16_F32ACC: the
 * two layers run on MFMA with bfloat16 operands (c, the weights and the
 * gated hidden layer rounded to bfloat16) and float accumulation; the gate
 * in float; p~ from the float c~ (where K, hidden <= 128 are multiples of
 * 4 and n_out <= 32, as a Gram matrix on MFMA with a bfloat16 high/low
 * split of c~, relative error about 2^-16).                           */
soap_status soap_compress_forward(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                                  int32_t n_out, int32_t hidden, int64_t n_atoms, const float* weights,
                                  const float* coeffs, float* coeffs_out, float* p_out);

/* soap_compress_forward with a device workspace of at least
 * soap_compress_workspace_size bytes.  With SOAP_BF16_F32ACC (and the
 * shapes of the one-wave-per-centre kernel: K, hidden <= 128 and multiples
 * of 4, n_out <= 32, 1 <= lmax <= 12) the weights are first laid out once in
 * the workspace as the kernel holds them in LDS (bfloat16 rows, the same
 * rounding), and each work-group copies the next degree's image while it
 * computes the current one; the results are those of soap_compress_forward
 * bit for bit.  The workspace is overwritten; calls that overlap must not
 * share it.                                                             */
soap_status soap_compress_forward_ws(const soap_calculator* calc, const soap_exec* exec, soap_precision precision,
                                     int32_t n_out, int32_t hidden, int64_t n_atoms, const float* weights,
                                     const float* coeffs, float* coeffs_out, float* p_out, void* workspace,
                                     size_t workspace_bytes);

/* Reverse mode for training: given grad_p = dL/dp~ [N][lmax+1][n_out
 * (n_out+1)/2] of the forward pass at (weights, coeffs), writes
 * grad_weights (n_params floats, overwritten) = sum over the N centres of
 * dL/dweights.  Float arithmetic; deterministic (fixed summation order). */
soap_status soap_compress_backward(const soap_calculator* calc, const soap_exec* exec, int32_t n_out,
                                   int32_t hidden, int64_t n_atoms, const float* weights, const float* coeffs,
                                   const float* grad_p, void* workspace, size_t workspace_bytes,
                                   float* grad_weights);

/* Linear kernel of power spectra stored packed, X [n][lmax+1][Q(Q+1)/2]:
 *   K_ij = sum_{l,q1,q2} p_{l q1 q2}(i) p_{l q1 q2}(j)
 * over the full symmetric spectrum (packed off-diagonal entries weighted
 * 2; this kernel does not depend on the orthonormal basis of the channel
 * space).  out K [n][n].  n_channels = Q: the calculator's K for the plain
 * spectrum, n_out for the compressed one.                              */
soap_status soap_spectrum_gram(const soap_exec* exec, int32_t n, int32_t n_channels, int32_t lmax,
                               const float* X, float* K);

/* Training loss of the compression over a batch and its gradient:
 *   L = |K~ - Kref|_F^2 / |Kref|_F^2,  K~ = soap_spectrum_gram(X),
 *   grad_X = dL/dX [n][lmax+1][Q(Q+1)/2].
 * work: n*n + 1 floats of device scratch; loss: device float.           */
soap_status soap_spectrum_kernel_loss(const soap_exec* exec, int32_t n, int32_t n_channels, int32_t lmax,
                                      const float* X, const float* Kref, float* work, float* loss,
                                      float* grad_X);

/* One Adam step (Kingma & Ba, bias-corrected; step counts from 1) on n
 * parameters: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
 * params <- params - lr mhat / (sqrt(vhat) + eps).                     */
soap_status soap_adam_step(const soap_exec* exec, int64_t n, float* params, const float* grads, float* m,
                           float* v, float lr, float beta1, float beta2, float eps, int32_t step);

/* Synchronises exec->stream and returns *exec->dev_status (SOAP_OK if
 * dev_status is NULL), or SOAP_EDEVICE on a runtime error.             */
soap_status soap_read_device_status(const soap_exec* exec);

#ifdef __cplusplus
}
#endif

#endif /* SOAP_MI355X_H */
