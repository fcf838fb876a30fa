"""FP64 CPU oracle of the SOAP hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It wraps ``soap_oracle.c`` (plain C, double precision,
written from the paper's definitions; see the header of that file) through
ctypes and shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "soap_oracle.c")
# another build of the same source (for example one with sanitizers) can be
# named in SOAP_ORACLE_LIBRARY
_LIB_PATH = os.environ.get("SOAP_ORACLE_LIBRARY") or os.path.join(_HERE, "libsoap_oracle.so")
_lib = None


FLAGS = ["-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True, path: str = _LIB_PATH, native: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over centres; generic x86-64, or
    tuned for the host it runs on with native=True, for timing there)."""
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        flags = FLAGS + (["-march=native"] if native else [])
        subprocess.check_call(["gcc"] + flags + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


def use_build(path: str):
    """Load the oracle from another build of the same source (for example a
    -march=native one); later calls go to it."""
    global _lib
    _lib = None
    return lib(path)


def lib(path: str = _LIB_PATH):
    global _lib
    if _lib is None:
        if not os.path.exists(path) or (path == _LIB_PATH and os.path.getmtime(path) < os.path.getmtime(_SRC)):
            build(path=path)
        L = ctypes.CDLL(path)
        d, i, i64, u8 = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_uint8
        P = ctypes.POINTER
        L.orc_num_threads.restype = i
        L.orc_set_num_threads.argtypes = [i]
        L.orc_fcut.restype = d
        L.orc_fcut.argtypes = [d, d, d, P(d)]
        L.orc_gto_constants.argtypes = [i, d, P(d), P(d), P(d)]
        L.orc_overlap.argtypes = [i, d, P(d)]
        L.orc_inverse_sqrt.restype = i
        L.orc_inverse_sqrt.argtypes = [i, P(d), P(d)]
        L.orc_hyp1f1.restype = d
        L.orc_hyp1f1.argtypes = [d, d, d]
        L.orc_radial_integral.argtypes = [i, i, d, d, d, P(d), P(d)]
        L.orc_orth_matrix.restype = i
        L.orc_orth_matrix.argtypes = [i, d, P(d)]
        L.orc_radial_integral_orth.restype = i
        L.orc_radial_integral_orth.argtypes = [i, i, d, d, d, P(d), P(d)]
        L.orc_ylm.argtypes = [i, P(d), P(d), P(d)]
        L.orc_neighbors.restype = i
        L.orc_neighbors.argtypes = [i, P(i64), P(d), P(d), P(u8), P(ctypes.c_int32), d, P(i64),
                                    P(ctypes.c_int32), P(ctypes.c_int32), P(d)]
        hy = [i, i, i, i, d, d, d, i]
        L.orc_gauss_legendre.argtypes = [i, P(d), P(d)]
        L.orc_sph_bessel_i.restype = d
        L.orc_sph_bessel_i.argtypes = [i, d, P(d)]
        L.orc_dvr_points.argtypes = [i, d, d, P(d), P(d)]
        L.orc_dvr_radial_integral.argtypes = [i, i, d, d, d, P(d), P(d)]
        L.orc_expansion.restype = i
        L.orc_expansion.argtypes = hy + [P(ctypes.c_int32), P(i64), P(ctypes.c_int32), P(d), i64, P(i64), P(d)]
        L.orc_power_spectrum.argtypes = [i, i, i, i64, P(d), P(d)]
        L.orc_gradients.restype = i
        L.orc_gradients.argtypes = hy + [P(ctypes.c_int32), P(i64), P(ctypes.c_int32), P(d), i64, P(i64),
                                         P(d), P(d), P(d), P(d)]
        L.orc_vjp.restype = i
        L.orc_vjp.argtypes = hy + [i64, P(ctypes.c_int32), P(i64), P(ctypes.c_int32), P(d), P(d), P(d), P(d)]
        _lib = L
    return _lib


def _p(a, ct=ctypes.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _hy(h):
    return (int(h["n_species"]), int(h["nmax"]), int(h["lmax"]), int(h.get("include_center", 1)),
            float(h["rcut"]), float(h.get("cutoff_width", 0.5)), float(h["sigma"]),
            int(h.get("radial_basis", 0)))


# ---------------------------------------------------------------- elements
def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int):
    lib().orc_set_num_threads(int(n))


def fcut(r, rcut, width):
    df = ctypes.c_double()
    f = lib().orc_fcut(float(r), float(rcut), float(width), ctypes.byref(df))
    return f, df.value


def gto_constants(nmax, rcut):
    s, d, n = np.zeros(nmax), np.zeros(nmax), np.zeros(nmax)
    lib().orc_gto_constants(nmax, rcut, _p(s), _p(d), _p(n))
    return s, d, n


def overlap(nmax, rcut):
    S = np.zeros((nmax, nmax))
    lib().orc_overlap(nmax, rcut, _p(S))
    return S


def inverse_sqrt(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    X = np.zeros_like(A)
    st = lib().orc_inverse_sqrt(A.shape[0], _p(A), _p(X))
    if st:
        raise ValueError("matrix not positive definite")
    return X


def orth_matrix(nmax, rcut):
    X = np.zeros((nmax, nmax))
    if lib().orc_orth_matrix(nmax, rcut, _p(X)):
        raise ValueError("overlap not positive definite")
    return X


def hyp1f1(a, b, z):
    return lib().orc_hyp1f1(float(a), float(b), float(z))


def radial_integral(nmax, lmax, rcut, sigma, r, deriv=False):
    I = np.zeros((nmax, lmax + 1))
    dI = np.zeros((nmax, lmax + 1)) if deriv else None
    lib().orc_radial_integral(nmax, lmax, rcut, sigma, float(r), _p(I), _p(dI))
    return (I, dI) if deriv else I


def radial_integral_orth(nmax, lmax, rcut, sigma, r, deriv=False):
    I = np.zeros((nmax, lmax + 1))
    dI = np.zeros((nmax, lmax + 1)) if deriv else None
    lib().orc_radial_integral_orth(nmax, lmax, rcut, sigma, float(r), _p(I), _p(dI))
    return (I, dI) if deriv else I


def gauss_legendre(n):
    """Gauss-Legendre points and weights on [-1, 1] (ascending)."""
    t, w = np.zeros(n), np.zeros(n)
    lib().orc_gauss_legendre(int(n), _p(t), _p(w))
    return t, w


def sph_bessel_i(l, z, deriv=False):
    """Modified spherical Bessel function i_l(z) (and d/dz) by its series."""
    d = ctypes.c_double()
    v = lib().orc_sph_bessel_i(int(l), float(z), ctypes.byref(d))
    return (v, d.value) if deriv else v


def dvr_points(nmax, rcut, sigma):
    """DVR points x_n and weights w_n on [0, rcut + 3 sigma] (Sec. 4.C)."""
    x, w = np.zeros(nmax), np.zeros(nmax)
    lib().orc_dvr_points(int(nmax), float(rcut), float(sigma), _p(x), _p(w))
    return x, w


def dvr_radial_integral(nmax, lmax, rcut, sigma, r, deriv=False):
    """DVR radial integral I_nl(r) [nmax, lmax+1] (and d/dr), Sec. 4.C."""
    I = np.zeros((nmax, lmax + 1))
    dI = np.zeros((nmax, lmax + 1)) if deriv else None
    lib().orc_dvr_radial_integral(nmax, lmax, rcut, sigma, float(r), _p(I), _p(dI))
    return (I, dI) if deriv else I


def ylm(lmax, v, deriv=False):
    v = np.ascontiguousarray(v, dtype=np.float64)
    L2 = (lmax + 1) ** 2
    Y = np.zeros(L2)
    dY = np.zeros((3, L2)) if deriv else None
    lib().orc_ylm(lmax, _p(v), _p(Y), _p(dY))
    return (Y, dY) if deriv else Y


# ---------------------------------------------------------------- pipeline
class Neighbors:
    def __init__(self, pair_offsets, pair_j, pair_shift, pair_vec):
        self.pair_offsets, self.pair_j, self.pair_shift, self.pair_vec = pair_offsets, pair_j, pair_shift, pair_vec

    @property
    def n_pairs(self):
        return int(self.pair_offsets[-1])


def neighbors(batch, rcut=None):
    rcut = float(batch.hypers["rcut"] if rcut is None else rcut)
    N = batch.n_atoms
    offs = np.zeros(N + 1, dtype=np.int64)
    pos = np.ascontiguousarray(batch.positions, dtype=np.float64)
    cells = np.ascontiguousarray(batch.cells, dtype=np.float64)
    pbc = np.ascontiguousarray(batch.pbc, dtype=np.uint8)
    spc = np.ascontiguousarray(batch.species, dtype=np.int32)
    ao = np.ascontiguousarray(batch.atom_offsets, dtype=np.int64)
    L = lib()
    args = (batch.n_structures, _p(ao, ctypes.c_int64), _p(pos), _p(cells), _p(pbc, ctypes.c_uint8),
            _p(spc, ctypes.c_int32), rcut)
    st = L.orc_neighbors(*args, _p(offs, ctypes.c_int64), None, None, None)
    if st:
        raise ValueError(f"oracle neighbours failed ({st})")
    P = int(offs[-1])
    pj = np.zeros(max(P, 1), dtype=np.int32)
    ps = np.zeros((max(P, 1), 3), dtype=np.int32)
    pv = np.zeros((max(P, 1), 3))
    st = L.orc_neighbors(*args, _p(offs, ctypes.c_int64), _p(pj, ctypes.c_int32), _p(ps, ctypes.c_int32), _p(pv))
    if st:
        raise ValueError(f"oracle neighbours failed ({st})")
    return Neighbors(offs, pj[:P], ps[:P], pv[:P])


def _centres(nl, centres):
    N = nl.pair_offsets.shape[0] - 1
    if centres is None:
        centres = np.arange(N, dtype=np.int64)
    return np.ascontiguousarray(centres, dtype=np.int64)


def expansion(hypers, species, nl, centres=None):
    S, nmax, lmax = int(hypers["n_species"]), int(hypers["nmax"]), int(hypers["lmax"])
    cen = _centres(nl, centres)
    c = np.zeros((cen.shape[0], S, nmax, (lmax + 1) ** 2))
    spc = np.ascontiguousarray(species, dtype=np.int32)
    pv = np.ascontiguousarray(nl.pair_vec, dtype=np.float64).reshape(-1, 3)
    if pv.shape[0] == 0:
        pv = np.zeros((1, 3))
    pj = nl.pair_j if nl.pair_j.shape[0] else np.zeros(1, dtype=np.int32)
    st = lib().orc_expansion(*_hy(hypers), _p(spc, ctypes.c_int32), _p(nl.pair_offsets, ctypes.c_int64),
                             _p(np.ascontiguousarray(pj), ctypes.c_int32), _p(pv), cen.shape[0],
                             _p(cen, ctypes.c_int64), _p(c))
    if st:
        raise ValueError("oracle expansion failed")
    return c


def power_spectrum(hypers, coeffs):
    S, nmax, lmax = int(hypers["n_species"]), int(hypers["nmax"]), int(hypers["lmax"])
    K = S * nmax
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    n = c.shape[0]
    p = np.zeros((n, lmax + 1, K * (K + 1) // 2))
    lib().orc_power_spectrum(S, nmax, lmax, n, _p(c), _p(p))
    return p


def power_spectrum_selected(hypers, coeffs, selected):
    """Sec. 4.H: only the chosen invariants q = (k1, k2, l), each the sum
    over m of c[k1, lm] c[k2, lm] (channels k = a n, R4's normalisation),
    for every centre.  coeffs [N, S, nmax, L2]; selected [n_sel, 3];
    returns [N, n_sel]."""
    S, nmax = int(hypers["n_species"]), int(hypers["nmax"])
    c = np.asarray(coeffs, dtype=np.float64)
    c = c.reshape(c.shape[0], S * nmax, -1)
    out = np.zeros((c.shape[0], len(selected)))
    for q, (k1, k2, l) in enumerate(np.asarray(selected, dtype=np.int64)):
        m = slice(l * l, l * l + 2 * l + 1)
        out[:, q] = (c[:, k1, m] * c[:, k2, m]).sum(axis=1)
    return out


def power_spectrum_selected_vjp(hypers, coeffs, selected, grad):
    """Adjoint of power_spectrum_selected: dL/dc for L = sum_i sum_q
    grad[i, q] p_sel[i, q]; each invariant q = (k1, k2, l) gives
    grad[q] c[k2, lm] to (k1, lm) and grad[q] c[k1, lm] to (k2, lm)."""
    S, nmax = int(hypers["n_species"]), int(hypers["nmax"])
    c = np.asarray(coeffs, dtype=np.float64)
    shape = c.shape
    c = c.reshape(shape[0], S * nmax, -1)
    g = np.asarray(grad, dtype=np.float64)
    out = np.zeros_like(c)
    for q, (k1, k2, l) in enumerate(np.asarray(selected, dtype=np.int64)):
        m = slice(l * l, l * l + 2 * l + 1)
        out[:, k1, m] += g[:, q:q + 1] * c[:, k2, m]
        out[:, k2, m] += g[:, q:q + 1] * c[:, k1, m]
    return out.reshape(shape)


def gradients(hypers, species, nl, centres=None):
    """Forward-mode gradient rows for the listed centres.  Returns
    (dc [rows,3,nmax,L2], dc_self [n,3,S,nmax,L2], dp [rows,3,lmax+1,KK],
    dp_self [n,3,lmax+1,KK]) with the pair rows of the centres concatenated
    in their pair order."""
    S, nmax, lmax = int(hypers["n_species"]), int(hypers["nmax"]), int(hypers["lmax"])
    K, L2 = S * nmax, (lmax + 1) ** 2
    KK = K * (K + 1) // 2
    cen = _centres(nl, centres)
    rows = int(sum(nl.pair_offsets[c + 1] - nl.pair_offsets[c] for c in cen))
    dc = np.zeros((max(rows, 1), 3, nmax, L2))
    dcs = np.zeros((cen.shape[0], 3, S, nmax, L2))
    dp = np.zeros((max(rows, 1), 3, lmax + 1, KK))
    dps = np.zeros((cen.shape[0], 3, lmax + 1, KK))
    spc = np.ascontiguousarray(species, dtype=np.int32)
    pv = np.ascontiguousarray(nl.pair_vec, dtype=np.float64).reshape(-1, 3)
    if pv.shape[0] == 0:
        pv = np.zeros((1, 3))
    pj = nl.pair_j if nl.pair_j.shape[0] else np.zeros(1, dtype=np.int32)
    st = lib().orc_gradients(*_hy(hypers), _p(spc, ctypes.c_int32), _p(nl.pair_offsets, ctypes.c_int64),
                             _p(np.ascontiguousarray(pj), ctypes.c_int32), _p(pv), cen.shape[0],
                             _p(cen, ctypes.c_int64), _p(dc), _p(dcs), _p(dp), _p(dps))
    if st:
        raise ValueError("oracle gradients failed")
    return dc[:rows], dcs, dp[:rows], dps


def vjp(hypers, species, nl, grad_p):
    """dL/dr [N,3] and dL/dr_ji [P,3] for L = sum_i <grad_p_i, p_i>."""
    N = nl.pair_offsets.shape[0] - 1
    P = nl.n_pairs
    g = np.ascontiguousarray(grad_p, dtype=np.float64)
    out = np.zeros((N, 3))
    gp = np.zeros((max(P, 1), 3))
    spc = np.ascontiguousarray(species, dtype=np.int32)
    pv = np.ascontiguousarray(nl.pair_vec, dtype=np.float64).reshape(-1, 3)
    if pv.shape[0] == 0:
        pv = np.zeros((1, 3))
    pj = nl.pair_j if nl.pair_j.shape[0] else np.zeros(1, dtype=np.int32)
    st = lib().orc_vjp(*_hy(hypers), N, _p(spc, ctypes.c_int32), _p(nl.pair_offsets, ctypes.c_int64),
                       _p(np.ascontiguousarray(pj), ctypes.c_int32), _p(pv), _p(g), _p(out), _p(gp))
    if st:
        raise ValueError("oracle vjp failed")
    return out, gp[:P]


def virial(atom_offsets, nl, grad_pair):
    """App. B, Eq. energy-virial: per structure s, W_s[a][b] = sum over the
    pairs q of the centres of s of dL/dr_q[a] * r_q[b] (r_q the pair vector,
    images included), the derivative of L under the deformation
    r -> (1 + eps) r of positions and cell."""
    offs = np.asarray(atom_offsets, dtype=np.int64)
    po = np.asarray(nl.pair_offsets, dtype=np.int64)
    vec = np.asarray(nl.pair_vec, dtype=np.float64).reshape(-1, 3)
    g = np.asarray(grad_pair, dtype=np.float64).reshape(-1, 3)
    W = np.zeros((len(offs) - 1, 3, 3))
    for s in range(len(offs) - 1):
        q0, q1 = po[offs[s]], po[offs[s + 1]]
        W[s] = g[q0:q1].T @ vec[q0:q1]
    return W


def gpr_predict(species, feats, active_species, active_feats, weights, zeta):
    """Sparse kernel model of Sec. 5.B.  Per centre i (Eq. sparse-gp with the
    polynomial kernel k = (M_I . p_i)^zeta):
        E_i = sum over active points I of species a_i of w_I (M_I . p_i)^zeta,
    and the derivative of E_i with respect to the features, with the sum
    over the active set taken first (Eq. gpr-force-order):
        dE_i/dp_i = sum over the same I of w_I zeta (M_I . p_i)^(zeta-1) M_I.
    feats [N, F], active_feats [n_active, F]; returns (E [N], dE/dp [N, F]).
    Structure energies are the sums of E_i over their centres (Eq.
    additive-energy-model); forces and virial follow from dE/dp through the
    adjoint (vjp, virial)."""
    p = np.asarray(feats, dtype=np.float64).reshape(len(species), -1)
    M = np.asarray(active_feats, dtype=np.float64).reshape(len(active_species), -1)
    w = np.asarray(weights, dtype=np.float64)
    same = np.asarray(species)[:, None] == np.asarray(active_species)[None, :]
    k1 = p @ M.T                                    # M_I . p_i
    coef = np.where(same, w[None, :], 0.0)
    E = (coef * k1 ** zeta).sum(axis=1)
    dk = coef * zeta * k1 ** (zeta - 1)
    return E, dk @ M


def features(batch, centres=None):
    """Neighbours, coefficients and power spectrum of a batch (FP64)."""
    nl = neighbors(batch)
    c = expansion(batch.hypers, batch.species, nl, centres)
    return nl, c, power_spectrum(batch.hypers, c)
