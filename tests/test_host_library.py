"""Host-side checks of the HIP library that need no GPU: every symbol the
header declares is exported, every host-side error path returns its status
before anything is enqueued, and the FP64 table builder (the library's own
1F1 recurrence, eigen-solver and spline) agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

import oracle
import paper_2101_08814_amd as P
from paper_2101_08814_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "soap_mi355x.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(soap_[a-z_0-9]+)\s*\(", txt)))


def test_library_loads_and_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _declared()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(L, name), f"{name} declared in the header but not exported"
    assert sorted(_lib.EXPORTS) == declared
    assert L.soap_abi_version() == 2


def _create(**kw):
    h = dict(n_species=1, nmax=8, lmax=6, include_center=1, rcut=5.0, cutoff_width=0.5, sigma=0.5,
             spline_accuracy=1e-8, radial_basis=0, reserved=0)
    h.update(kw)
    hy = _lib.soap_hypers(h["n_species"], h["nmax"], h["lmax"], h["include_center"], h["rcut"],
                          h["cutoff_width"], h["sigma"], h["spline_accuracy"], h["radial_basis"], h["reserved"])
    out = ctypes.c_void_p()
    st = _lib.lib().soap_calculator_create(ctypes.byref(hy), ctypes.byref(out))
    return st, out


@pytest.mark.parametrize("bad", [dict(n_species=0), dict(nmax=0), dict(nmax=17), dict(lmax=-1), dict(lmax=13),
                                 dict(rcut=0.0), dict(rcut=float("nan")), dict(sigma=-1.0),
                                 dict(cutoff_width=0.0), dict(cutoff_width=6.0), dict(include_center=2),
                                 dict(spline_accuracy=0.0)])
def test_invalid_hypers_rejected(bad):
    st, out = _create(**bad)
    assert st == _lib.SOAP_EINVAL
    assert not out.value
    assert _lib.lib().soap_last_error()


def test_null_arguments_rejected():
    L = _lib.lib()
    assert L.soap_calculator_create(None, None) == _lib.SOAP_EINVAL
    info = _lib.soap_table_info()
    assert L.soap_calculator_info(None, ctypes.byref(info)) == _lib.SOAP_EINVAL
    assert L.soap_calculator_destroy(None) == _lib.SOAP_OK


@pytest.fixture(scope="module")
def calc():
    return P.Calculator(2, 6, 4, 4.0, 0.5)


def _nb_call(calc, **over):
    L = _lib.lib()
    dummy = ctypes.c_void_p(256)   # never dereferenced: validation fails first
    args = dict(n_structures=1, n_atoms=4, atom_offsets=dummy, cells=dummy, pbc=dummy, positions=dummy,
                species=dummy, workspace=dummy, workspace_bytes=1 << 30, capacity=100, prec=_lib.SOAP_F32,
                pair_offsets=dummy, pair_j=dummy, pair_shift=dummy, pair_vec=dummy, pair_transpose=None)
    args.update(over)
    e = _lib.soap_exec(None, None)
    return L.soap_compute_neighbors(calc.handle, ctypes.byref(e), args["n_structures"], args["n_atoms"],
                                    args["atom_offsets"], args["cells"], args["pbc"], args["positions"],
                                    args["species"], args["workspace"], args["workspace_bytes"], args["capacity"],
                                    args["prec"], args["pair_offsets"], args["pair_j"], args["pair_shift"],
                                    args["pair_vec"], args["pair_transpose"])


@pytest.mark.parametrize("over", [
    dict(capacity=-1), dict(n_structures=-1), dict(n_atoms=-1), dict(prec=_lib.SOAP_BF16_F32ACC),
    dict(n_structures=0), dict(workspace_bytes=16), dict(positions=None), dict(pair_offsets=None),
    dict(pair_j=None), dict(atom_offsets=None), dict(cells=None),
    dict(pair_vec=ctypes.c_void_p(258)),                             # misaligned
    dict(workspace=ctypes.c_void_p(264)),                            # workspace must be 256-aligned
])
def test_neighbor_host_errors(calc, over):
    assert _nb_call(calc, **over) == _lib.SOAP_EINVAL
    assert _lib.lib().soap_last_error()


def test_workspace_size(calc):
    n1 = calc.neighbors_workspace_size(1, 10)
    n2 = calc.neighbors_workspace_size(4, 1000)
    assert 0 < n1 < n2
    L = _lib.lib()
    n = ctypes.c_size_t()
    assert L.soap_neighbors_workspace_size(calc.handle, -1, 10, ctypes.byref(n)) == _lib.SOAP_EINVAL


def test_feature_entry_points_host_errors(calc):
    L = _lib.lib()
    e = _lib.soap_exec(None, None)
    d = ctypes.c_void_p(256)
    # bad precision, negative atoms, mismatched optional outputs, null required arrays
    assert L.soap_spherical_expansion(calc.handle, ctypes.byref(e), 7, 4, d, d, d, d, 10, d, None, None) == -1
    assert L.soap_spherical_expansion(calc.handle, ctypes.byref(e), 1, -4, d, d, d, d, 10, d, None, None) == -1
    assert L.soap_spherical_expansion(calc.handle, ctypes.byref(e), 1, 4, d, d, d, d, 10, d, d, None) == -1
    assert L.soap_spherical_expansion(calc.handle, ctypes.byref(e), 1, 4, None, d, d, d, 10, d, None, None) == -1
    assert L.soap_spherical_expansion(calc.handle, ctypes.byref(e), 1, 4, d, d, d, d, -10, d, None, None) == -1
    assert L.soap_power_spectrum(calc.handle, ctypes.byref(e), 2, 4, d, d, d, d, d, 10, d, d, d, d) == -1
    assert L.soap_power_spectrum(calc.handle, ctypes.byref(e), 1, 4, None, d, None, None, None, 0, None, None,
                                 None, None) == -1
    assert L.soap_features(calc.handle, ctypes.byref(e), 1, 4, d, d, d, d, 10, d, d, d, None, d, d) == -1
    assert L.soap_features(calc.handle, ctypes.byref(e), 0, 4, d, d, d, ctypes.c_void_p(260), 10, d, d,
                           None, None, None, None) == -1          # float64 pair_vec misaligned
    assert L.soap_power_spectrum_backward(calc.handle, ctypes.byref(e), 1, 4, d, None, d) == -1
    assert L.soap_spherical_expansion_backward(calc.handle, ctypes.byref(e), 1, 4, d, d, d, d, None, 10, d, d,
                                               d) == -1
    # zero atoms is a valid no-op
    assert L.soap_features(calc.handle, ctypes.byref(e), 1, 0, None, None, None, None, 0, None, None, None,
                           None, None, None) == 0


# ------------------------------------------------------------ table builder
HYPERS = [
    dict(n_species=2, nmax=6, lmax=4, rcut=4.0, sigma=0.5),
    dict(n_species=1, nmax=8, lmax=6, rcut=5.0, sigma=0.5),
    dict(n_species=4, nmax=8, lmax=6, rcut=5.0, sigma=0.4),
    dict(n_species=2, nmax=10, lmax=8, rcut=6.0, sigma=0.5),
    dict(n_species=8, nmax=12, lmax=8, rcut=5.0, sigma=0.5),
]


@pytest.mark.parametrize("h", HYPERS)
def test_library_radial_integral_matches_oracle(h):
    """The library's recurrence-based 1F1 (with its series/asymptotic switch)
    and its own S^{-1/2} reproduce the oracle's direct-series radial integral."""
    c = P.Calculator(h["n_species"], h["nmax"], h["lmax"], h["rcut"], h["sigma"])
    # two FP64 computations of S^{-1/2} I differ by ~eps * ||S^{-1/2}|| ~ eps sqrt(cond S)
    tol = 1e-13 * np.sqrt(c.info()["overlap_condition"])
    rs = np.concatenate([[0.0, 1e-3], np.linspace(0.05, h["rcut"], 37)])
    I, dI = c.radial_integral_host(rs, exact=True)
    for k, r in enumerate(rs):
        Io, dIo = oracle.radial_integral_orth(h["nmax"], h["lmax"], h["rcut"], h["sigma"], r, deriv=True)
        scale = max(1.0, np.abs(Io).max())
        assert np.abs(I[k] - Io).max() <= tol * scale, (r, np.abs(I[k] - Io).max())
        assert np.abs(dI[k] - dIo).max() <= 10 * tol * max(1.0, np.abs(dIo).max()), r


@pytest.mark.parametrize("h", HYPERS)
def test_spline_table_accuracy(h):
    """Sec. 4.D: the spline the kernels evaluate stays within the requested
    1e-8 of the exact orthogonalised radial integral (checked against the
    oracle at points off the knots)."""
    c = P.Calculator(h["n_species"], h["nmax"], h["lmax"], h["rcut"], h["sigma"])
    info = c.info()
    assert info["max_error"] <= 1e-8
    assert info["n_intervals"] >= 1024
    rng = np.random.default_rng(0)
    rs = rng.uniform(0, h["rcut"], 60)
    I, dI = c.radial_integral_host(rs, exact=False)
    for k, r in enumerate(rs):
        Io, dIo = oracle.radial_integral_orth(h["nmax"], h["lmax"], h["rcut"], h["sigma"], r, deriv=True)
        assert np.abs(I[k] - Io).max() <= 1e-8
        assert np.abs(dI[k] - dIo).max() <= 2e-6


def test_radial_host_rejects_out_of_range(calc):
    with pytest.raises(P.SoapError):
        calc.radial_integral_host([5.0], exact=True)       # beyond rcut = 4


def test_spline_accuracy_is_honoured():
    coarse = P.Calculator(1, 8, 6, 5.0, 0.5, spline_accuracy=1e-6)
    fine = P.Calculator(1, 8, 6, 5.0, 0.5, spline_accuracy=1e-12)
    assert coarse.info()["n_intervals"] == 1024
    assert fine.info()["n_intervals"] > 1024
    assert fine.info()["max_error"] <= 1e-12


def test_selected_backward_plan_host():
    """The host plan of the selected-invariant adjoint: per row (k, l) the
    entries (q, partner) of every triple touching channel k at degree l, in
    q order, two per triple (k1 = k2 gives two entries in the same row);
    out-of-range triples are rejected with SOAP_EINVAL."""
    import ctypes
    from paper_2101_08814_amd import _lib
    L = _lib.lib()
    K, lmax = 4, 2
    tri = np.array([[0, 1, 0], [2, 2, 1], [1, 0, 0], [3, 1, 2]], dtype=np.int32)
    offs = np.zeros(K * (lmax + 1) + 1, dtype=np.int32)
    ent = np.zeros((2 * len(tri), 2), dtype=np.int32)
    st = L.soap_power_spectrum_selected_plan(K, lmax, len(tri), tri.ctypes.data, offs.ctypes.data,
                                             ent.ctypes.data)
    assert st == _lib.SOAP_OK
    expect = {}
    for q, (k1, k2, l) in enumerate(tri):
        expect.setdefault(k1 * (lmax + 1) + l, []).append((q, k2))
        expect.setdefault(k2 * (lmax + 1) + l, []).append((q, k1))
    for r in range(K * (lmax + 1)):
        got = [tuple(x) for x in ent[offs[r]:offs[r + 1]]]
        assert got == expect.get(r, [])
    bad = tri.copy()
    bad[2] = (0, 4, 0)
    st = L.soap_power_spectrum_selected_plan(K, lmax, len(bad), bad.ctypes.data, offs.ctypes.data,
                                             ent.ctypes.data)
    assert st == _lib.SOAP_EINVAL


def test_new_entry_points_reject_bad_arguments_on_host():
    """Host-side checks of the virial, sparse-model and selected-invariant
    entry points return SOAP_EINVAL before any device work."""
    import ctypes
    L = _lib.lib()
    e = _lib.soap_exec(None, None)
    ref = ctypes.byref(e)
    nb = ctypes.c_size_t()
    # virial: BF16 is not a virial precision; negative structure count
    assert L.soap_virial(ref, _lib.SOAP_BF16_F32ACC, 1, None, 0, None, None, None, 0, None, None) == _lib.SOAP_EINVAL
    assert L.soap_virial(ref, _lib.SOAP_F32, -1, None, 0, None, None, None, 0, None, None) == _lib.SOAP_EINVAL
    # sparse model: zeta out of range, too many features, workspace too small
    assert L.soap_gpr_predict(ref, _lib.SOAP_F32, 4, 8, None, None, 2, None, None, None, 0, None, 0, None,
                              None) == _lib.SOAP_EINVAL
    assert L.soap_gpr_predict(ref, _lib.SOAP_F32, 4, 64 * 65535 + 1, None, None, 2, None, None, None, 2, None, 0,
                              None, None) == _lib.SOAP_EINVAL
    assert L.soap_gpr_workspace_size(_lib.SOAP_F32, 4, 8, 2, ctypes.byref(nb)) == _lib.SOAP_OK and nb.value > 0
    assert L.soap_gpr_predict(ref, _lib.SOAP_F32, 4, 8, None, None, 2, None, None, None, 2, None, nb.value - 1,
                              None, None) == _lib.SOAP_EINVAL
    assert L.soap_gpr_workspace_size(_lib.SOAP_F32, 4, 8, 0, ctypes.byref(nb)) == _lib.SOAP_EINVAL
    # selected invariants: lmax above 12; one centre's coefficients beyond 160 KB of LDS
    assert L.soap_power_spectrum_selected(ref, _lib.SOAP_F32, 1, 4, 13, None, 1, None, None) == _lib.SOAP_EINVAL
    assert L.soap_power_spectrum_selected(ref, _lib.SOAP_F64, 1, 400, 12, None, 1, None, None) == _lib.SOAP_EINVAL
    assert L.soap_power_spectrum_selected_backward(ref, _lib.SOAP_F32, 1, 4, 2, None, -1, None, None, None,
                                                   None) == _lib.SOAP_EINVAL
    msg = L.soap_last_error().decode()
    assert "n_selected" in msg


def test_forced_allocation_failure(calc, monkeypatch):
    """SOAP_FAIL_ALLOC=1 makes the calculator creation and every workspace
    query report SOAP_ENOMEM (the library's out-of-memory path), and the
    library recovers once it is unset."""
    L = _lib.lib()
    n = ctypes.c_size_t()
    nparam = ctypes.c_int64()
    monkeypatch.setenv("SOAP_FAIL_ALLOC", "1")
    st, out = _create()
    assert st == _lib.SOAP_ENOMEM and not out.value
    assert b"SOAP_FAIL_ALLOC" in L.soap_last_error()
    assert L.soap_neighbors_workspace_size(calc.handle, 1, 10, ctypes.byref(n)) == _lib.SOAP_ENOMEM
    assert L.soap_gpr_workspace_size(_lib.SOAP_F32, 10, 20, 30, ctypes.byref(n)) == _lib.SOAP_ENOMEM
    assert L.soap_compress_workspace_size(calc.handle, 4, 8, ctypes.byref(n)) == _lib.SOAP_ENOMEM
    # queries that size nothing are unaffected
    assert L.soap_compress_n_params(calc.handle, 4, 8, ctypes.byref(nparam)) == _lib.SOAP_OK
    with pytest.raises(_lib.SoapError) as err:
        calc.neighbors_workspace_size(1, 10)
    assert err.value.status == _lib.SOAP_ENOMEM
    monkeypatch.delenv("SOAP_FAIL_ALLOC")
    st, out = _create()
    assert st == _lib.SOAP_OK and out.value
    assert L.soap_calculator_destroy(out) == _lib.SOAP_OK
    assert L.soap_neighbors_workspace_size(calc.handle, 1, 10, ctypes.byref(n)) == _lib.SOAP_OK and n.value > 0


@pytest.mark.parametrize("h", HYPERS)
def test_library_dvr_radial_integral_matches_oracle(h):
    """DVR basis (Sec. 4.C): the library's Golub-Welsch points and its
    scaled Bessel functions (series below a switch point, closed forms and
    upward recurrence above) reproduce the oracle's Newton points and power
    series, for the direct values and, within the requested accuracy, for
    the spline the kernels use."""
    c = P.Calculator(h["n_species"], h["nmax"], h["lmax"], h["rcut"], h["sigma"], radial_basis="dvr")
    info = c.info()
    assert info["overlap_condition"] == 1.0
    assert info["max_error"] <= 1e-8
    rs = np.concatenate([[0.0, 1e-3], np.linspace(0.05, h["rcut"], 37)])
    I, dI = c.radial_integral_host(rs, exact=True)
    Is, dIs = c.radial_integral_host(rs, exact=False)
    for k, r in enumerate(rs):
        Io, dIo = oracle.dvr_radial_integral(h["nmax"], h["lmax"], h["rcut"], h["sigma"], r, deriv=True)
        scale = max(1.0, np.abs(Io).max())
        assert np.abs(I[k] - Io).max() <= 1e-13 * scale, (r, np.abs(I[k] - Io).max())
        assert np.abs(dI[k] - dIo).max() <= 1e-12 * max(1.0, np.abs(dIo).max()), r
        assert np.abs(Is[k] - Io).max() <= 1e-8
        assert np.abs(dIs[k] - dIo).max() <= 2e-6


def test_radial_basis_validated():
    st, out = _create(radial_basis=2)
    assert st == _lib.SOAP_EINVAL and not out.value
    st, out = _create(reserved=1)
    assert st == _lib.SOAP_EINVAL and not out.value
    st, out = _create(radial_basis=1)
    assert st == _lib.SOAP_OK and out.value
    assert _lib.lib().soap_calculator_destroy(out) == _lib.SOAP_OK


class _StubNeighbors:
    pass


class _StubCalc:
    """Stands in for a calculator on the CPU: returns zero tensors from every
    kernel call and a chosen value from the device status word."""

    check_device = P.Calculator.check_device

    def __init__(self, forward_status, backward_status):
        self.statuses = [forward_status, backward_status]

    def device_status(self):
        return self.statuses.pop(0) if len(self.statuses) > 1 else self.statuses[0]

    def compute_neighbors(self, positions, species, *a, **k):
        return _StubNeighbors()

    def features(self, nl, species, dtype):
        n = species.shape[0]
        return torch.zeros((n, 4), dtype=dtype), torch.zeros((n, 3), dtype=dtype)

    def power_spectrum_backward(self, c, grad_p):
        return torch.zeros_like(c)

    def spherical_expansion_backward(self, nl, species, gc):
        return torch.zeros((species.shape[0], 3), dtype=gc.dtype), None


@pytest.mark.parametrize("where", ["forward", "backward"])
def test_autograd_function_raises_on_device_status(where):
    """SOAPFunction reads the status word after each pass: a kernel error
    (here SOAP_EGEOMETRY) raises instead of returning features or forces."""
    from paper_2101_08814_amd.soap import SOAPFunction
    calc = _StubCalc(_lib.SOAP_EGEOMETRY if where == "forward" else 0,
                     _lib.SOAP_EGEOMETRY if where == "backward" else 0)
    pos = torch.zeros((5, 3), dtype=torch.float64, requires_grad=True)
    spc = torch.zeros(5, dtype=torch.int32)
    if where == "forward":
        with pytest.raises(_lib.SoapError, match="SOAP_EGEOMETRY"):
            SOAPFunction.apply(pos, calc, spc, None, None, None, torch.float32)
        return
    p = SOAPFunction.apply(pos, calc, spc, None, None, None, torch.float32)
    with pytest.raises(_lib.SoapError, match="SOAP_EGEOMETRY"):
        p.sum().backward()


def test_autograd_function_passes_clean_status():
    from paper_2101_08814_amd.soap import SOAPFunction
    calc = _StubCalc(0, 0)
    pos = torch.zeros((5, 3), dtype=torch.float64, requires_grad=True)
    p = SOAPFunction.apply(pos, calc, torch.zeros(5, dtype=torch.int32), None, None, None, torch.float32)
    p.sum().backward()
    assert pos.grad is not None and pos.grad.shape == (5, 3)


def _checkpoint_bytes(n_out, hidden, channels, lmax, n_params, step=3, version=1, magic=b"SOAPCMP1", seed=0):
    """A compression checkpoint in the documented file format (header,
    three float arrays, FNV-1a 64-bit hash of everything before it)."""
    import struct
    head = magic + struct.pack("<6i2q", version, n_out, hidden, channels, lmax, 0, step, n_params)
    body = np.random.default_rng(seed).normal(size=3 * n_params).astype("<f4").tobytes()
    h = 14695981039346656037
    for b in head + body:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return head + body + struct.pack("<Q", h)


def test_compress_checkpoint_validation(tmp_path):
    """soap_compress_load checks the file before any device copy: missing,
    foreign, wrong shape, truncated, trailing data and hash mismatch are all
    SOAP_EINVAL; a well-formed file passes to the copy (which has no device
    here)."""
    c = P.Calculator(2, 4, 3, 4.0, 0.5)
    L = _lib.lib()
    n = ctypes.c_int64()
    assert L.soap_compress_n_params(c.handle, 4, 8, ctypes.byref(n)) == 0
    npar = int(n.value)
    fake = ctypes.c_void_p(1 << 20)      # aligned, never dereferenced on these paths
    step = ctypes.c_int64()

    def load(data):
        path = tmp_path / "x.ckpt"
        if data is None:
            path = tmp_path / "missing.ckpt"
        else:
            path.write_bytes(data)
        return L.soap_compress_load(c.handle, 4, 8, os.fsencode(str(path)), fake, fake, fake, ctypes.byref(step))

    good = _checkpoint_bytes(4, 8, c.K, c.lmax, npar)
    assert load(None) == _lib.SOAP_EINVAL
    assert load(b"not a checkpoint at all" * 4) == _lib.SOAP_EINVAL
    assert load(_checkpoint_bytes(4, 9, c.K, c.lmax, npar)) == _lib.SOAP_EINVAL
    assert load(_checkpoint_bytes(4, 8, c.K, c.lmax, npar, version=2)) == _lib.SOAP_EINVAL
    assert load(good[:-9]) == _lib.SOAP_EINVAL
    assert load(good + b"\0") == _lib.SOAP_EINVAL
    flipped = bytearray(good)
    flipped[60] ^= 1
    assert load(bytes(flipped)) == _lib.SOAP_EINVAL
    assert b"corrupted" in L.soap_last_error()
    st = load(good)
    assert st in (_lib.SOAP_OK, _lib.SOAP_EDEVICE), st
