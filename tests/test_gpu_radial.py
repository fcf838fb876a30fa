"""GPU parity of the radial part: the DVR basis (Sec. 4.C) through every
kernel, and the device entry point soap_radial_integral (spline and direct
evaluation, GTO and DVR) against the FP64 oracle.

Tolerances: features as in the other parity tests (FP64 1e-7, FP32 1e-6 on
c and p, 1e-5 on gradient rows and the adjoint).  Radial integrals: the
direct device evaluation runs the host's FP64 code, so it matches the
host's values to rounding (1e-14 relative, times sqrt(cond S) for the GTO
orthogonalisation) and the oracle's to the host's own bound; the FP64
spline to the requested spline accuracy 1e-8 (values) and 2e-6 (its
derivative, one order of the cubic lower); the FP32 spline to 2e-6 of the
largest value (FP32 rounding of the cubic's terms).
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic
import paper_2101_08814_amd as P

pytestmark = pytest.mark.gpu


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    assert P.LIB_PATH


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def dvr(batch):
    return synthetic.Batch(batch.positions, batch.species, batch.atom_offsets, batch.cells, batch.pbc,
                           dict(batch.hypers, radial_basis=1), batch.name + "_dvr")


def gpu_features(batch, dtype, gradients=False):
    calc = P.Calculator.from_hypers(batch.hypers)
    pos = torch.tensor(batch.positions, dtype=torch.float64, device="cuda")
    spc = torch.tensor(batch.species, dtype=torch.int32, device="cuda")
    nl = calc.compute_neighbors(pos, spc, batch.atom_offsets, batch.cells, batch.pbc, vec_dtype=dtype)
    out = calc.features(nl, spc, dtype, gradients)
    assert calc.device_status() == 0
    return calc, nl, spc, [o.double().cpu().numpy() for o in out]


# ------------------------------------------------------------ DVR features
def test_dvr_clusters_fp64_parity():
    b = dvr(synthetic.clusters_2species())
    print("[dvr clusters f64]", flush=True)
    _, _, _, (c, p) = gpu_features(b, torch.float64)
    _, ref_c, ref_p = oracle.features(b)
    ec, ep = rel(c, ref_c), rel(p, ref_p)
    print(f"  rel c={ec:.3e} p={ep:.3e}")
    assert ec <= 1e-7 and ep <= 1e-7


def test_dvr_diamond_fp32_gradients_parity():
    """1024-atom diamond with the DVR basis, FP32: c, p and the gradient
    rows against the oracle."""
    b = dvr(synthetic.diamond_bulk())
    print("[dvr diamond f32 grads]", flush=True)
    _, _, _, (c, p, dc, dcs, dp, dps) = gpu_features(b, torch.float32, gradients=True)
    ref_nl = oracle.neighbors(b)
    ref_c = oracle.expansion(b.hypers, b.species, ref_nl)
    ref_p = oracle.power_spectrum(b.hypers, ref_c)
    rdc, rdcs, rdp, rdps = oracle.gradients(b.hypers, b.species, ref_nl)
    n = ref_nl.n_pairs
    errs = dict(c=rel(c, ref_c), p=rel(p, ref_p), dc=rel(dc[:n], rdc), dcs=rel(dcs, rdcs), dp=rel(dp[:n], rdp),
                dps=rel(dps, rdps))
    print("  " + " ".join(f"{k}={v:.3e}" for k, v in errs.items()))
    assert errs["c"] <= 1e-6 and errs["p"] <= 1e-6
    assert max(errs["dc"], errs["dcs"], errs["dp"], errs["dps"]) <= 1e-5


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_dvr_vjp_matches_oracle(dt):
    """Adjoint dL/dr with the DVR basis, L = <W, p>, 512-atom liquid."""
    b = dvr(synthetic.liquid_bulk(n_atoms=512))
    print(f"[dvr vjp {dt}]", flush=True)
    calc, nl, spc, (c, p) = gpu_features(b, dt)
    W = np.random.default_rng(2104).normal(size=p.shape)
    cd, _ = calc.features(nl, spc, dt)
    gc = calc.power_spectrum_backward(cd, torch.tensor(W, dtype=dt, device="cuda"))
    gpos, gpair = calc.spherical_expansion_backward(nl, spc, gc)
    assert calc.device_status() == 0
    ref_nl = oracle.neighbors(b)
    g_ref, gp_ref = oracle.vjp(b.hypers, b.species, ref_nl, W)
    e = rel(gpos.double().cpu().numpy(), g_ref)
    ep = rel(gpair[:ref_nl.n_pairs].double().cpu().numpy(), gp_ref)
    print(f"  rel dL/dr={e:.3e} per-pair={ep:.3e}")
    tol = 1e-7 if dt == torch.float64 else 1e-5
    assert e <= tol and ep <= tol


def test_dvr_differs_from_gto():
    """The basis switch reaches the kernels: the same structure gives other
    coefficients (and the same for both when the switch is off)."""
    b = synthetic.clusters_2species().subset([0, 1])
    _, _, _, (c0, _) = gpu_features(b, torch.float64)
    _, _, _, (c1, _) = gpu_features(dvr(b), torch.float64)
    assert rel(c1, c0) > 1e-2


# ------------------------------------------------------------ soap_radial_integral
RADIAL_HYPERS = [
    dict(n_species=1, nmax=8, lmax=6, rcut=5.0, sigma=0.5),
    dict(n_species=2, nmax=10, lmax=8, rcut=6.0, sigma=0.5),
    dict(n_species=1, nmax=12, lmax=12, rcut=5.0, sigma=0.4),
    dict(n_species=1, nmax=4, lmax=0, rcut=3.0, sigma=0.3),
]


def _radii(h):
    """0, tiny r, a ragged count of points across (0, rcut] and rcut itself."""
    rng = np.random.default_rng(2105)
    return np.concatenate([[0.0, 1e-6, 1e-3], np.sort(rng.uniform(0.0, h["rcut"], 197)), [h["rcut"]]])


def _oracle_radial(h, basis, rs):
    f = oracle.dvr_radial_integral if basis == "dvr" else oracle.radial_integral_orth
    out = [f(h["nmax"], h["lmax"], h["rcut"], h["sigma"], r, deriv=True) for r in rs]
    I = np.stack([o[0] for o in out], axis=-1)
    dI = np.stack([o[1] for o in out], axis=-1)
    return I, dI


@pytest.mark.parametrize("basis", ["gto", "dvr"])
@pytest.mark.parametrize("hi", range(len(RADIAL_HYPERS)))
def test_radial_integral_entry_point(basis, hi):
    h = RADIAL_HYPERS[hi]
    print(f"[radial {basis} {h}]", flush=True)
    calc = P.Calculator(h["n_species"], h["nmax"], h["lmax"], h["rcut"], h["sigma"], radial_basis=basis)
    cond = calc.info()["overlap_condition"]
    rs = _radii(h)
    rd = torch.tensor(rs, dtype=torch.float64, device="cuda")
    Ie, dIe = (t.cpu().numpy() for t in calc.radial_integral(rd, exact=True))
    I64, dI64 = (t.cpu().numpy() for t in calc.radial_integral(rd, exact=False, dtype=torch.float64))
    I32, dI32 = (t.double().cpu().numpy() for t in calc.radial_integral(rd, exact=False, dtype=torch.float32))
    Ionly = calc.radial_integral(rd, exact=False, dtype=torch.float64, deriv=False).cpu().numpy()
    assert calc.device_status() == 0
    Ih, dIh = calc.radial_integral_host(rs, exact=True)
    Ih, dIh = np.moveaxis(Ih, 0, -1), np.moveaxis(dIh, 0, -1)
    Io, dIo = _oracle_radial(h, basis, rs)
    s, ds = max(1.0, np.abs(Io).max()), max(1.0, np.abs(dIo).max())
    # direct device values: the host's code on the device; the two differ
    # in rounding (contractions into FMA, exp and log to an ulp), which
    # S^{-1/2} amplifies by up to ||S^{-1/2}|| ~ sqrt(cond S)
    amp = max(1.0, np.sqrt(cond))
    assert np.abs(Ie - Ih).max() <= 1e-14 * amp * s, np.abs(Ie - Ih).max()
    assert np.abs(dIe - dIh).max() <= 1e-13 * amp * ds, np.abs(dIe - dIh).max()
    bound = 1e-13 * amp
    assert np.abs(Ie - Io).max() <= bound * s, np.abs(Ie - Io).max()
    assert np.abs(dIe - dIo).max() <= 10 * bound * ds, np.abs(dIe - dIo).max()
    # splines
    assert np.abs(I64 - Io).max() <= 1e-8 * s and np.abs(dI64 - dIo).max() <= 2e-6 * ds
    assert np.abs(I32 - Io).max() <= 2e-6 * s and np.abs(dI32 - dIo).max() <= 1e-4 * ds
    assert np.array_equal(Ionly, I64)


def test_radial_integral_empty_and_rejections():
    calc = P.Calculator(1, 6, 4, 4.0, 0.5)
    rd = torch.zeros(0, dtype=torch.float64, device="cuda")
    I, dI = calc.radial_integral(rd, exact=True)
    assert I.shape == (6, 5, 0) and dI.shape == (6, 5, 0)
    rbad = torch.tensor([1.0], dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        calc.radial_integral(rbad, exact=True, dtype=torch.float32)
    assert calc.device_status() == 0
