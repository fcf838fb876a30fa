"""GPU parity of the expansion with pairs packed across centres (c alone):
against the FP64 oracle for several (nmax, lmax) shapes, including nmax not
a multiple of four, nmax = 1 and lmax = 0, with centres that have no pairs
at all, against c from the one-wave-per-centre kernel that forms c and p
together (same sums in the same order; used below 4096 centres), and at the
molecules' full size (four centres per wave), where features come from the
packed c and the power-spectrum kernel, against the oracle's c and p.

Tolerances as in test_gpu_parity.py: FP64 <= 1e-7, FP32 c <= 1e-6
(relative Frobenius error), per centre WORST_ROW_F32 in FP32."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
import paper_2101_08814_amd as P

from test_gpu_parity import gpu_neighbors, rel, WORST_ROW_F32

pytestmark = pytest.mark.gpu


def _np(t):
    return t.double().cpu().numpy()


def _with_isolated(b, hyp, at_front=True):
    """The batch with a non-periodic structure of five atoms 10 A apart
    (no neighbours within the cutoff) placed first (or last)."""
    iso = synthetic.Batch(np.arange(15, dtype=np.float64).reshape(5, 3) * np.array([10.0, 0.0, 0.0]),
                          np.array([0, 1, 2, 3, 1], dtype=np.int32) % hyp["n_species"],
                          np.array([0, 5], dtype=np.int64), np.zeros((1, 3, 3)), np.zeros((1, 3), dtype=np.uint8),
                          hyp)
    parts = [iso, b] if at_front else [b, iso]
    pos = np.concatenate([x.positions for x in parts])
    spc = np.concatenate([x.species for x in parts]).astype(np.int32)
    offs = np.concatenate([[0], parts[0].atom_offsets[1:], parts[0].n_atoms + parts[1].atom_offsets[1:]])
    return synthetic.Batch(pos, spc, offs.astype(np.int64), np.concatenate([x.cells for x in parts]),
                           np.concatenate([x.pbc for x in parts]).astype(np.uint8), hyp)


def _worst_centre(x, y):
    x = x.reshape(x.shape[0], -1)
    y = y.reshape(y.shape[0], -1)
    scale = np.linalg.norm(y, axis=1).max()
    return float(np.linalg.norm(x - y, axis=1).max() / scale)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("nmax,lmax", [(8, 6), (13, 3), (1, 0), (6, 8)])
def test_packed_expansion_matches_oracle(dt, nmax, lmax):
    """24 molecules (about 2,600 atoms: two centres per wave) with five
    isolated atoms in front, c alone against the oracle; the centres
    without pairs hold only the central atom's term."""
    mol = synthetic.molecule_batch().subset(list(range(24)))
    hyp = dict(mol.hypers, nmax=nmax, lmax=lmax)
    b = _with_isolated(mol, hyp)
    calc = P.Calculator.from_hypers(hyp)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c = calc.spherical_expansion(nl, spc, dt).clone()
    c2, _ = calc.features(nl, spc, dt)
    assert calc.device_status() == 0
    d = rel(_np(c), _np(c2))
    ref_nl = oracle.neighbors(b)
    ref_c = oracle.expansion(hyp, b.species, ref_nl)
    assert np.all(np.diff(ref_nl.pair_offsets)[:5] == 0)
    e, w = rel(_np(c), ref_c), _worst_centre(_np(c), ref_c)
    print(f"[packed {dt} nmax={nmax} lmax={lmax}] N={b.n_atoms} rel={e:.3e} worst centre={w:.3e} "
          f"vs one wave per centre={d:.3e}")
    f64 = dt == torch.float64
    assert e <= (1e-7 if f64 else 1e-6)
    assert w <= (1e-7 if f64 else WORST_ROW_F32)
    assert d <= (1e-12 if f64 else 1e-6)
    # isolated centres: only the centre term (lm = 0 of their own species),
    # to the spline's accuracy
    ci = _np(c)[:5]
    assert np.count_nonzero(ci) <= 5 * nmax
    scale = np.abs(ref_c[:5]).max()
    assert np.allclose(ci, ref_c[:5], rtol=0, atol=(1e-7 if f64 else 1e-6) * scale)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_packed_full_molecules_matches_oracle(dt):
    """All 256 molecules (28,929 atoms with five isolated ones at the end:
    four centres per wave, a partly filled last wave) at nmax 13, lmax 3:
    c alone, and c and p from soap_features (the packed c, then p from it),
    against the oracle."""
    mol = synthetic.molecule_batch()
    hyp = dict(mol.hypers, nmax=13, lmax=3)
    b = _with_isolated(mol, hyp, at_front=False)
    calc = P.Calculator.from_hypers(hyp)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c = calc.spherical_expansion(nl, spc, dt).clone()
    c2, p2 = calc.features(nl, spc, dt)
    assert calc.device_status() == 0
    ref_nl = oracle.neighbors(b)
    ref_c = oracle.expansion(hyp, b.species, ref_nl)
    ref_p = oracle.power_spectrum(hyp, ref_c)
    e, w = rel(_np(c), ref_c), _worst_centre(_np(c), ref_c)
    ep, wp = rel(_np(p2), ref_p), _worst_centre(_np(p2), ref_p)
    print(f"[packed full {dt}] N={b.n_atoms} c rel={e:.3e} worst centre={w:.3e}; features c same="
          f"{bool(torch.equal(c, c2))}, p rel={ep:.3e} worst centre={wp:.3e}")
    f64 = dt == torch.float64
    assert e <= (1e-7 if f64 else 1e-6)
    assert w <= (1e-7 if f64 else WORST_ROW_F32)
    assert torch.equal(c, c2)
    assert ep <= (1e-7 if f64 else 1e-6)
    assert wp <= (1e-7 if f64 else WORST_ROW_F32)
