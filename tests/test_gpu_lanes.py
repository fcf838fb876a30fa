"""GPU parity of the one-lane-per-pair expansion and adjoint kernels against
the FP64 oracle: the full 4096-atom liquid adjoint, centres with several
chunks of pairs, pair lists not grouped by species, and neighbours one
micrometre-scale step (1e-6 A) inside and outside the cutoff.

Tolerances as in test_gpu_parity.py (relative Frobenius error):
FP64 <= 1e-7, FP32 c and p <= 1e-6, FP32 gradients <= 1e-5."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
import paper_2101_08814_amd as P
from paper_2101_08814_amd.soap import Neighbors

from test_gpu_parity import gpu_neighbors, rel, worst_centre

pytestmark = pytest.mark.gpu


def _np(t):
    return t.double().cpu().numpy()


def _dense_cell():
    """About 100 neighbours per centre (two chunks of 64 pairs), 2 species."""
    hyp = dict(n_species=2, nmax=4, lmax=4, rcut=6.0, sigma=0.5, cutoff_width=0.5, include_center=1)
    return synthetic.random_cell_structure(41, 40, np.array([[7.0, 0, 0], [0.4, 6.8, 0], [-0.3, 0.5, 7.2]]), 2,
                                           min_sep=1.2, hypers=hyp)


def test_vjp_liquid_full_size_matches_oracle():
    """The 4096-atom liquid (2 species, nmax 10, lmax 8, rcut 6 A), FP32
    forward and adjoint for W ~ N(0, 1) (seed 2004), against the oracle's
    vector-Jacobian product at full size."""
    b = synthetic.liquid_bulk()
    calc = P.Calculator.from_hypers(b.hypers)
    nl, pos, spc = gpu_neighbors(calc, b, torch.float32)
    c, p = calc.features(nl, spc, torch.float32)
    W = np.random.default_rng(2004).normal(size=tuple(p.shape))
    gc = calc.power_spectrum_backward(c, torch.tensor(W, dtype=torch.float32, device="cuda"))
    gpos, gpair = calc.spherical_expansion_backward(nl, spc, gc)
    assert calc.device_status() == 0
    ref_nl = oracle.neighbors(b)
    ref_c = oracle.expansion(b.hypers, b.species, ref_nl)
    ref_p = oracle.power_spectrum(b.hypers, ref_c)
    g_ref, gp_ref = oracle.vjp(b.hypers, b.species, ref_nl, W)
    # per atom, the error against the size of the pair terms its gradient
    # sums (sum_q |g_q| over the pairs that touch it): the terms cancel, so
    # this, not |dL/dr_k| itself, is the scale FP32 rounding works on
    off, pj = ref_nl.pair_offsets, ref_nl.pair_j
    centre = np.repeat(np.arange(b.n_atoms), np.diff(off))
    mag = np.linalg.norm(gp_ref, axis=1)
    scale = np.bincount(centre, mag, b.n_atoms) + np.bincount(pj, mag, b.n_atoms)
    atom_err = np.linalg.norm(_np(gpos) - g_ref, axis=1) / scale
    errs = dict(c=rel(_np(c), ref_c), p=rel(_np(p), ref_p), p_worst=worst_centre(_np(p), ref_p),
                grad=rel(_np(gpos), g_ref), grad_pair=rel(_np(gpair[:ref_nl.n_pairs]), gp_ref),
                grad_worst_atom=float(atom_err.max()))
    print("[liquid 4096 f32] " + " ".join(f"{k}={v:.3e}" for k, v in errs.items()))
    assert errs["c"] <= 1e-6 and errs["p"] <= 1e-6 and errs["p_worst"] <= 1e-6
    assert errs["grad"] <= 1e-5 and errs["grad_pair"] <= 1e-5 and errs["grad_worst_atom"] <= 1e-5


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_many_pairs_per_centre(dt):
    """c, p and the adjoint where every centre has about 100 pairs (the
    expansion stages them in two chunks, the adjoint's lanes take them in
    two passes)."""
    b = _dense_cell()
    calc = P.Calculator.from_hypers(b.hypers)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    assert nl.count() / b.n_atoms > 80
    c, p = calc.features(nl, spc, dt)
    W = np.random.default_rng(7).normal(size=tuple(p.shape))
    gc = calc.power_spectrum_backward(c, torch.tensor(W, dtype=dt, device="cuda"))
    gpos, gpair = calc.spherical_expansion_backward(nl, spc, gc)
    assert calc.device_status() == 0
    ref_nl = oracle.neighbors(b)
    ref_c = oracle.expansion(b.hypers, b.species, ref_nl)
    ref_p = oracle.power_spectrum(b.hypers, ref_c)
    g_ref, gp_ref = oracle.vjp(b.hypers, b.species, ref_nl, W)
    f64 = dt == torch.float64
    for name, x, y, tol in [("c", c, ref_c, 1e-7 if f64 else 1e-6), ("p", p, ref_p, 1e-7 if f64 else 1e-6),
                            ("grad", gpos, g_ref, 1e-7 if f64 else 1e-5),
                            ("grad_pair", gpair[:ref_nl.n_pairs], gp_ref, 1e-7 if f64 else 1e-5)]:
        e = rel(_np(x), y)
        print(f"[many pairs {dt}] {name} {e:.3e}")
        assert e <= tol, name


def _permuted(nl, seed):
    """The same list with the pairs of every centre in a random order (so
    not grouped by neighbour species); returns it and the permutation
    new -> old."""
    off = nl.pair_offsets.cpu().numpy()
    rng = np.random.default_rng(seed)
    perm = np.concatenate([lo + rng.permutation(hi - lo) for lo, hi in zip(off[:-1], off[1:])]).astype(np.int64)
    Pn = perm.shape[0]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(Pn)
    pt = torch.tensor(perm, device="cuda")
    t_old = nl.pair_transpose[:Pn].long().cpu().numpy()
    t_new = inv[t_old[perm]].astype(np.int32)
    out = Neighbors(nl.pair_offsets.clone(), nl.pair_j[pt].contiguous(), nl.pair_shift[pt].contiguous(),
                    nl.pair_vec[pt].contiguous(), torch.tensor(t_new, device="cuda"), Pn)
    return out, perm


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_pairs_not_grouped_by_species(dt):
    """A list whose pairs are not grouped by neighbour species gives the c,
    p and adjoint of the grouped list (the expansion redoes such a centre
    one species at a time)."""
    hyp = dict(n_species=3, nmax=5, lmax=4, rcut=4.5, sigma=0.45, cutoff_width=0.5, include_center=1)
    b = synthetic.random_cell_structure(21, 60, np.array([[11.0, 0, 0], [1.0, 10.5, 0], [0.5, -0.8, 12.0]]), 3,
                                        min_sep=1.3, hypers=hyp)
    calc = P.Calculator.from_hypers(hyp)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c, p = [t.clone() for t in calc.features(nl, spc, dt)]
    W = torch.tensor(np.random.default_rng(3).normal(size=tuple(p.shape)), dtype=dt, device="cuda")
    gpos, gpair = calc.spherical_expansion_backward(nl, spc, calc.power_spectrum_backward(c, W))
    nl2, perm = _permuted(nl, 5)
    sp_sorted = spc[nl2.pair_j.long()].cpu().numpy()
    off = nl.pair_offsets.cpu().numpy()
    assert any(np.any(np.diff(sp_sorted[lo:hi]) < 0) for lo, hi in zip(off[:-1], off[1:]))
    c2, p2 = calc.features(nl2, spc, dt)
    c3 = calc.spherical_expansion(nl2, spc, dt)
    gpos2, gpair2 = calc.spherical_expansion_backward(nl2, spc, calc.power_spectrum_backward(c2, W))
    assert calc.device_status() == 0
    same = 1e-12 if dt == torch.float64 else 1e-6
    Pn = nl.count()
    for name, x, y in [("c", c2, c), ("c alone", c3, c), ("p", p2, p), ("grad", gpos2, gpos),
                       ("grad_pair", gpair2[:Pn], gpair[:Pn][torch.tensor(perm, device="cuda")])]:
        e = rel(_np(x), _np(y))
        print(f"[not grouped {dt}] {name} {e:.3e}")
        assert e <= same, name


def _edge_batch(inside: bool, hyp):
    """Non-periodic cluster: atom 1 at rcut - 1e-6 A from atom 0 (or
    rcut + 1e-6 A with inside=False), atom 2 at rcut + 1e-6 A from atom 0,
    three more atoms well inside; every other distance is away from rcut."""
    rc = hyp["rcut"]
    u1 = np.array([0.48, -0.6, 0.64])
    u2 = np.array([-0.36, 0.0, 0.933])
    u1 /= np.linalg.norm(u1)
    u2 /= np.linalg.norm(u2)
    d1 = rc - 1e-6 if inside else rc + 1e-6
    pos = np.array([[0.0, 0.0, 0.0], d1 * u1, (rc + 1e-6) * u2, [1.1, 0.9, -0.7], [-1.3, 0.4, 1.2],
                    [0.5, -1.6, 0.3]]) + np.array([3.0, 2.0, 1.0])
    spc = np.array([0, 1, 1, 0, 1, 0], dtype=np.int32)
    d = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
    away = np.abs(d - rc)
    away[0, 1] = away[1, 0] = away[0, 2] = away[2, 0] = 1.0
    assert away.min() > 1e-2
    return synthetic.Batch(pos, spc, np.array([0, 6], dtype=np.int64), np.zeros((1, 3, 3)),
                           np.zeros((1, 3), dtype=np.uint8), hyp)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_neighbour_crossing_the_cutoff(dt):
    """A neighbour 1e-6 A inside rcut is in the list with a vanishing
    contribution and the one 1e-6 A outside is not; c, p, the gradient rows
    and the adjoint match the oracle, and moving the neighbour across rcut
    changes them continuously (by the size of the cutoff function there)."""
    hyp = dict(n_species=2, nmax=6, lmax=4, rcut=4.0, sigma=0.5, cutoff_width=0.5, include_center=1)
    res = {}
    for inside in (True, False):
        b = _edge_batch(inside, hyp)
        calc = P.Calculator.from_hypers(hyp)
        nl, pos, spc = gpu_neighbors(calc, b, dt)
        c, p, dc, dcs, dp, dps = [t.clone() for t in calc.features(nl, spc, dt, gradients=True)]
        W = np.random.default_rng(11).normal(size=tuple(p.shape))
        gpos, _ = calc.spherical_expansion_backward(
            nl, spc, calc.power_spectrum_backward(c, torch.tensor(W, dtype=dt, device="cuda")))
        assert calc.device_status() == 0
        ref_nl = oracle.neighbors(b)
        Pn = ref_nl.n_pairs
        assert nl.count() == Pn
        j0 = ref_nl.pair_j[ref_nl.pair_offsets[0]:ref_nl.pair_offsets[1]]
        assert (1 in j0) == inside and 2 not in j0
        ref_c = oracle.expansion(hyp, b.species, ref_nl)
        ref_p = oracle.power_spectrum(hyp, ref_c)
        rdc, rdcs, rdp, rdps = oracle.gradients(hyp, b.species, ref_nl)
        g_ref, _ = oracle.vjp(hyp, b.species, ref_nl, W)
        f64 = dt == torch.float64
        for name, x, y, tol in [("c", c, ref_c, 1e-7 if f64 else 1e-6), ("p", p, ref_p, 1e-7 if f64 else 1e-6),
                                ("dc", dc[:Pn], rdc, 1e-7 if f64 else 1e-5),
                                ("dcs", dcs, rdcs, 1e-7 if f64 else 1e-5),
                                ("dp", dp[:Pn], rdp, 1e-7 if f64 else 1e-5),
                                ("dps", dps, rdps, 1e-7 if f64 else 1e-5),
                                ("grad", gpos, g_ref, 1e-7 if f64 else 1e-5)]:
            e = rel(_np(x), y)
            print(f"[cutoff edge {dt} inside={inside}] {name} {e:.3e}")
            assert e <= tol, name
        res[inside] = (_np(c), _np(p), _np(dcs), _np(dps), _np(gpos))
    # continuity across rcut: f_cut(rcut - 1e-6) ~ 1e-11 and its derivative
    # ~ 2e-5 (shifted cosine of width 0.5 A), so the two sides differ by
    # about that times the size of one neighbour's terms
    for k, name in enumerate(("c", "p", "dcs", "dps", "grad")):
        a, bb = res[True][k], res[False][k]
        d = np.linalg.norm(a - bb) / np.linalg.norm(bb)
        print(f"[cutoff edge {dt}] continuity {name} {d:.3e}")
        assert d <= 1e-4, name
