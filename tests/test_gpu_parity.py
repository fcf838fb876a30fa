"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative Frobenius error of each result tensor, ||d||_F/||ref||_F,
plus the worst single centre):
  FP64 path                         <= 1e-7   (spline accuracy 1e-8 dominates)
  FP32 path, c and p                <= 1e-6   (the stated FP32 bound on p)
  FP32 gradient rows / adjoint      <= 1e-5   (derivatives lose ~1 digit)
  bfloat16 hi/lo MFMA power spectrum <= 2e-3  (the stated bound; ~1e-5 expected)
Neighbour lists (integers) are compared bit-exactly.
"""
import math

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


def worst_centre(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    nb = np.linalg.norm(b, axis=1)
    scale = np.maximum(nb, 1e-3 * np.linalg.norm(b) / math.sqrt(b.shape[0]) + 1e-300)
    return float(np.max(np.linalg.norm(a - b, axis=1) / scale))


def worst_row(a, b):
    """Largest per-row error ||a_q - b_q|| / max(||b_q||, 1e-3 * rms row
    norm) over the rows q (first axis) of a gradient-row tensor."""
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    nb = np.linalg.norm(b, axis=1)
    floor = 1e-3 * np.sqrt(np.mean(nb ** 2)) + 1e-300
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.maximum(nb, floor)))


# Worst single gradient row in FP32 (relative to the row's norm, floored at
# 1e-3 of the rms row norm): each element is a sum of a few products whose
# factors carry FP32 rounding (~6e-8) amplified by the harmonic recurrence
# up to lmax and by cancellation in the product rule; rows of pairs near
# the cutoff, where f and f' are small, are the worst.  Measured on the
# 1024-atom diamond: dc and dp rows 9.9e-6, self rows 1.7e-6 and 4.6e-6;
# the bound is three times the worst.
WORST_ROW_F32 = 3e-5


def to_dev(batch):
    pos = torch.tensor(batch.positions, dtype=torch.float64, device="cuda")
    spc = torch.tensor(batch.species, dtype=torch.int32, device="cuda")
    return pos, spc


def gpu_neighbors(calc, batch, dtype=torch.float32):
    pos, spc = to_dev(batch)
    nl = calc.compute_neighbors(pos, spc, batch.atom_offsets, batch.cells, batch.pbc, vec_dtype=dtype)
    assert calc.device_status() == 0
    return nl, pos, spc


def assert_same_list(nl, ref, batch, f64):
    P_ = ref.n_pairs
    assert nl.count() == P_
    assert np.array_equal(nl.pair_offsets.cpu().numpy(), ref.pair_offsets)
    assert np.array_equal(nl.pair_j[:P_].cpu().numpy(), ref.pair_j)
    assert np.array_equal(nl.pair_shift[:P_].cpu().numpy(), ref.pair_shift)
    vec = nl.pair_vec[:P_].double().cpu().numpy()
    tol = 1e-12 if f64 else 4e-7
    assert np.abs(vec - ref.pair_vec).max() <= tol * max(1.0, np.abs(ref.pair_vec).max())
    if nl.pair_transpose is not None and P_:
        t = nl.pair_transpose[:P_].cpu().numpy().astype(np.int64)
        centre = np.repeat(np.arange(batch.n_atoms), np.diff(ref.pair_offsets))
        assert np.array_equal(ref.pair_j[t], centre)
        assert np.array_equal(ref.pair_shift[t], -ref.pair_shift)
        assert np.array_equal(t[t], np.arange(P_))


# ------------------------------------------------------------------ neighbours
NEIGHBOR_CASES = {
    "clusters": lambda: synthetic.clusters_2species(),
    "diamond": lambda: synthetic.diamond_bulk(),
    "molecules": lambda: synthetic.molecule_batch(),
    "liquid": lambda: synthetic.liquid_bulk(),
    "multispecies_64cells": lambda: synthetic.multi_species_cells().subset(list(range(64))),
    "triclinic_self_images": lambda: synthetic.random_cell_structure(
        3, 2, np.array([[3.1, 0.0, 0.0], [1.2, 2.9, 0.0], [-0.7, 0.9, 3.4]]), 2, min_sep=1.0,
        hypers=dict(n_species=2, nmax=4, lmax=3, rcut=5.0, sigma=0.5, cutoff_width=0.5, include_center=1)),
    "diamond_primitive": lambda: synthetic.random_cell_structure(
        4, 2, np.array([[0.0, 2.715, 2.715], [2.715, 0.0, 2.715], [2.715, 2.715, 0.0]]), 1, min_sep=1.0,
        hypers=dict(n_species=1, nmax=4, lmax=3, rcut=5.0, sigma=0.5, cutoff_width=0.5, include_center=1)),
    "slab_pbc_xy": lambda: synthetic.random_cell_structure(
        5, 40, np.array([[9.0, 0.0, 0.0], [0.0, 8.0, 0.0], [0.0, 0.0, 12.0]]), 2, min_sep=1.2, pbc=(1, 1, 0),
        hypers=dict(n_species=2, nmax=4, lmax=3, rcut=3.5, sigma=0.5, cutoff_width=0.5, include_center=1)),
}


@pytest.mark.parametrize("name", sorted(NEIGHBOR_CASES))
@pytest.mark.parametrize("f64", [False, True])
def test_neighbors_match_oracle(name, f64):
    print(f"[neighbors] case={name} f64={f64}", flush=True)
    b = NEIGHBOR_CASES[name]()
    calc = P.Calculator.from_hypers(b.hypers)
    nl, _, _ = gpu_neighbors(calc, b, torch.float64 if f64 else torch.float32)
    ref = oracle.neighbors(b)
    assert_same_list(nl, ref, b, f64)


def test_neighbors_unwrapped_positions_and_empty_structures():
    """Positions outside the cell (any number of cells away) and structures
    with zero or one atom."""
    b = synthetic.random_cell_structure(9, 12, np.array([[6.0, 0, 0], [0.5, 5.5, 0], [0, -0.4, 6.5]]), 2,
                                        min_sep=1.0)
    shifts = np.random.default_rng(0).integers(-3, 4, size=(12, 3))
    pos = b.positions + shifts @ b.cells[0]
    lone = synthetic.clusters_2species().subset([0])
    parts = [synthetic.Batch(pos, b.species, b.atom_offsets, b.cells, b.pbc, b.hypers)]
    empty = synthetic.Batch(np.zeros((0, 3)), np.zeros(0, np.int32), np.array([0, 0]), np.zeros((1, 3, 3)),
                            np.zeros((1, 3), np.uint8), b.hypers)
    single = synthetic.Batch(np.array([[1.0, 2.0, 3.0]]), np.array([1], np.int32), np.array([0, 1]),
                             np.zeros((1, 3, 3)), np.zeros((1, 3), np.uint8), b.hypers)
    parts += [empty, single, lone]
    pos = np.concatenate([p.positions for p in parts])
    spc = np.concatenate([p.species for p in parts]).astype(np.int32)
    offs = np.cumsum([0] + [p.n_atoms for p in parts])
    cells = np.concatenate([p.cells for p in parts])
    pbc = np.concatenate([p.pbc for p in parts])
    batch = synthetic.Batch(pos, spc, offs, cells, pbc, b.hypers)
    calc = P.Calculator.from_hypers(b.hypers)
    nl, _, _ = gpu_neighbors(calc, batch, torch.float64)
    assert_same_list(nl, oracle.neighbors(batch), batch, True)


# ------------------------------------------------------------ expansion + p
def run_features(batch, dtype, gradients=False):
    calc = P.Calculator.from_hypers(batch.hypers)
    nl, pos, spc = gpu_neighbors(calc, batch, dtype)
    out = calc.features(nl, spc, dtype, gradients)
    assert calc.device_status() == 0
    return calc, nl, spc, [o.double().cpu().numpy() for o in out]


def test_clusters_fp64_full_parity():
    """8 x 64-atom clusters, 2 species, FP64: c and p against the oracle."""
    b = synthetic.clusters_2species()
    calc, nl, spc, (c, p) = run_features(b, torch.float64)
    ref_nl, ref_c, ref_p = oracle.features(b)
    ec, ep = rel(c, ref_c), rel(p, ref_p)
    print(f"[clusters f64] rel c={ec:.3e} p={ep:.3e} worst-centre p={worst_centre(p, ref_p):.3e}")
    assert ec <= 1e-7 and ep <= 1e-7
    assert worst_centre(p, ref_p) <= 1e-7


def test_diamond_fp32_gradients_full_parity():
    """1024-atom periodic diamond, FP32: c, p and all forward-mode gradient
    rows against the oracle, at the size and launch the benchmark times."""
    b = synthetic.diamond_bulk()
    calc, nl, spc, (c, p, dc, dcs, dp, dps) = run_features(b, torch.float32, gradients=True)
    ref_nl = oracle.neighbors(b)
    ref_c = oracle.expansion(b.hypers, b.species, ref_nl)
    ref_p = oracle.power_spectrum(b.hypers, ref_c)
    rdc, rdcs, rdp, rdps = oracle.gradients(b.hypers, b.species, ref_nl)
    P_ = ref_nl.n_pairs
    errs = dict(c=rel(c, ref_c), p=rel(p, ref_p), dc=rel(dc[:P_], rdc), dcs=rel(dcs, rdcs), dp=rel(dp[:P_], rdp),
                dps=rel(dps, rdps), p_worst=worst_centre(p, ref_p),
                dc_row=worst_row(dc[:P_], rdc), dp_row=worst_row(dp[:P_], rdp),
                dcs_row=worst_row(dcs, rdcs), dps_row=worst_row(dps, rdps))
    print("[diamond f32 grads] " + " ".join(f"{k}={v:.3e}" for k, v in errs.items()))
    assert errs["c"] <= 1e-6 and errs["p"] <= 1e-6 and errs["p_worst"] <= 1e-6
    assert errs["dc"] <= 1e-5 and errs["dcs"] <= 1e-5 and errs["dp"] <= 1e-5 and errs["dps"] <= 1e-5
    # every single row, not only the whole tensor
    assert max(errs["dc_row"], errs["dp_row"], errs["dcs_row"], errs["dps_row"]) <= WORST_ROW_F32


def test_separate_entry_points_match_fused():
    """soap_spherical_expansion + soap_power_spectrum (with rows) give the
    results of soap_features; checked on a multi-species periodic structure
    against the oracle."""
    hyp = dict(n_species=3, nmax=5, lmax=4, rcut=4.5, sigma=0.45, cutoff_width=0.5, include_center=1)
    b = synthetic.random_cell_structure(21, 60, np.array([[11.0, 0, 0], [1.0, 10.5, 0], [0.5, -0.8, 12.0]]), 3,
                                        min_sep=1.3, hypers=hyp)
    for dt in (torch.float32, torch.float64):
        calc = P.Calculator.from_hypers(hyp)
        nl, pos, spc = gpu_neighbors(calc, b, dt)
        c, dc, dcs = calc.spherical_expansion(nl, spc, dt, gradients=True)
        p, dp, dps = calc.power_spectrum(c, dt, rows=(dc, dcs), nl=nl, species=spc)
        fused = calc.features(nl, spc, dt, gradients=True)
        assert calc.device_status() == 0
        ref_nl = oracle.neighbors(b)
        ref_c = oracle.expansion(hyp, b.species, ref_nl)
        ref_p = oracle.power_spectrum(hyp, ref_c)
        rdc, rdcs, rdp, rdps = oracle.gradients(hyp, b.species, ref_nl)
        Pn = ref_nl.n_pairs
        tol = 1e-7 if dt == torch.float64 else 1e-5
        for got, ref in [(c, ref_c), (p, ref_p), (dc[:Pn], rdc), (dcs, rdcs), (dp[:Pn], rdp), (dps, rdps)]:
            assert rel(got.double().cpu().numpy(), ref) <= tol
        # rows past the pair count are not written (their contents are undefined)
        fc, fp, fdc, fdcs, fdp, fdps = fused
        for a, f in [(c, fc), (p, fp), (dc[:Pn], fdc[:Pn]), (dcs, fdcs), (dp[:Pn], fdp[:Pn]), (dps, fdps)]:
            assert rel(a.double().cpu().numpy(), f.double().cpu().numpy()) <= (1e-12 if dt == torch.float64 else 1e-6)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_fused_rows_over_many_chunks(dt):
    """A dense small periodic cell (about 100 neighbours per centre, several
    LDS chunks per centre, the last one partial): the pair rows written by
    soap_features, whose kernel loads each chunk ahead while the previous
    one is in use, against the oracle and against soap_gradient_rows."""
    hyp = dict(n_species=2, nmax=4, lmax=4, rcut=6.0, sigma=0.5, cutoff_width=0.5, include_center=1)
    b = synthetic.random_cell_structure(41, 40, np.array([[7.0, 0, 0], [0.4, 6.8, 0], [-0.3, 0.5, 7.2]]), 2,
                                        min_sep=1.2, hypers=hyp)
    calc = P.Calculator.from_hypers(hyp)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c, p, dc, dcs, dp, dps = calc.features(nl, spc, dt, gradients=True)
    r_dc, r_dp = calc.gradient_rows(nl, spc, c)
    assert calc.device_status() == 0
    Pn = nl.count()
    assert Pn / b.n_atoms > 80
    ref_nl = oracle.neighbors(b)
    ref_c = oracle.expansion(hyp, b.species, ref_nl)
    ref_p = oracle.power_spectrum(hyp, ref_c)
    rdc, rdcs, rdp, rdps = oracle.gradients(hyp, b.species, ref_nl)
    tol = 1e-7 if dt == torch.float64 else 1e-5
    for name, x, y in [("c", c, ref_c), ("p", p, ref_p), ("dc", dc[:Pn], rdc), ("dcs", dcs, rdcs),
                       ("dp", dp[:Pn], rdp), ("dps", dps, rdps)]:
        e = rel(x.double().cpu().numpy(), y)
        print(f"[many chunks {dt}] {name} {e:.3e}")
        assert e <= tol, name
    same = 1e-12 if dt == torch.float64 else 1e-6
    for name, x, y in [("dc", dc[:Pn], r_dc[:Pn]), ("dp", dp[:Pn], r_dp[:Pn])]:
        assert rel(x.double().cpu().numpy(), y.double().cpu().numpy()) <= same, name
    # c alone (in float the sums stay in registers across the chunks)
    c_only = calc.spherical_expansion(nl, spc, dt)
    assert rel(c_only.double().cpu().numpy(), ref_c) <= tol
    assert rel(c_only.double().cpu().numpy(), c.double().cpu().numpy()) <= same


def test_gradient_rows_entry_point():
    """soap_gradient_rows (dc and dp rows from c) gives the rows of
    soap_features, together or one at a time."""
    hyp = dict(n_species=2, nmax=6, lmax=5, rcut=4.5, sigma=0.45, cutoff_width=0.5, include_center=1)
    b = synthetic.random_cell_structure(31, 48, np.array([[10.0, 0, 0], [0.8, 9.5, 0], [0.3, -0.6, 10.5]]), 2,
                                        min_sep=1.3, hypers=hyp)
    calc = P.Calculator.from_hypers(hyp)
    nl, pos, spc = gpu_neighbors(calc, b, torch.float32)
    c, p, dc, dcs, dp, dps = calc.features(nl, spc, torch.float32, gradients=True)
    c2, p2, _, dcs2, _, dps2 = calc.features(nl, spc, torch.float32, gradients=True, rows=False)
    r_dc, r_dp = calc.gradient_rows(nl, spc, c2)
    o_dc, _ = calc.gradient_rows(nl, spc, c2, want_dp=False)
    _, o_dp = calc.gradient_rows(nl, spc, c2, want_dc=False)
    assert calc.device_status() == 0
    Pn = nl.count()
    # the row kernel is the one behind soap_gradient_rows, alone or for both
    # rows: same arithmetic, same bits
    for name, x, y in [("dc", r_dc[:Pn], o_dc[:Pn]), ("dp", r_dp[:Pn], o_dp[:Pn])]:
        assert torch.equal(x, y), name
    # soap_features may write the rows from the expansion kernel, whose LDS
    # layout stages fewer pairs at a time (partial sums rounded in another
    # grouping) and where the compiler contracts the same products into other
    # fused multiply-adds: equal to rounding
    for name, x, y in [("c", c, c2), ("p", p, p2), ("dcs", dcs, dcs2), ("dps", dps, dps2), ("dc", dc[:Pn], r_dc[:Pn]),
                       ("dp", dp[:Pn], r_dp[:Pn])]:
        assert rel(x.double().cpu().numpy(), y.double().cpu().numpy()) <= 1e-6, name
    ref_nl = oracle.neighbors(b)
    rdc, rdcs, rdp, rdps = oracle.gradients(hyp, b.species, ref_nl)
    for x, y in [(r_dc[:Pn], rdc), (r_dp[:Pn], rdp), (dc[:Pn], rdc), (dp[:Pn], rdp), (dcs, rdcs), (dps, rdps)]:
        assert rel(x.double().cpu().numpy(), y) <= 1e-5


def test_molecules_bf16_mfma_power_spectrum():
    """256 molecules of 20-200 atoms, 4 species, one launch: p from the
    bfloat16 hi/lo MFMA contraction against the FP64 oracle (bound 2e-3)."""
    b = synthetic.molecule_batch()
    calc = P.Calculator.from_hypers(b.hypers)
    nl, pos, spc = gpu_neighbors(calc, b, torch.float32)
    c = calc.spherical_expansion(nl, spc, torch.float32)
    p_bf16 = calc.power_spectrum(c, "bf16")
    p_f32 = calc.power_spectrum(c, torch.float32)
    assert calc.device_status() == 0
    ref_nl, ref_c, ref_p = oracle.features(b)
    e16 = rel(p_bf16.double().cpu().numpy(), ref_p)
    e32 = rel(p_f32.double().cpu().numpy(), ref_p)
    ec = rel(c.double().cpu().numpy(), ref_c)
    w16 = worst_centre(p_bf16.double().cpu().numpy(), ref_p)
    print(f"[molecules] rel c={ec:.3e} p_f32={e32:.3e} p_bf16={e16:.3e} worst-centre bf16={w16:.3e}")
    assert ec <= 1e-6 and e32 <= 1e-6
    assert e16 <= 2e-3 and w16 <= 2e-3


@pytest.mark.parametrize("n_cells", [8])
def test_multispecies_fp32_parity(n_cells):
    """8 species, nmax 12, lmax 8 (K = 96, 41904 features per centre)."""
    b = synthetic.multi_species_cells().subset(list(range(n_cells)))
    calc, nl, spc, (c, p) = run_features(b, torch.float32)
    c_t = calc.spherical_expansion(nl, spc, torch.float32)
    p16 = calc.power_spectrum(c_t, "bf16")   # K = 96: several waves per centre on the matrix cores
    assert calc.device_status() == 0
    ref_nl, ref_c, ref_p = oracle.features(b)
    ec, ep, e16 = rel(c, ref_c), rel(p, ref_p), rel(p16.double().cpu().numpy(), ref_p)
    ect = rel(c_t.double().cpu().numpy(), ref_c)
    w16 = worst_centre(p16.double().cpu().numpy(), ref_p)
    print(f"[multispecies {n_cells} cells] rel c={ec:.3e} c alone={ect:.3e} p={ep:.3e} p_bf16={e16:.3e} "
          f"worst-centre bf16={w16:.3e}")
    assert ec <= 1e-6 and ect <= 1e-6 and ep <= 1e-6
    assert e16 <= 2e-3 and w16 <= 2e-3


def test_rotation_invariance_on_gpu():
    b = synthetic.clusters_2species().subset([2, 5])
    _, _, _, (c, p) = run_features(b, torch.float32)
    q, _ = np.linalg.qr(np.random.default_rng(4).normal(size=(3, 3)))
    b2 = synthetic.Batch(b.positions @ q.T + 1.7, b.species, b.atom_offsets, b.cells, b.pbc, b.hypers)
    _, _, _, (c2, p2) = run_features(b2, torch.float32)
    assert rel(p2, p) <= 1e-6


def test_results_are_bitwise_reproducible():
    b = synthetic.diamond_bulk()
    calc = P.Calculator.from_hypers(b.hypers)
    nl, pos, spc = gpu_neighbors(calc, b)
    a = [t.clone() for t in calc.features(nl, spc, torch.float32, gradients=True)]
    nl2 = calc.compute_neighbors(pos, spc, b.atom_offsets, b.cells, b.pbc, out=nl)
    b_ = calc.features(nl2, spc, torch.float32, gradients=True)
    for x, y in zip(a, b_):
        assert torch.equal(x, y)


def test_graph_replays_match_eager():
    """The neighbour list and the fused feature kernel captured in HIP graphs:
    several replays, with eager work and synchronisations in between, each
    equal to the eager result."""
    b = synthetic.diamond_bulk()
    calc = P.Calculator.from_hypers(b.hypers)
    dev = torch.device("cuda")
    pos, spc = to_dev(b)
    ao, ce, pb = P.soap.structures_to_device(b.atom_offsets, b.cells, b.pbc, dev)
    nl = calc.compute_neighbors(pos, spc, ao, ce, pb)
    out = calc.allocate_features(b.n_atoms, nl.capacity, torch.float32, dev, True)
    calc.features(nl, spc, torch.float32, gradients=True, out=out)
    torch.cuda.synchronize()
    Pn = nl.count()
    # rows past the pair count are not written: compare the first Pn
    rows = lambda ts: [t[:Pn] if k in (2, 4) else t for k, t in enumerate(ts)]
    ref = [t.clone() for t in rows(out)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calc.compute_neighbors(pos, spc, ao, ce, pb, out=nl)
        calc.features(nl, spc, torch.float32, gradients=True, out=out)
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        calc.compute_neighbors(pos, spc, ao, ce, pb, out=nl)
        calc.features(nl, spc, torch.float32, gradients=True, out=out)
    for rep in range(4):
        for t in out:
            t.zero_()
        nl.pair_j.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, r in zip(rows(out), ref):
            assert torch.equal(a, r), f"replay {rep}"
        _ = (pos * 2).sum().item()      # eager work between replays
    assert calc.device_status() == 0


# ------------------------------------------------------------ adjoint
def _liquid_small():
    return synthetic.liquid_bulk(n_atoms=512)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_vjp_matches_oracle(dt):
    """dL/dr for L = <W, p> with W ~ N(0, 1) (seed 2004), 2 species, nmax 10,
    lmax 8, rcut 6, at the liquid density (512 atoms)."""
    b = _liquid_small()
    calc = P.Calculator.from_hypers(b.hypers)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c, p = calc.features(nl, spc, dt)
    W = np.random.default_rng(2004).normal(size=tuple(p.shape))
    gc = calc.power_spectrum_backward(c, torch.tensor(W, dtype=dt, device="cuda"))
    gpos, gpair = calc.spherical_expansion_backward(nl, spc, gc)
    assert calc.device_status() == 0
    ref_nl = oracle.neighbors(b)
    g_ref, gp_ref = oracle.vjp(b.hypers, b.species, ref_nl, W)
    e = rel(gpos.double().cpu().numpy(), g_ref)
    ep = rel(gpair[:ref_nl.n_pairs].double().cpu().numpy(), gp_ref)
    print(f"[vjp {dt}] rel dL/dr={e:.3e} per-pair={ep:.3e}")
    assert e <= (1e-7 if dt == torch.float64 else 1e-5)
    assert ep <= (1e-7 if dt == torch.float64 else 1e-5)


def _virial_batch():
    """A 256-atom liquid cube, an empty structure and a 40-atom triclinic
    cell, all with the liquid's hypers (2 species, nmax 10, lmax 8, rcut 6)."""
    a = synthetic.liquid_bulk(n_atoms=256)
    cell = np.array([[9.1, 0.0, 0.0], [1.7, 8.6, 0.0], [-0.9, 1.2, 9.4]])
    t = synthetic.random_cell_structure(31, 40, cell, 2, min_sep=1.5, hypers=a.hypers)
    na, nt = a.n_atoms, t.n_atoms
    return synthetic.Batch(np.concatenate([a.positions, t.positions]), np.concatenate([a.species, t.species]),
                           np.array([0, na, na, na + nt], dtype=np.int64),
                           np.concatenate([a.cells, np.zeros((1, 3, 3)), t.cells]),
                           np.concatenate([a.pbc, np.zeros((1, 3), dtype=np.uint8), t.pbc]), a.hypers)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_virial_matches_oracle(dt):
    """Per-structure virial (App. B, Eq. energy-virial) of L = <W, p>,
    W ~ N(0, 1) (seed 2005): GPU adjoint then soap_virial against the
    oracle's VJP and virial; the empty structure gives exactly zero."""
    b = _virial_batch()
    calc = P.Calculator.from_hypers(b.hypers)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c, p = calc.features(nl, spc, dt)
    W = np.random.default_rng(2005).normal(size=tuple(p.shape))
    gc = calc.power_spectrum_backward(c, torch.tensor(W, dtype=dt, device="cuda"))
    _, gpair = calc.spherical_expansion_backward(nl, spc, gc)
    vir = calc.virial(nl, gpair, b.atom_offsets)
    assert calc.device_status() == 0
    ref_nl = oracle.neighbors(b)
    _, gp_ref = oracle.vjp(b.hypers, b.species, ref_nl, W)
    ref = oracle.virial(b.atom_offsets, ref_nl, gp_ref)
    got = vir.double().cpu().numpy()
    assert got.shape == (3, 3, 3)
    assert np.all(got[1] == 0.0)
    tol = 1e-7 if dt == torch.float64 else 1e-5
    for s in (0, 2):
        e = rel(got[s], ref[s])
        print(f"[virial {dt}] structure {s} rel={e:.3e}")
        assert e <= tol


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_gpr_predict_matches_oracle(dt):
    """Sparse kernel model (Eq. sparse-gp, polynomial kernel, zeta = 3) on
    seeded inputs (seed 2006) with ragged tiles: 300 centres, 1890 features,
    150 active points; centres of species 3 have no active point and active
    points of species 2 no centre, so those energies and gradients are 0."""
    rng = np.random.default_rng(2006)
    N, F, nA = 300, 1890, 150
    sp = rng.choice([0, 1, 3], size=N, p=[0.5, 0.4, 0.1]).astype(np.int32)
    asp = rng.choice([0, 1, 2], size=nA).astype(np.int32)
    p = rng.normal(size=(N, F))
    M = rng.normal(size=(nA, F))
    M /= np.linalg.norm(M, axis=1, keepdims=True)
    w = rng.normal(size=nA)
    E_ref, g_ref = oracle.gpr_predict(sp, p, asp, M, w, 3)
    calc = P.Calculator.from_hypers(synthetic.liquid_bulk(n_atoms=64).hypers)
    dev = lambda a, t=dt: torch.tensor(a, dtype=t, device="cuda")
    E, g = calc.gpr_predict(dev(sp, torch.int32), dev(p), dev(asp, torch.int32), dev(M), dev(w), 3)
    E2, g2 = calc.gpr_predict(dev(sp, torch.int32), dev(p), dev(asp, torch.int32), dev(M), dev(w), 3,
                              want_grad=False)
    assert calc.device_status() == 0 and g2 is None
    E, g, E2 = (x.double().cpu().numpy() for x in (E, g, E2))
    tol = 1e-12 if dt == torch.float64 else 1e-5
    print(f"[gpr {dt}] rel E={rel(E, E_ref):.3e} dE/dp={rel(g, g_ref):.3e}")
    assert rel(E, E_ref) <= tol and rel(g, g_ref) <= tol
    assert np.array_equal(E, E2)
    none = sp == 3
    assert np.all(E[none] == 0.0) and np.all(g[none] == 0.0)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_gpr_energy_forces_virial_end_to_end(dt):
    """Energies per structure (Eq. additive-energy-model), forces and virial
    (Eqs. gpr-force-order, gpr-stress) of a zeta = 2 sparse model on the
    liquid cube, an empty structure and a triclinic cell: GPU features,
    soap_gpr_predict, the adjoint and soap_virial against the same chain in
    the oracle.  Active points: the normalised oracle features of 24 atoms
    of another liquid cube, weights N(0, 1) (seed 2007)."""
    b = _virial_batch()
    other = synthetic.liquid_bulk(seed=77, n_atoms=64)
    _, _, pa = oracle.features(other)
    pa = pa.reshape(other.n_atoms, -1)[:24]
    M = pa / np.linalg.norm(pa, axis=1, keepdims=True)
    asp = other.species[:24]
    w = np.random.default_rng(2007).normal(size=24)
    calc = P.Calculator.from_hypers(b.hypers)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c, p = calc.features(nl, spc, dt)
    dev = lambda a, t=dt: torch.tensor(a, dtype=t, device="cuda")
    E, dEdp = calc.gpr_predict(spc, p, dev(asp, torch.int32), dev(M), dev(w), 2)
    gc = calc.power_spectrum_backward(c, dEdp.reshape(p.shape))
    grad, gpair = calc.spherical_expansion_backward(nl, spc, gc)
    vir = calc.virial(nl, gpair, b.atom_offsets)
    assert calc.device_status() == 0
    ref_nl, _, p_ref = oracle.features(b)
    E_ref, g_ref = oracle.gpr_predict(b.species, p_ref.reshape(b.n_atoms, -1), asp, M, w, 2)
    grad_ref, gp_ref = oracle.vjp(b.hypers, b.species, ref_nl, g_ref.reshape(p_ref.shape))
    vir_ref = oracle.virial(b.atom_offsets, ref_nl, gp_ref)
    offs = b.atom_offsets
    Es = np.array([E.double().cpu().numpy()[offs[s]:offs[s + 1]].sum() for s in range(3)])
    Es_ref = np.array([E_ref[offs[s]:offs[s + 1]].sum() for s in range(3)])
    tol = 1e-7 if dt == torch.float64 else 1e-5
    ef = rel(grad.double().cpu().numpy(), grad_ref)
    print(f"[gpr e2e {dt}] rel E={rel(Es, Es_ref):.3e} forces={ef:.3e} "
          f"virial={rel(vir.double().cpu().numpy(), vir_ref):.3e}")
    assert rel(Es, Es_ref) <= tol and ef <= tol
    assert rel(vir.double().cpu().numpy(), vir_ref) <= tol
    assert Es[1] == 0.0


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_selected_invariants_match_oracle(dt):
    """Selected invariants (Sec. 4.H) on two 8-species cells (K = 96,
    lmax 8): 700 seeded triples (seed 2009, both k1 <= k2 and k1 > k2, every
    l) plus 64 columns picked by farthest-point sampling over the oracle's
    spectra, from GPU coefficients against the oracle's selection of its own
    coefficients; a triple out of range gives 0 and SOAP_EINVAL."""
    from paper_2101_08814_amd.selection import fps_columns, packed_to_triples
    b = synthetic.multi_species_cells(n_cells=2)
    h = b.hypers
    K, lmax = h["n_species"] * h["nmax"], h["lmax"]
    calc = P.Calculator.from_hypers(h)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c = calc.spherical_expansion(nl, spc, dt)
    ref_nl, c_ref, p_ref = oracle.features(b)
    rng = np.random.default_rng(2009)
    tri = np.stack([rng.integers(0, K, 700), rng.integers(0, K, 700), rng.integers(0, lmax + 1, 700)], 1)
    cols = fps_columns(p_ref.reshape(p_ref.shape[0], -1)[:64], 64)
    tri = np.concatenate([tri, packed_to_triples(K, lmax, cols)]).astype(np.int32)
    got = calc.power_spectrum_selected(c, tri)
    assert calc.device_status() == 0
    ref = oracle.power_spectrum_selected(h, c_ref, tri)
    e = rel(got.double().cpu().numpy(), ref)
    print(f"[selected {dt}] rel={e:.3e} worst centre={worst_centre(got.double().cpu().numpy(), ref):.3e}")
    assert e <= (1e-7 if dt == torch.float64 else 1e-6)
    bad = tri[:3].copy()
    bad[1] = (0, K, 0)
    out = calc.power_spectrum_selected(c, bad)
    assert calc.device_status() == P._lib.SOAP_EINVAL
    assert torch.all(out[:, 1] == 0)
    calc.reset_status()


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_selected_invariants_backward_matches_oracle(dt):
    """Adjoint of the selected invariants on two 8-species cells: 700
    seeded triples (seed 2011, repeats and k1 = k2 possible) and an upstream
    gradient N(0, 1), from GPU coefficients against the oracle's adjoint of
    its own coefficients."""
    b = synthetic.multi_species_cells(n_cells=2)
    h = b.hypers
    K, lmax = h["n_species"] * h["nmax"], h["lmax"]
    calc = P.Calculator.from_hypers(h)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c = calc.spherical_expansion(nl, spc, dt)
    _, c_ref, _ = oracle.features(b)
    rng = np.random.default_rng(2011)
    tri = np.stack([rng.integers(0, K, 700), rng.integers(0, K, 700), rng.integers(0, lmax + 1, 700)],
                   1).astype(np.int32)
    G = rng.normal(size=(b.n_atoms, 700))
    gc = calc.power_spectrum_selected_backward(c, tri, torch.tensor(G, dtype=dt, device="cuda"))
    assert calc.device_status() == 0
    ref = oracle.power_spectrum_selected_vjp(h, c_ref, tri, G)
    e = rel(gc.double().cpu().numpy(), ref)
    print(f"[selected backward {dt}] rel={e:.3e}")
    assert e <= (1e-7 if dt == torch.float64 else 1e-5)


def _selected_backward_raw(calc, c, tri, G, corrupt=None):
    """soap_power_spectrum_selected_backward through the C ABI with the
    host plan, optionally corrupted by corrupt(offsets, entries) first."""
    import ctypes
    from paper_2101_08814_amd.soap import _ptr, _np_ptr, _precision
    L = P._lib.lib()
    n_sel = tri.shape[0]
    offs = np.zeros(calc.K * (calc.lmax + 1) + 1, dtype=np.int32)
    ent = np.zeros((max(2 * n_sel, 1), 2), dtype=np.int32)
    assert L.soap_power_spectrum_selected_plan(calc.K, calc.lmax, n_sel, _np_ptr(tri), _np_ptr(offs),
                                               _np_ptr(ent)) == 0
    if corrupt is not None:
        corrupt(offs, ent)
    offs_d, ent_d = torch.from_numpy(offs).cuda(), torch.from_numpy(ent).cuda()
    g = torch.tensor(G, dtype=c.dtype, device="cuda")
    gc = torch.empty_like(c)
    e = calc._exec()
    assert L.soap_power_spectrum_selected_backward(ctypes.byref(e), _precision(c.dtype), c.shape[0], calc.K,
                                                   calc.lmax, _ptr(c), n_sel, _ptr(g), _ptr(offs_d), _ptr(ent_d),
                                                   _ptr(gc)) == 0
    return gc, offs, ent


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_selected_backward_corrupted_plan(dt):
    """An entry of the plan out of range is reported (SOAP_EINVAL) and
    contributes nothing; every other term is summed as before (FP32: the
    plan held in LDS; FP64: the plan read through L2)."""
    b = synthetic.multi_species_cells(n_cells=1)
    h = b.hypers
    K, lmax = h["n_species"] * h["nmax"], h["lmax"]
    calc = P.Calculator.from_hypers(h)
    nl, pos, spc = gpu_neighbors(calc, b, dt)
    c = calc.spherical_expansion(nl, spc, dt)
    rng = np.random.default_rng(2012)
    tri = np.stack([rng.integers(0, K, 300), rng.integers(0, K, 300), rng.integers(0, lmax + 1, 300)],
                   1).astype(np.int32)
    G = rng.normal(size=(b.n_atoms, 300))
    good, offs, ent = _selected_backward_raw(calc, c, tri, G)
    assert calc.device_status() == 0
    r = int(np.argmax(np.diff(offs) > 0))     # a row with entries
    t = int(offs[r])
    q, partner = int(ent[t, 0]), int(ent[t, 1])
    k, l = divmod(r, lmax + 1)

    def corrupt(o, e):
        e[t, 0] = tri.shape[0] + 5

    bad, _, _ = _selected_backward_raw(calc, c, tri, G, corrupt)
    assert calc.device_status() == P._lib.SOAP_EINVAL
    calc.reset_status()
    expect = good.clone().reshape(b.n_atoms, K, (lmax + 1) ** 2)
    cf = c.reshape(b.n_atoms, K, (lmax + 1) ** 2)
    Gd = torch.tensor(G, dtype=dt, device="cuda")
    expect[:, k, l * l:(l + 1) ** 2] -= Gd[:, q:q + 1] * cf[:, partner, l * l:(l + 1) ** 2]
    atol = 1e-12 if dt == torch.float64 else 1e-5 * float(good.abs().max())
    assert torch.allclose(bad.reshape(expect.shape), expect, rtol=0, atol=atol)


def test_selected_backward_overlapping_rows():
    """Row offsets that are not monotonic pass the per-row check but make
    rows overlap: more entries than the plan holds.  FP32 (plan in LDS):
    reported as SOAP_EINVAL, the rows that no longer fit left empty, the
    output finite."""
    b = synthetic.multi_species_cells(n_cells=1)
    h = b.hypers
    K, lmax = h["n_species"] * h["nmax"], h["lmax"]
    calc = P.Calculator.from_hypers(h)
    nl, pos, spc = gpu_neighbors(calc, b, torch.float32)
    c = calc.spherical_expansion(nl, spc, torch.float32)
    rng = np.random.default_rng(2014)
    tri = np.stack([rng.integers(0, K, 300), rng.integers(0, K, 300), rng.integers(0, lmax + 1, 300)],
                   1).astype(np.int32)
    G = rng.normal(size=(b.n_atoms, 300))
    good, offs, ent = _selected_backward_raw(calc, c, tri, G)
    assert calc.device_status() == 0

    def corrupt(o, e):
        # rows 0, 2, 4, 6 each claim every entry (rows 1, 3, 5, 7 run
        # backwards and fail the check): with the rows after them about
        # twice what the plan holds
        o[1:8] = [o[-1], 0, o[-1], 0, o[-1], 0, o[-1]]

    bad, _, _ = _selected_backward_raw(calc, c, tri, G, corrupt)
    assert calc.device_status() == P._lib.SOAP_EINVAL
    calc.reset_status()
    assert torch.isfinite(bad).all()


@pytest.mark.parametrize("n_sel", [6000, 9000])
def test_selected_backward_large_selection(n_sel):
    """Large selections against the oracle: at 6000 triples the LDS plan
    takes 118 KB, one work-group per CU instead of two; at 9000 the gradient
    row no longer fits beside the coefficients in the plan's 16-bit
    addresses, so the per-centre kernel that reads the plan through L2
    runs."""
    b = synthetic.multi_species_cells(n_cells=1)
    h = b.hypers
    K, lmax = h["n_species"] * h["nmax"], h["lmax"]
    calc = P.Calculator.from_hypers(h)
    nl, pos, spc = gpu_neighbors(calc, b, torch.float32)
    c = calc.spherical_expansion(nl, spc, torch.float32)
    _, c_ref, _ = oracle.features(b)
    rng = np.random.default_rng(2013)
    tri = np.stack([rng.integers(0, K, n_sel), rng.integers(0, K, n_sel), rng.integers(0, lmax + 1, n_sel)],
                   1).astype(np.int32)
    G = rng.normal(size=(b.n_atoms, n_sel))
    gc = calc.power_spectrum_selected_backward(c, tri, torch.tensor(G, dtype=torch.float32, device="cuda"))
    assert calc.device_status() == 0
    ref = oracle.power_spectrum_selected_vjp(h, c_ref, tri, G)
    e = rel(gc.double().cpu().numpy(), ref)
    print(f"[selected backward {n_sel}] rel={e:.3e}")
    assert e <= 1e-5


def test_vjp_full_size_against_finite_differences():
    """4096-atom liquid (2 species, nmax 10, lmax 8, rcut 6): the FP32 adjoint
    against central differences (h = 1e-4 A) of the FP64 GPU forward on 32
    seeded coordinates; the FP64 adjoint against the same differences."""
    b = synthetic.liquid_bulk()
    calc = P.Calculator.from_hypers(b.hypers)
    pos, spc = to_dev(b)
    rng = np.random.default_rng(2004)
    ao, ce, pb = b.atom_offsets, b.cells, b.pbc
    nl64 = calc.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=torch.float64)
    c64, p64 = calc.features(nl64, spc, torch.float64)
    W = torch.tensor(rng.normal(size=tuple(p64.shape)), dtype=torch.float64, device="cuda")
    g64, _ = calc.spherical_expansion_backward(nl64, spc, calc.power_spectrum_backward(c64, W))
    nl32 = calc.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=torch.float32)
    c32, p32 = calc.features(nl32, spc, torch.float32)
    g32, _ = calc.spherical_expansion_backward(nl32, spc, calc.power_spectrum_backward(c32, W.float()))
    assert calc.device_status() == 0
    h = 1e-4
    picks = [(int(k), int(x)) for k, x in zip(rng.integers(0, b.n_atoms, 32), rng.integers(0, 3, 32))]
    fd = []
    for k, x in picks:
        vals = []
        for sgn in (1, -1):
            pp = pos.clone()
            pp[k, x] += sgn * h
            nlp = calc.compute_neighbors(pp, spc, ao, ce, pb, vec_dtype=torch.float64)
            _, pp_ = calc.features(nlp, spc, torch.float64)
            vals.append(float((W * pp_).sum()))
        fd.append((vals[0] - vals[1]) / (2 * h))
    fd = np.array(fd)
    a64 = np.array([float(g64[k, x]) for k, x in picks])
    a32 = np.array([float(g32[k, x]) for k, x in picks])
    scale = np.abs(g64.cpu().numpy()).max()
    print(f"[fd] max|fd-a64|/scale={np.abs(fd - a64).max() / scale:.3e} "
          f"max|a32-a64|/scale={np.abs(a32 - a64).max() / scale:.3e}")
    assert np.abs(fd - a64).max() <= 1e-6 * scale
    assert rel(g32.double().cpu().numpy(), g64.cpu().numpy()) <= 1e-5


def test_autograd_function_matches_adjoint():
    b = synthetic.liquid_bulk(n_atoms=256)
    calc = P.Calculator.from_hypers(b.hypers)
    pos, spc = to_dev(b)
    x = pos.clone().requires_grad_(True)
    p = P.soap_power_spectrum_of_positions(x, calc, spc, b.atom_offsets, b.cells, b.pbc, torch.float32)
    W = torch.randn(p.shape, device="cuda", generator=torch.Generator(device="cuda").manual_seed(5))
    (g,) = torch.autograd.grad((W * p).sum(), x)
    ref_nl = oracle.neighbors(b)
    g_ref, _ = oracle.vjp(b.hypers, b.species, ref_nl, W.double().cpu().numpy())
    assert rel(g.cpu().numpy(), g_ref) <= 1e-5


# ------------------------------------------------------------ device errors
def test_capacity_exceeded_reports_status():
    b = synthetic.diamond_bulk()
    calc = P.Calculator.from_hypers(b.hypers)
    pos, spc = to_dev(b)
    nl = calc.compute_neighbors(pos, spc, b.atom_offsets, b.cells, b.pbc, capacity=1000)
    assert calc.device_status() == P._lib.SOAP_ECAPACITY
    assert int(nl.pair_offsets[-1]) > 1000
    calc.reset_status()
    calc.features(nl, spc, torch.float32)
    assert calc.device_status() == P._lib.SOAP_ECAPACITY


def test_species_out_of_range_reports_status():
    b = synthetic.clusters_2species().subset([0])
    calc = P.Calculator.from_hypers(b.hypers)
    pos, spc = to_dev(b)
    spc[3] = 5
    calc.compute_neighbors(pos, spc, b.atom_offsets, b.cells, b.pbc)
    assert calc.device_status() == P._lib.SOAP_ESPECIES


@pytest.mark.parametrize("what", ["singular_cell", "bad_offsets"])
def test_invalid_structures_report_status(what):
    b = synthetic.diamond_bulk()
    calc = P.Calculator.from_hypers(b.hypers)
    pos, spc = to_dev(b)
    cells, offs = b.cells.copy(), b.atom_offsets.copy()
    if what == "singular_cell":
        cells[0, 2] = cells[0, 0]
    else:
        offs[-1] -= 1
    nl = calc.compute_neighbors(pos, spc, offs, cells, b.pbc, capacity=100)
    assert calc.device_status() == P._lib.SOAP_EINVAL
    assert int(nl.pair_offsets[-1]) == 0


def _all_pairs_batch(path):
    """A batch that the neighbour list builds without bins: a 40-atom slab
    (one wave checks the input itself), or 64 cells of 256 atoms (geometry
    kernel, then counts, scan and fill)."""
    if path == "small":
        return NEIGHBOR_CASES["slab_pbc_xy"]()
    return synthetic.multi_species_cells().subset(list(range(64)))


@pytest.mark.parametrize("path", ["small", "many"])
@pytest.mark.parametrize("what", ["singular_cell", "bad_offsets"])
def test_invalid_structures_report_status_all_pairs(path, what):
    """The all-pairs neighbour paths check the input as the bin build does:
    SOAP_EINVAL and an empty list."""
    b = _all_pairs_batch(path)
    calc = P.Calculator.from_hypers(b.hypers)
    pos, spc = to_dev(b)
    cells, offs = b.cells.copy(), b.atom_offsets.copy()
    if what == "singular_cell":
        s = cells.shape[0] - 1
        cells[s, 1] = cells[s, 0]
    else:
        offs[-1] -= 1
    nl = calc.compute_neighbors(pos, spc, offs, cells, b.pbc, capacity=100)
    assert calc.device_status() == P._lib.SOAP_EINVAL
    assert int(nl.pair_offsets[-1]) == 0


@pytest.mark.parametrize("path", ["small", "many"])
def test_capacity_exceeded_reports_status_all_pairs(path):
    b = _all_pairs_batch(path)
    calc = P.Calculator.from_hypers(b.hypers)
    pos, spc = to_dev(b)
    nl = calc.compute_neighbors(pos, spc, b.atom_offsets, b.cells, b.pbc, capacity=50)
    assert calc.device_status() == P._lib.SOAP_ECAPACITY
    assert int(nl.pair_offsets[-1]) > 50
    assert int(nl.pair_offsets[-1]) == oracle.neighbors(b).n_pairs


def test_coincident_atoms_report_status():
    b = synthetic.clusters_2species().subset([0])
    pos = b.positions.copy()
    pos[1] = pos[0]
    calc = P.Calculator.from_hypers(b.hypers)
    p_, s_ = to_dev(synthetic.Batch(pos, b.species, b.atom_offsets, b.cells, b.pbc, b.hypers))
    calc.compute_neighbors(p_, s_, b.atom_offsets, b.cells, b.pbc)
    assert calc.device_status() == P._lib.SOAP_EGEOMETRY


def test_isolated_atoms_and_absent_species():
    """Atoms with no neighbours get only the centre term; a species with no
    atoms gives zero channels."""
    hyp = dict(n_species=3, nmax=4, lmax=3, rcut=3.0, sigma=0.5, cutoff_width=0.5, include_center=1)
    pos = np.array([[0.0, 0, 0], [10.0, 0, 0], [10.0, 1.5, 0]])
    b = synthetic.Batch(pos, np.array([0, 0, 2], np.int32), np.array([0, 3]), np.zeros((1, 3, 3)),
                        np.zeros((1, 3), np.uint8), hyp)
    _, nl, _, (c, p) = run_features(b, torch.float64)
    ref_nl, ref_c, ref_p = oracle.features(b)
    assert rel(c, ref_c) <= 1e-7 and rel(p, ref_p) <= 1e-7
    assert np.all(c[:, 1] == 0.0)
