#!/usr/bin/env python3
"""Throughput of the SOAP hot path on one MI355X, in atom-centres per second.

Workload (one step): a periodic perturbed-diamond cell of 1024 atoms
(4 x 4 x 8 conventional cells, a = 5.43 A, 0.1 A Gaussian displacements),
1 species, rcut 5 A, cutoff width 0.5 A, sigma 0.5 A, nmax 8, lmax 6:
full neighbour list with periodic images, FP32 spherical expansion, power
spectrum and forward-mode position gradients of both (every pair row and
every self row).  Inputs are resident in HBM when the timed region starts;
each step launches two phases on one stream: the neighbour list and
soap_features, whose one kernel writes c, p, the self rows and the pair
rows (~97% of the bytes).  --two-pass times the older split instead: the
per-centre pass, then the pair rows from soap_gradient_rows.

Prints ONE JSON line on stdout; diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
DOMINANT_KERNEL = "k_features_rows<float, 6>"
TWO_PASS_KERNEL = "k_pair_rows<float, 6, true, true>"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "features_diamond1024_traffic.txt")
KERNEL_SOURCES = ["features_rows.hip", "lane_pair.hpp", "chunk.hpp", "sph.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SPECTRUM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spectrum_bf16_molecules_counters.txt")
SPECTRUM_SOURCES = ["power_spectrum.hip"]


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2101_08814_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n_launch_bytes_alg: float, path: str = TRAFFIC_FILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch of a kernel from its committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.lstrip().startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash(sources):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes(N: int, P: int, S: int, nmax: int, lmax: int, es: int = 4):
    """Bytes each pass must move per launch, inputs read once and outputs
    written once; the L2-resident spline table is not counted.
    Per-centre pass: pair vectors, neighbour indices and species, CSR
    offsets, centre species in; c, p and both self rows out.
    Row pass: pair vectors, neighbour indices and species, CSR offsets and c
    of each centre in; the dc and dp rows of every pair out.
    Fused pass (soap_features with rows): the inputs of the per-centre pass
    in; c, p, both self rows and both pair rows out."""
    L2 = (lmax + 1) ** 2
    K = S * nmax
    KK = K * (K + 1) // 2
    pair_in = 12 + 4 + 4
    centre_out = es * (K * L2 + (lmax + 1) * KK + 3 * K * L2 + 3 * (lmax + 1) * KK)
    pair_out = es * (3 * nmax * L2 + 3 * (lmax + 1) * KK)
    centres = N * (centre_out + 8 + 4) + P * pair_in
    rows = N * (es * K * L2 + 8) + P * (pair_out + pair_in)
    fused = N * (centre_out + 8 + 4) + P * (pair_in + pair_out)
    return centres, rows, fused


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, seconds: float):
    """The FP64 oracle, as it stands, on the host cores: the same step
    (neighbours, expansion, power spectrum, every gradient row) on the whole
    workload, from a -march=native build of the oracle's source made here.
    Three samples with every thread and three with one thread (the paper's
    code is serial), each repeating whole steps until its share of
    `seconds` has passed; the medians are reported."""
    import statistics
    import tempfile

    import oracle
    path = os.path.join(tempfile.mkdtemp(prefix="soap_oracle_"), "libsoap_oracle_native.so")
    build = "gcc " + " ".join(oracle.FLAGS + ["-march=native"])
    try:
        oracle.build(path=path, native=True)
        oracle.use_build(path)
    except Exception as e:     # no gcc: the generic build that ships
        log(f"[cpu_baseline] native build failed ({e}); timing the generic build")
        build = "gcc " + " ".join(oracle.FLAGS)
        oracle.use_build(oracle._LIB_PATH)
    h = batch.hypers
    n_all = oracle.num_threads()

    def sample(budget):
        reps, t0 = 0, time.perf_counter()
        while True:
            nl = oracle.neighbors(batch)
            c = oracle.expansion(h, batch.species, nl)
            oracle.power_spectrum(h, c)
            oracle.gradients(h, batch.species, nl)
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return batch.n_atoms * reps / el, reps, el

    multi = [sample(seconds / 6) for _ in range(3)]
    oracle.set_num_threads(1)
    single = [sample(seconds / 6) for _ in range(3)]
    oracle.set_num_threads(n_all)
    v_multi = statistics.median(m[0] for m in multi)
    v_single = statistics.median(m[0] for m in single)
    return {"value": v_multi, "unit": "atom-centres/s", "cores": n_all, "kind": "oracle",
            "sample": f"median of 3 samples of whole 1024-atom steps (neighbours, expansion, power spectrum, all "
                      f"gradient rows) in FP64 on {n_all} threads: "
                      + ", ".join(f"{r} steps in {el:.1f} s" for _, r, el in multi),
            "single_thread": {"value": v_single, "unit": "atom-centres/s", "cores": 1,
                              "sample": "median of 3: " + ", ".join(f"{r} steps in {el:.1f} s" for _, r, el in single)},
            "cpu_model": cpu_model(), "build": build}


def run_compression(args) -> int:
    """The learned-compression workload: 512 periodic cells x 256 atoms, 8
    species (equal counts), rcut 5 A, sigma 0.5 A, nmax 12, lmax 8 (96
    channels).  Trains the per-l network (16 outputs, 128 hidden, float) on
    the coefficients of cells 0-409 (80%), scores the linear-kernel error of
    the full symmetric spectrum on held-out centres of cells 410-511, and
    times the plain path (expansion + full power spectrum) against the
    compressed one (expansion + bfloat16 MFMA compression and spectrum)."""
    import numpy as np
    import torch

    import synthetic
    import paper_2101_08814_amd as P

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    batch = synthetic.multi_species_cells()
    h = batch.hypers
    calc = P.Calculator.from_hypers(h)
    pos = torch.tensor(batch.positions, dtype=torch.float64, device=dev)
    spc = torch.tensor(batch.species, dtype=torch.int32, device=dev)
    ao, ce, pb = P.soap.structures_to_device(batch.atom_offsets, batch.cells, batch.pbc, dev)
    nl = calc.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=torch.float32, transpose=False)
    N = batch.n_atoms
    c = calc.spherical_expansion(nl, spc, dtype=torch.float32)
    torch.cuda.synchronize()
    log(f"[compression] {N} centres, {nl.count()} pairs, coefficients {c.numel() * 4 / 1e9:.2f} GB "
        f"({time.perf_counter() - t0:.1f} s)")
    n_train = int(batch.atom_offsets[410])
    held = torch.arange(n_train, N, max(1, (N - n_train) // 2048), device=dev)[:2048]
    c_held = c[held].contiguous()
    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(1, args.steps)
    H = 128
    results = {}
    for Q in (16, 32):
        cmp_ = P.Compressor(calc, Q, H)
        cmp_.init_pca(c[:n_train], seed=0, noise=0.0)
        eps_pca = cmp_.kernel_error(c_held)
        cmp_.init_pca(c[:n_train], seed=1005, noise=0.05)
        gen = torch.Generator(device="cpu").manual_seed(1005)
        t1 = time.perf_counter()
        steps = args.train_steps
        for k in range(steps):
            idx = torch.randint(0, n_train, (512,), generator=gen).to(dev)
            lr = 2e-3 * (0.05 ** (k / max(1, steps - 1)))
            cmp_.train_step(c[idx].contiguous(), lr=lr)
            if (k + 1) % 200 == 0:
                log(f"[compression] Q={Q} step {k + 1}/{steps}")
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        eps32 = cmp_.kernel_error(c_held)
        eps16 = cmp_.kernel_error(c_held, precision="bf16")
        t_comp = timed(lambda: cmp_.forward(c, precision="bf16"), reps)
        results[Q] = {"eps_K_pca": eps_pca, "eps_K_trained_fp32": eps32, "eps_K_trained_bf16": eps16,
                      "compressed_spectrum_ms": t_comp, "train_seconds": t_train,
                      "features_per_centre": (h["lmax"] + 1) * Q * (Q + 1) // 2}
        log(f"[compression] Q={Q}: eps_K pca {eps_pca:.4f}  trained fp32 {eps32:.4f}  bf16 {eps16:.4f}  "
            f"compressed p {t_comp:.3f} ms  ({t_train:.1f} s training)")
    t_exp = timed(lambda: calc.spherical_expansion(nl, spc, dtype=torch.float32), reps)
    t_plain32 = timed(lambda: calc.power_spectrum(c, precision=torch.float32), reps)
    t_plain16 = timed(lambda: calc.power_spectrum(c, precision="bf16"), reps)
    t_plain = t_exp + min(t_plain32, t_plain16)
    t_cpath = t_exp + results[16]["compressed_spectrum_ms"]
    for Q in results:
        results[Q]["speedup_vs_plain"] = t_plain / (t_exp + results[Q]["compressed_spectrum_ms"])
    log(f"[compression] expansion {t_exp:.3f} ms  full p fp32 {t_plain32:.3f} ms  bf16 {t_plain16:.3f} ms")
    line = {
        "metric": "atom-centres/s, expansion + compressed power spectrum (16 learned channels, bf16 MFMA) "
                  "vs expansion + full power spectrum",
        "value": N / (t_cpath * 1e-3),
        "unit": "atom-centres/s",
        "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": t_cpath,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {
            "workload": "512 periodic cells x 256 atoms (side 16.22 A), 8 species x 32, rcut 5 A, sigma 0.5 A, "
                        "nmax 12, lmax 8; network 96 -> 128 -> Q channels per l, trained on cells 0-409, "
                        "kernel error on 2048 centres of cells 410-511",
            "centres": N, "plain_ms_per_step": t_plain, "speedup": t_plain / t_cpath,
            "expansion_ms": t_exp, "full_spectrum_ms_fp32": t_plain32, "full_spectrum_ms_bf16": t_plain16,
            "full_features_per_centre": (h["lmax"] + 1) * calc.KK,
            "compressed": {str(Q): v for Q, v in results.items()},
            "train_steps": args.train_steps, "train_batch": 512,
        },
    }
    print(json.dumps(line), flush=True)
    return 0


def run_selected(args) -> int:
    """Selected invariants (Sec. 4.H) on the 8-species workload: 512
    periodic cells x 256 atoms, nmax 12, lmax 8 (96 channels, 41,904 packed
    features).  From FP32 coefficients already in HBM, times the full FP32
    spectrum against 2000 seeded packed columns (seed 2010, uniform over the
    packed features) computed alone, and the adjoint of those columns for an
    N(0, 1) upstream gradient (its host plan built inside the timed call)."""
    import numpy as np
    import torch

    import synthetic
    import paper_2101_08814_amd as P
    from paper_2101_08814_amd.selection import packed_to_triples

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    batch = synthetic.multi_species_cells()
    h = batch.hypers
    calc = P.Calculator.from_hypers(h)
    pos = torch.tensor(batch.positions, dtype=torch.float64, device=dev)
    spc = torch.tensor(batch.species, dtype=torch.int32, device=dev)
    ao, ce, pb = P.soap.structures_to_device(batch.atom_offsets, batch.cells, batch.pbc, dev)
    nl = calc.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=torch.float32, transpose=False)
    N = batch.n_atoms
    K, lmax = calc.K, calc.lmax
    KK = K * (K + 1) // 2
    n_sel = 2000
    cols = np.sort(np.random.default_rng(2010).choice((lmax + 1) * KK, size=n_sel, replace=False))
    tri = torch.tensor(packed_to_triples(K, lmax, cols), device=dev)
    c = calc.spherical_expansion(nl, spc, torch.float32)
    g_sel = torch.randn((N, n_sel), generator=torch.Generator(device="cpu").manual_seed(2010)).to(dev)
    tri_host = tri.cpu().numpy()
    phases = [("full_spectrum", lambda: calc.power_spectrum(c)),
              ("selected", lambda: calc.power_spectrum_selected(c, tri)),
              ("selected_backward", lambda: calc.power_spectrum_selected_backward(c, tri_host, g_sel))]
    for _ in range(max(2, args.warmup)):
        for _, f in phases:
            f()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 20))
    ms = {}
    for name, f in phases:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            f()
        e1.record()
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / steps
    if calc.device_status() != 0:
        log(f"device status {calc.device_status()}")
        return 4
    L2 = (lmax + 1) ** 2
    sel_bytes = N * (K * L2 + n_sel) * 4 + n_sel * 12
    full_bytes = N * (K * L2 + (lmax + 1) * KK) * 4
    gbs = sel_bytes / (ms["selected"] * 1e-3) / 1e9
    log(f"[bench:selected] N={N} full={ms['full_spectrum']:.3f} ms selected({n_sel})={ms['selected']:.3f} ms "
        f"({gbs:.0f} GB/s) selected backward={ms['selected_backward']:.3f} ms")
    line = {
        "metric": "atom-centres/s (2000 selected invariants from c)", "value": N / (ms["selected"] * 1e-3),
        "unit": "atom-centres/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": ms["selected"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512 periodic cells x 256 atoms (side 16.22 A), 8 species x 32, rcut 5 A, sigma 0.5 A, "
                               "nmax 12, lmax 8 (96 channels, 41,904 packed features); 2000 seeded packed columns "
                               "from FP32 c in HBM",
                   "centres": N, "n_selected": n_sel,
                   "full_spectrum_ms": ms["full_spectrum"], "full_spectrum_GB_s":
                       full_bytes / (ms["full_spectrum"] * 1e-3) / 1e9,
                   "speedup_vs_full": ms["full_spectrum"] / ms["selected"],
                   "selected_backward_ms": ms["selected_backward"],
                   "selected_backward_GB_s": N * (2 * K * L2 + n_sel) * 4 / (ms["selected_backward"] * 1e-3) / 1e9},
        "roofline": {"bound": "hbm", "kernel": "k_ps_selected<float>", "achieved": gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel_ms": ms["selected"],
                     "algorithmic_bytes_per_launch": sel_bytes},
    }
    print(json.dumps(line), flush=True)
    return 0


def config_bytes(kind: str, N: int, P: int, S: int, nmax: int, lmax: int, es: int):
    """Algorithmic bytes of one launch of a phase of the parity workloads
    (inputs read once, outputs written once; the L2-resident spline table
    not counted).  es: bytes per element of c and p."""
    L2 = (lmax + 1) ** 2
    K = S * nmax
    KK = K * (K + 1) // 2
    c, p = es * K * L2, es * (lmax + 1) * KK
    pair_in = 3 * es + 4 + 4
    if kind == "expansion":          # c from the pairs
        return N * (c + 12) + P * pair_in
    if kind == "features":           # c and p from the pairs
        return N * (c + p + 12) + P * pair_in
    if kind == "spectrum":           # p from c
        return N * (c + p)
    if kind == "spectrum_backward":  # grad_c from c and grad_p
        return N * (2 * c + p)
    if kind == "expansion_backward":  # per-pair g and grad_r from grad_c and the pairs
        return N * (c + 8 + 3 * es) + P * (pair_in + 4 + 3 * es)
    if kind == "virial":             # 3x3 per structure from the pairs' g and r
        return P * 6 * es + N * 8
    raise ValueError(kind)


def measure_config(wl: str, steps: int, warmup: int):
    """The parity workloads as timed steps (neighbours included, as in the
    headline step); each phase is timed with HIP events on the launch stream.
    clusters: 8 x 64-atom clusters, FP64 c and p.
    molecules: 256 molecules of 20-200 atoms, 4 species, FP32 c then p from
      the bfloat16 hi/lo MFMA contraction (one launch for all structures).
    liquid: 4096-atom periodic liquid, 2 species, FP32 c and p, then the
      adjoint for an upstream gradient drawn N(0, 1) (seed 2004).
    gpr: the 1024-atom diamond cell with the bulk-silicon feature set
      (nmax 10, lmax 12: 715 features), a polynomial sparse model (zeta 4,
      2000 active points, |N(0, 1)| rows normalised, weights N(0, 1), seed
      2008): energies, forces and virial (features, model with dE/dp, the
      adjoint, the virial)."""
    import numpy as np
    import torch

    import synthetic
    import paper_2101_08814_amd as P

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    batch = {"clusters": synthetic.clusters_2species, "molecules": synthetic.molecule_batch,
             "liquid": synthetic.liquid_bulk, "gpr": synthetic.diamond_bulk}[wl]()
    if wl == "gpr":
        batch.hypers = dict(batch.hypers, nmax=10, lmax=12)
    h = batch.hypers
    calc = P.Calculator.from_hypers(h)
    td = torch.float64 if wl == "clusters" else torch.float32
    es = 8 if td == torch.float64 else 4
    pos = torch.tensor(batch.positions, dtype=torch.float64, device=dev)
    spc = torch.tensor(batch.species, dtype=torch.int32, device=dev)
    ao, ce, pb = P.soap.structures_to_device(batch.atom_offsets, batch.cells, batch.pbc, dev)
    adjoint = wl in ("liquid", "gpr")
    nl = calc.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=td, transpose=adjoint)
    N, Pn = batch.n_atoms, nl.count()
    S, nmax, lmax = h["n_species"], h["nmax"], h["lmax"]
    state = {}

    def ph_neighbors():
        calc.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=td, out=nl)

    phases = [("neighbours", ph_neighbors, None)]
    if wl == "molecules":
        out_c = torch.empty((N, S, nmax, (lmax + 1) ** 2), dtype=td, device=dev)

        def ph_expansion():
            state["c"] = calc.spherical_expansion(nl, spc, td)

        def ph_spectrum():
            state["p"] = calc.power_spectrum(state["c"], "bf16")

        phases += [("expansion", ph_expansion, ("k_expansion_packed<float, 6, 2>", "expansion")),
                   ("spectrum_bf16_mfma", ph_spectrum, ("k_power_spectrum_bf16", "spectrum"))]
    else:
        out = calc.allocate_features(N, nl.capacity, td, dev, False)

        def ph_features():
            calc.features(nl, spc, td, out=out)

        tn = 'double' if td == torch.float64 else 'float'
        if N >= 4096:   # c with pairs packed across centres, then p from c (two kernels)
            kname = f"k_expansion_packed<{tn}, {lmax}, {max(2, (nmax + 3) // 4)}> + k_power_spectrum<{tn}, false>"
        else:
            kname = f"k_expansion_lanes<{tn}, {lmax}, true>"
        phases.append(("features", ph_features, (kname, "features")))
        if wl == "gpr":
            n_active, zeta = 2000, 4
            g = torch.Generator(device="cpu").manual_seed(2008)
            F = out[1][0].numel()
            M = torch.randn((n_active, F), generator=g, dtype=torch.float64).abs()
            M = (M / M.norm(dim=1, keepdim=True)).to(dev, td)
            wts = torch.randn(n_active, generator=g, dtype=torch.float64).to(dev, td)
            asp = torch.zeros(n_active, dtype=torch.int32, device=dev)

            def ph_gpr():
                state["E"], state["dEdp"] = calc.gpr_predict(spc, out[1], asp, M, wts, zeta)

            phases.append(("gpr_predict", ph_gpr, ("k_gpr_dots<float> + k_gpr_energy + k_gpr_grad", "gpr")))
            grad_p = None
        elif adjoint:
            g = torch.Generator(device="cpu").manual_seed(2004)
            grad_p = torch.randn(out[1].shape, generator=g, dtype=torch.float64).to(dev, td)
        if adjoint:

            def ph_ps_backward():
                state["gc"] = calc.power_spectrum_backward(out[0], grad_p if grad_p is not None else
                                                           state["dEdp"].reshape(out[1].shape))

            def ph_exp_backward():
                state["gpos"], state["gpair"] = calc.spherical_expansion_backward(nl, spc, state["gc"])

            phases += [("spectrum_backward", ph_ps_backward, ("k_ps_backward<float>", "spectrum_backward")),
                       ("expansion_backward", ph_exp_backward,
                        ("k_exp_backward_lanes + k_exp_backward_gather", "expansion_backward"))]
            if wl == "gpr":
                def ph_virial():
                    state["virial"] = calc.virial(nl, state["gpair"], ao)

                phases.append(("virial", ph_virial, ("k_virial_centres + k_virial_structures", "virial")))
    # events made and the status word cleared before the warm-up, so that
    # the timed steps follow it directly
    K = steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)] for _ in range(K)]
    t_all0, t_all1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    calc.reset_status()
    for _ in range(max(3, warmup)):
        for _, f, _ in phases:
            f()
    torch.cuda.synchronize()
    t_all0.record()
    for k in range(K):
        ev[k][0].record()
        for j, (_, f, _) in enumerate(phases):
            f()
            ev[k][j + 1].record()
    t_all1.record()
    torch.cuda.synchronize()
    status = calc.device_status()
    if status != 0:
        log(f"device status {status}")
        return None
    total_ms = t_all0.elapsed_time(t_all1)
    ph_ms = {name: float(np.median([e[j].elapsed_time(e[j + 1]) for e in ev])) for j, (name, _, _) in
             enumerate(phases)}
    ms_per_step = total_ms / K
    rows = {}
    for name, _, info in phases:
        if info is None:
            continue
        kern, kind = info
        if kind == "gpr":
            KK = (S * nmax) * (S * nmax + 1) // 2
            F = (lmax + 1) * KK
            fl = 4.0 * N * n_active * F     # the two products, one multiply-add per term each
            rows[name] = {"kernel": kern, "ms": ph_ms[name], "algorithmic_flops": fl,
                          "TFLOP_s": fl / (ph_ms[name] * 1e-3) / 1e12,
                          "algorithmic_bytes": es * (N * F * 2 + n_active * F + N + n_active)}
            rows[name]["GB_s"] = rows[name]["algorithmic_bytes"] / (ph_ms[name] * 1e-3) / 1e9
            continue
        b = config_bytes(kind, N, Pn, S, nmax, lmax, es)
        rows[name] = {"kernel": kern, "ms": ph_ms[name], "algorithmic_bytes": b,
                      "GB_s": b / (ph_ms[name] * 1e-3) / 1e9}
    dom = max(rows, key=lambda k: rows[k]["ms"])
    d = rows[dom]
    if "TFLOP_s" in d:
        # dense FP32 products on the vector units: 157.3 TFLOP/s
        roof = {"bound": "alu", "kernel": d["kernel"], "achieved": d["TFLOP_s"], "peak": 157.3, "unit": "TFLOP/s",
                "frac": d["TFLOP_s"] / 157.3, "traffic": None, "kernel_ms": d["ms"],
                "algorithmic_flops_per_launch": d["algorithmic_flops"]}
    else:
        roof = {"bound": "hbm", "kernel": d["kernel"], "achieved": d["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["GB_s"] / HBM_PEAK_GBS, "traffic": None, "kernel_ms": d["ms"],
                "algorithmic_bytes_per_launch": d["algorithmic_bytes"]}
    if wl == "molecules":
        if d["kernel"].startswith("k_power_spectrum_bf16"):
            roof["traffic"] = measured_traffic(d["algorithmic_bytes"], SPECTRUM_TRAFFIC_FILE, SPECTRUM_SOURCES)
        KK = (S * nmax) * (S * nmax + 1) // 2
        flops = 2.0 * N * KK * (lmax + 1) ** 2                 # packed p: K(K+1)/2 dot products of L2 terms
        tf = flops / (rows["spectrum_bf16_mfma"]["ms"] * 1e-3) / 1e12
        rows["spectrum_bf16_mfma"].update({"algorithmic_tflops": tf, "frac_of_bf16_peak": tf / 2500.0,
                                           "attainable_tflops_at_hbm": flops / rows["spectrum_bf16_mfma"][
                                               "algorithmic_bytes"] * HBM_PEAK_GBS / 1e3})
    if adjoint:
        # VALU work of the adjoint's pair pass: per pair and (n, lm) the three
        # components of G * grad(f I Y), about 12 flops (2 FMA x 3 + the product)
        fl = 12.0 * Pn * nmax * (lmax + 1) ** 2
        tf = fl / (rows["expansion_backward"]["ms"] * 1e-3) / 1e12
        rows["expansion_backward"].update({"algorithmic_tflops": tf, "frac_of_fp32_valu_peak": tf / 157.3})
    log(f"[bench:{wl}] N={N} P={Pn} step={ms_per_step * 1e3:.1f} us  " +
        "  ".join(f"{k}={v * 1e3:.1f} us" for k, v in ph_ms.items()))
    names = {"clusters": "8 clusters x 64 atoms (cube 8.618 A), 2 species 32/32, rcut 4 A, sigma 0.5 A, nmax 6, "
                         "lmax 4; neighbours + FP64 expansion and power spectrum",
             "molecules": "256 molecules of 20-200 atoms at 0.08 A^-3, 4 species, rcut 5 A, sigma 0.4 A, nmax 8, "
                          "lmax 6; neighbours + FP32 expansion + bfloat16 hi/lo MFMA power spectrum, one launch",
             "liquid": "4096-atom periodic liquid (side 43.44 A), 2 species 2867/1229, rcut 6 A, sigma 0.5 A, "
                       "nmax 10, lmax 8; neighbours with reverse-pair index + FP32 expansion and power spectrum + "
                       "adjoint (vector-Jacobian product for an N(0,1) upstream gradient)",
             "gpr": "periodic perturbed diamond, 1024 atoms, 1 species, rcut 5 A, sigma 0.5 A, nmax 10, lmax 12 "
                    "(715 features); sparse polynomial model zeta 4 with 2000 active points; neighbours with "
                    "reverse-pair index + FP32 expansion and power spectrum + model energies and dE/dp + adjoint "
                    "(forces) + virial"}
    line = {
        "metric": "atom-centres/s (neighbours + " + {"clusters": "FP64 expansion + power spectrum)",
                                                    "molecules": "expansion + bf16 MFMA power spectrum)",
                                                    "liquid": "expansion + power spectrum + adjoint)",
                                                    "gpr": "expansion + power spectrum + sparse model energies, "
                                                           "forces and virial)"}[wl],
        "value": N / (ms_per_step * 1e-3), "unit": "atom-centres/s", "n_gpus": 1, "steps": K,
        "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if es == 8 else ("bf16" if wl == "molecules" else "f32"),
        "data": "synthetic",
        "config": {"workload": names[wl], "centres": N, "pairs": Pn, "phases_ms": ph_ms, "phases": rows},
        "roofline": roof,
    }
    return line


def run_config(args) -> int:
    line = measure_config(args.workload, args.steps, args.warmup)
    if line is None:
        return 4
    print(json.dumps(line), flush=True)
    return 0


def run_radial(args) -> int:
    """Cost of one radial-integral evaluation per radius (Sec. 4.D): the
    pair distances of the 4096-atom liquid (rcut 6 A, sigma 0.5 A, nmax 10,
    lmax 8, about 45 neighbours per atom) evaluated through
    soap_radial_integral from the FP32 and FP64 splines the kernels use and
    directly in FP64, for the orthogonalised GTO basis (restricted 1F1 and
    S^{-1/2}) and for the DVR basis (modified spherical Bessel functions).
    Values and derivatives are written, [nmax][lmax+1][n_r]."""
    import torch

    import synthetic
    import paper_2101_08814_amd as P

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    batch = synthetic.liquid_bulk()
    h = batch.hypers
    gto = P.Calculator.from_hypers(h)
    dvr = P.Calculator.from_hypers(dict(h, radial_basis=1))
    pos = torch.tensor(batch.positions, dtype=torch.float64, device=dev)
    spc = torch.tensor(batch.species, dtype=torch.int32, device=dev)
    ao, ce, pb = P.soap.structures_to_device(batch.atom_offsets, batch.cells, batch.pbc, dev)
    nl = gto.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=torch.float64, transpose=False)
    n_r = nl.count()
    r = nl.pair_vec[:n_r].norm(dim=1).contiguous()
    nlm = gto.nmax * (gto.lmax + 1)
    cases = [("spline_f32", gto, False, torch.float32), ("spline_f64", gto, False, torch.float64),
             ("direct_gto_f64", gto, True, torch.float64), ("direct_dvr_f64", dvr, True, torch.float64)]
    steps = max(1, min(args.steps, 50))
    ms = {}
    for name, calc, exact, dt in cases:
        def f():
            return calc.radial_integral(r, exact=exact, dtype=dt)
        for _ in range(max(2, min(args.warmup, 10))):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            f()
        e1.record()
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / steps
        if calc.device_status() != 0:
            log(f"device status {calc.device_status()} in {name}")
            return 4
    ns = {k: v * 1e6 / n_r for k, v in ms.items()}
    log("[bench:radial] n_r=%d " % n_r + " ".join(f"{k}={v:.3f} ms ({ns[k]:.3f} ns/radius)" for k, v in ms.items()))
    out_bytes = 2 * nlm * 4 * n_r + 8 * n_r
    gbs = out_bytes / (ms["spline_f32"] * 1e-3) / 1e9
    line = {
        "metric": "radii/s (FP32 spline, nmax x (lmax+1) values and derivatives per radius)",
        "value": n_r / (ms["spline_f32"] * 1e-3), "unit": "radii/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms["spline_f32"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "pair distances of the 4096-atom periodic liquid (0.05 atoms/A^3, rcut 6 A, "
                               "sigma 0.5 A, nmax 10, lmax 8)",
                   "radii": n_r, "ms": ms, "ns_per_radius": ns,
                   "direct_over_spline": {k: ms[k] / ms["spline_f64"] for k in ("direct_gto_f64", "direct_dvr_f64")}},
        "roofline": {"bound": "hbm", "kernel": "k_radial_spline<float, 8>", "achieved": gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel_ms": ms["spline_f32"],
                     "algorithmic_bytes_per_launch": out_bytes},
    }
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--graph", action="store_true", help="replay the phases as HIP graphs instead of "
                    "launching them eagerly (measured slower: each graph launch adds a gap)")
    ap.add_argument("--two-pass", action="store_true", help="per-centre pass and pair rows as two kernels "
                    "(soap_features without rows, then soap_gradient_rows) instead of the one fused kernel")
    ap.add_argument("--calibrate-copy", action="store_true", help="only copy 256 MiB device-to-device five times "
                    "(the reference kernel for scaling memory counters) and exit")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the sub-records of the clusters, molecules "
                    "and liquid workloads in the headline line")
    ap.add_argument("--config-steps", type=int, default=200, help="timed steps of each sub-record workload")
    ap.add_argument("--workload", choices=["diamond", "clusters", "molecules", "liquid", "gpr", "selected",
                                           "compression", "radial"],
                    default="diamond",
                    help="diamond: the headline step (default); clusters, molecules, liquid: the FP64, MFMA and "
                         "adjoint parity workloads as timed steps; compression: the learned channel compression "
                         "of the 8-species cells, trained and timed against the full power spectrum; radial: the cost per "
                         "radius of the splined and the directly evaluated radial integrals")
    ap.add_argument("--train-steps", type=int, default=600)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; sharding over several GPUs is not "
                                   "built", "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import synthetic
    import paper_2101_08814_amd as P

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.workload == "selected":
        return run_selected(args)
    if args.workload == "compression":
        return run_compression(args)
    if args.workload == "radial":
        return run_radial(args)
    if args.workload in ("clusters", "molecules", "liquid", "gpr"):
        return run_config(args)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[calibrate] copied {src.numel() * 4} bytes 5 times")
        return 0
    batch = synthetic.diamond_bulk()
    h = batch.hypers
    calc = P.Calculator.from_hypers(h)
    dev = torch.device("cuda", 0)
    pos = torch.tensor(batch.positions, dtype=torch.float64, device=dev)
    spc = torch.tensor(batch.species, dtype=torch.int32, device=dev)
    ao, ce, pb = P.soap.structures_to_device(batch.atom_offsets, batch.cells, batch.pbc, dev)
    # forward-mode rows need no reverse-pair index, so the step does not build it
    nl = calc.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=torch.float32, transpose=False)
    N, Pn = batch.n_atoms, nl.count()
    out = calc.allocate_features(N, nl.capacity, torch.float32, dev, True)
    calc.reset_status()

    def step_neighbors():
        calc.compute_neighbors(pos, spc, ao, ce, pb, vec_dtype=torch.float32, out=nl)

    def step_centres():
        calc.features(nl, spc, torch.float32, gradients=True, out=out, rows=not args.two_pass)

    def step_rows():
        calc.gradient_rows(nl, spc, out[0], dc=out[2], dp=out[4])

    steps = [step_neighbors, step_centres] + ([step_rows] if args.two_pass else [])
    # eager warm-up (also sets LDS attributes before any capture)
    for _ in range(3):
        for f in steps:
            f()
    torch.cuda.synchronize()
    ref = [t.clone() for t in out]
    if args.graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for f in steps:
                f()
        torch.cuda.current_stream().wait_stream(side)
        graphs = [torch.cuda.CUDAGraph() for _ in steps]
        for g, f in zip(graphs, steps):
            with torch.cuda.graph(g):
                f()
        runs = [g.replay for g in graphs]
    else:
        runs = steps
    n_ph = len(runs)

    # the replayed (or launched) results against the eager ones, before the
    # warm-up, so that the timed steps follow the warm-up directly
    for f in runs:
        f()
    torch.cuda.synchronize()
    for a, b in zip(out, ref):
        if not torch.equal(a, b):
            log("graph replay differs from the eager result")
            return 3

    K = args.steps
    # ev[k][j] is recorded after phase j of step k (same stream as the kernels)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(n_ph)] for _ in range(K)]
    start_all = torch.cuda.Event(enable_timing=True)
    end_all = torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup):
        for f in runs:
            f()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start_all.record()
    for k in range(K):
        for j, f in enumerate(runs):
            f()
            ev[k][j].record()
    end_all.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start_all.elapsed_time(end_all)
    centres_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    rows_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev])) if args.two_pass else 0.0
    status = calc.device_status()
    if status != 0:
        log(f"device status {status}")
        return 4
    for a, b in zip(out, ref):
        if not torch.equal(a, b):
            log("timed results differ from the eager result")
            return 5

    ms_per_step = total_ms / K
    value = N / (ms_per_step * 1e-3)
    alg_centres, alg_rows, alg_fused = algorithmic_bytes(N, Pn, h["n_species"], h["nmax"], h["lmax"])
    if args.two_pass:
        kernel, alg, kernel_ms = TWO_PASS_KERNEL, alg_rows, rows_ms
        log(f"[bench] two-pass N={N} P={Pn} steps={K} total={total_ms:.2f} ms (host wall {wall * 1e3:.1f} ms) "
            f"step={ms_per_step * 1e3:.1f} us  centres={centres_ms * 1e3:.1f} us "
            f"({alg_centres / (centres_ms * 1e-3) / 1e9:.0f} GB/s)  rows={rows_ms * 1e3:.1f} us "
            f"({alg_rows / (rows_ms * 1e-3) / 1e9:.0f} GB/s)  "
            f"neighbours+gaps={(ms_per_step - rows_ms - centres_ms) * 1e3:.1f} us")
    else:
        kernel, alg, kernel_ms = DOMINANT_KERNEL, alg_fused, centres_ms
        log(f"[bench] N={N} P={Pn} steps={K} total={total_ms:.2f} ms (host wall {wall * 1e3:.1f} ms) "
            f"step={ms_per_step * 1e3:.1f} us  features={centres_ms * 1e3:.1f} us "
            f"({alg_fused / (centres_ms * 1e-3) / 1e9:.0f} GB/s)  "
            f"neighbours+gaps={(ms_per_step - centres_ms) * 1e3:.1f} us  bytes/launch={alg_fused / 1e6:.1f} MB")
    achieved = alg / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(alg) if not args.two_pass else None

    line = {
        "metric": "atom-centres/s (expansion+power spectrum+grads) at stated error vs FP64 oracle",
        "value": value,
        "unit": "atom-centres/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "two_pass": bool(args.two_pass),
            "workload": "periodic perturbed diamond, 1024 atoms (4x4x8 cells, a=5.43 A, 0.1 A displacements), "
                        "1 species, rcut 5 A, sigma 0.5 A, nmax 8, lmax 6; neighbour list with images + FP32 "
                        "expansion + power spectrum + forward-mode position gradients",
            "centres": N, "pairs": Pn, "n_species": h["n_species"], "nmax": h["nmax"], "lmax": h["lmax"],
            "rcut": h["rcut"], "sigma": h["sigma"], "graphs": bool(args.graph),
            "parity": "FP32 vs FP64 oracle: p <= 1e-6, gradient rows <= 1e-5 relative (tests/test_gpu_parity.py)",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel_ms": kernel_ms,
            "algorithmic_bytes_per_launch": alg,
        },
    }
    if not args.no_configs:
        # the other single-GPU parity workloads as sub-records: each its own
        # timed steps (neighbours included) and its dominant kernel against
        # its roofline
        subs = {}
        for wl in ("clusters", "molecules", "liquid"):
            sub = measure_config(wl, args.config_steps, 5)
            if sub is None:
                return 4
            subs[wl] = {"workload": sub["config"]["workload"], "metric": sub["metric"], "value": sub["value"],
                        "unit": sub["unit"], "dtype": sub["dtype"], "steps": sub["steps"],
                        "ms_per_step": sub["ms_per_step"], "centres": sub["config"]["centres"],
                        "pairs": sub["config"]["pairs"], "phases_ms": sub["config"]["phases_ms"],
                        "roofline": sub["roofline"]}
        line["configs"] = subs
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(batch, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
