"""Seeded synthetic atomic structures.

This module only places atoms, assigns species and builds cells.  It holds
none of the representation's arithmetic, so both the FP64 oracle and the GPU
library may be fed from it.

A batch of structures is a ``Batch``:

* ``positions``    float64 [N, 3]   Cartesian, Angstrom
* ``species``      int32   [N]      species index in [0, n_species)
* ``atom_offsets`` int64   [n_struct + 1]  atoms of structure s are
  ``atom_offsets[s] : atom_offsets[s + 1]``
* ``cells``        float64 [n_struct, 3, 3]  rows are the lattice vectors
  h1, h2, h3 (zeros for a non-periodic structure)
* ``pbc``          uint8   [n_struct, 3]  periodicity per lattice vector

The paper benchmarks on datasets (bulk Si, methane, molecular crystals,
QM9) that are not available here; the five workloads below are synthetic
stand-ins with their densities, species mixes and neighbour counts.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Batch:
    positions: np.ndarray
    species: np.ndarray
    atom_offsets: np.ndarray
    cells: np.ndarray
    pbc: np.ndarray
    hypers: Dict
    name: str = ""

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])

    @property
    def n_structures(self) -> int:
        return int(self.atom_offsets.shape[0] - 1)

    def subset(self, structures: List[int]) -> "Batch":
        """The batch restricted to the listed structures (renumbered)."""
        pos, spc, cells, pbc, offs = [], [], [], [], [0]
        for s in structures:
            a, b = int(self.atom_offsets[s]), int(self.atom_offsets[s + 1])
            pos.append(self.positions[a:b])
            spc.append(self.species[a:b])
            cells.append(self.cells[s])
            pbc.append(self.pbc[s])
            offs.append(offs[-1] + b - a)
        return Batch(np.ascontiguousarray(np.concatenate(pos)),
                     np.ascontiguousarray(np.concatenate(spc)).astype(np.int32),
                     np.asarray(offs, dtype=np.int64),
                     np.ascontiguousarray(np.stack(cells)),
                     np.ascontiguousarray(np.stack(pbc)).astype(np.uint8),
                     dict(self.hypers), self.name + f"[{len(structures)} structures]")


def _exact_species(rng, n, counts):
    s = np.concatenate([np.full(c, a, dtype=np.int32) for a, c in enumerate(counts)])
    assert s.shape[0] == n
    rng.shuffle(s)
    return s


def _rsa(rng, n, side, min_sep, periodic, max_tries=1_000_000):
    """Random sequential addition in a cube of edge ``side``: a uniform
    candidate is rejected when it lies closer than ``min_sep`` (minimum image
    when ``periodic``) to an atom already placed."""
    pts = np.empty((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        cand = rng.uniform(0.0, side, size=3)
        if k:
            d = pts[:k] - cand
            if periodic:
                d -= side * np.round(d / side)
            if np.min(np.einsum("ij,ij->i", d, d)) < min_sep * min_sep:
                continue
        pts[k] = cand
        k += 1
    return pts


def _pack(structs, hypers, name):
    pos = np.concatenate([s[0] for s in structs])
    spc = np.concatenate([s[1] for s in structs]).astype(np.int32)
    cells = np.stack([s[2] for s in structs]).astype(np.float64)
    pbc = np.stack([s[3] for s in structs]).astype(np.uint8)
    offs = np.zeros(len(structs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([s[0].shape[0] for s in structs])
    return Batch(np.ascontiguousarray(pos), np.ascontiguousarray(spc), offs,
                 np.ascontiguousarray(cells), np.ascontiguousarray(pbc), hypers, name)


def _hypers(n_species, rcut, sigma, nmax, lmax, width=0.5, include_center=1):
    return dict(n_species=n_species, nmax=nmax, lmax=lmax, rcut=rcut,
                cutoff_width=width, sigma=sigma, include_center=include_center,
                spline_accuracy=1e-8)


def clusters_2species(seed: int = 1001, n_clusters: int = 8, n_atoms: int = 64) -> Batch:
    """8 non-periodic clusters of 64 atoms, 2 species (exactly 50/50), uniform
    in a cube at 0.1 atoms/A^3, 0.8 A minimum separation; rcut 4 A, cutoff
    width 0.5 A, sigma 0.5 A, nmax 6, lmax 4."""
    rng = np.random.default_rng(seed)
    side = (n_atoms / 0.1) ** (1.0 / 3.0)
    structs = []
    for _ in range(n_clusters):
        p = _rsa(rng, n_atoms, side, 0.8, periodic=False)
        s = _exact_species(rng, n_atoms, [n_atoms // 2, n_atoms - n_atoms // 2])
        structs.append((p, s, np.zeros((3, 3)), np.zeros(3, dtype=np.uint8)))
    return _pack(structs, _hypers(2, 4.0, 0.5, 6, 4), "clusters 8x64, 2 species")


def diamond_bulk(seed: int = 1002, reps=(4, 4, 8), a: float = 5.43, disp: float = 0.1) -> Batch:
    """Periodic perturbed diamond lattice: 4x4x8 conventional cells of edge
    5.43 A (1024 atoms), Gaussian displacements of 0.1 A per coordinate,
    wrapped into the cell; 1 species; rcut 5 A, sigma 0.5 A, nmax 8, lmax 6."""
    rng = np.random.default_rng(seed)
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
                      [.25, .25, .25], [.25, .75, .75], [.75, .25, .75], [.75, .75, .25]])
    grid = np.stack(np.meshgrid(*[np.arange(r) for r in reps], indexing="ij"), -1).reshape(-1, 3)
    frac = (grid[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    pos = frac * a + rng.normal(0.0, disp, size=frac.shape)
    cell = np.diag(np.asarray(reps, dtype=np.float64) * a)
    lengths = np.diag(cell)
    pos = pos - lengths * np.floor(pos / lengths)
    spc = np.zeros(pos.shape[0], dtype=np.int32)
    return _pack([(pos, spc, cell, np.ones(3, dtype=np.uint8))],
                 _hypers(1, 5.0, 0.5, 8, 6), f"diamond bulk {pos.shape[0]} atoms")


def molecule_batch(seed: int = 1003, n_structures: int = 256, lo: int = 20, hi: int = 200) -> Batch:
    """256 non-periodic molecule-like clusters of 20-200 atoms (uniform),
    4 species drawn i.i.d. with fractions 0.5/0.3/0.1/0.1, 0.08 atoms/A^3,
    0.9 A minimum separation; rcut 5 A, sigma 0.4 A, nmax 8, lmax 6."""
    rng = np.random.default_rng(seed)
    structs = []
    for _ in range(n_structures):
        n = int(rng.integers(lo, hi + 1))
        side = (n / 0.08) ** (1.0 / 3.0)
        p = _rsa(rng, n, side, 0.9, periodic=False)
        s = rng.choice(4, size=n, p=[0.5, 0.3, 0.1, 0.1]).astype(np.int32)
        structs.append((p, s, np.zeros((3, 3)), np.zeros(3, dtype=np.uint8)))
    return _pack(structs, _hypers(4, 5.0, 0.4, 8, 6), f"{n_structures} molecules 20-200 atoms, 4 species")


def liquid_bulk(seed: int = 1004, n_atoms: int = 4096) -> Batch:
    """Periodic liquid-like cube at 0.05 atoms/A^3 (edge 43.44 A for 4096
    atoms), 1.8 A minimum separation, 2 species exactly 70/30; rcut 6 A,
    sigma 0.5 A, nmax 10, lmax 8."""
    rng = np.random.default_rng(seed)
    side = (n_atoms / 0.05) ** (1.0 / 3.0)
    p = _rsa(rng, n_atoms, side, 1.8, periodic=True)
    n0 = int(0.7 * n_atoms)
    s = _exact_species(rng, n_atoms, [n0, n_atoms - n0])
    return _pack([(p, s, np.eye(3) * side, np.ones(3, dtype=np.uint8))],
                 _hypers(2, 6.0, 0.5, 10, 8), f"liquid bulk {n_atoms} atoms, 2 species")


def multi_species_cells(seed: int = 1005, n_cells: int = 512, n_atoms: int = 256) -> Batch:
    """512 periodic cubic cells of 256 atoms at 0.06 atoms/A^3 (edge 16.22 A),
    8 species with 32 atoms each, 0.8 A minimum separation; rcut 5 A,
    sigma 0.5 A, nmax 12, lmax 8."""
    rng = np.random.default_rng(seed)
    side = (n_atoms / 0.06) ** (1.0 / 3.0)
    structs = []
    for _ in range(n_cells):
        p = _rsa(rng, n_atoms, side, 0.8, periodic=True)
        s = _exact_species(rng, n_atoms, [n_atoms // 8] * 8)
        structs.append((p, s, np.eye(3) * side, np.ones(3, dtype=np.uint8)))
    return _pack(structs, _hypers(8, 5.0, 0.5, 12, 8), f"{n_cells} cells x {n_atoms} atoms, 8 species")


WORKLOADS = {
    "clusters": clusters_2species,
    "diamond": diamond_bulk,
    "molecules": molecule_batch,
    "liquid": liquid_bulk,
    "multispecies": multi_species_cells,
}


def random_cell_structure(seed: int, n_atoms: int, cell: np.ndarray, n_species: int,
                          min_sep: float = 0.7, pbc=(1, 1, 1), hypers: Optional[Dict] = None) -> Batch:
    """A small structure with atoms uniform in an arbitrary (possibly
    triclinic) cell, for edge-case tests.  Positions are drawn in fractional
    coordinates and a candidate closer than ``min_sep`` to any periodic image
    of a placed atom is rejected."""
    rng = np.random.default_rng(seed)
    cell = np.asarray(cell, dtype=np.float64)
    pts = []
    tries = 0
    shifts = np.stack(np.meshgrid(*[np.arange(-1, 2)] * 3, indexing="ij"), -1).reshape(-1, 3)
    while len(pts) < n_atoms:
        tries += 1
        if tries > 100000:
            raise RuntimeError("placement failed")
        f = rng.uniform(0, 1, size=3)
        c = f @ cell
        ok = True
        for q in pts:
            d = (q - c)[None, :] + shifts @ cell
            if np.min(np.linalg.norm(d, axis=1)) < min_sep:
                ok = False
                break
        if ok:
            pts.append(c)
    pos = np.asarray(pts)
    spc = rng.integers(0, n_species, size=n_atoms).astype(np.int32)
    if hypers is None:
        hypers = _hypers(n_species, 4.0, 0.5, 4, 3)
    return _pack([(pos, spc, cell, np.asarray(pbc, dtype=np.uint8))], hypers, "random cell")
