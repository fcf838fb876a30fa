"""Seeded synthetic inputs shared by the oracle tests and the GPU library tests."""
from .structures import (Batch, WORKLOADS, clusters_2species, diamond_bulk, molecule_batch,
                         liquid_bulk, multi_species_cells, random_cell_structure)
