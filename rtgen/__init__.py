"""Seeded synthetic inputs for the M1 radiative-transfer subcycle: jittered
periodic lattice meshes in Peano-Hilbert (or random) order, lognormal density
fields, density-peak point sources with power-law rates and per-bin
cross-sections.  Holds no step of the method itself."""
from .configs import (CHEM_H, CHEM_HHE, CHEM_NONE, RATES_CASEB_CONST, RATES_HG97, adjoint_262k,
                      by_name, cosmological, default_params, degree_sorted, expanding_hii, face_counts, hhe_2m,
                      neutral_state, random_order, reorder, reorder_cells, stromgren, throughput_16m,
                      travelling_wave)
from .hilbert import bits_for, hilbert_key
from .mesh import Mesh, jittered_lattice, split_faces, staggered_bcc

__all__ = ["CHEM_H", "CHEM_HHE", "CHEM_NONE", "RATES_CASEB_CONST", "RATES_HG97", "Mesh",
           "adjoint_262k", "bits_for", "by_name", "cosmological", "default_params", "degree_sorted",
           "expanding_hii", "face_counts", "hhe_2m", "hilbert_key", "jittered_lattice", "neutral_state",
           "random_order", "reorder", "reorder_cells", "split_faces", "staggered_bcc", "stromgren",
           "throughput_16m", "travelling_wave"]
