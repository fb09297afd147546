"""Jittered periodic lattice meshes in the library's mesh format.

The mesh is the one the synthetic workloads use: cells of a regular
Cartesian lattice with spacing h, each cell's centre displaced by a seeded
uniform jitter of at most ``jitter*h`` per axis, and the faces of the
unjittered lattice (area h^2, normal +e_k pointing from the left cell to its
+k neighbour, centre at the lattice face midpoint).  This is the paper's
"irregular mesh" of the travelling-wave test (Section 4.2.1): a Cartesian grid
whose generating points deviate from the cell centroids.

Cell order is chosen here, never by the library: ``order="hilbert"`` sorts
cells along the Peano-Hilbert curve of their lattice index, ``"random"`` is a
seeded permutation, ``"lattice"`` is x-fastest lexicographic order.  Faces are
listed by their left cell (in cell order), then axis x, y, z.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .hilbert import bits_for, hilbert_key


@dataclass
class Mesh:
    n_cells: int
    volume: np.ndarray        # [nc]
    centre: np.ndarray        # [3][nc]
    n_faces: int
    face_cells: np.ndarray    # [2][nf] int64, (L, R)
    area: np.ndarray          # [nf]
    normal: np.ndarray        # [3][nf], unit, L -> R
    face_centre: np.ndarray   # [3][nf]
    box: np.ndarray           # [3] periodic lengths
    lattice_index: np.ndarray  # [3][nc] int64 (ix, iy, iz) of each cell
    dims: tuple               # (nx, ny, nz)
    h: float

    def as_dict(self) -> dict:
        return dict(n_cells=self.n_cells, volume=self.volume, centre=self.centre,
                    n_faces=self.n_faces, face_cells=self.face_cells, area=self.area,
                    normal=self.normal, face_centre=self.face_centre, box=self.box)


def lattice_order(dims, order: str, seed: int | None = None) -> np.ndarray:
    """Return lexicographic lattice ids (x fastest) in the requested cell order."""
    nx, ny, nz = dims
    lex = np.arange(nx * ny * nz, dtype=np.int64)
    ix = lex % nx
    iy = (lex // nx) % ny
    iz = lex // (nx * ny)
    if order == "lattice":
        return lex
    if order == "hilbert":
        key = hilbert_key(ix, iy, iz, bits_for(max(dims)))
        return lex[np.argsort(key, kind="stable")]
    if order == "random":
        rng = np.random.default_rng(seed)
        return rng.permutation(lex)
    raise ValueError(f"unknown order {order!r}")


def jittered_lattice(dims, h: float, jitter: float, seed: int, order: str = "hilbert",
                     perm_seed: int = 4000) -> Mesh:
    nx, ny, nz = (int(d) for d in dims)
    nc = nx * ny * nz
    lex_of_cell = lattice_order((nx, ny, nz), order, perm_seed)   # cell -> lex id
    cell_of_lex = np.empty(nc, dtype=np.int64)
    cell_of_lex[lex_of_cell] = np.arange(nc, dtype=np.int64)

    ix = lex_of_cell % nx
    iy = (lex_of_cell // nx) % ny
    iz = lex_of_cell // (nx * ny)
    idx = np.stack([ix, iy, iz])

    # Jitter is drawn per lattice site (lexicographic), so a reordering of the
    # same lattice moves no point.
    rng = np.random.default_rng(seed)
    jit_lex = rng.uniform(-jitter, jitter, size=(3, nc)) * h
    centre = (idx + 0.5) * h + jit_lex[:, lex_of_cell]

    volume = np.full(nc, h ** 3)

    dims_arr = np.array([nx, ny, nz])
    face_cells = np.empty((2, 3 * nc), dtype=np.int64)
    normal = np.zeros((3, 3 * nc))
    face_centre = np.empty((3, 3 * nc))
    for k in range(3):
        nb_idx = idx.copy()
        nb_idx[k] = (nb_idx[k] + 1) % dims_arr[k]
        nb_lex = nb_idx[0] + nx * (nb_idx[1] + ny * nb_idx[2])
        sl = slice(k, 3 * nc, 3)
        face_cells[0, sl] = np.arange(nc)
        face_cells[1, sl] = cell_of_lex[nb_lex]
        normal[k, sl] = 1.0
        fc = (idx + 0.5) * h
        fc[k] = (idx[k] + 1.0) * h
        face_centre[:, sl] = fc
    area = np.full(3 * nc, h * h)
    box = dims_arr.astype(np.float64) * h
    return Mesh(nc, volume, np.ascontiguousarray(centre), 3 * nc, face_cells, area,
                normal, face_centre, box, idx, (nx, ny, nz), float(h))
