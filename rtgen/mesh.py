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


def staggered_bcc(n: int, a: float, jitter: float, seed: int, order: str = "hilbert") -> Mesh:
    """The paper's "staggered" 2 n^3 grid (Sections 3.1, 4.2.2): points of a
    periodic body-centred cubic lattice with cube edge a, i.e. a corner point
    (i, j, k) a and a body-centre point (i+1/2, j+1/2, k+1/2) a per cube.  Its
    Voronoi cells are truncated octahedra of volume a^3/2 with 14 faces: 8
    regular hexagons (area 3 sqrt(3) a^2 / 16) towards the nearest points
    along the cube diagonals, and 6 squares (area a^2 / 8) towards the next
    nearest points along the axes.  Faces are those of the unjittered lattice
    (centre at the midpoint of the two points, normal along their
    separation); the generating points are jittered by at most jitter*a per
    axis.  Cells are ordered along the Hilbert curve of the doubled lattice."""
    nn = n
    nc = 2 * nn ** 3
    t = np.repeat([0, 1], nn ** 3)                     # sublattice: 0 corner, 1 body centre
    lex = np.tile(np.arange(nn ** 3), 2)
    ix, iy, iz = lex % nn, (lex // nn) % nn, lex // (nn * nn)
    d2 = np.stack([2 * ix + t, 2 * iy + t, 2 * iz + t])   # doubled-lattice coordinates
    if order == "hilbert":
        key = hilbert_key(d2[0], d2[1], d2[2], bits_for(2 * nn))
        site_of_cell = np.argsort(key, kind="stable")
    elif order == "random":
        site_of_cell = np.random.default_rng(4000).permutation(nc)
    else:
        site_of_cell = np.arange(nc)
    cell_of_site = np.empty(nc, dtype=np.int64)
    cell_of_site[site_of_cell] = np.arange(nc)

    def site(tt, i, j, k):
        return tt * nn ** 3 + (i % nn) + nn * ((j % nn) + nn * (k % nn))

    pos0 = d2 * (0.5 * a)                               # unjittered positions, sites order
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-jitter, jitter, size=(3, nc)) * a
    centre = (pos0 + 0.5 * a + jit)[:, site_of_cell]    # +a/2 keeps corner points off the box edge

    L_sites, R_sites, kinds = [], [], []
    corner = np.arange(nn ** 3)
    ci, cj, ck = corner % nn, (corner // nn) % nn, corner // (nn * nn)
    # squares: every site to its +x, +y, +z neighbour on the same sublattice
    for tt in (0, 1):
        s0 = tt * nn ** 3 + corner
        for k, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            L_sites.append(s0)
            R_sites.append(site(tt, ci + di, cj + dj, ck + dk))
            kinds.append(np.full(nn ** 3, k))
    # hexagons: every corner to its 8 surrounding body centres
    for di in (0, -1):
        for dj in (0, -1):
            for dk in (0, -1):
                L_sites.append(corner)
                R_sites.append(site(1, ci + di, cj + dj, ck + dk))
                kinds.append(np.full(nn ** 3, 3))
    Ls = np.concatenate(L_sites)
    Rs = np.concatenate(R_sites)
    kind = np.concatenate(kinds)
    box = np.full(3, nn * a)
    sep = pos0[:, Rs] - pos0[:, Ls]
    sep -= box[:, None] * np.round(sep / box[:, None])
    dist = np.linalg.norm(sep, axis=0)
    normal = sep / dist
    fc = pos0[:, Ls] + 0.5 * a + 0.5 * sep
    area = np.where(kind == 3, 3 * np.sqrt(3.0) * a * a / 16, a * a / 8)
    # faces grouped by their L cell in cell order, then in generation order
    Lc, Rc = cell_of_site[Ls], cell_of_site[Rs]
    fo = np.lexsort((np.arange(Lc.size), Lc))
    face_cells = np.stack([Lc[fo], Rc[fo]])
    idx = np.stack([ix, iy, iz])[:, site_of_cell]
    return Mesh(nc, np.full(nc, 0.5 * a ** 3), np.ascontiguousarray(centre), int(Lc.size), face_cells,
                np.ascontiguousarray(area[fo]), np.ascontiguousarray(normal[:, fo]),
                np.ascontiguousarray(fc[:, fo]), box, idx, (nn, nn, nn), float(a))


def split_faces(mesh: Mesh, fraction: float, seed: int) -> Mesh:
    """A mesh with variable face counts: a seeded share of the faces of
    ``mesh`` is split into two faces of half the area, joining the same two
    cells with the same normal, centred a quarter of the spacing either side
    of the original centre along the next axis of the face's plane.  Each
    cell keeps sum A n = 0 and its geometry matrix; a cell gets one more face
    for each of its split faces (degrees 6 to 12 on a lattice).  Faces stay
    grouped by their L cell, the halves in place of the face they replace."""
    nf = mesh.n_faces
    rng = np.random.default_rng(seed)
    split = rng.random(nf) < fraction
    reps = np.where(split, 2, 1)
    src = np.repeat(np.arange(nf), reps)                   # original face of each new face
    first = np.concatenate([[True], src[1:] != src[:-1]])  # first (or only) face of its group
    half = split[src]
    sign = np.where(half, np.where(first, -1.0, 1.0), 0.0)
    n = mesh.normal[:, src]
    k = np.argmax(np.abs(n), axis=0)                       # axis of the normal
    t = np.zeros_like(n)
    t[(k + 1) % 3, np.arange(src.size)] = 1.0              # an axis of the face's plane
    fc = mesh.face_centre[:, src] + sign[None, :] * 0.25 * mesh.h * t
    area = mesh.area[src] * np.where(half, 0.5, 1.0)
    return Mesh(mesh.n_cells, mesh.volume, mesh.centre, int(src.size),
                np.ascontiguousarray(mesh.face_cells[:, src]), np.ascontiguousarray(area),
                np.ascontiguousarray(n), np.ascontiguousarray(fc), mesh.box, mesh.lattice_index, mesh.dims,
                mesh.h)
