"""Single cells of a large lattice run, recomputed by the oracle on a small
patch (test infrastructure).

One subcycle of a cell depends on its own state and that of the cells within
two faces of it: its face states need its neighbours' limited gradients, and
those need the neighbours' neighbours (the limiter's extrema too).  On a
jittered lattice that cone lies inside the 5x5x5 block of lattice sites
centred on the cell, and the cone of k subcycles inside the block of
half-width w = 2k.  The patch is that block as a periodic mesh of its own:
its interior faces are the lattice's faces (translated), and the faces that
leave the block close it onto the opposite side.  Only the block's outer
layer gets wrong neighbours.  After the first subcycle the wrong values
reach one layer in (the faces that use an outer cell's gradient), and every
later subcycle takes them two layers further, so after k subcycles on the
block of half-width 2k they stop one layer short of the centre: the
oracle's k subcycles on the patch give the centre cell's exact result on
the whole mesh (to rounding order).  The block must not wrap onto itself,
so its edge is at most the lattice's.
"""
from __future__ import annotations

import numpy as np

W = 2                     # cells from the centre to the block's edge, one subcycle


def edge(w: int) -> int:
    return 2 * w + 1


def centre_index(w: int) -> int:
    """Local index of the centre (x fastest) of the block of half-width w."""
    p = edge(w)
    return w + p * (w + p * w)


class LatticeIndex:
    """Lattice site of every cell of a jittered lattice mesh (jitter below
    half a spacing), and the cell at every site."""

    def __init__(self, mesh: dict):
        self.h = float(np.cbrt(mesh["volume"][0]))
        self.dims = np.rint(np.asarray(mesh["box"], float) / self.h).astype(np.int64)
        self.idx = np.floor(np.asarray(mesh["centre"]) / self.h).astype(np.int64)
        nx, ny, _ = self.dims
        lex = self.idx[0] + nx * (self.idx[1] + ny * self.idx[2])
        self.cell_at = np.empty(lex.size, np.int64)
        self.cell_at[lex] = np.arange(lex.size)

    def block(self, c: int, w: int = W) -> np.ndarray:
        """Cells of the (2w+1)^3 block centred on cell c, in local order (x fastest)."""
        if edge(w) > self.dims.min():
            raise ValueError(f"block of edge {edge(w)} wraps on a lattice of {self.dims.tolist()}")
        a = np.arange(edge(w)) - w
        lx, ly, lz = np.meshgrid(a, a, a, indexing="ij")
        lx, ly, lz = (v.transpose(2, 1, 0).ravel() for v in (lx, ly, lz))   # x fastest
        g = (self.idx[:, c][:, None] + np.stack([lx, ly, lz])) % self.dims[:, None]
        nx, ny, _ = self.dims
        return self.cell_at[g[0] + nx * (g[1] + ny * g[2])]


def patch_config(cfg: dict, fields: dict, lat: LatticeIndex, c: int, n_sub: int = 1) -> dict:
    """The oracle's config of the periodic block around cell c of half-width
    2 n_sub, with the state `fields` (N, F, species, T, n_H of the whole mesh)
    and the sources inside the block, for n_sub subcycles."""
    m = cfg["mesh"]
    h = lat.h
    w = 2 * n_sub
    P = edge(w)
    cells = lat.block(c, w)
    n = cells.size
    loc = np.arange(n)
    l = np.stack([loc % P, (loc // P) % P, loc // (P * P)])          # local lattice coords
    site = lat.idx[:, cells]
    centre = l * h + (np.asarray(m["centre"])[:, cells] - site * h)  # jitter kept
    face_cells = np.empty((2, 3 * n), np.int64)
    normal = np.zeros((3, 3 * n))
    face_centre = np.empty((3, 3 * n))
    for k in range(3):
        nb = l.copy()
        nb[k] = (nb[k] + 1) % P
        sl = slice(k, 3 * n, 3)
        face_cells[0, sl] = loc
        face_cells[1, sl] = nb[0] + P * (nb[1] + P * nb[2])
        normal[k, sl] = 1.0
        fc = (l + 0.5) * h
        fc[k] = (l[k] + 1.0) * h
        face_centre[:, sl] = fc
    mesh = dict(n_cells=n, volume=np.asarray(m["volume"])[cells].copy(), centre=np.ascontiguousarray(centre),
                n_faces=3 * n, face_cells=face_cells, area=np.full(3 * n, h * h), normal=normal,
                face_centre=face_centre, box=np.full(3, P * h))
    state = dict(N=np.ascontiguousarray(fields["N"][:, cells]), F=np.ascontiguousarray(fields["F"][:, :, cells]),
                 n_H=np.ascontiguousarray(fields["n_H"][cells]),
                 species=np.ascontiguousarray(fields["species"][:, cells]),
                 T=np.ascontiguousarray(fields["T"][cells]))
    src_cell = np.asarray(cfg["sources"]["cell"], np.int64)
    rate = np.asarray(cfg["sources"]["rate"], float).reshape(cfg["params"]["nb"], -1)
    where = {int(g): j for j, g in enumerate(cells)}
    keep = [k for k in range(src_cell.size) if int(src_cell[k]) in where]
    sources = dict(cell=np.array([where[int(src_cell[k])] for k in keep], np.int64),
                   rate=np.ascontiguousarray(rate[:, keep]))
    return dict(name="patch", mesh=mesh, params=cfg["params"], state=state, sources=sources, n_subcycles=n_sub,
                precision="fp64")


def centre_values(st: dict, n_sub: int = 1) -> dict:
    """The centre cell's fields from an oracle result on a patch of n_sub
    subcycles."""
    k = centre_index(2 * n_sub)
    return dict(N=st["N"][:, k], F=st["F"][:, :, k], species=st["species"][:, k], T=st["T"][k])


def sample_cells(fields: dict, n_lit: int, n_any: int, seed: int, src_cells) -> np.ndarray:
    """Seeded sample: n_lit cells where bin 0's N is at least 1e-8 of its
    maximum (lit gas and fronts), n_any cells from the whole mesh, and the
    source cells among them first."""
    rng = np.random.default_rng(seed)
    N0 = fields["N"][0]
    lit = np.nonzero(N0 >= 1e-8 * N0.max())[0]
    pick = list(np.asarray(src_cells, np.int64)[:4])
    pick += list(rng.choice(lit, size=min(n_lit, lit.size), replace=False))
    pick += list(rng.choice(N0.size, size=n_any, replace=False))
    return np.unique(np.array(pick, np.int64))
