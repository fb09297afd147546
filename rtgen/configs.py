"""The synthetic workloads the radiative-transfer subcycle is tested and
measured on, built deterministically from seeds.

Each builder returns a plain dict::

    {"name", "mesh": {...}, "params": {...}, "state": {...},
     "sources": {"cell", "rate"}, "n_subcycles", "precision", "meta": {...}}

with numpy arrays in the library's layouts (SoA, cgs units, caller's cell
order).  ``params`` holds every constant the paper leaves open; the names
mirror the library's parameter struct.

Workloads (paper Sections 3.1, 4.2; sizes per the workload definitions):

* ``stromgren``  - 32^3 jittered lattice, 16 kpc box, uniform n_H = 1e-3,
  isothermal 1e4 K hydrogen, one bin, one 5e48 s^-1 source in lattice cell
  (16,16,16), reduced light speed 0.01c, 100 subcycles, FP64.
* ``hhe_2m``      - 128^3 (2.1M cells), 1 kpc spacing, lognormal density
  (sigma_ln = 1.0, mean 2e-4), H+He with evolving temperature from 100 K,
  three bins, 256 power-law sources at density peaks, 0.01c, 50 subcycles.
* ``stromgren_mixed`` / ``stromgren_hhe_mixed`` - the Stromgren workload in
  mixed precision, H-only (as above) and with 3-bin H+He physics, 50 subcycles.
* ``throughput_16m`` - 256^3 (16.8M cells), sigma_ln = 1.5, 4096 sources,
  0.1c, 200 subcycles, Hilbert or random cell order, mixed or FP64.
* ``adjoint_262k`` - 64^3, sigma_ln = 1.0, 64 sources, 0.01c, 50 FP64
  subcycles, checkpoints every 10.
* ``travelling_wave`` - the paper's optically thin periodic travelling wave
  (Section 4.2.1): unit box, c = 1, E = 1 + 1e-6 sin(2 pi (x+y+z)),
  F parallel to (1,1,1) with |F| = cE, 10% jitter, transport only.
"""
from __future__ import annotations

import numpy as np

from . import fields
from .fields import C_LIGHT, KPC
from .hilbert import bits_for, hilbert_key
from .mesh import jittered_lattice, split_faces, staggered_bcc

CHEM_NONE, CHEM_H, CHEM_HHE = 0, 1, 2
RATES_CASEB_CONST, RATES_HG97 = 0, 1

Y_HE = 0.24
BIN_EDGES_EV = (13.6, 24.6, 54.4)
BIN_SPLIT = (1.0, 0.05, 0.03)     # photons per bin relative to the H-ionising bin
T_BLACKBODY = 5.0e4


def default_params(nb: int) -> dict:
    return dict(
        nb=nb, chem_mode=CHEM_H, isothermal=1, rate_set=RATES_CASEB_CONST,
        use_limiter=1, chem_max_substeps=100000,
        c_reduced=0.01 * C_LIGHT, cfl_eta=0.3, T_iso=1.0e4, Y_He=0.0,
        alpha_B_const=2.59e-13, gamma=5.0 / 3.0,
        chem_fmax=0.1, chem_fs=0.05, chem_growth=2.0, chem_xfloor=1.0e-6,
        sigma=np.zeros((nb, 3)), e_heat=np.zeros((nb, 3)),
    )


def neutral_state(nb: int, nc: int, n_h, t0) -> dict:
    species = np.zeros((5, nc))
    species[0] = 1.0   # x_HI
    species[2] = 1.0   # y_HeI
    return dict(N=np.zeros((nb, nc)), F=np.zeros((nb, 3, nc)),
                n_H=np.broadcast_to(np.asarray(n_h, dtype=float), (nc,)).copy(),
                species=species, T=np.full(nc, float(t0)))


def _lex_ids(mesh):
    nx, ny, _ = mesh.dims
    ix, iy, iz = mesh.lattice_index
    return ix + nx * (iy + ny * iz)


def _pack(name, mesh, params, state, src_cell, src_rate, n_sub, precision, **meta):
    return dict(name=name, mesh=mesh.as_dict(), params=params, state=state,
                sources=dict(cell=np.asarray(src_cell, dtype=np.int64),
                             rate=np.ascontiguousarray(src_rate, dtype=np.float64)),
                n_subcycles=int(n_sub), precision=precision,
                meta=dict(dims=mesh.dims, h=mesh.h, lattice_index=mesh.lattice_index, **meta))


def stromgren(n: int = 32, n_sub: int = 100, precision: str = "fp64", hhe: bool = False,
              order: str = "hilbert", seed_offset: int = 1, dims=None) -> dict:
    """Point source in uniform hydrogen (or H+He) gas."""
    h = 0.5 * KPC
    dims = (n, n, n) if dims is None else tuple(dims)
    mesh = jittered_lattice(dims, h, 0.2, 1000 + seed_offset, order)
    lex = _lex_ids(mesh)
    cx, cy, cz = (d // 2 for d in dims)
    src_lex = cx + dims[0] * (cy + dims[1] * cz)
    src_cell = np.flatnonzero(lex == src_lex)
    c = (cx, cy, cz)
    if hhe:
        nb = 3
        p = default_params(nb)
        sig, eh = fields.blackbody_bin_constants(T_BLACKBODY, BIN_EDGES_EV)
        p.update(chem_mode=CHEM_HHE, isothermal=0, rate_set=RATES_HG97, Y_He=Y_HE,
                 sigma=sig, e_heat=eh)
        rate = (5.0e48 * np.asarray(BIN_SPLIT))[:, None]
    else:
        nb = 1
        p = default_params(nb)
        p["sigma"][0, 0] = fields.SIGMA0_HI
        rate = np.array([[5.0e48]])
    state = neutral_state(nb, mesh.n_cells, 1.0e-3, 1.0e4)
    name = "stromgren_hhe" if hhe else "stromgren"
    return _pack(name, mesh, p, state, src_cell, rate, n_sub, precision,
                 source_lex=c)


def cosmological(n: int, spacing_kpc: float, sigma_ln: float, n_src: int, c_frac: float,
                 n_sub: int, cfg_id: int, precision: str = "fp64", order: str = "hilbert",
                 name: str = "cosmo", t0: float = 100.0, mean_nh: float = 2.0e-4, dims=None,
                 split_fraction: float = 0.0) -> dict:
    """Lognormal H+He gas with power-law point sources at density peaks.
    With split_fraction > 0 that share of the lattice's faces is split in two
    (seed 6000 + cfg_id), giving cells of 6 to 12 faces."""
    h = spacing_kpc * KPC
    mesh = jittered_lattice((n, n, n) if dims is None else tuple(dims), h, 0.2, 1000 + cfg_id, order)
    if split_fraction > 0:
        mesh = split_faces(mesh, split_fraction, 6000 + cfg_id)
    dims = mesh.dims
    g = fields.gaussian_random_field(dims, h, 2.0 * h, 2000 + cfg_id)
    n_lex = fields.lognormal_density(g, mean_nh, sigma_ln)
    lex = _lex_ids(mesh)
    n_h = n_lex[lex]
    nx, ny, nz = dims
    all_lex = np.arange(nx * ny * nz)
    key_lex = hilbert_key(all_lex % nx, (all_lex // nx) % ny, all_lex // (nx * ny), bits_for(max(dims)))
    peaks_lex = fields.density_peaks(n_lex, dims, key_lex, n_src)
    cell_of_lex = np.empty_like(lex)
    cell_of_lex[lex] = np.arange(lex.size)
    src_cell = cell_of_lex[peaks_lex]
    lum = fields.power_law_luminosities(n_src, 1.0e47, 1.0e50, 3000 + cfg_id)
    rate = np.asarray(BIN_SPLIT)[:, None] * lum[None, :]
    nb = 3
    p = default_params(nb)
    sig, eh = fields.blackbody_bin_constants(T_BLACKBODY, BIN_EDGES_EV)
    p.update(chem_mode=CHEM_HHE, isothermal=0, rate_set=RATES_HG97, Y_He=Y_HE,
             sigma=sig, e_heat=eh, c_reduced=c_frac * C_LIGHT)
    state = neutral_state(nb, mesh.n_cells, n_h, t0)
    return _pack(name, mesh, p, state, src_cell, rate, n_sub, precision,
                 luminosity=lum, sigma_ln=sigma_ln)


def hhe_2m(n: int = 128, n_src: int = 256, n_sub: int = 50, order: str = "hilbert") -> dict:
    return cosmological(n, 1.0, 1.0, n_src, 0.01, n_sub, 2, "fp64", order, "hhe_2m")


def throughput_16m(n: int = 256, n_src: int = 4096, n_sub: int = 200, order: str = "hilbert",
                   precision: str = "mixed") -> dict:
    return cosmological(n, 1.0, 1.5, n_src, 0.1, n_sub, 4, precision, order, "throughput_16m")


def adjoint_262k(n: int = 64, n_src: int = 64, n_sub: int = 50, order: str = "hilbert") -> dict:
    cfg = cosmological(n, 1.0, 1.0, n_src, 0.01, n_sub, 5, "fp64", order, "adjoint_262k")
    cfg["checkpoint_every"] = 10
    # Target luminosities: each source perturbed by a seeded +-20%.
    u = np.random.default_rng(5000).uniform(-1.0, 1.0, size=n_src)
    cfg["meta"]["target_rate_factor"] = 1.0 + 0.2 * u
    return cfg


def travelling_wave(n: int = 16, n_sub: int = 64, amplitude: float = 1.0e-6,
                    order: str = "hilbert", jitter: float = 0.1) -> dict:
    """Optically thin free-streaming wave in a periodic unit box, c = 1."""
    mesh = jittered_lattice((n, n, n), 1.0 / n, jitter, 1000, order)
    nb = 1
    p = default_params(nb)
    p.update(chem_mode=CHEM_NONE, c_reduced=1.0)
    x = mesh.centre
    N = 1.0 + amplitude * np.sin(2 * np.pi * (x[0] + x[1] + x[2]))
    F = np.empty((1, 3, mesh.n_cells))
    F[0, :, :] = N[None, :] / np.sqrt(3.0)
    state = neutral_state(nb, mesh.n_cells, 1.0, 1.0e4)
    state["N"] = N[None, :].copy()
    state["F"] = F * p["c_reduced"]
    return _pack("travelling_wave", mesh, p, state, np.zeros(0, np.int64), np.zeros((1, 0)),
                 n_sub, "fp64", amplitude=amplitude)


def expanding_hii(n: int = 44, n_sub: int = 64, precision: str = "fp64", c_frac: float = 1.0e-3,
                  order: str = "hilbert", jitter: float = 0.1) -> dict:
    """The paper's expanding H II region with hydrogen and helium (Sections
    3.1 and 4.2.2) on its staggered 2 n^3 grid: a 1.6 kpc periodic box of
    neutral gas at 100 K with n_H = n0 inside r0 and n0 (r0 / r)^2 outside
    (n0 = 3.2 cm^-3, r0 = 91.5 pc); photons injected uniformly in a 0.05 kpc
    sphere about the centre at 1e50, 5e48 and 3e48 s^-1 in the three bins;
    cross-sections and heating of a 5e4 K black body; reduced light speed
    1e-3 c."""
    L = 1.6 * KPC
    a = L / n
    mesh = staggered_bcc(n, a, jitter, 1000 + 7, order)
    c = np.full(3, 0.5 * L)
    # distance of each generating point from the box centre
    rel = mesh.centre - c[:, None]
    r = np.linalg.norm(rel, axis=0)
    n0, r0 = 3.2, 0.0915 * KPC
    n_h = np.where(r < r0, n0, n0 * (r0 / np.maximum(r, 1e-30)) ** 2)
    src = np.flatnonzero(r < 0.05 * KPC)
    if src.size == 0:
        src = np.array([int(np.argmin(r))])
    rate = np.array([1.0e50, 5.0e48, 3.0e48])[:, None] * np.full((1, src.size), 1.0 / src.size)
    nb = 3
    p = default_params(nb)
    sig, eh = fields.blackbody_bin_constants(T_BLACKBODY, BIN_EDGES_EV)
    p.update(chem_mode=CHEM_HHE, isothermal=0, rate_set=RATES_HG97, Y_He=Y_HE, sigma=sig, e_heat=eh,
             c_reduced=c_frac * C_LIGHT)
    state = neutral_state(nb, mesh.n_cells, n_h, 100.0)
    return _pack("expanding_hii", mesh, p, state, src, rate, n_sub, precision, radius=r)


def by_name(name: str, **kw) -> dict:
    table = {
        "stromgren": lambda **k: stromgren(**k),
        "hhe_2m": hhe_2m,
        "stromgren_mixed": lambda **k: stromgren(n_sub=k.pop("n_sub", 50), precision="mixed", **k),
        "stromgren_hhe_mixed": lambda **k: stromgren(n_sub=k.pop("n_sub", 50), precision="mixed",
                                                     hhe=True, **k),
        "throughput_16m": throughput_16m,
        "adjoint_262k": adjoint_262k,
        "travelling_wave": travelling_wave,
        "expanding_hii": expanding_hii,
    }
    return table[name](**kw)


def reorder(cfg: dict, perm: np.ndarray) -> dict:
    """The same workload with cells relabelled: new cell k is old cell perm[k].
    Faces stay grouped by their L cell (lattice meshes: three faces per cell)."""
    perm = np.asarray(perm, dtype=np.int64)
    m = cfg["mesh"]
    nc, nf = m["n_cells"], m["n_faces"]
    if nf != 3 * nc or not np.array_equal(m["face_cells"][0], np.repeat(np.arange(nc), 3)):
        raise ValueError("reorder expects a lattice mesh from jittered_lattice")
    new_of_old = np.empty(nc, dtype=np.int64)
    new_of_old[perm] = np.arange(nc)
    fperm = (3 * perm[:, None] + np.arange(3)[None, :]).reshape(-1)
    mesh = dict(m, volume=np.ascontiguousarray(m["volume"][perm]),
                centre=np.ascontiguousarray(m["centre"][:, perm]),
                face_cells=np.ascontiguousarray(new_of_old[m["face_cells"][:, fperm]]),
                area=np.ascontiguousarray(m["area"][fperm]), normal=np.ascontiguousarray(m["normal"][:, fperm]),
                face_centre=np.ascontiguousarray(m["face_centre"][:, fperm]))
    st = cfg["state"]
    state = dict(N=np.ascontiguousarray(st["N"][:, perm]), F=np.ascontiguousarray(st["F"][..., perm]),
                 n_H=np.ascontiguousarray(st["n_H"][perm]), species=np.ascontiguousarray(st["species"][:, perm]),
                 T=np.ascontiguousarray(st["T"][perm]))
    meta = dict(cfg["meta"], lattice_index=np.ascontiguousarray(cfg["meta"]["lattice_index"][:, perm]))
    src = dict(cfg["sources"], cell=new_of_old[cfg["sources"]["cell"]])
    return dict(cfg, mesh=mesh, state=state, sources=src, meta=meta)


def random_order(cfg: dict, seed: int = 4000) -> dict:
    """The workload in a seeded random cell order."""
    return reorder(cfg, np.random.default_rng(seed).permutation(cfg["mesh"]["n_cells"]))


def reorder_cells(cfg: dict, perm: np.ndarray) -> dict:
    """The same workload with cells relabelled (new cell k is old cell perm[k])
    on any mesh: faces are relabelled and listed by their new L cell, in
    their previous order within a cell."""
    perm = np.asarray(perm, dtype=np.int64)
    m = cfg["mesh"]
    nc = m["n_cells"]
    new_of_old = np.empty(nc, dtype=np.int64)
    new_of_old[perm] = np.arange(nc)
    fc = new_of_old[m["face_cells"]]
    fperm = np.lexsort((np.arange(m["n_faces"]), fc[0]))
    mesh = dict(m, volume=np.ascontiguousarray(m["volume"][perm]),
                centre=np.ascontiguousarray(m["centre"][:, perm]),
                face_cells=np.ascontiguousarray(fc[:, fperm]),
                area=np.ascontiguousarray(m["area"][fperm]), normal=np.ascontiguousarray(m["normal"][:, fperm]),
                face_centre=np.ascontiguousarray(m["face_centre"][:, fperm]))
    st = cfg["state"]
    state = dict(N=np.ascontiguousarray(st["N"][:, perm]), F=np.ascontiguousarray(st["F"][..., perm]),
                 n_H=np.ascontiguousarray(st["n_H"][perm]), species=np.ascontiguousarray(st["species"][:, perm]),
                 T=np.ascontiguousarray(st["T"][perm]))
    meta = dict(cfg["meta"], lattice_index=np.ascontiguousarray(cfg["meta"]["lattice_index"][:, perm]),
                cell_perm=perm)
    src = dict(cfg["sources"], cell=new_of_old[cfg["sources"]["cell"]])
    return dict(cfg, mesh=mesh, state=state, sources=src, meta=meta)


def face_counts(mesh: dict) -> np.ndarray:
    return np.bincount(mesh["face_cells"].ravel(), minlength=mesh["n_cells"])


def degree_sorted(cfg: dict) -> dict:
    """Cells sorted by their number of faces, in their previous order within
    one count (the paper sorts cells by number of interfaces, Sec. 4.1.4), so
    that the 64 cells of a slice share a degree and a slice pads to no more
    slots than its cells have."""
    return reorder_cells(cfg, np.argsort(face_counts(cfg["mesh"]), kind="stable"))
