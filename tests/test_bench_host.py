"""bench.py's host-side accounting (no GPU): the byte models its roofline
figures use, and its refusal of more than one GPU."""
import subprocess
import sys
from pathlib import Path

import numpy as np

import bench

ROOT = Path(__file__).resolve().parents[1]


def test_whole_subcycle_bytes_per_cell():
    # two-pass: 36 nb p + 2 (52 g + 48) + 104; compulsory: 8 nb p + (52 g + 48) + 104
    assert bench.subcycle_bytes_per_cell(3, 4, 4) == {"two_pass": 1048, "compulsory": 456}
    assert bench.subcycle_bytes_per_cell(3, 8, 8) == {"two_pass": 1896, "compulsory": 760}
    assert bench.subcycle_bytes_per_cell(1, 8, 8) == {"two_pass": 1320, "compulsory": 632}


def test_kernel_bytes_per_lattice_cell():
    """Per cell of a six-face lattice (3 faces, 6 face sides), 3 bins, FP32."""
    per_cell = {k: bench.algorithmic_bytes(k, 1, 3, 3, 6, 0, 4, 4)
                for k in ("k_facestate", "k_flux", "k_transport", "k_chem")}
    assert per_cell == {"k_facestate": 548, "k_flux": 520, "k_transport": 488, "k_chem": 208}
    # linear in the cell count
    assert bench.algorithmic_bytes("k_flux", 1000, 3, 3000, 6000, 0, 4, 4) == 520 * 1000


def test_model_bytes_of_each_pass_add_up_to_the_two_pass_subcycle():
    # gradient pass 16 nb p + 52 g + 48, flux pass 20 nb p + 52 g + 48, chemistry 104
    m = {k: bench.model_bytes_per_cell(k, 3, 4, 4) for k in ("k_facestate", "k_flux", "k_chem", "k_transport")}
    assert m == {"k_facestate": 448, "k_flux": 496, "k_chem": 104, "k_transport": 944}
    assert m["k_facestate"] + m["k_flux"] + m["k_chem"] == bench.subcycle_bytes_per_cell(3, 4, 4)["two_pass"]
    assert bench.model_bytes_per_cell("k_flux", 3, 8, 8) == 20 * 3 * 8 + 52 * 8 + 48


def test_field_errors_find_planted_differences():
    import numpy as np
    rng = np.random.default_rng(3)
    nb, nc, c = 2, 50, 3.0e9
    N = rng.uniform(1.0, 2.0, size=(nb, nc))
    r = dict(N=N, F=0.5 * c * N[:, None, :] * np.ones((nb, 3, nc)) / np.sqrt(3), species=rng.uniform(size=(5, nc)),
             T=rng.uniform(1e3, 1e4, nc))
    a = {k: v.copy() for k, v in r.items()}
    a["N"][1, 7] *= 1 + 5e-3          # one cell over the N bar
    a["F"][0, 2, 9] += 1e-2 * c * r["N"][0, 9]
    a["species"][1, 3] += 2e-4
    att_r = np.ones(nc, np.int64)
    att_a = att_r.copy()
    att_a[7] = 2
    e, over = bench.field_errors(a, r, None, c, att_a, att_r)
    assert abs(e["N_rel_max(N>1e-10 max)"] - 5e-3) < 1e-12
    assert e["cells_N_rel>1e-3"] == 1 and over[7] and over.sum() == 1
    assert abs(e["F_rel_to_cN_max(N>1e-10 max)"] - 1e-2) < 1e-9
    assert abs(e["x_HII_abs_max"] - 2e-4) < 1e-12
    assert not e["meets_stated_bar"]
    assert e["cells_N_rel>1e-3_with_other_attempt_count"] == 1 and e["cells_with_other_attempt_count"] == 1
    e2, _ = bench.field_errors(r, r, None, c)
    assert e2["meets_stated_bar"] and e2["cells_N_rel>1e-3"] == 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_tile_byte_model_counts_every_face_side():
    """On a Hilbert-ordered lattice the split runs by tile: the boundary items
    and twice the tile-interior faces are every face side of the mesh, and
    the per-kernel bytes follow the tile formulas (fields in, partly updated
    fields out and back in, boundary states and cap numerators, geometry
    once)."""
    import rtgen
    from paper_2404_17630_amd import rt
    m = rtgen.jittered_lattice((16, 16, 16), 1.0, 0.2, 3, "hilbert").as_dict()
    h = rt.Mesh(m, device=rt.RT_DEVICE_HOST_ONLY)
    tiles = bench.tile_counts(h)
    h.close()
    nc = m["n_cells"]
    n_bnd, n_pairs = tiles
    assert n_bnd + 2 * n_pairs == 6 * nc
    assert n_bnd <= 2 * nc                       # compact tiles
    nb, p, g = 3, 4, 4
    fs = bench.algorithmic_bytes("k_facestate", nc, nb, 3 * nc, 6 * nc, 0, p, g, tiles)
    fl = bench.algorithmic_bytes("k_flux", nc, nb, 3 * nc, 6 * nc, 0, p, g, tiles)
    assert fs == nb * (16 * nc + 16 * nc + 20 * n_bnd) + nc * 33 + 6 * nc * 28 + n_pairs * 20
    assert fl == nb * (16 * nc + 16 * nc + 40 * n_bnd) + nc * 5 + n_bnd * 20
    # an unordered lattice keeps the per-slice kernels
    r = rtgen.jittered_lattice((16, 16, 16), 1.0, 0.2, 3, "random").as_dict()
    h = rt.Mesh(r, device=rt.RT_DEVICE_HOST_ONLY)
    assert bench.tile_counts(h) is None
    h.close()


def test_attempt_histogram_bins():
    """Every count lands in exactly one bin, at the bins' edges too."""
    a = np.array([1, 1, 2, 3, 4, 5, 8, 9, 16, 17, 64, 65, 256, 257, 1000])
    h = bench.attempt_histogram(a)
    assert list(h) == ["1", "2", "3-4", "5-8", "9-16", "17-64", "65-256", ">256"]
    assert list(h.values()) == [2, 1, 2, 2, 2, 2, 2, 2]
    assert sum(h.values()) == a.size
