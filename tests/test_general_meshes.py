"""Meshes with variable face counts (no GPU): the split-face lattice, whose
cells have 6 to 12 faces, and the degree-sorted cell order.

The split mesh replaces a seeded share of a jittered lattice's faces by two
half-area faces with distinct centres.  What fixes the oracle on it,
independently of its own formulas: every cell still closes (sum A n = 0),
so a uniform radiation field is left unchanged by the transport; the
geometry matrix sum A u u^T is that of the unsplit lattice; fluxes are
antisymmetric, so the photon content of optically thin periodic transport
is conserved; and the degree-sorted relabelling gives the same physics."""
import numpy as np
import pytest

import oracle
import rtgen


def split_wave(n=8, n_sub=6):
    cfg = rtgen.travelling_wave(n=n, n_sub=n_sub)
    mesh = rtgen.split_faces(rtgen.jittered_lattice((n, n, n), 1.0 / n, 0.1, 1000, "hilbert"), 0.25, 11)
    return dict(cfg, mesh=mesh.as_dict())


def test_split_mesh_cells_close_and_keep_their_geometry_matrix():
    base = rtgen.jittered_lattice((7, 6, 5), 1.0, 0.2, 4, "hilbert")
    sm = rtgen.split_faces(base, 0.3, 9)
    m = sm.as_dict()
    deg = rtgen.face_counts(m)
    assert deg.min() == 6 and deg.max() > 7 and m["n_faces"] > base.n_faces
    s = np.zeros((3, m["n_cells"]))
    for k in range(3):
        np.add.at(s[k], m["face_cells"][0], m["area"] * m["normal"][k])
        np.add.at(s[k], m["face_cells"][1], -m["area"] * m["normal"][k])
    assert np.abs(s).max() <= 1e-12 * m["area"].max()
    assert np.allclose(oracle.geometry_minv(m), oracle.geometry_minv(base.as_dict()), rtol=1e-12, atol=0)


def test_uniform_state_is_invariant_on_the_split_mesh():
    cfg = split_wave()
    cfg["state"]["N"][:] = 2.5
    cfg["state"]["F"][:] = 0.3 * cfg["params"]["c_reduced"] * 2.5 / np.sqrt(3.0)
    out = oracle.run(cfg)
    assert np.allclose(out["N"], 2.5, rtol=1e-13, atol=0)
    assert np.allclose(out["F"], cfg["state"]["F"], rtol=1e-12, atol=0)


def test_photon_content_is_conserved_on_the_split_mesh():
    cfg = split_wave(n_sub=1)
    V = cfg["mesh"]["volume"]
    total = float((cfg["state"]["N"][0] * V).sum())
    for n_sub in (1, 5):
        out = oracle.run(cfg, n_sub=n_sub)
        assert abs(out["diag"]["photon_sum"][0] - total) <= 1e-14 * n_sub * total


def test_degree_sorted_order_gives_the_same_physics():
    cfg = rtgen.cosmological(0, 1.0, 1.0, 5, 0.01, 3, 3, dims=(9, 8, 7), split_fraction=0.2, name="split")
    srt = rtgen.degree_sorted(cfg)
    assert np.all(np.diff(rtgen.face_counts(srt["mesh"])) >= 0)
    perm = srt["meta"]["cell_perm"]
    a = oracle.run(cfg)
    b = oracle.run(srt)
    # sums over a cell's faces run in another face order: rounding only
    for b_ in range(3):
        ref = a["N"][b_][perm]
        scale = np.maximum(np.abs(ref), 1e-6 * np.abs(ref).max())
        assert np.max(np.abs(b["N"][b_] - ref) / scale) < 1e-11
    assert np.allclose(b["species"], a["species"][:, perm], rtol=1e-11, atol=1e-15)
    assert a["diag"]["substeps"] == b["diag"]["substeps"]
