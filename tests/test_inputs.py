"""The seeded input generator: Hilbert order, mesh geometry, determinism."""
import numpy as np
import pytest

import rtgen
from rtgen.hilbert import hilbert_key


def test_hilbert_curve_steps_between_lattice_neighbours():
    for bits in (1, 2, 3, 5):
        n = 1 << bits
        lex = np.arange(n ** 3)
        ix, iy, iz = lex % n, (lex // n) % n, lex // (n * n)
        k = hilbert_key(ix, iy, iz, bits)
        assert np.array_equal(np.sort(k), lex)
        o = np.argsort(k)
        step = np.abs(np.diff(np.stack([ix[o], iy[o], iz[o]]), axis=1)).sum(0)
        assert np.all(step == 1)


def test_lattice_mesh_is_closed_and_consistent():
    m = rtgen.jittered_lattice((5, 4, 3), 2.0, 0.2, 3, "random")
    nc, nf = m.n_cells, m.n_faces
    assert nf == 3 * nc
    # each cell has six faces and sum A n over its faces (outward) vanishes
    s = np.zeros((3, nc))
    cnt = np.zeros(nc, int)
    for f in range(nf):
        L, R = m.face_cells[:, f]
        s[:, L] += m.area[f] * m.normal[:, f]
        s[:, R] -= m.area[f] * m.normal[:, f]
        cnt[L] += 1
        cnt[R] += 1
    assert np.all(cnt == 6)
    assert np.allclose(s, 0, atol=1e-12)
    assert np.allclose(m.volume.sum(), np.prod(m.box))
    # jitter bounded by 0.2 h per axis about the lattice centre
    off = m.centre - (m.lattice_index + 0.5) * m.h
    assert np.all(np.abs(off) <= 0.2 * m.h + 1e-12)


def test_orders_share_the_same_points():
    a = rtgen.jittered_lattice((4, 4, 4), 1.0, 0.2, 5, "hilbert")
    b = rtgen.jittered_lattice((4, 4, 4), 1.0, 0.2, 5, "random")
    ka = a.lattice_index[0] + 4 * (a.lattice_index[1] + 4 * a.lattice_index[2])
    kb = b.lattice_index[0] + 4 * (b.lattice_index[1] + 4 * b.lattice_index[2])
    assert np.array_equal(a.centre[:, np.argsort(ka)], b.centre[:, np.argsort(kb)])


def test_workloads_are_deterministic():
    a = rtgen.hhe_2m(n=16, n_src=8)
    b = rtgen.hhe_2m(n=16, n_src=8)
    assert np.array_equal(a["state"]["n_H"], b["state"]["n_H"])
    assert np.array_equal(a["sources"]["cell"], b["sources"]["cell"])
    assert np.array_equal(a["sources"]["rate"], b["sources"]["rate"])
    # lognormal density keeps its mean
    big = rtgen.hhe_2m(n=48, n_src=8)
    assert abs(big["state"]["n_H"].mean() / 2e-4 - 1) < 0.05


def test_bin_constants_are_physical():
    c = rtgen.stromgren(hhe=True, n=8)
    sig, eh = c["params"]["sigma"], c["params"]["e_heat"]
    assert np.all(sig >= 0) and np.all(eh >= 0)
    assert sig[0, 1] == 0 and sig[0, 2] == 0 and sig[1, 2] == 0     # below He thresholds
    assert 1e-18 < sig[0, 0] < 6.3e-18


def test_staggered_bcc_cells_are_truncated_octahedra():
    m = rtgen.staggered_bcc(4, 2.0, 0.1, 3, "hilbert")
    nc, nf = m.n_cells, m.n_faces
    assert nc == 2 * 4 ** 3 and nf == 7 * nc
    s = np.zeros((3, nc))
    cnt = np.zeros(nc, int)
    surf = np.zeros(nc)
    for f in range(nf):
        L, R = m.face_cells[:, f]
        s[:, L] += m.area[f] * m.normal[:, f]
        s[:, R] -= m.area[f] * m.normal[:, f]
        cnt[L] += 1
        cnt[R] += 1
        surf[L] += m.area[f]
        surf[R] += m.area[f]
    a = 2.0
    assert np.all(cnt == 14)
    assert np.allclose(s, 0, atol=1e-12)
    # truncated octahedron of a BCC Voronoi cell: volume a^3/2, surface (3 sqrt(3)/2 + 3/4) a^2
    assert np.allclose(m.volume, a ** 3 / 2)
    assert np.allclose(surf, (1.5 * np.sqrt(3) + 0.75) * a * a)
    assert m.volume.sum() == pytest.approx(np.prod(m.box))
