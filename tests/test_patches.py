"""The patch recomputation of single cells (tests/patches.py) against whole-
mesh oracle runs, on the CPU: what the full-size GPU test relies on."""
import numpy as np

import oracle
import rtgen
import pytest

from tests.patches import LatticeIndex, centre_index, centre_values, patch_config, sample_cells


@pytest.mark.parametrize("n, n_sub", [(12, 1), (16, 2), (16, 3)])
def test_patch_recomputes_subcycles_of_sampled_cells(n, n_sub):
    """An n^3 H+He lattice with 8 sources, advanced 6 subcycles by the
    oracle; n_sub more subcycles on the whole mesh against the same
    subcycles on the periodic patch of half-width 2 n_sub around each
    sampled cell (lit cells, fronts, source cells and unlit gas): equal to
    1e-12 in every field, N and F relative to the largest N in the 3^3
    block around the cell (the size of the terms its update sums, in another
    order on the patch)."""
    cfg = rtgen.throughput_16m(n=n, n_src=8, n_sub=6, precision="fp64")
    st6 = oracle.run(cfg)
    fields = {k: st6[k] for k in ("N", "F", "species", "T")}
    fields["n_H"] = np.asarray(cfg["state"]["n_H"], float)
    cfg1 = dict(cfg, state=dict(fields), n_subcycles=n_sub)
    dt = oracle.cfl_dt(cfg)
    st7 = oracle.run(cfg1, dt=dt)
    lat = LatticeIndex(cfg["mesh"])
    cells = sample_cells(fields, 12, 6, 7, cfg["sources"]["cell"])
    assert cells.size >= 16
    worst = 0.0
    for c in cells:
        ref = centre_values(oracle.run(patch_config(cfg, fields, lat, int(c), n_sub=n_sub), dt=dt), n_sub=n_sub)
        ring = lat.block(int(c), 1)
        for b in range(cfg["params"]["nb"]):
            s = max(np.abs(st7["N"][b, ring]).max(), 1e-12 * st7["N"][b].max(), 1e-300)
            worst = max(worst, abs(ref["N"][b] - st7["N"][b, c]) / s)
            for k in range(3):
                worst = max(worst, abs(ref["F"][b, k] - st7["F"][b, k, c]) / (cfg["params"]["c_reduced"] * s))
        for q in range(5):
            worst = max(worst, abs(ref["species"][q] - st7["species"][q, c]) / max(abs(st7["species"][q, c]), 1e-9))
        worst = max(worst, abs(ref["T"] - st7["T"][c]) / st7["T"][c])
    assert worst <= 1e-12, worst


def test_patch_block_is_the_cell_and_its_two_face_rings():
    cfg = rtgen.throughput_16m(n=12, n_src=8, n_sub=1, precision="fp64")
    lat = LatticeIndex(cfg["mesh"])
    fc = cfg["mesh"]["face_cells"]
    nbrs = [set() for _ in range(cfg["mesh"]["n_cells"])]
    for L, R in fc.T:
        nbrs[L].add(int(R))
        nbrs[R].add(int(L))
    for c in (0, 17, 1000):
        ring1 = nbrs[c]
        ring2 = set().union(*(nbrs[j] for j in ring1))
        block = set(int(v) for v in lat.block(c))
        assert len(block) == 125
        assert {c} | ring1 | ring2 <= block
        assert lat.block(c)[62] == c
        for w in (1, 4):
            assert lat.block(c, w)[centre_index(w)] == c
    with pytest.raises(ValueError):
        lat.block(0, 6)          # 13 cells across a 12^3 lattice would wrap
