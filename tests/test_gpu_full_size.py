"""The throughput workload at full size (256^3 = 16,777,216 cells, 3 bins,
4096 sources, Hilbert order), in the launch configuration bench.py times
(the library's default transport: the split by tile), checked against the
oracle on sampled cells: after 20 FP64 subcycles on the GPU, one and four
more subcycles in FP64 and in the mixed form, each sampled cell against the
oracle's same subcycles on its periodic patch of half-width twice the
subcycle count (tests/patches.py; pinned against whole-mesh oracle runs in
tests/test_patches.py).  The sample takes the source cells, lit cells and
fronts (N >= 1e-8 of its maximum) and cells from anywhere.  Plus one
property at full size: the fused and split paths agree bit for bit."""
import numpy as np
import pytest

import oracle
import rtgen
from paper_2404_17630_amd import rt
from tests.gpu_common import say
from tests.patches import LatticeIndex, centre_values, patch_config, sample_cells

pytestmark = pytest.mark.gpu

N_SUB0 = 20
K_MULTI = 4


@pytest.fixture(scope="module")
def full():
    say("full size: generating the 256^3 throughput workload")
    cfg = rtgen.throughput_16m(n_sub=N_SUB0, precision="fp64")
    mesh = rt.Mesh(cfg["mesh"])
    say(f"full size: {N_SUB0} FP64 subcycles")
    st = rt.State.from_config(mesh, cfg, precision=rt.RT_FP64)
    st.subcycle(N_SUB0)
    f0 = st.fields()
    dt = st.diagnostics()["dt"]
    lat = LatticeIndex(cfg["mesh"])
    cells = sample_cells(f0, 48, 24, 11, cfg["sources"]["cell"])
    rings = np.stack([lat.block(int(c), 1) for c in cells])        # the 3^3 block around each cell

    def keep(f):
        """The sampled cells' fields, the largest N of each one's 3^3 block
        and every bin's largest N."""
        return dict(N=f["N"][:, cells], F=f["F"][:, :, cells], species=f["species"][:, cells], T=f["T"][cells],
                    ring_N=np.abs(f["N"][:, rings]).max(axis=2), bin_max=f["N"].max(axis=1))

    out = {}
    say(f"full size: 1 and {K_MULTI} more FP64 subcycles")
    st.subcycle(1, dt)
    out["fp64", 1] = keep(st.fields())
    st.subcycle(K_MULTI - 1, dt)
    out["fp64", K_MULTI] = keep(st.fields())
    st.close()
    say(f"full size: the same 1 and {K_MULTI} subcycles in the mixed form")
    cfg1 = dict(cfg, state=dict(f0), n_subcycles=1)
    stm = rt.State.from_config(mesh, cfg1, precision=rt.RT_MIXED)
    assert not stm.fused
    stm.subcycle(1, dt)
    out["mixed", 1] = keep(stm.fields())
    stm.subcycle(K_MULTI - 1, dt)
    out["mixed", K_MULTI] = keep(stm.fields())
    stm.close()
    yield dict(cfg=cfg, mesh=mesh, f0=f0, dt=dt, lat=lat, cells=cells, out=out)
    mesh.close()


def cell_errors(got, ref, ring_N, bin_max, c_red):
    """Errors of one cell: N against s = max(N, 1e-6 of the largest N in the
    cell's 3^3 block, 1e-10 bin max), F against c~ s, fractions relative to
    |x| times the cell's photon conditioning (floored at 1e-9; y_HeII at
    1e-5), T relative."""
    e = {}
    cond = 1.0
    for b in range(ref["N"].shape[0]):
        Nr = ref["N"][b]
        s = max(abs(Nr), 1e-6 * max(abs(Nr), ring_N[b]), 1e-10 * bin_max[b])
        s = s if s > 0 else 1.0
        if Nr > 0:
            cond = max(cond, min(s / Nr, 1e6))
        e[f"N[{b}]"] = abs(got["N"][b] - Nr) / s
        e[f"F[{b}]"] = float(np.abs(got["F"][b] - ref["F"][b]).max()) / (c_red * s)
    for q, name in enumerate(("x_HI", "x_HII", "y_HeI", "y_HeII", "y_HeIII")):
        floor = 1e-5 if name == "y_HeII" else 1e-9
        e[name] = abs(got["species"][q] - ref["species"][q]) / max(abs(ref["species"][q]) * cond, floor)
        e[name + " abs"] = abs(got["species"][q] - ref["species"][q])
    e["T"] = abs(got["T"] - ref["T"]) / ref["T"]
    return e


@pytest.mark.parametrize("k", [1, K_MULTI])
def test_sampled_cells_match_the_oracle(full, k):
    cfg, f0, lat, cells = full["cfg"], full["f0"], full["lat"], full["cells"]
    c_red = cfg["params"]["c_reduced"]
    say(f"full size: {cells.size} sampled cells after {k} subcycles against the oracle on their patches")
    r64, rmix = full["out"]["fp64", k], full["out"]["mixed", k]
    e64, emix = {}, {}
    for j, c in enumerate(cells):
        ref = centre_values(oracle.run(patch_config(cfg, f0, lat, int(c), n_sub=k), dt=full["dt"]), n_sub=k)
        for r, e in ((r64, e64), (rmix, emix)):
            got = dict(N=r["N"][:, j], F=r["F"][:, :, j], species=r["species"][:, j], T=r["T"][j])
            for q, v in cell_errors(got, ref, r64["ring_N"][:, j], r64["bin_max"], c_red).items():
                e[q] = max(e.get(q, 0.0), v)
    for q in e64:
        say(f"  {q:12s} fp64 {e64[q]:.3e}   mixed {emix[q]:.3e}")
    for q in ("N[0]", "N[1]", "N[2]", "F[0]", "F[1]", "F[2]", "x_HI", "x_HII", "y_HeI", "y_HeII", "y_HeIII", "T"):
        assert e64[q] <= 1e-10, (q, e64[q])
    for b in range(3):
        assert emix[f"N[{b}]"] <= 1e-3 and emix[f"F[{b}]"] <= 1e-3, (b, emix)
    for name in ("x_HI", "x_HII", "y_HeI", "y_HeII", "y_HeIII"):
        assert emix[name + " abs"] <= 1e-4, (name, emix)
    assert emix["T"] <= 1e-4, emix


def test_fused_equals_split_at_full_size(full):
    """Two mixed subcycles from the 20-subcycle state on both transport
    paths: every field equal bit for bit."""
    cfg = dict(full["cfg"], state=dict(full["f0"]), n_subcycles=2)
    out = []
    for mode in (rt.RT_TRANSPORT_SPLIT, rt.RT_TRANSPORT_FUSED):
        s = rt.State.from_config(full["mesh"], cfg, precision=rt.RT_MIXED)
        s.set_transport(mode)
        s.subcycle(2, full["dt"])
        out.append(s.fields())
        s.close()
    for k in ("N", "F", "species", "T"):
        assert np.array_equal(out[0][k], out[1][k]), k
