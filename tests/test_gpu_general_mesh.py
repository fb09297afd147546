"""General (non-lattice) meshes: the paper's staggered 2 n^3 grid, whose
cells are truncated octahedra with 14 faces, and the expanding H II region
with hydrogen and helium run on it (Sections 3.1 and 4.2.2)."""
import numpy as np
import pytest

import oracle
import rtgen
from paper_2404_17630_amd import rt
from paper_2404_17630_amd.autograd import Problem
from tests.gpu_common import field_errors, run_gpu, say
from tests.test_gpu_adjoint import adjoint
from tests.test_gpu_mixed import assert_other_fields, mixed_errors

pytestmark = pytest.mark.gpu


def test_expanding_hii_fp64_matches_oracle():
    cfg = rtgen.expanding_hii(n=12, n_sub=12)
    say("expanding H II region, BCC 2x12^3, 12 subcycles, fp64")
    gpu = run_gpu(cfg)
    ref = oracle.run(cfg)
    errs = field_errors(gpu, ref, cfg["params"]["c_reduced"], cfg["mesh"]["face_cells"])
    worst = max(errs, key=errs.get)
    say("worst", worst, f"{errs[worst]:.3e}")
    assert max(errs.values()) <= 1e-10, errs
    assert gpu["diag"]["substeps"] == ref["diag"]["substeps"]


def test_expanding_hii_mixed_meets_stated_error():
    cfg = rtgen.expanding_hii(n=12, n_sub=12, precision="mixed")
    gpu = run_gpu(cfg, precision=rt.RT_MIXED)
    ref = oracle.run(cfg)
    errs = mixed_errors(gpu, ref, cfg["params"]["c_reduced"])
    for k, v in errs.items():
        say(f"  {k:16s} {v:.3e}")
    assert max(errs[f"N[{b}] rel"] for b in range(3)) <= 1e-3
    assert errs["x_HII abs"] <= 1e-4
    assert_other_fields(errs)


def test_adjoint_on_fourteen_face_cells():
    cfg = rtgen.expanding_hii(n=6, n_sub=4)
    pb = Problem(cfg, checkpoint_every=3)
    nc = cfg["mesh"]["n_cells"]
    ns = cfg["sources"]["cell"].size
    rng = np.random.default_rng(7)
    w = rng.normal(size=nc)
    gq, gn, _ = adjoint(pb, pb.log_lum0.copy(), np.log(cfg["state"]["n_H"]), w)
    dq = np.zeros((2, ns))
    dq[0] = rng.normal(size=ns)
    dn = np.zeros((2, nc))
    dn[1] = rng.normal(size=nc)
    jv = oracle.run_jvp(cfg, dq, dn)["dxHI"]
    for d in range(2):
        ref = w @ jv[d]
        got = gq @ dq[d] + gn @ dn[d]
        say(f"bcc direction {d}: adjoint {got:.12e} oracle {ref:.12e}")
        assert got == pytest.approx(ref, rel=1e-8, abs=0.0)


def test_expanding_hii_ionisation_zones():
    """Zone structure the paper describes for this test (Section 4.2.2, Fig. 12):
    helium is ionised twice nearest the source, then once, and the outermost
    layer of the H II region has ionised hydrogen with neutral helium.  The
    paper's run moves the gas with hydrodynamics, which empties the centre;
    with the density held fixed the doubly ionised zone stays inside the
    source sphere, so the check is on the ordering of the shell-averaged
    profiles and of the fronts."""
    cfg = rtgen.expanding_hii(n=24, n_sub=150)
    say("expanding H II region, BCC 2x24^3, 150 subcycles")
    g = run_gpu(cfg)
    x = g["species"]
    V = cfg["mesh"]["volume"]
    pc = 3.086e18
    r = cfg["meta"]["radius"] / pc
    edges = np.arange(0.0, 321.0, 40.0)
    shells = [(r >= lo) & (r < hi) for lo, hi in zip(edges[:-1], edges[1:])]
    prof = {name: np.array([v[m].mean() for m in shells])
            for name, v in (("x_HII", x[1]), ("He ionised", 1.0 - x[2]), ("y_HeIII", x[4]), ("T", g["T"]))}
    for k, v in prof.items():
        say(f"  {k:10s}", " ".join(f"{e:.3g}" for e in v))
    for k in ("x_HII", "He ionised", "y_HeIII"):
        assert np.all(np.diff(prof[k]) <= 1e-12), k
    assert prof["y_HeIII"][0] > 0.05 and prof["x_HII"][0] > 0.99

    def front(frac):
        # volume-equivalent radius of the region where frac > 1/2
        return (3.0 / (4 * np.pi) * np.sum(V[frac > 0.5])) ** (1 / 3) / pc

    r_h, r_he = front(x[1]), front(1.0 - x[2])
    say(f"fronts: helium {r_he:.1f} pc, hydrogen {r_h:.1f} pc")
    assert 0 < r_he < r_h
    assert np.all(g["T"] > 0)


def split_cfg(order="hilbert", precision="fp64"):
    """H+He on a jittered lattice with a fifth of its faces split in two:
    cells of 6 to 11 faces, so every slice pads to its largest degree and the
    general-degree kernels run."""
    cfg = rtgen.cosmological(0, 1.0, 1.0, 6, 0.01, 6, 3, dims=(14, 12, 11), split_fraction=0.2,
                             name="split_faces", precision=precision)
    return rtgen.degree_sorted(cfg) if order == "degree" else cfg


@pytest.mark.parametrize("order", ["hilbert", "degree"])
def test_variable_degree_mesh_fp64_matches_oracle(order):
    cfg = split_cfg(order)
    m = rt.Mesh(cfg["mesh"])
    sdeg = m.table("sdeg")
    assert len(set(sdeg.tolist())) > 1           # slices of several degrees: the general kernels
    m.close()
    say("split faces", order, cfg["mesh"]["n_cells"], "cells", cfg["mesh"]["n_faces"], "faces")
    gpu = run_gpu(cfg)
    ref = oracle.run(cfg)
    errs = field_errors(gpu, ref, cfg["params"]["c_reduced"], cfg["mesh"]["face_cells"])
    worst = max(errs, key=errs.get)
    say("worst", worst, f"{errs[worst]:.3e}")
    assert max(errs.values()) <= 1e-10, errs
    assert gpu["diag"]["substeps"] == ref["diag"]["substeps"]
    assert gpu["diag"]["flux_caps"] > 0


def test_variable_degree_mesh_mixed_meets_stated_error():
    cfg = split_cfg(precision="mixed")
    gpu = run_gpu(cfg, precision=rt.RT_MIXED)
    ref = oracle.run(cfg)
    errs = mixed_errors(gpu, ref, cfg["params"]["c_reduced"])
    for k, v in errs.items():
        say(f"  {k:16s} {v:.3e}")
    assert max(errs[f"N[{b}] rel"] for b in range(3)) <= 1e-3
    assert errs["x_HII abs"] <= 1e-4
    assert_other_fields(errs)


@pytest.mark.parametrize("precision", [rt.RT_FP64, rt.RT_MIXED], ids=["fp64", "mixed"])
def test_variable_degree_mesh_fused_equals_split(precision):
    cfg = split_cfg()
    a = run_gpu(cfg, precision=precision, transport=rt.RT_TRANSPORT_FUSED)
    b = run_gpu(cfg, precision=precision, transport=rt.RT_TRANSPORT_SPLIT)
    assert a["fused"] and not b["fused"]
    for key in ("N", "F", "species", "T"):
        assert np.array_equal(a[key], b[key]), key


def open_slab_cfg(precision="fp64"):
    """H+He on a 12 x 12 x 10 jittered lattice, periodic in x and y and open
    in z (box_z = 0): the faces that would close the lattice across z are
    dropped, so the cells of the two z layers have five faces and nothing
    flows out through them."""
    cfg = rtgen.cosmological(0, 1.0, 1.0, 6, 0.01, 6, 4, dims=(12, 12, 10), name="open_slab", precision=precision)
    m = dict(cfg["mesh"])
    h = float(np.cbrt(m["volume"][0]))
    zc = np.floor(np.asarray(m["centre"])[2] / h).astype(np.int64)
    L, R = m["face_cells"]
    keep = ~((np.asarray(m["normal"])[2] == 1.0) & (zc[L] == 9) & (zc[R] == 0))
    m.update(n_faces=int(keep.sum()), face_cells=np.ascontiguousarray(m["face_cells"][:, keep]),
             area=np.ascontiguousarray(m["area"][keep]), normal=np.ascontiguousarray(m["normal"][:, keep]),
             face_centre=np.ascontiguousarray(m["face_centre"][:, keep]),
             box=np.array([m["box"][0], m["box"][1], 0.0]))
    cfg["mesh"] = m
    return cfg


def test_open_boundary_fp64_matches_oracle():
    cfg = open_slab_cfg()
    deg = rtgen.face_counts(cfg["mesh"])
    assert deg.min() == 5 and deg.max() == 6
    gpu = run_gpu(cfg)
    ref = oracle.run(cfg)
    errs = field_errors(gpu, ref, cfg["params"]["c_reduced"], cfg["mesh"]["face_cells"])
    worst = max(errs, key=errs.get)
    say("open slab: worst", worst, f"{errs[worst]:.3e}")
    assert max(errs.values()) <= 1e-10, errs
    assert gpu["diag"]["substeps"] == ref["diag"]["substeps"]


def test_open_boundary_mixed_and_both_paths():
    cfg = open_slab_cfg(precision="mixed")
    gpu = run_gpu(cfg, precision=rt.RT_MIXED)
    errs = mixed_errors(gpu, oracle.run(cfg), cfg["params"]["c_reduced"])
    assert max(errs[f"N[{b}] rel"] for b in range(3)) <= 1e-3
    assert errs["x_HII abs"] <= 1e-4
    assert_other_fields(errs)
    for precision in (rt.RT_FP64, rt.RT_MIXED):
        a = run_gpu(cfg, precision=precision, transport=rt.RT_TRANSPORT_FUSED)
        b = run_gpu(cfg, precision=precision, transport=rt.RT_TRANSPORT_SPLIT)
        for key in ("N", "F", "species", "T"):
            assert np.array_equal(a[key], b[key]), (precision, key)
