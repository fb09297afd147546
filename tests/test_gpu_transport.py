"""The fused transport kernel (gradients, face states and fluxes per
256-cell tile with the face states in LDS) against the split kernels and
against the oracle."""
import numpy as np
import pytest

import oracle
import rtgen
from paper_2404_17630_amd import rt
from tests.gpu_common import field_errors, run_gpu, say
from tests.test_gpu_mixed import assert_other_fields, mixed_errors

pytestmark = pytest.mark.gpu


def ragged_hhe(order="hilbert"):
    return rtgen.cosmological(0, 1.0, 1.0, 6, 0.01, 8, 2, dims=(20, 18, 17), order=order, name="hhe_ragged")


@pytest.mark.parametrize("precision", [rt.RT_FP64, rt.RT_MIXED], ids=["fp64", "mixed"])
def test_fused_and_split_agree(precision):
    cfg = ragged_hhe()
    a = run_gpu(cfg, precision=precision, transport=rt.RT_TRANSPORT_FUSED)
    b = run_gpu(cfg, precision=precision, transport=rt.RT_TRANSPORT_SPLIT)
    assert a["fused"] and not b["fused"]
    errs = field_errors(a, b, cfg["params"]["c_reduced"], cfg["mesh"]["face_cells"])
    worst = max(errs, key=errs.get)
    say("fused vs split", "fp64" if precision == rt.RT_FP64 else "mixed", worst, f"{errs[worst]:.3e}")
    # Both paths run the same per-cell arithmetic in the same order (the
    # fused kernel only keeps the face states in LDS), so they agree bit for
    # bit after any number of subcycles.
    for key in ("N", "F", "species", "T"):
        assert np.array_equal(a[key], b[key]), (key, errs)
    ref = oracle.run(cfg)
    e_ref = field_errors(a, ref, cfg["params"]["c_reduced"], cfg["mesh"]["face_cells"])
    if precision == rt.RT_FP64:
        assert max(e_ref.values()) <= 1e-10, e_ref
    else:
        m = mixed_errors(a, ref, cfg["params"]["c_reduced"])
        assert max(m[f"N[{k}] rel"] for k in range(3)) <= 1e-3 and m["x_HII abs"] <= 1e-4, m
        assert_other_fields(m)


def test_fused_photon_conservation_is_exact_to_rounding():
    """Transport only: the fused kernel computes a face state in every tile
    that needs it with the same code, so the two cells of a face still add
    and subtract the same flux and sum N V changes only by the rounding of
    the cell updates."""
    cfg = rtgen.travelling_wave(n=16, n_sub=20, amplitude=0.3)
    g = run_gpu(cfg, transport=rt.RT_TRANSPORT_FUSED)
    assert g["fused"]
    total0 = float(np.sum(cfg["state"]["N"][0] * cfg["mesh"]["volume"]))
    drift = abs(g["diag"]["photon_sum"][0] - total0) / total0
    say(f"fused fp64 conservation drift after 20 subcycles: {drift:.3e}")
    assert drift < 1e-13


def test_fused_on_a_cell_order_without_locality():
    """Random cell order: every neighbour is in another tile, so each tile's
    halo is as large as it can be.  AUTO picks the split path there; forcing
    the fused one must still give the oracle's answer."""
    cfg = ragged_hhe(order="random")
    auto = run_gpu(cfg, precision=rt.RT_MIXED)
    assert not auto["fused"]
    g = run_gpu(cfg, precision=rt.RT_MIXED, transport=rt.RT_TRANSPORT_FUSED)
    assert g["fused"]
    ref = oracle.run(cfg)
    m = mixed_errors(g, ref, cfg["params"]["c_reduced"])
    for k, v in m.items():
        say(f"  {k:16s} {v:.3e}")
    assert max(m[f"N[{k}] rel"] for k in range(3)) <= 1e-3 and m["x_HII abs"] <= 1e-4
    assert_other_fields(m)


def test_fused_on_the_staggered_mesh():
    """14-face cells; the path taken depends on the device's LDS per
    workgroup (the test reports it), the answer must not."""
    cfg = rtgen.expanding_hii(n=12, n_sub=8)
    ref = oracle.run(cfg)
    for prec in (rt.RT_FP64, rt.RT_MIXED):
        g = run_gpu(cfg, precision=prec)
        say("staggered mesh,", "fp64" if prec == rt.RT_FP64 else "mixed", "fused" if g["fused"] else "split")
        if prec == rt.RT_FP64:
            errs = field_errors(g, ref, cfg["params"]["c_reduced"], cfg["mesh"]["face_cells"])
            assert max(errs.values()) <= 1e-10, errs
        else:
            m = mixed_errors(g, ref, cfg["params"]["c_reduced"])
            assert max(m[f"N[{k}] rel"] for k in range(3)) <= 1e-3 and m["x_HII abs"] <= 1e-4, m
            assert_other_fields(m)


def test_transport_mode_errors():
    cfg = rtgen.stromgren(n=8, n_sub=1)
    m = rt.Mesh(cfg["mesh"])
    s = rt.State.from_config(m, cfg)
    with pytest.raises(rt.RtError) as e:
        s.set_transport(7)
    assert e.value.code == rt.RT_EINVAL
    s.set_transport(rt.RT_TRANSPORT_SPLIT)
    assert not s.fused
    c = s.clone()
    assert not c.fused
    c.close()
    s.close()
    m.close()
