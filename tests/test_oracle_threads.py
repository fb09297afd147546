"""The oracle's threaded subcycle against its single-thread loops.

With more than one host thread the face loop becomes a pass over the faces
and a per-cell pass that adds each cell's faces in face-index order, the
order in which the single-thread face loop adds them, so every field, every
counter and every forward derivative must be the same bit for bit.  The
workload is a ragged H+He lattice on which the cap, the admissibility fix
and the guards fire."""
import numpy as np
import pytest

import oracle
import rtgen


@pytest.fixture
def threads():
    yield
    oracle.set_threads(1)


def ragged():
    return rtgen.cosmological(0, 1.0, 1.0, 6, 0.01, 4, 2, dims=(20, 18, 17), name="threads")


def test_threaded_run_is_bitwise_the_single_thread_run(threads):
    cfg = ragged()
    a = oracle.run(cfg)
    assert a["diag"]["flux_caps"] > 0 and a["diag"]["adm_F"] > 0 and a["diag"]["guard_F"] > 0
    for n in (2, 5):
        oracle.set_threads(n)
        b = oracle.run(cfg)
        for k in ("N", "F", "species", "T"):
            assert np.array_equal(a[k], b[k]), (n, k)
        for k in ("adm_N", "adm_F", "flux_caps", "guard_N", "guard_F", "substeps", "max_substeps", "status"):
            assert a["diag"][k] == b["diag"][k], (n, k)
        assert np.array_equal(a["diag"]["photon_sum"], b["diag"]["photon_sum"])


def test_threaded_jvp_is_bitwise_the_single_thread_jvp(threads):
    cfg = ragged()
    rng = np.random.default_rng(7)
    nc, ns = cfg["mesh"]["n_cells"], len(cfg["sources"]["cell"])
    dq = rng.normal(size=(2, ns))
    dn = rng.normal(size=(2, nc))
    a = oracle.run_jvp(cfg, dq, dn, n_sub=2)
    oracle.set_threads(4)
    b = oracle.run_jvp(cfg, dq, dn, n_sub=2)
    assert np.array_equal(a["dxHI"], b["dxHI"])
    assert np.array_equal(a["species"], b["species"])


def test_substep_cap_reported_with_threads(threads):
    cfg = rtgen.stromgren(n=8, n_sub=2)
    cfg["params"] = dict(cfg["params"], chem_max_substeps=2)
    oracle.set_threads(3)
    with pytest.raises(RuntimeError):
        oracle.run(cfg)


def test_derivative_run_advances_the_same_state():
    """The forward-mode run holds some derivatives constant but no value: its
    primal state equals the plain run's (to the rounding of the isotropic
    Eddington tensor it takes for |Fh|^2 <= 1e-16 N^2)."""
    cfg = ragged()
    nc, ns = cfg["mesh"]["n_cells"], len(cfg["sources"]["cell"])
    rng = np.random.default_rng(8)
    a = oracle.run(cfg)
    b = oracle.run_jvp(cfg, rng.normal(size=(1, ns)), rng.normal(size=(1, nc)))
    for k in ("species", "T"):
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-300), k
    for bb in range(3):
        ref = a["N"][bb]
        assert np.max(np.abs(b["N"][bb] - ref) / np.maximum(ref, 1e-6 * ref.max())) < 1e-12
    assert np.all(np.isfinite(b["dxHI"]))
