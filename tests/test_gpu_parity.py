"""GPU parity of the FP64 path (through the C ABI) against the CPU oracle:
1e-10 relative per element, field and bin (scale: the value itself, floored
at 1e-6 of the largest value in its stencil and at 1e-10 of the field's
maximum, see tests/gpu_common.field_errors), plus determinism, conservation
and the documented error paths."""
import numpy as np
import pytest

import oracle
import rtgen
from paper_2404_17630_amd import rt
from tests.gpu_common import cached_oracle_run, field_errors, rel_err, run_gpu, say

pytestmark = pytest.mark.gpu

TOL = 1e-10


def assert_parity(cfg, gpu, ref, tol=TOL):
    errs = field_errors(gpu, ref, cfg["params"]["c_reduced"], cfg["mesh"]["face_cells"])
    worst = max(errs, key=errs.get)
    say(cfg["name"], "worst", worst, f"{errs[worst]:.3e}")
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    # photon sums per bin
    assert np.allclose(gpu["diag"]["photon_sum"], ref["diag"]["photon_sum"], rtol=1e-12, atol=0)
    assert gpu["diag"]["dt"] == pytest.approx(ref["diag"]["dt"], rel=1e-14, abs=0.0)
    say(cfg["name"], "caps gpu", gpu["diag"]["flux_caps"], "oracle", ref["diag"]["flux_caps"],
        "adm_F", gpu["diag"]["adm_F"], ref["diag"]["adm_F"], "guard_F", gpu["diag"]["guard_F"], ref["diag"]["guard_F"])


def test_stromgren_fp64_matches_oracle():
    cfg = rtgen.stromgren()
    say("stromgren 32^3, 100 subcycles, fp64")
    gpu = run_gpu(cfg)
    ref = oracle.run(cfg)
    assert_parity(cfg, gpu, ref)
    # same controller path: identical attempt counts
    assert gpu["diag"]["substeps"] == ref["diag"]["substeps"]
    assert gpu["diag"]["max_substeps"] == ref["diag"]["max_substeps"]
    # The guard and admissibility counters count decisions taken on values at
    # rounding level: a limited face state aimed exactly at a neighbour's
    # N = 0 lands on -1e-30 or +1e-30 depending on the order of its sums, and
    # a free-streaming cell's |Fh| equals N to the last bit.  They are
    # reported, not compared; the fields above are the parity check.
    for k in ("guard_N", "guard_F", "adm_N", "adm_F", "flux_caps"):
        say(f"  {k}: gpu {gpu['diag'][k]} oracle {ref['diag'][k]}")


@pytest.mark.parametrize("order", ["hilbert", "random"])
def test_hhe_ragged_mesh_matches_oracle(order):
    """H+He, 3 bins, evolving T on a 20x18x17 lattice (6120 cells: several
    256-cell blocks and a ragged last wavefront), two sources in one cell."""
    cfg = rtgen.cosmological(0, 1.0, 1.0, 6, 0.01, 8, 2, dims=(20, 18, 17), order=order, name="hhe_ragged")
    cfg["sources"]["cell"][1] = cfg["sources"]["cell"][0]
    say("hhe ragged", order)
    gpu = run_gpu(cfg)
    ref = oracle.run(cfg)
    assert_parity(cfg, gpu, ref)
    assert gpu["diag"]["substeps"] == ref["diag"]["substeps"]


def test_transport_only_travelling_wave():
    cfg = rtgen.travelling_wave(n=12, n_sub=10, amplitude=0.1)
    say("travelling wave")
    gpu = run_gpu(cfg)
    ref = oracle.run(cfg)
    assert_parity(cfg, gpu, ref)


def test_photon_conservation_on_gpu():
    """Optically thin periodic transport conserves sum N V to rounding: each
    face flux is computed bit-identically by both of its cells."""
    cfg = rtgen.travelling_wave(n=16, n_sub=1, amplitude=0.1)
    V = cfg["mesh"]["volume"]
    total0 = float(np.sum(cfg["state"]["N"][0] * V))
    m = rt.Mesh(cfg["mesh"])
    s = rt.State.from_config(m, cfg)
    for k in range(20):
        s.subcycle(1)
        tot = s.diagnostics()["photon_sum"][0]
        assert abs(tot - total0) <= 1e-14 * total0 * (k + 1)
    s.close()
    m.close()


def test_single_subcycle_pieces():
    """One subcycle at a time for a few steps: catches an error that a long run
    could average out."""
    cfg = rtgen.cosmological(0, 1.0, 1.5, 4, 0.1, 1, 4, dims=(16, 16, 16), name="pieces")
    m = rt.Mesh(cfg["mesh"])
    s = rt.State.from_config(m, cfg)
    st = cfg
    for k in range(4):
        s.subcycle(1)
        g = s.fields()
        g["diag"] = s.diagnostics()
        ref = oracle.run(st, n_sub=1)
        assert_parity(cfg, g, ref)
        st = dict(cfg, state=dict(N=ref["N"], F=ref["F"], n_H=ref["n_H"], species=ref["species"], T=ref["T"]))
    s.close()
    m.close()


def test_determinism_bitwise():
    cfg = rtgen.cosmological(0, 1.0, 1.0, 6, 0.01, 6, 2, dims=(24, 24, 24), name="det")
    a = run_gpu(cfg)
    b = run_gpu(cfg)
    for k in ("N", "F", "species", "T"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["diag"]["photon_sum"], b["diag"]["photon_sum"])


def test_full_size_hhe_2m_all_subcycles():
    """The 2.1M-cell H+He workload at full size (3 bins, sigma_ln = 1.0, 256
    sources) over all 50 subcycles against the oracle (run on the host's
    threads, bitwise its single-thread result), then the invariants."""
    say("hhe_2m full size: generating")
    cfg = rtgen.hhe_2m()
    say("hhe_2m: gpu 50 subcycles")
    full = run_gpu(cfg)
    say("hhe_2m: oracle 50 subcycles on the host's threads")
    ref = cached_oracle_run("hhe_2m", cfg)
    assert_parity(cfg, full, ref)
    assert full["diag"]["substeps"] == ref["diag"]["substeps"]
    x = full["species"]
    assert np.all((x >= 0) & (x <= 1))
    assert np.abs(x[0] + x[1] - 1).max() < 1e-13
    assert np.abs(x[2:].sum(0) - 1).max() < 1e-13
    assert np.all(full["T"] > 0) and np.all(full["N"] >= 0)
    # |Fh| <= N, down to the level where the guards' squared norms underflow
    Fm = np.sqrt(((full["F"] / cfg["params"]["c_reduced"]) ** 2).sum(1))
    assert np.all(Fm <= full["N"] * (1 + 1e-12) + 1e-150)
    assert full["diag"]["status"] == 0


def test_clone_and_fields_roundtrip():
    cfg = rtgen.cosmological(0, 1.0, 1.0, 3, 0.01, 3, 2, dims=(8, 8, 8), name="clone")
    m = rt.Mesh(cfg["mesh"])
    s = rt.State.from_config(m, cfg)
    s.subcycle(2)
    c = s.clone()
    s.subcycle(1)
    c.subcycle(1)
    for f in (rt.RT_FIELD_N, rt.RT_FIELD_F, rt.RT_FIELD_SPECIES, rt.RT_FIELD_T):
        assert np.array_equal(s.get(f), c.get(f))
    # set/get round trip
    N = s.get(rt.RT_FIELD_N) * 1.5
    s.set(rt.RT_FIELD_N, N)
    assert np.array_equal(s.get(rt.RT_FIELD_N), N)
    T = s.get(rt.RT_FIELD_T)
    s.set(rt.RT_FIELD_T, T * 2)
    assert np.allclose(s.get(rt.RT_FIELD_T), 2 * T, rtol=1e-14)
    info = s.info()
    assert info["n_cells"] == 512 and info["nb"] == 3 and info["n_src"] == 3
    c.close()
    s.close()
    m.close()


def test_error_paths():
    cfg = rtgen.stromgren(n=8, n_sub=2)
    m = rt.Mesh(cfg["mesh"])
    s = rt.State.from_config(m, cfg)
    dt = s.info()["dt_cfl"]
    with pytest.raises(rt.RtError) as e:
        s.subcycle(1, dt=1.01 * dt)
    assert e.value.code == rt.RT_EINVAL
    # substep cap: the call fails and the state is unchanged
    p = dict(cfg["params"], chem_max_substeps=2)
    s2 = rt.State(m, p, rt.RT_FP64, cfg["state"]["N"], cfg["state"]["F"], cfg["state"]["n_H"],
                  cfg["state"]["species"], cfg["state"]["T"], cfg["sources"]["cell"], cfg["sources"]["rate"])
    before = s2.fields()
    with pytest.raises(rt.RtError) as e:
        s2.subcycle(3)      # ionising the source cell needs many more attempts
    assert e.value.code == rt.RT_ENUMERIC
    after = s2.fields()
    for k in ("N", "F", "species", "T"):
        assert np.array_equal(before[k], after[k]), k
    assert s2.diagnostics()["status"] & 2
    # invalid inputs at create
    bad = np.array(cfg["state"]["N"])
    bad[0, 3] = np.nan
    with pytest.raises(rt.RtError) as e:
        rt.State(m, cfg["params"], rt.RT_FP64, bad, cfg["state"]["F"], cfg["state"]["n_H"],
                 cfg["state"]["species"], cfg["state"]["T"], cfg["sources"]["cell"], cfg["sources"]["rate"])
    assert e.value.code == rt.RT_EINVAL
    with pytest.raises(rt.RtError) as e:
        rt.State(m, cfg["params"], rt.RT_FP64, cfg["state"]["N"], cfg["state"]["F"], cfg["state"]["n_H"],
                 cfg["state"]["species"], cfg["state"]["T"], np.array([cfg["mesh"]["n_cells"]]),
                 cfg["sources"]["rate"])
    assert e.value.code == rt.RT_EINVAL
    with pytest.raises(rt.RtError) as e:
        rt.State(m, dict(cfg["params"], nb=9), rt.RT_FP64, cfg["state"]["N"], cfg["state"]["F"],
                 cfg["state"]["n_H"], cfg["state"]["species"], cfg["state"]["T"], cfg["sources"]["cell"],
                 cfg["sources"]["rate"])
    assert e.value.code == rt.RT_EINVAL
    s2.close()
    s.close()
    m.close()


def test_no_sources_and_zero_subcycles():
    cfg = rtgen.travelling_wave(n=6, n_sub=0)
    gpu = run_gpu(cfg)
    assert np.array_equal(gpu["N"], cfg["state"]["N"])
    gpu = run_gpu(cfg, n_sub=3)
    ref = oracle.run(cfg, n_sub=3)
    assert rel_err(gpu["N"][0], ref["N"][0]) < TOL


@pytest.mark.parametrize("mode", [rt.RT_TRANSPORT_FUSED, rt.RT_TRANSPORT_SPLIT], ids=["fused", "split"])
def test_profile_counters(mode):
    cfg = rtgen.stromgren(n=8, n_sub=5)
    g = run_gpu(cfg, profile=True, transport=mode)
    prof = g["profile"]
    assert g["fused"] == (mode == rt.RT_TRANSPORT_FUSED)
    ran = [rt.RT_KERNEL_SOURCES, rt.RT_KERNEL_CHEM]
    idle = []
    if g["fused"]:
        ran.append(rt.RT_KERNEL_TRANSPORT)
        idle += [rt.RT_KERNEL_GRADIENT, rt.RT_KERNEL_FLUX]
    else:
        ran += [rt.RT_KERNEL_GRADIENT, rt.RT_KERNEL_FLUX]
        idle.append(rt.RT_KERNEL_TRANSPORT)
    for k in ran:
        assert prof[k][0] == 5 and prof[k][1] > 0
    for k in idle:
        assert prof[k][0] == 0
    assert prof[rt.RT_KERNEL_REDUCE][0] == 1


def test_many_block_mesh_matches_oracle():
    """81^3 = 531,441 cells, 3 bins, 2 FP64 subcycles: 2,076 partial rows
    per bin, so each first-stage workgroup of the reduction folds several;
    two cells a lane in the chemistry, so lanes refill from the workgroup's
    counter.  Fields, photon sums and attempt counts against the oracle."""
    cfg = rtgen.cosmological(81, 1.0, 1.0, 32, 0.01, 2, 7, name="blocks_531k")
    say("81^3, 2 subcycles, fp64")
    gpu = run_gpu(cfg)
    ref = oracle.run(cfg)
    assert_parity(cfg, gpu, ref)
    assert gpu["diag"]["substeps"] == ref["diag"]["substeps"]
    assert gpu["diag"]["max_substeps"] == ref["diag"]["max_substeps"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_chemistry_cells_per_lane_leaves_results_unchanged(precision):
    """The chemistry's share of cells per lane (rt_params.chem_cells_per_lane)
    changes only which lane integrates a cell: on an I-front workload one
    cell per lane (no refill), 7 and 1024 per lane give the default's fields,
    attempt counts and diagnostics bit for bit; values outside 0..1024 are
    refused."""
    cfg = rtgen.cosmological(0, 1.0, 1.0, 6, 0.01, 4, 3, dims=(20, 18, 17), name="per_lane")
    m = rt.Mesh(cfg["mesh"])
    prec = rt.RT_FP64 if precision == "fp64" else rt.RT_MIXED
    out = []
    for per_lane in (0, 1, 7, 1024):
        c = dict(cfg, params=dict(cfg["params"], chem_cells_per_lane=per_lane))
        s = rt.State.from_config(m, c, precision=prec)
        s.subcycle(cfg["n_subcycles"])
        out.append((s.fields(), s.attempts(), s.diagnostics()))
        s.close()
    f0, a0, d0 = out[0]
    for f, a, d in out[1:]:
        for k in ("N", "F", "species", "T"):
            assert np.array_equal(f[k], f0[k]), k
        assert np.array_equal(a, a0)
        assert d["substeps"] == d0["substeps"] and d["max_substeps"] == d0["max_substeps"]
    for bad in (-1, 1025):
        c = dict(cfg, params=dict(cfg["params"], chem_cells_per_lane=bad))
        with pytest.raises(rt.RtError) as e:
            rt.State.from_config(m, c, precision=prec)
        assert e.value.code == rt.RT_EINVAL
    m.close()


def test_per_cell_attempt_counts():
    """RT_FIELD_ATTEMPTS: each cell's chemistry attempts over the last call.
    They add up to the call's total, every cell takes at least one attempt a
    subcycle, the source cell at the ionisation front takes the most, and the
    counts start from zero at every call."""
    cfg = rtgen.cosmological(0, 1.0, 1.0, 6, 0.01, 4, 2, dims=(20, 18, 17), name="attempts")
    m = rt.Mesh(cfg["mesh"])
    s = rt.State.from_config(m, cfg)
    for n in (4, 1):
        s.subcycle(n)
        att = s.attempts()
        d = s.diagnostics()
        assert att.sum() == d["substeps"], (att.sum(), d["substeps"])
        assert att.min() >= n
        assert att.max() >= d["max_substeps"]
    with pytest.raises(rt.RtError) as e:
        s.set(rt.RT_FIELD_ATTEMPTS, np.zeros(cfg["mesh"]["n_cells"]))
    assert e.value.code == rt.RT_EINVAL
    s.close()
    m.close()


def lit_random_state(use_limiter: int) -> dict:
    """Pure transport (no chemistry or absorption, no sources) on the 12^3
    Strömgren lattice from a lit random state: N log-uniform over four
    decades in every cell, F in a random direction at a uniform fraction of
    c~N up to 0.99.  No cell is empty, so every cap, admissibility and guard
    decision compares values of their own size: none sits at rounding
    level."""
    cfg = rtgen.stromgren(n=12, n_sub=3)
    p = cfg["params"]
    nb, nc = p["nb"], cfg["mesh"]["n_cells"]
    cfg["params"] = dict(p, chem_mode=rtgen.CHEM_NONE, sigma=np.zeros((nb, 3)), use_limiter=use_limiter)
    rng = np.random.default_rng(5)
    N = 10.0 ** rng.uniform(-2, 2, size=(nb, nc))
    u = rng.normal(size=(nb, 3, nc))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    F = u * (rng.uniform(0, 0.99, size=(nb, nc)) * p["c_reduced"] * N)[:, None, :]
    cfg["state"] = dict(cfg["state"], N=N, F=F)
    cfg["sources"] = dict(cell=np.zeros(0, np.int64), rate=np.zeros((nb, 0)))
    return cfg


@pytest.mark.parametrize("use_limiter", [1, 0])
def test_counters_equal_the_oracle_on_a_lit_random_state(use_limiter):
    """Three subcycles from lit_random_state: the cap, admissibility and
    guard counts of the FP64 form equal the oracle's exactly, on the default
    split transport and on the fused one (with the limiter off the face
    states' N goes negative and its admissibility fix fires too); the mixed
    form's counts are within 1% of them."""
    cfg = lit_random_state(use_limiter)
    ref = oracle.run(cfg)
    keys = ("flux_caps", "adm_N", "adm_F", "guard_N", "guard_F")
    want = {k: ref["diag"][k] for k in keys}
    assert want["flux_caps"] > 0 and want["adm_F"] > 0 and want["guard_F"] > 0, want
    if not use_limiter:
        assert want["adm_N"] > 0, want
    for mode in (rt.RT_TRANSPORT_SPLIT, rt.RT_TRANSPORT_FUSED):
        gpu = run_gpu(cfg, precision=rt.RT_FP64, transport=mode)
        assert_parity(cfg, gpu, ref)
        got = {k: gpu["diag"][k] for k in keys}
        say(f"limiter {use_limiter} transport {mode}: gpu {got} oracle {want}")
        assert got == want
    mix = run_gpu(cfg, precision=rt.RT_MIXED)
    got = {k: mix["diag"][k] for k in keys}
    say(f"limiter {use_limiter} mixed: {got}")
    for k in keys:
        assert abs(got[k] - want[k]) <= 0.01 * want[k], (k, got, want)


def test_limiter_counters_fire_on_a_free_streaming_front():
    """The cap, admissibility and guard counters on pure transport from a
    point source: the free-streaming front is capped (theta = 0.9 on a face
    it leaves through) and its extrapolated states need the admissibility
    fix, in both implementations.  The counts themselves are not compared:
    the HLL flux of a free-streaming state is a difference of terms of its
    size, which leaves rounding-residue states (1e-18 of the maximum and
    below) from the second subcycle on, and the limited face state of a
    cell next to an empty one is its neighbour's 0 plus a rounding residue
    of either sign.  Measured here: caps 299 (GPU) against 412 (oracle),
    admissibility fixes of N 178 against 412, while every field agrees to
    the parity bar."""
    cfg = rtgen.stromgren(n=16, n_sub=8)
    cfg["params"] = dict(cfg["params"], chem_mode=rtgen.CHEM_NONE, sigma=np.zeros((1, 3)))
    gpu = run_gpu(cfg)
    ref = oracle.run(cfg)
    assert_parity(cfg, gpu, ref)
    keys = ("flux_caps", "adm_N", "adm_F", "guard_N", "guard_F")
    say("counters gpu", {k: gpu["diag"][k] for k in keys}, "oracle", {k: ref["diag"][k] for k in keys})
    n_faces = cfg["mesh"]["n_faces"] * cfg["n_subcycles"]
    for d in (gpu["diag"], ref["diag"]):
        assert 0 < d["flux_caps"] < n_faces and 0 < d["adm_F"] < 2 * n_faces
