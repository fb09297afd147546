"""rt_subcycle_noalloc against rt_subcycle through the C ABI.

The allocation-free entry point runs the same kernels with its partials in a
static device array, so its fields and diagnostics must equal rt_subcycle's
bit for bit.  Two calls in a row, the second on a smaller mesh, check that
what the first call left in the shared array does not leak into the second.
"""
import numpy as np
import pytest

import rtgen
from paper_2404_17630_amd import rt
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

FIELDS = ("N", "F", "species", "T")
DIAG = ("photon_sum", "guard_N", "guard_F", "adm_N", "adm_F", "flux_caps", "substeps", "max_substeps", "status",
        "n_subcycles", "dt")


def workload(dims, n_src, seed):
    """A ragged H+He lattice (tiles and slices with tails), 3 bins."""
    return rtgen.cosmological(0, 1.0, 1.0, n_src, 0.01, 4, 2, dims=dims, name=f"noalloc_{seed}")


def run_pair(cfg, precision, transport, n_sub):
    """The same state advanced by rt_subcycle and by rt_subcycle_noalloc."""
    m = rt.Mesh(cfg["mesh"])
    ref = rt.State.from_config(m, cfg, precision=precision)
    new = rt.State.from_config(m, cfg, precision=precision)
    ref.set_transport(transport)
    new.set_transport(transport)
    say("noalloc", cfg["name"], "cells", cfg["mesh"]["n_cells"], "precision", precision, "transport", transport,
        "subcycles", n_sub)
    ref.subcycle(n_sub)
    rt.rt_subcycle_noalloc(new.h, n_sub)
    a, b = ref.fields(), new.fields()
    da, db = ref.diagnostics(), new.diagnostics()
    for s in (ref, new):
        s.close()
    m.close()
    return a, b, da, db


def assert_same(a, b, da, db):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k
    for k in DIAG:
        assert np.array_equal(np.asarray(da[k]), np.asarray(db[k])), (k, da[k], db[k])


@pytest.mark.parametrize("precision", [rt.RT_FP64, rt.RT_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("transport", [rt.RT_TRANSPORT_SPLIT, rt.RT_TRANSPORT_FUSED], ids=["split", "fused"])
def test_noalloc_equals_subcycle_on_two_calls(precision, transport):
    big = workload((24, 20, 18), 8, 1)
    small = workload((9, 8, 7), 3, 2)
    assert small["mesh"]["n_cells"] < big["mesh"]["n_cells"]
    for cfg, n_sub in ((big, 3), (small, 2)):
        assert_same(*run_pair(cfg, precision, transport, n_sub))


def test_noalloc_does_not_restore_on_error():
    """A substep cap of 2 attempts fails the call (forced from the host):
    rt_subcycle restores the entry state, the allocation-free call keeps no
    entry copy and leaves the state advanced, and a later call on another
    state still matches rt_subcycle."""
    cfg = rtgen.stromgren(n=8, n_sub=2)
    p = dict(cfg["params"], chem_max_substeps=2)
    m = rt.Mesh(cfg["mesh"])
    st = cfg["state"]

    def make():
        return rt.State(m, p, rt.RT_FP64, st["N"], st["F"], st["n_H"], st["species"], st["T"],
                        cfg["sources"]["cell"], cfg["sources"]["rate"])

    s = make()
    before = s.fields()
    with pytest.raises(rt.RtError) as e:
        rt.rt_subcycle_noalloc(s.h, 3)
    assert e.value.code == rt.RT_ENUMERIC
    assert "not restored" in str(e.value)
    assert s.diagnostics()["status"] & 2
    after = s.fields()
    assert not np.array_equal(before["species"], after["species"])
    with pytest.raises(rt.RtError) as e:
        rt.rt_subcycle_noalloc(s.h, 1, dt=2.0 * s.info()["dt_cfl"])
    assert e.value.code == rt.RT_EINVAL
    s.close()
    m.close()
    assert_same(*run_pair(workload((9, 8, 7), 3, 3), rt.RT_MIXED, rt.RT_TRANSPORT_AUTO, 2))
