"""Host-only checks of the C ABI library: it loads, exports every function
that include/rt.h declares, its constants match the binding, and mesh
validation reports the documented error codes without touching a GPU."""
import re
from pathlib import Path

import numpy as np
import pytest

import rtgen
from paper_2404_17630_amd import rt

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "rt.h"


def declared_functions():
    text = HEADER.read_text()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*|double)\s+(rt_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    L = rt.lib()
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(L, n), n
    bound = {s[0] for s in rt._SIGNATURES}
    assert set(names) == bound


def test_header_constants_match_binding():
    text = HEADER.read_text()
    defs = dict(re.findall(r"#define\s+(RT_\w+)\s+(-?\d+)", text))
    for name, val in defs.items():
        if hasattr(rt, name):
            assert getattr(rt, name) == int(val), name
    assert int(defs["RT_MAX_BINS"]) == rt.MAX_BINS


def test_params_default():
    p = rt.rt_params_default(3)
    assert p.nb == 3 and p.cfl_eta == 0.3 and p.chem_fmax == 0.1 and p.chem_fs == 0.05
    assert p.chem_growth == 2.0 and p.chem_xfloor == 1e-6 and p.chem_max_substeps == 100000
    assert p.chem_cells_per_lane == 0 and p.reserved0 == 0
    assert rt.rt_params.c_reduced.offset == 32          # eight int32, then the doubles, as in rt.h
    with pytest.raises(rt.RtError) as e:
        rt.rt_params_default(0)
    assert e.value.code == rt.RT_EINVAL
    with pytest.raises(rt.RtError):
        rt.rt_params_default(rt.MAX_BINS + 1)


def mesh_arrays():
    m = rtgen.jittered_lattice((4, 4, 4), 1.0, 0.2, 1, "hilbert").as_dict()
    return {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in m.items()}


def create(m, device=0):
    return rt.rt_mesh_create(m["n_cells"], np.ascontiguousarray(m["volume"]), np.ascontiguousarray(m["centre"]),
                             m["n_faces"], np.ascontiguousarray(m["face_cells"]), np.ascontiguousarray(m["area"]),
                             np.ascontiguousarray(m["normal"]), np.ascontiguousarray(m["face_centre"]), m["box"],
                             device)


@pytest.mark.parametrize("breakage,code", [
    ("index", rt.RT_EMESH), ("self", rt.RT_EMESH), ("area", rt.RT_EMESH), ("volume", rt.RT_EMESH),
    ("normal", rt.RT_EMESH), ("few_faces", rt.RT_EMESH), ("singular", rt.RT_EMESH), ("size", rt.RT_EINVAL),
])
def test_mesh_validation_errors(breakage, code):
    m = mesh_arrays()
    if breakage == "index":
        m["face_cells"][1, 5] = m["n_cells"]
    elif breakage == "self":
        m["face_cells"][1, 5] = m["face_cells"][0, 5]
    elif breakage == "area":
        m["area"][3] = 0.0
    elif breakage == "volume":
        m["volume"][2] = -1.0
    elif breakage == "normal":
        m["normal"][:, 7] *= 1.0 + 1e-9
    elif breakage == "few_faces":
        # drop the +x, +y, +z faces of cell 0: three faces remain
        keep = np.ones(m["n_faces"], bool)
        keep[[0, 1, 2]] = False
        for k in ("face_cells", "normal", "face_centre"):
            m[k] = np.ascontiguousarray(m[k][:, keep])
        m["area"] = np.ascontiguousarray(m["area"][keep])
        m["n_faces"] = int(keep.sum())
    elif breakage == "singular":
        # every neighbour of cell 0 (and every face centre of cell 0) at the
        # height of cell 0: all separations lie in a plane, M_0 is singular
        fc = m["face_cells"]
        for f in range(m["n_faces"]):
            if 0 in fc[:, f]:
                other = fc[1, f] if fc[0, f] == 0 else fc[0, f]
                m["centre"][2, other] = m["centre"][2, 0]
                m["face_centre"][2, f] = m["centre"][2, 0]
    elif breakage == "size":
        m["n_cells"] = 0
    with pytest.raises(rt.RtError) as e:
        create(m)
    assert e.value.code == code, str(e.value)


def test_valid_mesh_reaches_device_check_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(rt.RtError) as e:
        create(mesh_arrays())
    assert e.value.code == rt.RT_EDEVICE
