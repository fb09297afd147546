"""ctypes wrapper of the plain FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library; the only thing both sides consume is the seeded input
dicts built by ``rtgen``.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
LIB_PATH = HERE / "liboracle.so"
MAX_BINS = 8

_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)


class Params(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("nb", "chem_mode", "isothermal", "rate_set", "use_limiter",
                                         "chem_max_substeps")] + \
               [(n, C.c_double) for n in ("c_reduced", "cfl_eta", "T_iso", "Y_He", "alpha_B_const", "gamma",
                                          "chem_fmax", "chem_fs", "chem_growth", "chem_xfloor")] + \
               [("sigma", C.c_double * 3 * MAX_BINS), ("e_heat", C.c_double * 3 * MAX_BINS)]


class MeshC(C.Structure):
    _fields_ = [("nc", C.c_int64), ("volume", _f64p), ("centre", _f64p), ("nf", C.c_int64),
                ("face_cells", _i64p), ("area", _f64p), ("normal", _f64p), ("face_centre", _f64p),
                ("box", C.c_double * 3)]


class Diag(C.Structure):
    _fields_ = [("dt", C.c_double), ("photon_sum", C.c_double * MAX_BINS),
                ("guard_N", C.c_int64), ("guard_F", C.c_int64), ("adm_N", C.c_int64), ("adm_F", C.c_int64),
                ("flux_caps", C.c_int64), ("substeps", C.c_int64), ("max_substeps", C.c_int64),
                ("status", C.c_int32), ("loop_seconds", C.c_double)]

    def as_dict(self, nb: int) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "photon_sum"}
        d["photon_sum"] = np.array(self.photon_sum[:nb])
        return d


def build(force: bool = False) -> Path:
    """Compile the oracle with the host compiler (g++)."""
    import subprocess
    src = HERE / "m1rt_oracle.cpp"
    if force or not LIB_PATH.exists() or LIB_PATH.stat().st_mtime < max(src.stat().st_mtime,
                                                                       (HERE / "m1rt_oracle.h").stat().st_mtime):
        tmp = LIB_PATH.with_suffix(".so.tmp")
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               str(src), "-o", str(tmp)])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            build()
        L = C.CDLL(str(LIB_PATH))
        L.oracle_cfl_dt.restype = C.c_double
        L.oracle_cfl_dt.argtypes = [C.POINTER(MeshC), C.POINTER(Params)]
        L.oracle_run.restype = C.c_int
        L.oracle_run.argtypes = [C.POINTER(MeshC), C.POINTER(Params), _f64p, _f64p, _f64p, _f64p, _f64p,
                                 C.c_int64, _i64p, _f64p, C.c_int, C.c_double, C.POINTER(Diag)]
        L.oracle_run_jvp.restype = C.c_int
        L.oracle_run_jvp.argtypes = [C.POINTER(MeshC), C.POINTER(Params), _f64p, _f64p, _f64p, _f64p, _f64p,
                                     C.c_int64, _i64p, _f64p, C.c_int, C.c_double, C.c_int, _f64p, _f64p,
                                     _f64p, C.POINTER(Diag)]
        L.oracle_gradients.restype = C.c_int
        L.oracle_gradients.argtypes = [C.POINTER(MeshC), _f64p, C.c_int, _f64p]
        L.oracle_geometry.restype = C.c_int
        L.oracle_geometry.argtypes = [C.POINTER(MeshC), _f64p]
        L.oracle_chi.restype = C.c_double
        L.oracle_chi.argtypes = [C.c_double]
        L.oracle_hll_flux.restype = None
        L.oracle_hll_flux.argtypes = [_f64p, _f64p, _f64p, C.c_double, _f64p]
        L.oracle_chem_cell.restype = C.c_int
        L.oracle_chem_cell.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _f64p, _f64p, _f64p, _f64p,
                                       _i64p]
        L.oracle_rates.restype = None
        L.oracle_rates.argtypes = [C.POINTER(Params), C.c_double, _f64p]
        L.oracle_cooling.restype = C.c_double
        L.oracle_cooling.argtypes = [C.POINTER(Params), C.c_double, C.c_double, _f64p]
        L.oracle_set_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Host threads of the oracle's subcycle loop (1 = the plain loops; more
    give the same results bit for bit).  Returns the previous setting."""
    global _threads
    if lib().oracle_set_threads(int(n)) != 0:
        raise ValueError(f"threads={n}")
    prev, _threads = _threads, int(n)
    return prev


_threads = 1


def _ptr(a: np.ndarray, ty=_f64p):
    return a.ctypes.data_as(ty)


def make_params(p: dict) -> Params:
    out = Params()
    for k in ("nb", "chem_mode", "isothermal", "rate_set", "use_limiter", "chem_max_substeps"):
        setattr(out, k, int(p[k]))
    for k in ("c_reduced", "cfl_eta", "T_iso", "Y_He", "alpha_B_const", "gamma", "chem_fmax", "chem_fs",
              "chem_growth", "chem_xfloor"):
        setattr(out, k, float(p[k]))
    sig = np.asarray(p["sigma"], dtype=float).reshape(-1, 3)
    eh = np.asarray(p["e_heat"], dtype=float).reshape(-1, 3)
    for b in range(sig.shape[0]):
        for s in range(3):
            out.sigma[b][s] = sig[b, s]
            out.e_heat[b][s] = eh[b, s]
    return out


class _Mesh:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, m: dict):
        self.arrays = dict(
            volume=np.ascontiguousarray(m["volume"], dtype=np.float64),
            centre=np.ascontiguousarray(m["centre"], dtype=np.float64),
            face_cells=np.ascontiguousarray(m["face_cells"], dtype=np.int64),
            area=np.ascontiguousarray(m["area"], dtype=np.float64),
            normal=np.ascontiguousarray(m["normal"], dtype=np.float64),
            face_centre=np.ascontiguousarray(m["face_centre"], dtype=np.float64))
        a = self.arrays
        self.c = MeshC(int(m["n_cells"]), _ptr(a["volume"]), _ptr(a["centre"]), int(m["n_faces"]),
                       _ptr(a["face_cells"], _i64p), _ptr(a["area"]), _ptr(a["normal"]),
                       _ptr(a["face_centre"]), (C.c_double * 3)(*[float(x) for x in m["box"]]))


def cfl_dt(cfg: dict) -> float:
    m = _Mesh(cfg["mesh"])
    return lib().oracle_cfl_dt(C.byref(m.c), C.byref(make_params(cfg["params"])))


def _state_copy(cfg: dict) -> dict:
    st = cfg["state"]
    return dict(N=np.array(st["N"], dtype=np.float64, order="C"),
                F=np.array(st["F"], dtype=np.float64, order="C"),
                n_H=np.array(st["n_H"], dtype=np.float64, order="C"),
                species=np.array(st["species"], dtype=np.float64, order="C"),
                T=np.array(st["T"], dtype=np.float64, order="C"))


def run(cfg: dict, n_sub: int | None = None, dt: float = 0.0, rate_scale=None, check: bool = True) -> dict:
    """Run the oracle on a config; returns the final state and diagnostics."""
    p = cfg["params"]
    m = _Mesh(cfg["mesh"])
    st = _state_copy(cfg)
    cell = np.ascontiguousarray(cfg["sources"]["cell"], dtype=np.int64)
    rate = np.array(cfg["sources"]["rate"], dtype=np.float64, order="C").reshape(p["nb"], -1)
    if rate_scale is not None:
        rate = np.ascontiguousarray(rate * np.asarray(rate_scale)[None, :])
    d = Diag()
    n = cfg["n_subcycles"] if n_sub is None else n_sub
    rc = lib().oracle_run(C.byref(m.c), C.byref(make_params(p)), _ptr(st["N"]), _ptr(st["F"]), _ptr(st["n_H"]),
                          _ptr(st["species"]), _ptr(st["T"]), len(cell), _ptr(cell, _i64p), _ptr(rate), int(n),
                          float(dt), C.byref(d))
    if check and rc != 0:
        raise RuntimeError(f"oracle_run failed with status {rc}")
    st["diag"] = d.as_dict(p["nb"])
    st["rc"] = rc
    return st


def run_jvp(cfg: dict, dlnQ: np.ndarray, dln_nH: np.ndarray, n_sub: int | None = None, dt: float = 0.0,
            n_H=None, rate_scale=None) -> dict:
    """Forward-mode derivatives of the final x_HI along up to 8 directions of
    (ln Q per source, ln n_H per cell)."""
    p = cfg["params"]
    m = _Mesh(cfg["mesh"])
    st = _state_copy(cfg)
    if n_H is not None:
        st["n_H"] = np.ascontiguousarray(n_H, dtype=np.float64)
    cell = np.ascontiguousarray(cfg["sources"]["cell"], dtype=np.int64)
    rate = np.array(cfg["sources"]["rate"], dtype=np.float64, order="C").reshape(p["nb"], -1)
    if rate_scale is not None:
        rate = np.ascontiguousarray(rate * np.asarray(rate_scale)[None, :])
    dlnQ = np.ascontiguousarray(np.atleast_2d(dlnQ), dtype=np.float64)
    dln_nH = np.ascontiguousarray(np.atleast_2d(dln_nH), dtype=np.float64)
    ndir = dlnQ.shape[0]
    assert dln_nH.shape[0] == ndir and 1 <= ndir <= 8
    out = np.zeros((ndir, m.c.nc))
    d = Diag()
    n = cfg["n_subcycles"] if n_sub is None else n_sub
    rc = lib().oracle_run_jvp(C.byref(m.c), C.byref(make_params(p)), _ptr(st["N"]), _ptr(st["F"]),
                              _ptr(st["n_H"]), _ptr(st["species"]), _ptr(st["T"]), len(cell), _ptr(cell, _i64p),
                              _ptr(rate), int(n), float(dt), ndir, _ptr(dlnQ), _ptr(dln_nH), _ptr(out), C.byref(d))
    if rc != 0:
        raise RuntimeError(f"oracle_run_jvp failed with status {rc}")
    st["dxHI"] = out
    st["diag"] = d.as_dict(p["nb"])
    return st


def gradients(mesh: dict, phi: np.ndarray, use_limiter: bool) -> np.ndarray:
    m = _Mesh(mesh)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros((3, m.c.nc))
    if lib().oracle_gradients(C.byref(m.c), _ptr(phi), int(use_limiter), _ptr(out)) != 0:
        raise RuntimeError("bad mesh")
    return out


def geometry_minv(mesh: dict) -> np.ndarray:
    m = _Mesh(mesh)
    out = np.zeros((6, m.c.nc))
    if lib().oracle_geometry(C.byref(m.c), _ptr(out)) != 0:
        raise RuntimeError("bad mesh")
    return out


def chi(f: float) -> float:
    return lib().oracle_chi(float(f))


def hll_flux(UL, UR, n, c: float) -> np.ndarray:
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    out = np.zeros(4)
    lib().oracle_hll_flux(_ptr(UL), _ptr(UR), _ptr(n), float(c), _ptr(out))
    return out


def chem_cell(params: dict, dt: float, n_H: float, N, Fh, x, T: float) -> dict:
    nb = params["nb"]
    N = np.array(N, dtype=np.float64).reshape(nb)
    Fh = np.array(Fh, dtype=np.float64).reshape(nb, 3).copy()
    x = np.array(x, dtype=np.float64).reshape(5)
    Tv = np.array([T], dtype=np.float64)
    att = np.zeros(1, dtype=np.int64)
    rc = lib().oracle_chem_cell(C.byref(make_params(params)), float(dt), float(n_H), _ptr(N), _ptr(Fh), _ptr(x),
                                _ptr(Tv), _ptr(att, _i64p))
    return dict(N=N, Fh=Fh, x=x, T=float(Tv[0]), attempts=int(att[0]), rc=rc)


def rates(params: dict, T: float) -> dict:
    out = np.zeros(7)
    lib().oracle_rates(C.byref(make_params(params)), float(T), _ptr(out))
    return dict(zip(("aHII", "aHeII", "aHeIII", "bHI", "bHeI", "bHeII", "ad"), out))


def cooling(params: dict, T: float, n_H: float, x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().oracle_cooling(C.byref(make_params(params)), float(T), float(n_H), _ptr(x))
