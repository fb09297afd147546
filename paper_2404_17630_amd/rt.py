"""ctypes binding of the C ABI in ``include/rt.h`` (argument marshalling only).

Every step of the subcycle runs in ``librt_m1.so``; this module converts
numpy arrays / torch tensors to pointers, raises ``RtError`` on a non-zero
status, and offers two small owning wrappers (``Mesh``, ``State``).  The
library must be built (``python -m paper_2404_17630_amd.build``): importing
the functions below without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "librt_m1.so"
MAX_BINS = 8

RT_OK, RT_EINVAL, RT_EMESH, RT_ESTATE, RT_EDEVICE, RT_ENOMEM, RT_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
RT_FP64, RT_MIXED = 0, 1
RT_CHEM_NONE, RT_CHEM_H, RT_CHEM_HHE = 0, 1, 2
RT_RATES_CASEB_CONST, RT_RATES_HG97 = 0, 1
RT_FIELD_N, RT_FIELD_F, RT_FIELD_NH, RT_FIELD_SPECIES, RT_FIELD_T, RT_FIELD_ATTEMPTS = 0, 1, 2, 3, 4, 5
RT_KERNEL_SOURCES, RT_KERNEL_CHEM, RT_KERNEL_GRADIENT, RT_KERNEL_FLUX, RT_KERNEL_REDUCE = 0, 1, 2, 3, 4
RT_KERNEL_TRANSPORT = 5
RT_N_KERNELS = 6
KERNEL_NAMES = ("k_sources", "k_chem", "k_facestate", "k_flux", "k_reduce", "k_transport")
RT_TRANSPORT_AUTO, RT_TRANSPORT_FUSED, RT_TRANSPORT_SPLIT = 0, 1, 2
RT_DEVICE_HOST_ONLY = -1
RT_TILE_CELLS = 256
RT_NOALLOC_SCRATCH_MB = 64
TABLES = ("nbr", "fsf", "opp", "sptr", "sdeg", "lds_opp", "halo_ptr", "halo_cell", "hside_ptr", "hside_entry",
          "fitem_ptr", "fitem", "tpair_ptr", "tpair", "tbnd_ptr", "tbnd", "tbnd_sptr")

ERROR_NAMES = {RT_EINVAL: "RT_EINVAL", RT_EMESH: "RT_EMESH", RT_ESTATE: "RT_ESTATE", RT_EDEVICE: "RT_EDEVICE",
               RT_ENOMEM: "RT_ENOMEM", RT_ENUMERIC: "RT_ENUMERIC"}


class RtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class rt_params(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("nb", "chem_mode", "isothermal", "rate_set", "use_limiter",
                                         "chem_max_substeps", "chem_cells_per_lane", "reserved0")] + \
               [(n, C.c_double) for n in ("c_reduced", "cfl_eta", "T_iso", "Y_He", "alpha_B_const", "gamma",
                                          "chem_fmax", "chem_fs", "chem_growth", "chem_xfloor")] + \
               [("sigma", C.c_double * 3 * MAX_BINS), ("e_heat", C.c_double * 3 * MAX_BINS)]


class rt_diag(C.Structure):
    _fields_ = [("dt", C.c_double), ("photon_sum", C.c_double * MAX_BINS), ("scale", C.c_double * MAX_BINS),
                ("guard_N", C.c_int64), ("guard_F", C.c_int64), ("adm_N", C.c_int64), ("adm_F", C.c_int64),
                ("flux_caps", C.c_int64), ("substeps", C.c_int64), ("max_substeps", C.c_int64),
                ("status", C.c_int32), ("n_subcycles", C.c_int32)]

    def as_dict(self, nb: int) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("photon_sum", "scale")}
        d["photon_sum"] = np.array(self.photon_sum[:nb])
        d["scale"] = np.array(self.scale[:nb])
        return d


_vp = C.c_void_p
_lib = None

# (name, restype, argtypes) of every exported function.
_SIGNATURES = [
    ("rt_last_error", C.c_char_p, []),
    ("rt_params_default", C.c_int, [C.c_int32, C.POINTER(rt_params)]),
    ("rt_mesh_create", C.c_int, [C.c_int64, _vp, _vp, C.c_int64, _vp, _vp, _vp, _vp, C.POINTER(C.c_double),
                                 C.c_int, C.POINTER(_vp)]),
    ("rt_mesh_destroy", C.c_int, [_vp]),
    ("rt_mesh_table", C.c_int, [_vp, C.c_int, C.POINTER(C.POINTER(C.c_int32)), C.POINTER(C.c_int64)]),
    ("rt_state_create", C.c_int, [_vp, C.POINTER(rt_params), C.c_int, _vp, _vp, _vp, _vp, _vp, C.c_int64, _vp,
                                  _vp, C.POINTER(_vp)]),
    ("rt_state_clone", C.c_int, [_vp, C.POINTER(_vp)]),
    ("rt_state_destroy", C.c_int, [_vp]),
    ("rt_subcycle", C.c_int, [_vp, C.c_int, C.c_double, _vp]),
    ("rt_subcycle_noalloc", C.c_int, [_vp, C.c_int, C.c_double, _vp]),
    ("rt_subcycle_adjoint", C.c_int, [_vp, C.c_int, C.c_int, C.c_double, _vp, _vp, _vp, _vp]),
    ("rt_state_get_field", C.c_int, [_vp, C.c_int, _vp, C.c_int]),
    ("rt_state_set_field", C.c_int, [_vp, C.c_int, _vp, C.c_int]),
    ("rt_state_info", C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("rt_state_set_transport", C.c_int, [_vp, C.c_int]),
    ("rt_state_transport", C.c_int, [_vp, C.POINTER(C.c_int32)]),
    ("rt_state_diagnostics", C.c_int, [_vp, C.POINTER(rt_diag)]),
    ("rt_profile_enable", C.c_int, [_vp, C.c_int]),
    ("rt_profile_reset", C.c_int, [_vp]),
    ("rt_profile_read", C.c_int, [_vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
]


def lib():
    """Load librt_m1.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2404_17630_amd.build`")
        L = C.CDLL(str(LIB_PATH))
        for name, res, args in _SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != RT_OK:
        raise RtError(rc, lib().rt_last_error().decode())


def _ptr(a, dtype):
    """Pointer of a contiguous numpy array or torch tensor (host or device)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):           # torch tensor
        import torch
        want = {np.float64: torch.float64, np.int64: torch.int64}[dtype]
        if a.dtype != want or not a.is_contiguous():
            raise TypeError(f"tensor must be contiguous {want}")
        return C.c_void_p(a.data_ptr())
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags.c_contiguous:
        raise TypeError(f"array must be a C-contiguous {np.dtype(dtype).name} ndarray")
    return C.c_void_p(a.ctypes.data)


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def params_from_dict(p: dict) -> rt_params:
    out = rt_params()
    _check(lib().rt_params_default(int(p["nb"]), C.byref(out)))
    for k in ("nb", "chem_mode", "isothermal", "rate_set", "use_limiter", "chem_max_substeps",
              "chem_cells_per_lane"):
        if k in p:
            setattr(out, k, int(p[k]))
    for k in ("c_reduced", "cfl_eta", "T_iso", "Y_He", "alpha_B_const", "gamma", "chem_fmax", "chem_fs",
              "chem_growth", "chem_xfloor"):
        if k in p:
            setattr(out, k, float(p[k]))
    sig = np.asarray(p.get("sigma", np.zeros((p["nb"], 3))), dtype=float).reshape(-1, 3)
    eh = np.asarray(p.get("e_heat", np.zeros((p["nb"], 3))), dtype=float).reshape(-1, 3)
    for b in range(sig.shape[0]):
        for s in range(3):
            out.sigma[b][s] = sig[b, s]
            out.e_heat[b][s] = eh[b, s]
    return out


# --- the C ABI, one function each ----------------------------------------------

def rt_params_default(nb: int) -> rt_params:
    out = rt_params()
    _check(lib().rt_params_default(int(nb), C.byref(out)))
    return out


def rt_mesh_create(n_cells, volume, centre, n_faces, face_cells, area, normal, face_centre, box, device=0):
    out = C.c_void_p()
    boxa = (C.c_double * 3)(*[float(x) for x in box])
    _check(lib().rt_mesh_create(int(n_cells), _ptr(volume, np.float64), _ptr(centre, np.float64), int(n_faces),
                                _ptr(face_cells, np.int64), _ptr(area, np.float64), _ptr(normal, np.float64),
                                _ptr(face_centre, np.float64), boxa, int(device), C.byref(out)))
    return out


def rt_mesh_destroy(mesh):
    _check(lib().rt_mesh_destroy(mesh))


def rt_state_create(mesh, params: rt_params, precision: int, N, F, n_H, species, T, src_cell, src_rate):
    out = C.c_void_p()
    n_src = 0 if src_cell is None else int(src_cell.shape[0])
    _check(lib().rt_state_create(mesh, C.byref(params), int(precision), _ptr(N, np.float64), _ptr(F, np.float64),
                                 _ptr(n_H, np.float64), _ptr(species, np.float64), _ptr(T, np.float64), n_src,
                                 _ptr(src_cell, np.int64) if n_src else None,
                                 _ptr(src_rate, np.float64) if n_src else None, C.byref(out)))
    return out


def rt_state_clone(state):
    out = C.c_void_p()
    _check(lib().rt_state_clone(state, C.byref(out)))
    return out


def rt_state_destroy(state):
    _check(lib().rt_state_destroy(state))


def rt_subcycle(state, n_subcycles: int, dt: float = 0.0, stream=None):
    _check(lib().rt_subcycle(state, int(n_subcycles), float(dt), _stream_ptr(stream)))


def rt_subcycle_noalloc(state, n_subcycles: int, dt: float = 0.0, stream=None):
    _check(lib().rt_subcycle_noalloc(state, int(n_subcycles), float(dt), _stream_ptr(stream)))


def rt_subcycle_adjoint(initial, n_subcycles: int, checkpoint_every: int, dL_dxHI_final, dL_dlnQ, dL_dln_nH,
                        stream=None, dt: float = 0.0):
    _check(lib().rt_subcycle_adjoint(initial, int(n_subcycles), int(checkpoint_every), float(dt),
                                     _ptr(dL_dxHI_final, np.float64), _ptr(dL_dlnQ, np.float64),
                                     _ptr(dL_dln_nH, np.float64), _stream_ptr(stream)))


def rt_state_get_field(state, field: int, out):
    on_dev = int(hasattr(out, "is_cuda") and out.is_cuda)
    _check(lib().rt_state_get_field(state, int(field), _ptr(out, np.float64), on_dev))
    return out


def rt_state_set_field(state, field: int, values):
    on_dev = int(hasattr(values, "is_cuda") and values.is_cuda)
    _check(lib().rt_state_set_field(state, int(field), _ptr(values, np.float64), on_dev))


def rt_state_info(state) -> dict:
    nc, nb, ns, prec, dt = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int32(), C.c_double()
    _check(lib().rt_state_info(state, C.byref(nc), C.byref(nb), C.byref(ns), C.byref(prec), C.byref(dt)))
    return dict(n_cells=nc.value, nb=nb.value, n_src=ns.value, precision=prec.value, dt_cfl=dt.value)


def rt_state_diagnostics(state, nb: int) -> dict:
    d = rt_diag()
    _check(lib().rt_state_diagnostics(state, C.byref(d)))
    return d.as_dict(nb)


def rt_profile_enable(state, enable: bool = True):
    _check(lib().rt_profile_enable(state, int(enable)))


def rt_mesh_table(mesh, name: str) -> np.ndarray:
    """Copy of one of the mesh's index tables (see TABLES)."""
    p = C.POINTER(C.c_int32)()
    n = C.c_int64()
    _check(lib().rt_mesh_table(mesh, TABLES.index(name), C.byref(p), C.byref(n)))
    if n.value == 0:
        return np.zeros(0, np.int32)
    return np.ctypeslib.as_array(p, shape=(n.value,)).copy()


def rt_state_set_transport(state, mode: int):
    _check(lib().rt_state_set_transport(state, int(mode)))


def rt_state_transport(state) -> bool:
    f = C.c_int32()
    _check(lib().rt_state_transport(state, C.byref(f)))
    return bool(f.value)


def rt_profile_reset(state):
    _check(lib().rt_profile_reset(state))


def rt_profile_read(state, kernel: int) -> tuple[int, float]:
    n, ms = C.c_int64(), C.c_double()
    _check(lib().rt_profile_read(state, int(kernel), C.byref(n), C.byref(ms)))
    return n.value, ms.value


# --- owning wrappers -----------------------------------------------------------

def _c64(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


class Mesh:
    """A device mesh built from a mesh dict (the layout of ``rt_mesh_create``)."""

    def __init__(self, m: dict, device: int = 0):
        self.n_cells = int(m["n_cells"])
        self.n_faces = int(m["n_faces"])
        self.h = rt_mesh_create(self.n_cells, _c64(m["volume"]), _c64(m["centre"]), self.n_faces,
                                _c64(m["face_cells"], np.int64), _c64(m["area"]), _c64(m["normal"]),
                                _c64(m["face_centre"]), m["box"], device)

    def table(self, name: str) -> np.ndarray:
        return rt_mesh_table(self.h, name)

    def close(self):
        if self.h is not None and _lib is not None:
            rt_mesh_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """A radiation + gas state (the arguments of ``rt_state_create``)."""

    def __init__(self, mesh: Mesh, params, precision: int, N, F, n_H, species, T, src_cell, src_rate,
                 handle=None):
        self.mesh = mesh
        self.params = params if isinstance(params, rt_params) else params_from_dict(params)
        self.nb = int(self.params.nb)
        self.n_cells = mesh.n_cells
        if handle is not None:
            self.h = handle
            return
        cell = None if src_cell is None or len(src_cell) == 0 else _c64(src_cell, np.int64)
        rate = None if cell is None else _c64(src_rate)
        self.h = rt_state_create(mesh.h, self.params, precision, _c64(N), _c64(F), _c64(n_H), _c64(species), _c64(T),
                                 cell, rate)

    @classmethod
    def from_config(cls, mesh: Mesh, cfg: dict, precision: int | None = None, rate_scale=None, n_H=None):
        st = cfg["state"]
        prec = precision if precision is not None else (RT_MIXED if cfg.get("precision") == "mixed" else RT_FP64)
        rate = np.asarray(cfg["sources"]["rate"], dtype=float).reshape(cfg["params"]["nb"], -1)
        if rate_scale is not None:
            rate = rate * np.asarray(rate_scale)[None, :]
        return cls(mesh, cfg["params"], prec, st["N"], st["F"], st["n_H"] if n_H is None else n_H, st["species"],
                   st["T"], cfg["sources"]["cell"], rate)

    def clone(self) -> "State":
        return State(self.mesh, self.params, 0, None, None, None, None, None, None, None,
                     handle=rt_state_clone(self.h))

    def subcycle(self, n: int, dt: float = 0.0, stream=None):
        rt_subcycle(self.h, n, dt, stream)

    def get(self, field: int) -> np.ndarray:
        nc, nb = self.n_cells, self.nb
        shape = {RT_FIELD_N: (nb, nc), RT_FIELD_F: (nb, 3, nc), RT_FIELD_NH: (nc,), RT_FIELD_SPECIES: (5, nc),
                 RT_FIELD_T: (nc,), RT_FIELD_ATTEMPTS: (nc,)}[field]
        out = np.zeros(shape)
        rt_state_get_field(self.h, field, out)
        return out

    def set(self, field: int, values):
        rt_state_set_field(self.h, field, _c64(values) if isinstance(values, np.ndarray) else values)

    def fields(self) -> dict:
        return dict(N=self.get(RT_FIELD_N), F=self.get(RT_FIELD_F), species=self.get(RT_FIELD_SPECIES),
                    T=self.get(RT_FIELD_T), n_H=self.get(RT_FIELD_NH))

    def attempts(self) -> np.ndarray:
        """Chemistry attempts of each cell over the last subcycle call (int64)."""
        return self.get(RT_FIELD_ATTEMPTS).astype(np.int64)

    def diagnostics(self) -> dict:
        return rt_state_diagnostics(self.h, self.nb)

    def set_transport(self, mode: int):
        rt_state_set_transport(self.h, mode)

    @property
    def fused(self) -> bool:
        return rt_state_transport(self.h)

    def info(self) -> dict:
        return rt_state_info(self.h)

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            rt_state_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
