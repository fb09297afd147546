"""Helpers shared by the GPU tests: running a config through the C ABI and
comparing with the oracle."""
import sys

import numpy as np

from paper_2404_17630_amd import rt


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def run_gpu(cfg, n_sub=None, precision=None, dt=0.0, mesh=None, rate_scale=None, n_H=None, profile=False,
            transport=None):
    """Create mesh + state from a config, advance, return fields and diagnostics.
    transport: None (the library's default), or an RT_TRANSPORT_* mode."""
    m = mesh if mesh is not None else rt.Mesh(cfg["mesh"])
    s = rt.State.from_config(m, cfg, precision=precision, rate_scale=rate_scale, n_H=n_H)
    if transport is not None:
        s.set_transport(transport)
    if profile:
        rt.rt_profile_enable(s.h, True)
    n = cfg["n_subcycles"] if n_sub is None else n_sub
    s.subcycle(n, dt)
    out = s.fields()
    out["diag"] = s.diagnostics()
    out["info"] = s.info()
    out["fused"] = s.fused
    if profile:
        out["profile"] = {k: rt.rt_profile_read(s.h, k) for k in range(rt.RT_N_KERNELS)}
    s.close()
    if mesh is None:
        m.close()
    return out


def rel_err(a, r, floor=1e-10):
    """max |a - r| / max(|r|, floor * max|r|) (elementwise relative error with a
    floor relative to the field's largest magnitude)."""
    a = np.asarray(a, float)
    r = np.asarray(r, float)
    mx = np.abs(r).max() if r.size else 0.0
    if mx == 0.0:
        return float(np.abs(a).max()) if a.size else 0.0
    scale = np.maximum(np.abs(r), floor * mx)
    return float((np.abs(a - r) / scale).max())


def stencil_max(values, face_cells):
    """max |v| over each cell and its face neighbours."""
    a = np.abs(np.asarray(values, float))
    m = a.copy()
    np.maximum.at(m, face_cells[0], a[face_cells[1]])
    np.maximum.at(m, face_cells[1], a[face_cells[0]])
    return m


def field_errors(gpu, ref, c_red, face_cells, kappa=1e-6, phi=1e-10):
    """Per-field, per-bin relative errors of a GPU run against the oracle.

    Photon fields are measured against s_i = max(N_i, kappa * M_i, phi * max N),
    M_i the largest N over the cell and its face neighbours: a cell far below
    its neighbours is the difference of fluxes of their size, so rounding
    reaches it at the level eps * M_i (with kappa = 1e-6 and a tolerance of
    1e-10 the floor is one FP64 rounding of M_i); phi = 1e-10 is the global
    floor.  Flux components use the same scale times c~ (|F| <= c~ N).
    Fractions are measured against max(|x|, 1e-6): a fraction far below 1 is
    set by the photon density of the same cell and inherits its conditioning;
    below 1e-6 the allowance is 1e-16 absolute.  T relative."""
    errs = {}
    nb = ref["N"].shape[0]
    for b in range(nb):
        Nr = np.asarray(ref["N"][b], float)
        scale = np.maximum(np.maximum(Nr, kappa * stencil_max(Nr, face_cells)), phi * Nr.max())
        scale = np.where(scale > 0, scale, 1.0)
        errs[f"N[{b}]"] = float((np.abs(gpu["N"][b] - Nr) / scale).max())
        for k in range(3):
            errs[f"F[{b}][{k}]"] = float((np.abs(gpu["F"][b, k] - ref["F"][b, k]) / (c_red * scale)).max())
    names = ("x_HI", "x_HII", "y_HeI", "y_HeII", "y_HeIII")
    for s in range(5):
        r = np.asarray(ref["species"][s], float)
        errs[names[s]] = float((np.abs(gpu["species"][s] - r) / np.maximum(np.abs(r), 1e-6)).max())
    errs["T"] = rel_err(gpu["T"], ref["T"])
    return errs
