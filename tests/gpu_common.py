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


def photon_conditioning(N_ref, face_cells, kappa=1e-6, phi=1e-10, cap=1e6):
    """Per cell, how much looser than its own size the photon density is
    known: the largest over bins of s_i / N_i with s_i the N scale of
    field_errors (1 where N_i is at least 1e-6 of its stencil maximum and
    1e-10 of the field's maximum, and for N_i = 0), at most `cap`."""
    N_ref = np.asarray(N_ref, float)
    c = np.ones(N_ref.shape[1])
    for b in range(N_ref.shape[0]):
        Nr = N_ref[b]
        s = np.maximum(np.maximum(Nr, kappa * stencil_max(Nr, face_cells)), phi * Nr.max())
        ratio = np.where(Nr > 0, s / np.where(Nr > 0, Nr, 1.0), 1.0)
        c = np.maximum(c, np.minimum(ratio, cap))
    return c


def field_errors(gpu, ref, c_red, face_cells, kappa=1e-6, phi=1e-10):
    """Per-field, per-bin relative errors of a GPU run against the oracle.

    Photon fields are measured against s_i = max(N_i, kappa * M_i, phi * max N),
    M_i the largest N over the cell and its face neighbours: a cell far below
    its neighbours is the difference of fluxes of their size, so rounding
    reaches it at the level eps * M_i (with kappa = 1e-6 and a tolerance of
    1e-10 the floor is one FP64 rounding of M_i); phi = 1e-10 is the global
    floor.  Flux components use the same scale times c~ (|F| <= c~ N).
    A fraction is set by the photon density of its own cell and inherits
    that density's conditioning: it is measured relative to |x| times the
    cell's photon_conditioning factor (1 wherever N is known to its own
    relative precision), floored at 1e-9 (an allowance of 1e-19; the FP64
    test workloads need up to 2.4e-11, in cells ahead of a front whose x_HII
    is set by photon densities near the underflow edge).  y_HeII is
    the complement 1 - y_HeI - y_HeIII, so its absolute error is a few
    roundings of 1: its scale is floored at 1e-5 (an allowance of 1e-15).
    T relative."""
    errs = {}
    nb = ref["N"].shape[0]
    for b in range(nb):
        Nr = np.asarray(ref["N"][b], float)
        scale = np.maximum(np.maximum(Nr, kappa * stencil_max(Nr, face_cells)), phi * Nr.max())
        scale = np.where(scale > 0, scale, 1.0)
        errs[f"N[{b}]"] = float((np.abs(gpu["N"][b] - Nr) / scale).max())
        for k in range(3):
            errs[f"F[{b}][{k}]"] = float((np.abs(gpu["F"][b, k] - ref["F"][b, k]) / (c_red * scale)).max())
    cond = photon_conditioning(ref["N"], face_cells, kappa, phi)
    names = ("x_HI", "x_HII", "y_HeI", "y_HeII", "y_HeIII")
    for s in range(5):
        r = np.asarray(ref["species"][s], float)
        floor = 1e-5 if names[s] == "y_HeII" else 1e-9
        errs[names[s]] = float((np.abs(gpu["species"][s] - r) / np.maximum(np.abs(r) * cond, floor)).max())
    errs["T"] = rel_err(gpu["T"], ref["T"])
    return errs


def host_threads() -> int:
    """Host threads for the oracle on the large workloads: the CPUs this
    process may run on, at most 16 (one GPU's share of the host)."""
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_run_threaded(cfg, **kw):
    """oracle.run on the host's threads (bitwise the single-thread result)."""
    import oracle
    prev = oracle.set_threads(host_threads())
    try:
        return oracle.run(cfg, **kw)
    finally:
        oracle.set_threads(prev)


_oracle_cache = {}


def cached_oracle_run(key, cfg, **kw):
    """oracle_run_threaded, kept for the session under `key` (large workloads
    that several tests compare against)."""
    if key not in _oracle_cache:
        _oracle_cache[key] = oracle_run_threaded(cfg, **kw)
    return _oracle_cache[key]
