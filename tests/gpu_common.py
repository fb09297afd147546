"""Helpers shared by the GPU tests: running a config through the C ABI and
comparing with the oracle."""
import sys

import numpy as np

from paper_2404_17630_amd import rt


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def run_gpu(cfg, n_sub=None, precision=None, dt=0.0, mesh=None, rate_scale=None, n_H=None, profile=False):
    """Create mesh + state from a config, advance, return fields and diagnostics."""
    m = mesh if mesh is not None else rt.Mesh(cfg["mesh"])
    s = rt.State.from_config(m, cfg, precision=precision, rate_scale=rate_scale, n_H=n_H)
    if profile:
        rt.rt_profile_enable(s.h, True)
    n = cfg["n_subcycles"] if n_sub is None else n_sub
    s.subcycle(n, dt)
    out = s.fields()
    out["diag"] = s.diagnostics()
    out["info"] = s.info()
    if profile:
        out["profile"] = {k: rt.rt_profile_read(s.h, k) for k in range(5)}
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


def field_errors(gpu, ref, c_red):
    """Per-field, per-bin relative errors of a GPU run against the oracle."""
    errs = {}
    nb = ref["N"].shape[0]
    for b in range(nb):
        errs[f"N[{b}]"] = rel_err(gpu["N"][b], ref["N"][b])
        for k in range(3):
            errs[f"F[{b}][{k}]"] = rel_err(gpu["F"][b, k], ref["F"][b, k])
    names = ("x_HI", "x_HII", "y_HeI", "y_HeII", "y_HeIII")
    for s in range(5):
        errs[names[s]] = rel_err(gpu["species"][s], ref["species"][s])
    errs["T"] = rel_err(gpu["T"], ref["T"])
    return errs
