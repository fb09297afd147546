"""Benchmark of the M1 radiative-transfer subcycle on one MI355X.

A step is one subcycle (sources, chemistry, gradients, fluxes + update) of
the throughput workload: a 256^3 jittered periodic lattice (16.8M cells) in
Peano-Hilbert order, lognormal H+He gas (sigma_ln = 1.5, mean n_H = 2e-4),
3 frequency bins, 4096 power-law sources, c~ = 0.1 c, 200 subcycles.  The
headline is the mixed-precision form (FP32 transport, FP64 chemistry and
sums); the FP64 form and the random cell order are timed beside it, and the
mixed result is compared with the FP64 one.

    python bench.py [--steps 200] [--warmup 5] [--gpus 1]

Prints one JSON line.  Inputs are resident in HBM before the timed region;
the timed region is one rt_subcycle call of K subcycles, bracketed by
device synchronisations.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = ROOT / "profiles" / "traffic.json"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel: str, nc: int, nb: int, nf: int, n_sides: int, n_src: int, p: int, g: int) -> float:
    """Compulsory HBM bytes of one launch: every array element the kernel must
    read or write, counted once (a neighbour's record gathered by several
    cells, and geometry re-read for each bin, are counted once).
    p = bytes per transport value, g = bytes per geometry value; indices are
    4 bytes.  Face sides per cell: n_sides / nc."""
    if kernel == "k_facestate":
        # fields (4) in, one 4-value face state per face side out, the cell's
        # N copied out; cell record (M^-1, V, V/n_f), face record (12 values),
        # neighbour index
        return nb * (5 * nc + 4 * n_sides) * p + nc * 8 * g + nf * 12 * g + n_sides * 4
    if kernel == "k_transport":
        # fused gradient + face states + fluxes: fields in and out; cell and
        # face records; neighbour, face and opposite-slot index per face side
        # (the face states stay in LDS; the halo tables, about a tenth of
        # the side count, are not counted)
        return nb * 8 * nc * p + nc * 8 * g + nf * 12 * g + n_sides * 12
    if kernel == "k_flux":
        # fields in and out, the cells' N copy, face states of every face side
        # in; cell volume, face record, neighbour + face + opposite-side index
        return nb * (9 * nc + 4 * n_sides) * p + nc * g + nf * 12 * g + n_sides * 12
    if kernel == "k_chem":
        # fields of all bins in and out, 5 fractions and u in and out, n_H in
        return nc * (8 * nb * p + 2 * 5 * 8 + 2 * 8 + 8)
    if kernel == "k_sources":
        return n_src * (nb * 8 + 16) + 2 * n_src * nb * p
    return 0.0


def subcycle_bytes_per_cell(nb: int, p: int, g: int) -> dict:
    """Whole-subcycle HBM bytes per cell on a six-face mesh, two accountings.
    Two-pass: the gradient pass stores 3 gradient rows per field (and the
    flux pass reads them), so fields move 36 nb p bytes; the geometry (cell:
    M^-1, V, s = 10 values; per face side 8 index bytes; per face A, n, x_f
    = 7 values read by each side) is read twice; the chemistry moves 13 FP64
    values.  Compulsory: fields read and written once, geometry once."""
    geo = 52 * g + 48
    return {"two_pass": 36 * nb * p + 2 * geo + 104, "compulsory": 8 * nb * p + geo + 104}


def kernel_source_digest() -> str:
    """First 16 hex digits of SHA-256 over the kernel sources and the build
    script (its compiler flags)."""
    h = hashlib.sha256()
    for f in sorted((ROOT / "paper_2404_17630_amd" / "csrc").glob("*")) + [ROOT / "paper_2404_17630_amd" / "build.py"]:
        h.update(f.read_bytes())
    return h.hexdigest()[:16]


def timed_run(rt, mesh, cfg, precision, steps, warmup, torch, transport=None):
    """Warm up on a clone, then time `steps` subcycles from the initial state."""
    state = rt.State.from_config(mesh, cfg, precision=precision)
    if transport is not None:
        state.set_transport(transport)
    stream = torch.cuda.current_stream()
    if warmup > 0:
        w = state.clone()
        w.subcycle(warmup, stream=stream)
        w.close()
    rt.rt_profile_enable(state.h, True)
    rt.rt_profile_reset(state.h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    state.subcycle(steps, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {rt.KERNEL_NAMES[k]: rt.rt_profile_read(state.h, k) for k in range(rt.RT_N_KERNELS)}
    return state, t1 - t0, prof


def cpu_baseline():
    """The oracle as it stands, single-threaded, on a bounded sample of the same
    recipe: a 64^3 lattice (262,144 cells) with 64 sources, 2 subcycles."""
    import oracle
    import rtgen
    cfg = rtgen.cosmological(64, 1.0, 1.5, 64, 0.1, 2, 4, name="throughput_sample")
    out = oracle.run(cfg)
    secs = out["diag"]["loop_seconds"]
    nc, nb = cfg["mesh"]["n_cells"], cfg["params"]["nb"]
    return dict(value=nc * nb * 2 / secs, unit="cell*bin updates/s", cores=1, kind="oracle",
                sample="throughput recipe at 64^3 (262,144 cells, sigma_ln=1.5, 64 sources, 3 bins, c~=0.1c), "
                       f"2 subcycles from the initial state, {secs:.2f} s single-threaded")


def adjoint_timing(rt, torch):
    """The adjoint workload (64^3 cells, 3 bins, 64 sources, 50 FP64
    subcycles, checkpoints every 10): seconds of the forward run and of one
    rt_subcycle_adjoint call (its own forward pass, the segment recomputes
    and the reverse sweep), with seeded weights as dL/dx_HI."""
    import rtgen
    from paper_2404_17630_amd.autograd import Problem
    log("adjoint workload 64^3, 50 FP64 subcycles")
    cfg = rtgen.adjoint_262k()
    pb = Problem(cfg, checkpoint_every=10)
    s0 = pb.state(pb.log_lum0, np.log(cfg["state"]["n_H"]))
    stream = torch.cuda.current_stream()
    run = s0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.subcycle(pb.n_subcycles, stream=stream)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    run.close()
    nc = cfg["mesh"]["n_cells"]
    g = torch.from_numpy(np.random.default_rng(11).normal(size=nc)).to("cuda")
    d_lum = torch.zeros(pb.log_lum0.size, dtype=torch.float64, device="cuda")
    d_nH = torch.zeros(nc, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rt.rt_subcycle_adjoint(s0.h, pb.n_subcycles, pb.checkpoint_every, g, d_lum, d_nH, stream)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    s0.close()
    pb.mesh.close()
    return {"cells": nc, "subcycles": pb.n_subcycles, "checkpoint_every": pb.checkpoint_every,
            "forward_s": t_fwd, "adjoint_call_s": t_adj, "adjoint_over_forward": t_adj / t_fwd}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per side (256 = the throughput workload)")
    ap.add_argument("--no-extras", action="store_true", help="time only the mixed Hilbert-order run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--transport", choices=("auto", "fused", "split"), default="auto",
                    help="transport path of the headline run (the library's default is auto)")
    ap.add_argument("--order", choices=("hilbert", "random"), default="hilbert",
                    help="cell order of the headline run (random: for profiling the unordered case; "
                         "the throughput figure is quoted in Hilbert order)")
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GIB",
                    help="first copy a GIB-sized device buffer three times (a plain copy kernel of known size, "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only (there is no multi-GPU path); run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    import rtgen
    from paper_2404_17630_amd import rt

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    rt.lib()
    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:
        n = int(args.calibrate_copy * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {n * 4} bytes (read {n * 4}, write {n * 4} each)")
        del src, dst
    n_src = max(1, int(round(4096 * (args.n / 256) ** 3)))
    log(f"generating throughput workload {args.n}^3, {n_src} sources")
    cfg = rtgen.throughput_16m(n=args.n, n_src=n_src, n_sub=args.steps)
    if args.order == "random":
        cfg = rtgen.random_order(cfg)
    nc, nb, nf = cfg["mesh"]["n_cells"], cfg["params"]["nb"], cfg["mesh"]["n_faces"]
    n_sides = 2 * nf
    log("creating mesh")
    mesh = rt.Mesh(cfg["mesh"])

    log(f"mixed, {args.order}: {args.steps} subcycles")
    mode = {"auto": None, "fused": rt.RT_TRANSPORT_FUSED, "split": rt.RT_TRANSPORT_SPLIT}[args.transport]
    st_mixed, t_mixed, prof_mixed = timed_run(rt, mesh, cfg, rt.RT_MIXED, args.steps, args.warmup, torch,
                                              transport=mode)
    value = nc * nb * args.steps / t_mixed
    diag = st_mixed.diagnostics()
    if diag["status"] != 0:
        raise SystemExit(f"mixed run status {diag['status']}")

    def kernel_table(prof, p, g):
        tab = {}
        for name, (launches, ms) in prof.items():
            if launches == 0:
                continue
            avg = ms / launches
            algo = algorithmic_bytes(name, nc, nb, nf, n_sides, cfg["sources"]["cell"].size, p, g)
            tab[name] = dict(launches=launches, avg_ms=avg, algo_bytes=algo,
                             gbs=algo / (avg * 1e-3) / 1e9 if algo else None)
        return tab

    kt_mixed = kernel_table(prof_mixed, 4, 4)
    dominant = max((k for k in kt_mixed if k != "k_reduce"), key=lambda k: kt_mixed[k]["avg_ms"] * kt_mixed[k]["launches"])
    dk = kt_mixed[dominant]

    traffic = None
    if TRAFFIC_FILE.exists():
        rec = json.loads(TRAFFIC_FILE.read_text())
        ent = rec.get("kernels", {}).get(dominant)
        if ent and rec.get("source_digest") == kernel_source_digest() and rec.get("workload") == f"throughput_{args.n}" \
                and args.order == "hilbert":
            traffic = ent["bytes_per_launch"]

    out = {
        "metric": "RT cell\u00b7bin updates/s per subcycle, mixed vs FP64 at stated error; % HBM peak",
        "value": value,
        "unit": "cell*bin updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"throughput_{args.n}", "cells": nc, "bins": nb, "sources": int(n_src),
                   "subcycles": args.steps, "order": args.order, "precision": "mixed", "c_reduced": "0.1c",
                   "transport": "fused" if st_mixed.fused else "split",
                   "sigma_ln": 1.5},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": traffic},
        "kernels_mixed": kt_mixed,
        "subcycle_effective": {
            name: {"bytes_per_cell": b, "GB/s": b * nc / (t_mixed / args.steps) / 1e9,
                   "frac": b * nc / (t_mixed / args.steps) / 1e9 / HBM_PEAK_GBS}
            for name, b in subcycle_bytes_per_cell(nb, 4, 4).items()},
        "chem_attempts_per_cell_subcycle": diag["substeps"] / (nc * args.steps),
    }

    if not args.no_extras and args.order == "hilbert":
        fields_mixed = st_mixed.fields()
        st_mixed.close()
        other = "split" if out["config"]["transport"] == "fused" else "fused"
        log(f"mixed, hilbert, {other} transport: {args.steps} subcycles")
        try:
            st_s, t_s, prof_s = timed_run(rt, mesh, cfg, rt.RT_MIXED, args.steps, args.warmup, torch,
                                          transport=rt.RT_TRANSPORT_SPLIT if other == "split"
                                          else rt.RT_TRANSPORT_FUSED)
            st_s.close()
            out[f"{other}_transport_value"] = nc * nb * args.steps / t_s
            out[f"kernels_mixed_{other}"] = kernel_table(prof_s, 4, 4)
        except rt.RtError as e:
            out[f"{other}_transport_value"] = f"unavailable: {e}"
        log(f"fp64, hilbert: {args.steps} subcycles")
        st64, t64, prof64 = timed_run(rt, mesh, cfg, rt.RT_FP64, args.steps, args.warmup, torch)
        f64 = st64.fields()
        st64_fused = st64.fused
        st64.close()
        v64 = nc * nb * args.steps / t64
        fc = cfg["mesh"]["face_cells"]

        def n_errors(Na, Nr):
            """Relative error of N against a reference, the way the stated bar
            measures it, plus the share of cells above 1e-3 and the error with
            a floor of 1e-4 of the stencil maximum."""
            errN, errC, p999, frac = 0.0, 0.0, 0.0, 0.0
            for b in range(nb):
                r = Nr[b]
                mask = r > 1e-10 * r.max()
                rel = np.abs(Na[b][mask] - r[mask]) / r[mask]
                errN = max(errN, float(rel.max()))
                p999 = max(p999, float(np.quantile(rel, 0.999)))
                frac = max(frac, float(np.mean(rel > 1e-3)))
                m = r.copy()
                np.maximum.at(m, fc[0], r[fc[1]])
                np.maximum.at(m, fc[1], r[fc[0]])
                scale = np.maximum(np.maximum(r, 1e-4 * m), 1e-10 * r.max())
                errC = max(errC, float((np.abs(Na[b] - r) / np.where(scale > 0, scale, 1.0)).max()))
            return errN, p999, frac, errC

        errN, p999, frac, errC = n_errors(fields_mixed["N"], f64["N"])
        # Conditioning of the workload itself: the FP64 run again from n_H
        # rounded to FP32 (a relative change of at most 6e-8, the size of one
        # FP32 rounding).  How far that moves N is what any 1e-7-level change,
        # such as FP32 storage, can be expected to do.
        try:
            nH32 = cfg["state"]["n_H"].astype(np.float32).astype(np.float64)
            st_p = rt.State.from_config(mesh, cfg, precision=rt.RT_FP64, n_H=nH32)
            st_p.subcycle(args.steps, stream=torch.cuda.current_stream())
            f_p = st_p.fields()
            st_p.close()
            pN, pp999, pfrac, pC = n_errors(f_p["N"], f64["N"])
            out["fp64_nH_rounded_to_fp32_vs_fp64"] = {
                "N_rel_max(N>1e-10 max)": pN, "N_rel_p99.9(N>1e-10 max)": pp999, "N_frac_cells_rel>1e-3": pfrac,
                "N_rel_max(stencil floor 1e-4)": pC,
                "x_HII_abs_max": float(np.abs(f_p["species"][1] - f64["species"][1]).max()),
            }
            del f_p
        except rt.RtError as e:
            out["fp64_nH_rounded_to_fp32_vs_fp64"] = f"unavailable: {e}"
        out["fp64_value"] = v64
        out["fp64_ms_per_step"] = t64 / args.steps * 1e3
        out["mixed_speedup_vs_fp64"] = value / v64
        out["mixed_error_vs_fp64"] = {
            "N_rel_max(N>1e-10 max)": errN,
            "N_rel_p99.9(N>1e-10 max)": p999,
            "N_frac_cells_rel>1e-3": frac,
            "N_rel_max(stencil floor 1e-4)": errC,
            "x_HII_abs_max": float(np.abs(fields_mixed["species"][1] - f64["species"][1]).max()),
            "y_HeII_abs_max": float(np.abs(fields_mixed["species"][3] - f64["species"][3]).max()),
            "T_rel_max": float((np.abs(fields_mixed["T"] - f64["T"]) / f64["T"]).max()),
        }
        out["kernels_fp64"] = kernel_table(prof64, 8, 8)
        out["fp64_subcycle_effective"] = {
            name: {"bytes_per_cell": b, "GB/s": b * nc / (t64 / args.steps) / 1e9,
                   "frac": b * nc / (t64 / args.steps) / 1e9 / HBM_PEAK_GBS}
            for name, b in subcycle_bytes_per_cell(nb, 8, 8).items()}
        out["fp64_transport"] = "fused" if st64_fused else "split"
        del fields_mixed, f64
        mesh.close()
        log("random cell order (mixed)")
        cfg_r = rtgen.random_order(cfg)
        mesh_r = rt.Mesh(cfg_r["mesh"])
        st_r, t_r, prof_r = timed_run(rt, mesh_r, cfg_r, rt.RT_MIXED, args.steps, args.warmup, torch)
        out["random_order_transport"] = "fused" if st_r.fused else "split"
        st_r.close()
        mesh_r.close()
        out["random_order_value"] = nc * nb * args.steps / t_r
        out["kernels_mixed_random"] = kernel_table(prof_r, 4, 4)
        del cfg_r
        out["adjoint_262k"] = adjoint_timing(rt, torch)
    else:
        st_mixed.close()
        mesh.close()

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
