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


def tile_counts(mesh):
    """(boundary items, tile-interior faces) of the split transport by
    256-cell tile, which the library uses on six-slot meshes; None on other
    meshes."""
    n_bnd, n_pairs = mesh.table("tbnd").size // 2, mesh.table("tpair").size
    return (n_bnd, n_pairs) if n_bnd + n_pairs > 0 else None


def algorithmic_bytes(kernel: str, nc: int, nb: int, nf: int, n_sides: int, n_src: int, p: int, g: int,
                      tile=None) -> float:
    """This design's compulsory HBM bytes of one launch: every array element
    the kernel must read or write, counted once (a neighbour's record
    gathered by several cells, and geometry re-read for each bin, are counted
    once).  p = bytes per transport value, g = bytes per geometry value;
    indices are 4 bytes.  Face sides per cell: n_sides / nc.  tile = (n_bnd,
    n_pairs) on six-slot meshes, where the split path runs by tile; else the
    figures are those of the per-slice kernels."""
    if tile is not None and kernel in ("k_facestate", "k_flux"):
        n_bnd, n_pairs = tile
        if kernel == "k_facestate":
            # fields in; the cells updated by their tile-interior faces out;
            # each boundary item's state and cap numerator out; cell record,
            # per side weight, offset and neighbour, the slot mask; per
            # interior face its (L, R) pair and A, n
            return (nb * (8 * nc * p + 5 * n_bnd * p) + nc * (8 * g + 1) + n_sides * (6 * g + 4)
                    + n_pairs * (4 + 4 * g))
        # the partly updated fields in and out; each boundary item's own and
        # opposite state and cap numerator; V and the slot mask per cell; per
        # item the opposite position and A, n
        return nb * (8 * nc * p + 10 * n_bnd * p) + nc * (g + 1) + n_bnd * (4 + 4 * g)
    if kernel == "k_facestate":
        # fields (4) in, one 4-value face state per face side out, the cell's
        # cap numerator N V / n_faces out; cell record (M^-1, V, V/n_f), per
        # side the weight and offset (6 values) and the neighbour index
        return nb * (5 * nc + 4 * n_sides) * p + nc * 8 * g + n_sides * 6 * g + n_sides * 4
    if kernel == "k_transport":
        # fused gradient + face states + fluxes: fields in and out; cell
        # record; per side the gradient's 6 values and the flux's A, n and
        # V/n_f of both cells (6); neighbour, face and opposite-slot index
        # (the face states stay in LDS; the halo tables are not counted)
        return nb * 8 * nc * p + nc * 8 * g + n_sides * 12 * g + n_sides * 12
    if kernel == "k_flux":
        # fields in and out, the cells' cap numerators, face states of every
        # face side in; cell volume, per side A and n (4 values) and the
        # signed opposite-entry index
        return nb * (9 * nc + 4 * n_sides) * p + nc * g + n_sides * 4 * g + n_sides * 4
    if kernel == "k_chem":
        # fields of all bins in and out, 5 fractions and u in and out, n_H in,
        # the per-cell attempt count in and out
        return nc * (8 * nb * p + 2 * 5 * 8 + 2 * 8 + 8 + 8)
    if kernel == "k_sources":
        return n_src * (nb * 8 + 16) + 2 * n_src * nb * p
    return 0.0


def model_bytes_per_cell(kernel: str, nb: int, p: int, g: int) -> float:
    """Bytes per cell of a six-face mesh that the reference two-pass
    accounting assigns to the kernel doing each step: the gradient pass
    stores 3 gradient rows per field (16 nb p: fields in, gradients out) and
    reads the geometry (cell: M^-1, V, s = 10 values; per face side 8 index
    bytes; per face A, n, x_f = 7 values read by each side: 52 g + 48); the
    flux pass reads fields and gradients and writes fields (20 nb p) with the
    same geometry; the chemistry moves 13 FP64 values (104).  The fused
    kernel does both transport passes."""
    geo = 52 * g + 48
    return {"k_facestate": 16 * nb * p + geo, "k_flux": 20 * nb * p + geo, "k_transport": 36 * nb * p + 2 * geo,
            "k_chem": 104}.get(kernel, 0)


def subcycle_bytes_per_cell(nb: int, p: int, g: int) -> dict:
    """Whole-subcycle HBM bytes per cell on a six-face mesh, two accountings.
    Two-pass: the sum of model_bytes_per_cell over gradient, flux and
    chemistry passes.  Compulsory: fields read and written once, geometry
    once."""
    geo = 52 * g + 48
    return {"two_pass": 36 * nb * p + 2 * geo + 104, "compulsory": 8 * nb * p + geo + 104}


def kernel_source_digest() -> str:
    """First 16 hex digits of SHA-256 over the kernel sources and the build
    script (its compiler flags)."""
    h = hashlib.sha256()
    for f in sorted((ROOT / "paper_2404_17630_amd" / "csrc").glob("*")) + [ROOT / "paper_2404_17630_amd" / "build.py"]:
        h.update(f.read_bytes())
    return h.hexdigest()[:16]


def timed_run(rt, mesh, cfg, precision, steps, warmup, torch, transport=None, profile=False, n_H=None):
    """Warm up on a clone, then time `steps` subcycles from the initial state
    (one rt_subcycle call between device synchronisations).  With `profile`
    every launch is bracketed by HIP events on the stream it runs on, and the
    per-kernel launch counts and summed milliseconds are returned."""
    state = rt.State.from_config(mesh, cfg, precision=precision, n_H=n_H)
    if transport is not None:
        state.set_transport(transport)
    stream = torch.cuda.current_stream()
    if warmup > 0:
        w = state.clone()
        w.subcycle(warmup, stream=stream)
        w.close()
    rt.rt_profile_enable(state.h, bool(profile))
    rt.rt_profile_reset(state.h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    state.subcycle(steps, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {rt.KERNEL_NAMES[k]: rt.rt_profile_read(state.h, k) for k in range(rt.RT_N_KERNELS)} if profile else {}
    return state, t1 - t0, prof


def cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Host threads for the all-cores leg: the CPUs this process may run on,
    at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline():
    """The oracle on the host's cores, on bounded samples of the same recipe:
    all cores on a 128^3 lattice (2.1M cells, 512 sources) and one thread on a
    64^3 lattice (262,144 cells, 64 sources), 2 subcycles each from the
    initial state.  The threaded oracle gives the single-thread results bit
    for bit."""
    import oracle
    import rtgen
    out = {}
    for label, n, n_src, threads in (("all_cores", 128, 512, host_threads()), ("single_thread", 64, 64, 1)):
        cfg = rtgen.cosmological(n, 1.0, 1.5, n_src, 0.1, 2, 4, name="throughput_sample")
        prev = oracle.set_threads(threads)
        try:
            res = oracle.run(cfg)
        finally:
            oracle.set_threads(prev)
        secs = res["diag"]["loop_seconds"]
        nc, nb = cfg["mesh"]["n_cells"], cfg["params"]["nb"]
        out[label] = dict(value=nc * nb * 2 / secs, unit="cell*bin updates/s", cores=threads, kind="oracle",
                          cpu=cpu_model(), host_cpus=os.cpu_count(),
                          sample=f"throughput recipe at {n}^3 ({nc:,} cells, sigma_ln=1.5, {n_src} sources, 3 bins, "
                                 f"c~=0.1c), 2 subcycles from the initial state, {secs:.2f} s on {threads} thread(s)")
    return out


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


ATTEMPT_BINS = (1, 2, 4, 8, 16, 64, 256)          # upper edges of the attempts histogram


def attempt_histogram(a: np.ndarray) -> dict:
    """Counts of attempts per cell and subcycle in the bins 1, 2, 3-4, 5-8,
    9-16, 17-64, 65-256 and >256."""
    a = np.asarray(a).ravel()
    edges = (0,) + ATTEMPT_BINS
    hist = {f"{lo + 1}-{hi}" if hi > lo + 1 else f"{hi}": int(((a > lo) & (a <= hi)).sum())
            for lo, hi in zip(edges[:-1], edges[1:])}
    hist[f">{ATTEMPT_BINS[-1]}"] = int((a > ATTEMPT_BINS[-1]).sum())
    return hist


def chem_refill_ab(rt, torch):
    """Lane refill against one cell per lane (rt_params.chem_cells_per_lane
    = 1) in the chemistry: the throughput workload and the 2.1M-cell H+He
    workload, mixed, the first 10 subcycles from the initial state (the
    I-fronts forming around the sources), one subcycle per call.  Per
    workload: the chemistry's mean launch time in both modes, the histogram
    of attempts per cell and subcycle, and whether both modes took the same
    attempts cell by cell."""
    import rtgen
    out = {}
    for name, cfg in (("throughput_256", rtgen.throughput_16m(n_sub=10)), ("hhe_2m", rtgen.hhe_2m(n_sub=10))):
        log(f"chemistry A/B on {name}")
        mesh = rt.Mesh(cfg["mesh"])
        rec, atts = {}, []
        for label, per_lane in (("refill", 0), ("one_cell_per_lane", 1)):
            c = dict(cfg, params=dict(cfg["params"], chem_cells_per_lane=per_lane))
            st = rt.State.from_config(mesh, c, precision=rt.RT_MIXED)
            rt.rt_profile_enable(st.h, True)
            att = []
            for _ in range(cfg["n_subcycles"]):
                st.subcycle(1, stream=torch.cuda.current_stream())
                att.append(st.attempts())
            launches, total_ms = rt.rt_profile_read(st.h, rt.RT_KERNEL_CHEM)
            rec[label + "_ms_per_launch"] = total_ms / launches
            atts.append(np.stack(att))
            st.close()
        mesh.close()
        a = atts[0].ravel()
        rec.update(cells=cfg["mesh"]["n_cells"], subcycles=cfg["n_subcycles"], attempt_histogram=attempt_histogram(a),
                   max_attempts=int(a.max()), mean_attempts=float(a.mean()),
                   same_attempts=bool(np.array_equal(atts[0], atts[1])),
                   refill_speedup=rec["one_cell_per_lane_ms_per_launch"] / rec["refill_ms_per_launch"])
        out[name] = rec
    return out


MIXED_BAR = {"N_rel": 1e-3, "x_HII_abs": 1e-4}    # the stated accuracy of the mixed form
ERROR_SUBCYCLES = 200                              # the throughput workload's own run length


def field_errors(a, r, fc, c_red, a_att=None, r_att=None):
    """Errors of fields `a` against reference `r` over the cells where the
    reference N of a bin exceeds 1e-10 of its maximum: N relative, F relative
    to c~ N, fractions absolute, T relative; the share of cells above the N
    bar, and (given per-cell attempt counts) how many of those cells took a
    different number of chemistry attempts than the reference."""
    nb = r["N"].shape[0]
    errN = p999 = frac = errF = 0.0
    over = np.zeros(r["N"].shape[1], bool)
    for b in range(nb):
        rN = r["N"][b]
        mask = rN > 1e-10 * rN.max()
        rel = np.abs(a["N"][b][mask] - rN[mask]) / rN[mask]
        errN = max(errN, float(rel.max()))
        p999 = max(p999, float(np.quantile(rel, 0.999)))
        frac = max(frac, float(np.mean(rel > MIXED_BAR["N_rel"])))
        idx = np.nonzero(mask)[0]
        over[idx[rel > MIXED_BAR["N_rel"]]] = True
        dF = np.sqrt(((a["F"][b][:, mask] - r["F"][b][:, mask]) ** 2).sum(axis=0))
        errF = max(errF, float((dF / (c_red * rN[mask])).max()))
    out = {
        "N_rel_max(N>1e-10 max)": errN, "N_rel_p99.9(N>1e-10 max)": p999, "N_frac_cells_rel>1e-3": frac,
        "F_rel_to_cN_max(N>1e-10 max)": errF,
        "x_HII_abs_max": float(np.abs(a["species"][1] - r["species"][1]).max()),
        "y_HeII_abs_max": float(np.abs(a["species"][3] - r["species"][3]).max()),
        "T_rel_max": float((np.abs(a["T"] - r["T"]) / r["T"]).max()),
        "cells_N_rel>1e-3": int(over.sum()),
    }
    out["meets_stated_bar"] = bool(errN <= MIXED_BAR["N_rel"] and out["x_HII_abs_max"] <= MIXED_BAR["x_HII_abs"])
    if a_att is not None:
        out["cells_N_rel>1e-3_with_other_attempt_count"] = int((a_att[over] != r_att[over]).sum())
        out["cells_with_other_attempt_count"] = int((a_att != r_att).sum())
    return out, over


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
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the adjoint workload and print its record (for profiling the adjoint kernels)")
    ap.add_argument("--chem-ab", action="store_true",
                    help="time only the chemistry's lane refill against one cell per lane and print its record")
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
    if args.adjoint_only:
        print(json.dumps({"adjoint_262k": adjoint_timing(rt, torch)}), flush=True)
        return 0
    if args.chem_ab:
        print(json.dumps({"chem_refill_ab": chem_refill_ab(rt, torch)}), flush=True)
        return 0
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
    n_src_cells = cfg["sources"]["cell"].size
    log("creating mesh")
    mesh = rt.Mesh(cfg["mesh"])
    mode = {"auto": None, "fused": rt.RT_TRANSPORT_FUSED, "split": rt.RT_TRANSPORT_SPLIT}[args.transport]

    # Headline: no per-launch events in the timed region.
    log(f"mixed, {args.order}: {args.steps} subcycles")
    st_mixed, t_mixed, _ = timed_run(rt, mesh, cfg, rt.RT_MIXED, args.steps, args.warmup, torch, transport=mode)
    value = nc * nb * args.steps / t_mixed
    diag = st_mixed.diagnostics()
    if diag["status"] != 0:
        raise SystemExit(f"mixed run status {diag['status']}")
    fused = st_mixed.fused
    # The same run again with every launch bracketed by HIP events on the
    # stream it runs on: per-kernel launch times.
    log(f"mixed, {args.order}, per-kernel events: {args.steps} subcycles")
    st_p, t_prof, prof_mixed = timed_run(rt, mesh, cfg, rt.RT_MIXED, args.steps, 0, torch, transport=mode,
                                         profile=True)
    st_p.close()

    tiles = tile_counts(mesh)

    def kernel_table(prof, p, g, tile=tiles):
        tab = {}
        for name, (launches, ms) in prof.items():
            if launches == 0:
                continue
            avg = ms / launches
            algo = algorithmic_bytes(name, nc, nb, nf, n_sides, n_src_cells, p, g, tile)
            model = model_bytes_per_cell(name, nb, p, g) * nc
            tab[name] = dict(launches=launches, avg_ms=avg, algo_bytes=algo,
                             gbs=algo / (avg * 1e-3) / 1e9 if algo else None,
                             model_bytes=model or None, model_gbs=model / (avg * 1e-3) / 1e9 if model else None)
        return tab

    kt_mixed = kernel_table(prof_mixed, 4, 4)
    dominant = max((k for k in kt_mixed if k != "k_reduce"), key=lambda k: kt_mixed[k]["avg_ms"] * kt_mixed[k]["launches"])
    dk = kt_mixed[dominant]

    traffic = valu_busy = None
    if TRAFFIC_FILE.exists():
        rec = json.loads(TRAFFIC_FILE.read_text())
        ent = rec.get("kernels", {}).get(dominant)
        if ent and rec.get("source_digest") == kernel_source_digest() and rec.get("workload") == f"throughput_{args.n}" \
                and args.order == "hilbert":
            traffic = ent["bytes_per_launch"]
            valu_busy = ent.get("valu_busy")
    model_bpc = model_bytes_per_cell(dominant, nb, 4, 4)
    step_model = subcycle_bytes_per_cell(nb, 4, 4)

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
                   "transport": "fused" if fused else "split", "sigma_ln": 1.5},
        # Dominant kernel against the reference two-pass accounting's bytes
        # for the step it performs; this design's own bytes and the counter
        # bytes beside it.
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": dk["model_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dk["model_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_cell": model_bpc, "avg_ms": dk["avg_ms"],
                     "design_bytes_per_launch": dk["algo_bytes"], "design_achieved": dk["gbs"],
                     "traffic_over_model": traffic / (model_bpc * nc) if traffic else None,
                     # share of SIMD cycles issuing VALU instructions (SQ counters, same kernel digest)
                     "valu_busy": valu_busy},
        "subcycle_roofline": {
            name: {"bytes_per_cell": b, "GB/s": b * nc / (t_mixed / args.steps) / 1e9,
                   "frac": b * nc / (t_mixed / args.steps) / 1e9 / HBM_PEAK_GBS}
            for name, b in step_model.items()},
        "ms_per_step_with_kernel_events": t_prof / args.steps * 1e3,
        "kernels_mixed": kt_mixed,
        "chem_attempts_per_cell_subcycle": diag["substeps"] / (nc * args.steps),
    }

    if not args.no_extras and args.order == "hilbert":
        steps_e = ERROR_SUBCYCLES
        if args.steps == steps_e:
            fields_mixed, att_mixed = st_mixed.fields(), st_mixed.attempts()
        else:
            log(f"mixed, hilbert: {steps_e} subcycles for the error comparison")
            st_e, _, _ = timed_run(rt, mesh, cfg, rt.RT_MIXED, steps_e, 0, torch, transport=mode)
            fields_mixed, att_mixed = st_e.fields(), st_e.attempts()
            st_e.close()
        st_mixed.close()
        other = "split" if fused else "fused"
        log(f"mixed, hilbert, {other} transport: {args.steps} subcycles")
        try:
            st_s, t_s, _ = timed_run(rt, mesh, cfg, rt.RT_MIXED, args.steps, args.warmup, torch,
                                     transport=rt.RT_TRANSPORT_SPLIT if other == "split" else rt.RT_TRANSPORT_FUSED)
            st_s.close()
            out[f"{other}_transport_value"] = nc * nb * args.steps / t_s
            st_s, _, prof_s = timed_run(rt, mesh, cfg, rt.RT_MIXED, 20, 0, torch,
                                        transport=rt.RT_TRANSPORT_SPLIT if other == "split" else rt.RT_TRANSPORT_FUSED,
                                        profile=True)
            st_s.close()
            out[f"kernels_mixed_{other}"] = kernel_table(prof_s, 4, 4)
        except rt.RtError as e:
            out[f"{other}_transport_value"] = f"unavailable: {e}"
        log(f"fp64, hilbert: {steps_e} subcycles")
        st64, t64, _ = timed_run(rt, mesh, cfg, rt.RT_FP64, steps_e, args.warmup, torch)
        f64, att64 = st64.fields(), st64.attempts()
        st64_fused = st64.fused
        st64.close()
        v64 = nc * nb * steps_e / t64
        st64p, _, prof64 = timed_run(rt, mesh, cfg, rt.RT_FP64, 20, 0, torch, profile=True)
        st64p.close()
        fc = cfg["mesh"]["face_cells"]
        c_red = cfg["params"]["c_reduced"]
        err_mixed, over_mixed = field_errors(fields_mixed, f64, fc, c_red, att_mixed, att64)
        # Conditioning of the workload itself: the FP64 run again from n_H
        # rounded to FP32 (a relative change of at most 6e-8, the size of one
        # FP32 rounding), cell by cell against the same FP64 run.
        log(f"fp64 from n_H rounded to fp32: {steps_e} subcycles")
        nH32 = cfg["state"]["n_H"].astype(np.float32).astype(np.float64)
        st_c, _, _ = timed_run(rt, mesh, cfg, rt.RT_FP64, steps_e, 0, torch, n_H=nH32)
        f_c, att_c = st_c.fields(), st_c.attempts()
        st_c.close()
        err_ctrl, over_ctrl = field_errors(f_c, f64, fc, c_red, att_c, att64)
        err_mixed["cells_N_rel>1e-3_also_in_fp64_from_fp32_nH"] = int((over_mixed & over_ctrl).sum())
        err_mixed["cells_N_rel>1e-3_with_other_attempt_count_in_fp64_from_fp32_nH"] = int(
            (att_c[over_mixed] != att64[over_mixed]).sum())
        err_mixed["subcycles"] = steps_e
        err_ctrl["subcycles"] = steps_e
        out["mixed_error_vs_fp64"] = err_mixed
        out["fp64_nH_rounded_to_fp32_vs_fp64"] = err_ctrl
        out["fp64_value"] = v64
        out["fp64_ms_per_step"] = t64 / steps_e * 1e3
        out["mixed_speedup_vs_fp64"] = value / v64
        out["kernels_fp64"] = kernel_table(prof64, 8, 8)
        out["fp64_subcycle_roofline"] = {
            name: {"bytes_per_cell": b, "GB/s": b * nc / (t64 / steps_e) / 1e9,
                   "frac": b * nc / (t64 / steps_e) / 1e9 / HBM_PEAK_GBS}
            for name, b in subcycle_bytes_per_cell(nb, 8, 8).items()}
        out["fp64_transport"] = "fused" if st64_fused else "split"
        del fields_mixed, f64, f_c
        mesh.close()
        log("random cell order (mixed)")
        cfg_r = rtgen.random_order(cfg)
        mesh_r = rt.Mesh(cfg_r["mesh"])
        st_r, t_r, _ = timed_run(rt, mesh_r, cfg_r, rt.RT_MIXED, args.steps, args.warmup, torch)
        out["random_order_transport"] = "fused" if st_r.fused else "split"
        st_r.close()
        out["random_order_value"] = nc * nb * args.steps / t_r
        st_r, _, prof_r = timed_run(rt, mesh_r, cfg_r, rt.RT_MIXED, 20, 0, torch, profile=True)
        st_r.close()
        out["kernels_mixed_random"] = kernel_table(prof_r, 4, 4, tile_counts(mesh_r))
        mesh_r.close()
        del cfg_r
        out["adjoint_262k"] = adjoint_timing(rt, torch)
    else:
        st_mixed.close()
        mesh.close()

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        legs = cpu_baseline()
        out["cpu_baseline"] = legs["all_cores"]
        out["cpu_baseline_single_thread"] = legs["single_thread"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
