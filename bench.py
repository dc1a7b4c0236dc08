"""Throughput of Quadrature-TreeSHAP Shapley values on one MI355X.

Workload (synthetic, seeded): 1000 random trees of depth 8 (at most 256
leaves) over 100 features, 20 of them integer-valued, covers from 100k
training rows, leaf values N(0, 0.05), 100k explained samples.  One step is
one qts_shap_values call over all samples and every root-to-leaf path, with
the ensemble and the samples already resident in HBM.

Prints one JSON line: sample-tree-leaf paths/s of the FP32 form (FP32
quadrature, FP64 accumulation), with the plain FP64 form, the error of both
against the FP64 oracle on sampled rows, the roofline of the values kernel,
and the oracle's own rate on the host cores as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sample-tree-leaf paths/s for SHAP, FP32 vs FP64 GPU, at max rel err ≤1e-5"

# MI355X published vector peaks (256 CUs at 2.4 GHz).  FP64: one wave64 FMA per
# CU per clock.  FP32: twice that.  Plain (not packed) FP32 FMAs and multiplies
# whose operands are all vector registers issue at up to 1.71 wave
# instructions per CU per clock in probes on this GPU, so the FP32 figure is the
# ceiling for this build too, although it uses no packed FP32 instructions.
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# LDS FP64 atomic add, measured on MI355X: 2.45 lanes per clock per CU, random
# addresses in an 80 KB table (the interactions kernel's accumulator)
LDS_F64_ATOMIC_RATE = 2.45 * 256 * 2.4e9

# HBM bytes per launch of the first-order kernel on this workload in its timed
# launch shape, from two rocprofv3 --pmc runs (FETCH_SIZE x 2 and WRITE_SIZE x 1,
# the factors a 1 GiB device copy reads in the same runs); see
# profiles/values_kernel_c2_values.md.  Valid only for the kernel source they
# were measured on (its SHA-256 prefix); otherwise traffic is reported as null.
TRAFFIC = {"kernel_source": "paper_2605_04497_amd/csrc/kernels/values.hip",
           "sha256_16": "61456a43db1a66e4", "fetch_bytes": 9.3678e+08, "write_bytes": 1.6800e+09,
           "shape": [8, 32768]}


def measured_traffic(shape):
    import hashlib
    path = os.path.join(ROOT, TRAFFIC["kernel_source"])
    try:
        with open(path, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    if h != TRAFFIC["sha256_16"] or list(shape) != TRAFFIC["shape"]:
        return None
    return TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]
FLOPS_PER_ELEMENT = 51  # per (sample, path, unique feature): 8 nodes x 6 + 3

# Executed flops per call of the other legs' kernels: SQ_INSTS_VALU_FLOPS_FP32
# (or _FP64) x 64 summed over one call's dispatches, from rocprofv3 --pmc runs
# of `bench.py --only <leg>` (profiles/ holds the commands and counts).  Valid
# only for the kernel sources they were measured on (SHA-256 prefix over the
# kernel files); otherwise the executed figures are reported as null.
KERNEL_SOURCES = ("paper_2605_04497_amd/csrc/kernels/values.hip",
                  "paper_2605_04497_amd/csrc/kernels/interactions.hip",
                  "paper_2605_04497_amd/csrc/kernels/dfs.hip",
                  "paper_2605_04497_amd/csrc/kernels/common.hip")
EXECUTED_FLOPS_SHA = "51c12ee84f59c8f8"
# (leg, precision) -> (FP32 flops, FP64 flops) per call
EXECUTED_FLOPS = {
    ("values", "fp32"): (2.9722e+12, 2.3578e+06),
    ("values", "fp64"): (1.0722e+08, 4.3635e+12),
    ("interactions", "fp32"): (2.0298e+12, 3.7527e+09),
    ("interactions", "fp64"): (1.0476e+08, 3.0189e+12),
    ("interactions_dfs", "fp32"): (8.7750e+11, 1.3826e+08),
    ("interactions_dfs", "fp64"): (3.8014e+08, 2.0795e+12),
    ("adjoint", "fp32"): (3.8300e+10, 1.7949e+09),
    ("adjoint", "fp64"): (1.2013e+07, 5.8223e+10),
    ("deep_values", "fp32"): (4.5586e+11, 6.7738e+05),
    ("deep_values", "fp64"): (3.9215e+07, 5.2106e+11),
    ("deep_interactions", "fp32"): (2.9683e+12, 3.7794e+08),
    ("deep_interactions", "fp64"): (1.7664e+08, 3.8937e+12),
    ("deep_interactions_dfs", "fp32"): (5.6340e+11, 2.0386e+08),
    ("deep_interactions_dfs", "fp64"): (2.5984e+08, 1.3728e+12),
    ("deep_third_order", "fp32"): (8.2126e+11, 2.2150e+07),
    ("deep_third_order", "fp64"): (1.4848e+08, 9.4479e+11),
    ("deep_third_order_dfs", "fp32"): (1.8750e+11, 3.3869e+05),
    ("deep_third_order_dfs", "fp64"): (7.5008e+06, 2.3076e+11),
}

# One call of each leg for the counter runs (`--flop-call LEG:PREC` under
# rocprofv3 --pmc): workload, samples ("pairs": --pair-samples, an int: the
# first that many, None: all), the call, the interactions traversal, and the
# sample count the leg tunes its launch shapes at (None: the call's).
FLOP_CALLS = {
    "values": ("c2_values", None, "values", None, None),
    "interactions": ("c3_interactions", "pairs", "interactions", "paths", None),
    "interactions_dfs": ("c3_interactions", "pairs", "interactions", "dfs", None),
    "adjoint": ("c4_adjoint", None, "backward", None, None),
    "deep_values": ("c5_deep", None, "values", None, None),
    "deep_interactions": ("c5_deep", None, "interactions", "paths", None),
    "deep_interactions_dfs": ("c5_deep", None, "interactions", "dfs", None),
    "deep_third_order": ("c5_deep", 200, "interactions3", "paths", 10000),
    "deep_third_order_dfs": ("c5_deep", 200, "interactions3", "dfs", 10000),
}
# kernels that only the autotuner launches (synthetic inputs), left out of a
# call's counts
TUNER_KERNELS = ("fill_uniform_kernel", "widen_kernel")


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def executed(leg, precision, seconds):
    """Executed flops of one call of a leg from its counters (FP32 and FP64
    vector flops together), as TFLOP/s over `seconds`, with the fraction of
    the published peak of the precision;
    None where the table does not hold the leg or the kernels have changed."""
    fl = EXECUTED_FLOPS.get((leg, precision))
    if fl is None or EXECUTED_FLOPS_SHA != kernel_sources_sha():
        return None
    tf = (fl[0] + fl[1]) / seconds / 1e12
    peak = PEAK_FP32_TFLOPS if precision == "fp32" else PEAK_FP64_TFLOPS
    return {"executed_tflops": tf, "frac_of_peak": tf / peak, "peak_tflops": peak,
            "flops_per_call": {"fp32": fl[0], "fp64": fl[1]},
            "source": "SQ_INSTS_VALU_FLOPS_FP32/_FP64 x 64 over one call's dispatches, "
                      "rocprofv3 --pmc of bench.py --flop-call %s:%s" % (leg, precision)}


def flop_call(args, torch, q, synth, dev):
    """One eager call of a leg, launch shapes from the tune cache (a miss would
    add the tuner's launches to the counts, so it is an error)."""
    leg, prec = args.flop_call.split(":")
    name, samples, call, trav, tune_m = FLOP_CALLS[leg]
    over = {"M": args.pair_samples} if samples == "pairs" else {}
    wl = synth.make_workload(name, **over)
    e = q.Ensemble(wl.ensemble, device=dev)
    X = torch.from_numpy(wl.X).to(dev)
    tune_m = tune_m or X.shape[0]
    if isinstance(samples, int):
        X = X[:samples].contiguous()
    M = X.shape[0]
    if trav:
        e.set_pair_traversal(trav)
    G = None
    if call == "backward":
        g = 2.0 * (0.0 - wl.target.astype(np.float64))
        G = torch.from_numpy(g.astype(np.float32) if prec == "fp32" else g).to(dev)
    _, m0 = q.tune_cache_stats()
    if not args.no_autotune:
        e.autotune(tune_m, prec)
    _, m1 = q.tune_cache_stats()
    if m1 > m0:
        raise SystemExit("tune cache miss (%d): the counts would include the tuner's launches"
                         % (m1 - m0))
    torch.cuda.synchronize()
    if call == "values":
        e.shap_values(X, prec)
    elif call == "interactions":
        e.shap_interactions(X, prec)
    elif call == "interactions3":
        e.shap_interactions3(X, prec)
    else:
        e.shap_backward(X, G, prec)
    torch.cuda.synchronize()
    print(json.dumps({"flop_call": leg, "precision": prec, "workload": name, "samples": M,
                      "kernel_sources_sha": kernel_sources_sha()}), flush=True)
    e.close()


def pmc_summary(paths):
    """Per kernel, dispatch count and the sum over its dispatches (and over a
    counter's instances within each) of every counter in rocprofv3 result
    databases; FP32/FP64 executed flops of all kernels but the tuner's."""
    import sqlite3
    for path in paths:
        con = sqlite3.connect(path)
        rows = con.execute(
            "select k.name, p.counter_name, p.dispatch_id, sum(p.counter_value), k.duration "
            "from pmc_events p join kernels k on p.dispatch_id = k.dispatch_id "
            "group by p.dispatch_id, p.counter_name").fetchall()
        per = {}
        for name, counter, disp, val, dur in rows:
            kn = name.split("(")[0].split("<")[0].split()[-1]
            d = per.setdefault(kn, {"dispatches": set(), "ns": {}, "counters": {}})
            d["dispatches"].add(disp)
            d["ns"][disp] = dur
            d["counters"][counter] = d["counters"].get(counter, 0.0) + val
        print("# %s" % path)
        flops = [0.0, 0.0]
        for kn, d in sorted(per.items()):
            ms = sum(d["ns"].values()) / 1e6
            print("%-28s dispatches %4d  %.3f ms  %s" % (
                kn, len(d["dispatches"]), ms,
                "  ".join("%s=%.4e" % kv for kv in sorted(d["counters"].items()))))
            if kn not in TUNER_KERNELS:
                flops[0] += 64.0 * d["counters"].get("SQ_INSTS_VALU_FLOPS_FP32", 0.0)
                flops[1] += 64.0 * d["counters"].get("SQ_INSTS_VALU_FLOPS_FP64", 0.0)
        print("executed flops (x64, tuner kernels excluded): fp32 %.4e fp64 %.4e" % tuple(flops))


def shared_kernel_flops(rows, elements, shared, kept):
    """FP32 flops (FMA = 2) per sample of the first-order kernel for rows of at
    most 8 features at 8 nodes: a row of d features whose first s slots after
    slot 0 are reused from the previous row costs
      16 (8 - s)          factor FMAs of the slots it evaluates (padding included)
      8 (6 - min(s, 6))   prefix products over slots 1..6 not kept from the
                          previous row
      16 d                a 15-flop node sum and a scale per feature
      48                  suffix products over slots 7..2
    = 224 + 16 d - 16 s - 8 min(s, 6); summed over the table:
    224 R + 16 E - 16 S - 8 K (K: min(s, 6) summed, qts_info's prefix_kept)."""
    return 224.0 * rows + 16.0 * elements - 16.0 * shared - 8.0 * kept


def pair_flops(d):
    """Algorithmic flops of one (sample, row) of d features in the
    interactions kernel: per node, d factors (FMA), d-1 products, d
    reciprocals, d scalings into r and g, d additions into phi, and d(d-1)/2
    pair FMAs; 8 (d^2 + 6 d - 1) in all."""
    d = np.asarray(d, np.float64)
    return 8.0 * (2 * d + (d - 1) + 4 * d + d * (d - 1))


TUNE_CACHE = os.path.join(ROOT, "paper_2605_04497_amd", "tune_cache_mi355x.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--samples", type=int, default=None, help="override M (testing)")
    ap.add_argument("--trees", type=int, default=None, help="override T (testing)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-rows", type=int, default=16)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the interactions and adjoint measurements")
    ap.add_argument("--pair-samples", type=int, default=1024)
    ap.add_argument("--no-full-interactions", action="store_true",
                    help="skip the interactions calls on all 50k samples (8 GB FP32 output)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotune cache file (shapes measured on MI355X ship with the "
                         "package; keys include the kernel sources, so edited kernels "
                         "tune afresh); '' turns the cache off")
    ap.add_argument("--no-merge", action="store_true",
                    help="first-order calls walk every leaf's path (no sibling merging)")
    ap.add_argument("--eager", action="store_true",
                    help="launch eagerly instead of replaying a captured HIP graph")
    ap.add_argument("--flop-call", default=None, metavar="LEG:PREC",
                    help="one call of a leg (%s) for counter runs" % ", ".join(FLOP_CALLS))
    ap.add_argument("--pmc-summary", nargs="+", default=None, metavar="DB",
                    help="summarise rocprofv3 --pmc result databases and exit (no GPU)")
    ap.add_argument("--only", default=None,
                    choices=["interactions", "interactions_full", "adjoint", "deep", "small",
                             "third_order", "wide", "groups"],
                    help="run one leg alone and print its JSON (profiling aid)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MB (a "
                         "known-size reference for the memory counters)")
    return ap.parse_args()


def time_steps(fn, steps, warmup, torch, kind="values"):
    """Run `warmup` untimed steps, then `steps` timed ones on the current
    stream: HIP events around each step (spread) and around the whole run,
    and the library's own event pairs around its launches (kernel time)."""
    import paper_2605_04497_amd as q
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    q.read_kernel_timing(kind)  # drop warmup events
    q.set_kernel_timing(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    q.set_kernel_timing(False)
    kern_ms, calls = q.read_kernel_timing(kind)
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return {"ms_per_step": ev[0].elapsed_time(ev[steps]) / steps, "wall_s": wall,
            "kernel_ms": kern_ms / max(1, calls), "calls": calls,
            "step_ms_median": float(np.median(per)), "step_ms_min": float(min(per)),
            "step_ms_max": float(max(per))}


def cpu_baseline(ens, X, seconds, oracle):
    threads = oracle.default_threads()
    n_leaves = ens.n_leaves()
    # probe with two rows per thread (the oracle threads over rows), then size
    # the timed sample for about `seconds` of work
    probe = min(X.shape[0], 2 * threads)
    t0 = time.perf_counter()
    oracle.shap_values(ens, X[:probe], n=8, threads=threads)
    rate = probe / max(time.perf_counter() - t0, 1e-6)   # rows per second
    rows = int(max(probe, min(X.shape[0], rate * seconds)))
    rows = max(threads, (rows // threads) * threads)
    t0 = time.perf_counter()
    oracle.shap_values(ens, X[:rows], n=8, threads=threads)
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    # one core, on a smaller sample sized for about a fifth of the time
    per_row_1core = dt / rows * threads
    rows1 = max(1, min(rows, int(seconds / 5.0 / max(per_row_1core, 1e-9))))
    t1 = time.perf_counter()
    oracle.shap_values(ens, X[:rows1], n=8, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": rows * n_leaves / dt, "unit": "paths/s", "cores": threads, "kind": "oracle",
            "sample": "%d of the workload's explained rows, all 1000 trees, FP64 8-node path "
                      "quadrature, %.1f s, %s" % (rows, dt, cpu),
            "single_core": {"value": rows1 * n_leaves / dt1, "unit": "paths/s", "cores": 1,
                            "sample": "%d rows, %.1f s" % (rows1, dt1)}}


def traversal(e, prec):
    """The form qts_shap_interactions takes for a precision ('paths' or 'dfs')."""
    return "dfs" if e.refresh_info()["pairs_dfs"] & (1 if prec == "fp32" else 2) else "paths"


def traversal3(e, prec):
    """The form qts_shap_interactions3 takes for a precision."""
    return "dfs" if e.refresh_info()["pairs_dfs"] & (4 if prec == "fp32" else 8) else "paths"


def measure_interactions(args, torch, q, synth, oracle, dev):
    """Pairwise interactions on the full 500-tree, 200-feature ensemble (depths
    3..20), over a slice of its explained samples; FP32 form."""
    wl = synth.make_workload("c3_interactions", M=args.pair_samples)
    ens = wl.ensemble
    e = q.Ensemble(ens, device=dev)
    X = torch.from_numpy(wl.X).to(dev)
    M = X.shape[0]
    tab = e.export_paths()
    # work of the rows the kernels walk (a row merges two sibling leaves of up
    # to 16 features, or is one path): sum over rows of pair_flops(d), from
    # the row counts: sum d^2 = 2 U + E
    N, E, U = (float(e.info[k]) for k in ("n_pair_rows", "n_pair_elements", "n_pair_updates"))
    flops = float(M) * 8.0 * (2.0 * U + 7.0 * E - N)
    pairs = float(M) * U
    F = e.n_features
    res = {}
    trav = {}
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        if not args.no_autotune:
            e.autotune(M, prec)
        trav[prec] = traversal(e, prec)
        e.set_graph_replay(not args.eager)
        Phi = torch.empty((M, F, F), dtype=dt, device=dev)
        res[prec] = time_steps(lambda: e.shap_interactions(X, prec, out=Phi), 3, 1, torch,
                               "interactions")
        del Phi
        e.set_graph_replay(False)
    Phi = e.shap_interactions(X[:2], "fp32").double().cpu().numpy()
    _, Phi_o = oracle.shap_interactions(ens, wl.X[:2], n=8)
    err = float((np.abs(Phi - Phi_o).reshape(2, -1).max(1)
                 / np.abs(Phi_o).reshape(2, -1).max(1)).max())
    dfs = measure_dfs_form(args, torch, e, X, Phi_o, "interactions_dfs")
    # LDS FP64 atomics of the path form: one per pair update
    lds_rate = pairs / (res["fp32"]["kernel_ms"] * 1e-3) if trav["fp32"] == "paths" else None
    leg = {"paths": "interactions", "dfs": "interactions_dfs"}
    out = {"workload": "c3_interactions: 500 grown trees, depths 3..20, leaf cap 4096, 200 "
                       "features; first %d of the 50k explained samples" % M,
           "traversal": trav,
           "samples": M, "leaves": e.n_leaves, "mean_unique": float(tab["path_len"].mean()),
           "kernel_rows": int(N), "pair_updates_per_sample": int(U),
           "value": M * e.n_leaves / (res["fp32"]["ms_per_step"] * 1e-3), "unit": "paths/s",
           "ms_per_step": res["fp32"]["ms_per_step"], "kernel_ms": res["fp32"]["kernel_ms"],
           "fp64_ms_per_step": res["fp64"]["ms_per_step"],
           "max_rel_err_fp32": err, "rows_checked": 2,
           "executed_fp32": executed(leg[trav["fp32"]], "fp32", res["fp32"]["kernel_ms"] * 1e-3),
           "executed_fp64": executed(leg[trav["fp64"]], "fp64", res["fp64"]["kernel_ms"] * 1e-3),
           "pair_updates_per_s": lds_rate,
           "frac_of_lds_f64_atomic_rate": lds_rate / LDS_F64_ATOMIC_RATE if lds_rate else None,
           "fp64_kernel_ms": res["fp64"]["kernel_ms"],
           "launch": "hipGraph replay" if not args.eager else "eager",
           "depth_first_form": dfs}
    e.close()
    return out


def measure_dfs_form(args, torch, e, X, Phi_o, leg, steps=3):
    """The interactions call in each traversal, forced: collapsed paths and
    the depth-first form (Algorithm 1 at order 2), step times in both
    precisions, the depth-first form's error on the first rows, and the form
    the autotuner keeps under the default ('auto')."""
    M, F = X.shape[0], e.n_features
    out = {}
    ms = {}
    for trav in ("paths", "dfs"):
        e.set_pair_traversal(trav)
        if trav == "dfs":
            out["pair_updates_per_sample"] = int(e.info["n_dfs_updates"])
            out["internal_nodes"] = int(e.info["n_dfs_nodes"])
        for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
            e.set_graph_replay(not args.eager)
            Phi = torch.empty((M, F, F), dtype=dt, device=X.device)
            r = time_steps(lambda: e.shap_interactions(X, prec, out=Phi), steps, 1, torch,
                           "interactions")
            ms[trav, prec] = r["ms_per_step"]
            if trav == "dfs":
                out[prec + "_ms_per_step"] = r["ms_per_step"]
                out[prec + "_kernel_ms"] = r["kernel_ms"]
                out["executed_" + prec] = executed(leg, prec, r["kernel_ms"] * 1e-3)
                if prec == "fp32":
                    n = Phi_o.shape[0]
                    G = Phi[:n].double().cpu().numpy()
                    out["max_rel_err_fp32"] = float(
                        (np.abs(G - Phi_o).reshape(n, -1).max(1)
                         / np.abs(Phi_o).reshape(n, -1).max(1)).max())
            else:
                out["paths_" + prec + "_ms_per_step"] = r["ms_per_step"]
            del Phi
            e.set_graph_replay(False)
    for prec in ("fp32", "fp64"):
        out[prec + "_speedup_over_paths"] = ms["paths", prec] / ms["dfs", prec]
    e.set_pair_traversal("auto")
    for prec in ("fp32", "fp64"):
        if not args.no_autotune:
            e.autotune(M, prec)
    out["auto_keeps"] = {p: ("dfs" if e.refresh_info()["pairs_dfs"] & b else "paths")
                         for p, b in (("fp32", 1), ("fp64", 2))}
    return out


def measure_adjoint(args, torch, q, synth, oracle, dev):
    """Adjoint to the 12,800 leaf values of 200 full depth-6 trees, 20k samples."""
    wl = synth.make_workload("c4_adjoint")
    ens = wl.ensemble
    e = q.Ensemble(ens, device=dev)
    X = torch.from_numpy(wl.X).to(dev)
    M = X.shape[0]
    G = torch.from_numpy(2.0 * (np.zeros_like(wl.target, dtype=np.float64)
                                - wl.target.astype(np.float64))).to(dev)
    G32 = G.float()
    res = {}
    gl = torch.empty(e.n_leaves, dtype=torch.float64, device=dev)
    for prec, g in (("fp32", G32), ("fp64", G)):
        if not args.no_autotune:
            e.autotune(M, prec)
        e.set_graph_replay(not args.eager)
        res[prec] = time_steps(lambda: e.shap_backward(X, g, prec, out=gl), 10, 2, torch,
                               "backward")
        e.set_graph_replay(False)
    rows = np.arange(0, M, 10)
    want = oracle.leaf_grad(ens, wl.X[rows], G32.double().cpu().numpy()[rows])
    got = e.shap_backward(X[torch.from_numpy(rows).to(dev)], G32[torch.from_numpy(rows).to(dev)],
                          "fp32").cpu().numpy()
    err = float(np.abs(got - want).max() / np.abs(want).max())
    out = {"workload": "c4_adjoint: 200 full depth-6 trees (12,800 leaves), 50 features, "
                       "20k samples, grad of ||phi - target||^2",
           "value": M * e.n_leaves / (res["fp32"]["ms_per_step"] * 1e-3), "unit": "paths/s",
           "ms_per_step": res["fp32"]["ms_per_step"], "kernel_ms": res["fp32"]["kernel_ms"],
           "fp64_ms_per_step": res["fp64"]["ms_per_step"],
           "max_rel_err_fp32": err, "rows_checked": int(len(rows)),
           "kernel_rows": int(e.info["n_value_paths"]),
           "executed_fp32": executed("adjoint", "fp32", res["fp32"]["kernel_ms"] * 1e-3),
           "executed_fp64": executed("adjoint", "fp64", res["fp64"]["kernel_ms"] * 1e-3)}
    e.close()
    return out


def path_unique_counts(ens):
    """Unique features of every root-to-leaf path of a synthetic ensemble."""
    out = []
    for t in range(ens.n_trees):
        a = int(ens.tree_offsets[t])
        stack = [(0, frozenset())]
        while stack:
            node, fs = stack.pop()
            g = a + node
            if ens.left[g] < 0:
                out.append(len(fs))
                continue
            fs = fs | {int(ens.feature[g])}
            stack.append((int(ens.left[g]), fs))
            stack.append((int(ens.right[g]), fs))
    return out


def measure_third_order(args, torch, q, synth, oracle, dev):
    """Third-order Shapley interaction indices (Theorem 1 with |S| = 3) on the
    adjoint workload's ensemble (200 full depth-6 trees, 50 features: 19,600
    feature triples per sample), 2000 samples, FP32 and FP64."""
    import math
    wl = synth.make_workload("c4_adjoint")
    ens = wl.ensemble
    e = q.Ensemble(ens, device=dev)
    M = 2000
    X = torch.from_numpy(wl.X[:M]).to(dev)
    F = e.n_features
    T3 = F * (F - 1) * (F - 2) // 6
    triples = sum(math.comb(d, 3) for d in path_unique_counts(ens))
    res = {}
    trav = {}
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        if not args.no_autotune:
            e.autotune(M, prec)
        trav[prec] = traversal3(e, prec)
        out = torch.empty((M, T3), dtype=dt, device=dev)
        e.set_graph_replay(not args.eager)
        res[prec] = time_steps(lambda: e.shap_interactions3(X, prec, out=out), 5, 1, torch,
                               "interactions3")
        e.set_graph_replay(False)
        del out
    # 16 rows spread over the samples (first and last included) against the
    # oracle, taken from a call over all the samples (the timed launches)
    rows = np.linspace(0, M - 1, 16).astype(np.int64)
    want = oracle.shap_sii3(ens, wl.X[rows], n=8)
    got = e.triples_dense(e.shap_interactions3(X, "fp32")[torch.from_numpy(rows).to(dev)],
                          F).double().cpu().numpy()
    n = len(rows)
    err = float((np.abs(got - want).reshape(n, -1).max(1)
                 / np.abs(want).reshape(n, -1).max(1)).max())
    t32 = res["fp32"]["ms_per_step"] * 1e-3
    out = {"workload": "third order on the c4_adjoint ensemble: 200 full depth-6 trees (12,800 "
                       "leaves), 50 features, first 2000 samples; packed [M, 19600] output",
           "samples": M, "triples_per_sample": triples, "traversal": trav,
           "value": M * e.n_leaves / t32, "unit": "paths/s",
           "ms_per_step": res["fp32"]["ms_per_step"], "kernel_ms": res["fp32"]["kernel_ms"],
           "fp64_ms_per_step": res["fp64"]["ms_per_step"],
           "triple_updates_per_s": M * triples / t32,
           "max_rel_err_fp32": err, "rows_checked": int(n),
           "launch": "hipGraph replay" if not args.eager else "eager"}
    e.close()
    return out


def measure_deep(args, torch, q, synth, oracle, dev):
    """Deep trees (100 grown trees of depth 32, leaf cap 512, 64 features, 10k
    samples): values and interactions, FP32 error against the 8-node FP64
    oracle and the 8-node rule's own gap to the exact rule (Theorem 2: exact
    for d <= 16 first order, d <= 17 pairs)."""
    wl = synth.make_workload("c5_deep")
    ens = wl.ensemble
    e = q.Ensemble(ens, device=dev)
    X = torch.from_numpy(wl.X).to(dev)
    M, F = X.shape[0], e.n_features
    out = {"workload": "c5_deep: 100 grown trees depth 32, leaf cap 512, 64 features, 10k "
                       "explained samples", "samples": M, "leaves": e.n_leaves,
           "max_unique": e.info["max_unique"]}
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        if not args.no_autotune:
            e.autotune(M, prec)
        tr = traversal(e, prec)
        e.set_graph_replay(not args.eager)
        phi = torch.empty((M, F), dtype=dt, device=dev)
        r = time_steps(lambda: e.shap_values(X, prec, out=phi), 5, 1, torch)
        Phi = torch.empty((M, F, F), dtype=dt, device=dev)
        ri = time_steps(lambda: e.shap_interactions(X, prec, out=Phi), 2, 1, torch, "interactions")
        e.set_graph_replay(False)
        vt = r["kernel_ms"] * 1e-3
        pt = ri["kernel_ms"] * 1e-3
        out["values_" + prec] = {"value": M * e.n_leaves / (r["ms_per_step"] * 1e-3),
                                 "ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"],
                                 "executed": executed("deep_values", prec, vt)}
        out["interactions_" + prec] = {"value": M * e.n_leaves / (ri["ms_per_step"] * 1e-3),
                                       "ms_per_step": ri["ms_per_step"],
                                       "kernel_ms": ri["kernel_ms"], "traversal": tr,
                                       "executed": executed(
                                           "deep_interactions" + ("_dfs" if tr == "dfs" else ""),
                                           prec, pt)}
        # third order on 200 of the samples (F = 64: 41,664 triples per sample)
        T3 = F * (F - 1) * (F - 2) // 6
        M3 = 200
        o3 = torch.empty((M3, T3), dtype=dt, device=dev)
        tr3 = traversal3(e, prec)
        X3 = X[:M3]
        e.set_graph_replay(not args.eager)
        r3 = time_steps(lambda: e.shap_interactions3(X3, prec, out=o3), 2, 1, torch,
                        "interactions3")
        out["third_order_" + prec] = {"samples": M3, "ms_per_step": r3["ms_per_step"],
                                      "kernel_ms": r3["kernel_ms"],
                                      "value": M3 * e.n_leaves / (r3["ms_per_step"] * 1e-3),
                                      "traversal": tr3,
                                      "updates_per_sample": int(e.info["n_dfs_updates3"])
                                      if tr3 == "dfs" else None,
                                      "executed": executed(
                                          "deep_third_order" + ("_dfs" if tr3 == "dfs" else ""),
                                          prec, r3["kernel_ms"] * 1e-3)}
        # the other form beside it
        e.set_pair_traversal("paths" if tr3 == "dfs" else "dfs")
        r3o = time_steps(lambda: e.shap_interactions3(X3, prec, out=o3), 2, 1, torch,
                         "interactions3")
        out["third_order_" + prec]["other_form_ms_per_step"] = r3o["ms_per_step"]
        e.set_pair_traversal("auto")
        e.set_graph_replay(False)
        o3 = e.shap_interactions3(X[:M3], prec, out=o3)
        if prec == "fp32":
            rows3 = np.array([0, M3 - 1])
            want3 = oracle.shap_sii3(ens, wl.X[rows3], n=8)
            got3 = e.triples_dense(o3[torch.from_numpy(rows3).to(dev)], F).double().cpu().numpy()
            out["third_order_fp32"]["max_rel_err"] = float(
                (np.abs(got3 - want3).reshape(2, -1).max(1)
                 / np.abs(want3).reshape(2, -1).max(1)).max())
        del o3
        if prec == "fp32":
            rows = np.arange(0, M, M // 8)[:8]
            phi_o = oracle.shap_values(ens, wl.X[rows], n=8)
            phi_x = oracle.shap_values(ens, wl.X[rows], n=32)
            _, Phi_o = oracle.shap_interactions(ens, wl.X[rows[:1]], n=8)
            _, Phi_x = oracle.shap_interactions(ens, wl.X[rows[:1]], n=32)
            g = phi[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
            G = Phi[torch.from_numpy(rows[:1]).to(dev)].double().cpu().numpy()

            def rel(a, b):
                a, b = a.reshape(a.shape[0], -1), b.reshape(b.shape[0], -1)
                return float((np.abs(a - b).max(1) / np.maximum(np.abs(b).max(1), 1e-30)).max())
            out["max_rel_err_fp32"] = {"phi": rel(g, phi_o), "Phi": rel(G, Phi_o),
                                       "rows_checked": [int(len(rows)), 1]}
            assert rows[0] == 0  # Phi_o is sample 0's
            out["gap_8_nodes_vs_exact"] = {"phi": rel(phi_o, phi_x), "Phi": rel(Phi_o, Phi_x),
                                           "measure": "row-normwise, FP64 oracle n=8 vs n=32"}
        del phi, Phi
    # the depth-first form of the interactions call (sample 0 against the oracle)
    out["interactions_depth_first_form"] = measure_dfs_form(args, torch, e, X, Phi_o,
                                                            "deep_interactions_dfs", steps=2)
    e.close()
    return out


def measure_small(args, torch, q, synth, oracle, dev):
    """The small plain-FP64 case (10 trees of depth 4, 8 features, 1000
    samples): per-call latency, eager launches vs HIP graph replay."""
    wl = synth.make_workload("c1_small")
    ens = wl.ensemble
    e = q.Ensemble(ens, device=dev)
    X = torch.from_numpy(wl.X).to(dev)
    M = X.shape[0]
    phi = torch.empty((M, e.n_features), dtype=torch.float64, device=dev)
    res = {}
    for mode in ("eager", "graph"):
        e.set_graph_replay(mode == "graph")
        res[mode] = time_steps(lambda: e.shap_values(X, "fp64", out=phi), 200, 20, torch)
    e.set_graph_replay(False)
    from oracle import brute
    want = oracle.shap_values(ens, wl.X, n=8)
    got = phi.cpu().numpy()
    err = float((np.abs(got - want).max(1) / np.maximum(np.abs(want).max(1), 1e-30)).max())
    err_b = float(np.abs(brute.shap_values(ens, wl.X[:20]) - got[:20]).max()
                  / np.abs(got[:20]).max())
    e.close()
    return {"workload": "c1_small: 10 random trees depth 4, 8 features, 1000 samples, FP64",
            "eager_us_per_call": res["eager"]["ms_per_step"] * 1e3,
            "graph_us_per_call": res["graph"]["ms_per_step"] * 1e3,
            "value": M * e.n_leaves / (res["graph"]["ms_per_step"] * 1e-3), "unit": "paths/s",
            "max_rel_err_fp64": err, "max_rel_err_vs_enumeration_20_rows": err_b}


def measure_wide(args, torch, q, synth, oracle, dev):
    """Fashion-MNIST's width: 784 features (the sample tile of every feature
    does not fit in LDS, so work items take segments of rows with at most 96
    distinct features).  200 random trees of depth 8 (20% integer columns),
    20k samples: values in FP32 and FP64 and the adjoint, with the error on
    sampled rows."""
    wl = synth.make_workload("c2_values", F=784, T=200, M=20000)
    ens = wl.ensemble
    e = q.Ensemble(ens, device=dev)
    X = torch.from_numpy(wl.X).to(dev)
    M, F = X.shape[0], e.n_features
    res = {}
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        if not args.no_autotune:
            e.autotune(M, prec)
        e.set_graph_replay(not args.eager)
        phi = torch.empty((M, F), dtype=dt, device=dev)
        res[prec] = time_steps(lambda: e.shap_values(X, prec, out=phi), 5, 1, torch)
        G = torch.ones((M, F), dtype=dt, device=dev)
        gl = torch.empty(e.n_leaves, dtype=torch.float64, device=dev)
        res["adj_" + prec] = time_steps(lambda: e.shap_backward(X, G, prec, out=gl), 5, 1, torch,
                                        "backward")
        e.set_graph_replay(False)
        if prec == "fp32":
            rows = np.array([0, M // 2, M - 1])
            want = oracle.shap_values(ens, wl.X[rows], n=8)
            got = phi[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
            res["err"] = float((np.abs(got - want).max(1) / np.abs(want).max(1)).max())
        del phi, G
    out = {"workload": "784 features (Fashion-MNIST's width): 200 random trees depth 8, "
                       "20%% integer columns, %d leaves, 20k samples" % e.n_leaves,
           "segments": int(e.info["n_value_segments"]),
           "value": M * e.n_leaves / (res["fp32"]["ms_per_step"] * 1e-3), "unit": "paths/s",
           "ms_per_step": res["fp32"]["ms_per_step"],
           "fp64_ms_per_step": res["fp64"]["ms_per_step"],
           "adjoint_ms_per_step": res["adj_fp32"]["ms_per_step"],
           "adjoint_fp64_ms_per_step": res["adj_fp64"]["ms_per_step"],
           "max_rel_err_fp32": res["err"], "rows_checked": 3}
    e.close()
    return out


def measure_groups(args, torch, q, synth, oracle, dev):
    """A three-output model (tree t adds to output t mod 3, as the rounds of
    a multiclass booster): the headline's tree recipe with 300 trees, 20k
    samples; phi[M, 3, 100] in FP32 and FP64."""
    wl = synth.make_workload("c2_values", T=300, M=20000, groups=3)
    ens = wl.ensemble
    e = q.Ensemble(ens, device=dev)
    X = torch.from_numpy(wl.X).to(dev)
    M, F, K = X.shape[0], e.n_features, e.n_groups
    res = {}
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        if not args.no_autotune:
            e.autotune(M, prec)
        e.set_graph_replay(not args.eager)
        phi = torch.empty((M, K, F), dtype=dt, device=dev)
        res[prec] = time_steps(lambda: e.shap_values(X, prec, out=phi), 5, 1, torch)
        e.set_graph_replay(False)
        if prec == "fp32":
            rows = np.array([0, M - 1])
            want = oracle.shap_values_grouped(ens, wl.X[rows], n=8).reshape(2 * K, F)
            got = phi[torch.from_numpy(rows).to(dev)].double().cpu().numpy().reshape(2 * K, F)
            res["err"] = float((np.abs(got - want).max(1) / np.abs(want).max(1)).max())
        del phi
    out = {"workload": "3 outputs: 300 random trees depth 8 (100 per output), 100 features, "
                       "20k samples, phi[M, 3, F]",
           "value": M * e.n_leaves / (res["fp32"]["ms_per_step"] * 1e-3), "unit": "paths/s",
           "ms_per_step": res["fp32"]["ms_per_step"],
           "fp64_ms_per_step": res["fp64"]["ms_per_step"],
           "max_rel_err_fp32": res["err"], "rows_checked": 2}
    e.close()
    return out


def measure_interactions_full(args, torch, q, synth, oracle, dev):
    """The interactions workload at its stated size: all 50k explained samples
    of the 500-tree, 200-feature ensemble, Phi[50k, 200, 200] in FP32 (8.0 GB)
    and FP64 (16 GB), under HIP graph replay into reused output buffers.  The
    error is taken on rows spread over the sample blocks against the 8-node
    FP64 oracle, which runs on the host cores while the GPU is timed."""
    import threading
    wl = synth.make_workload("c3_interactions")
    ens = wl.ensemble
    M, F = wl.X.shape[0], ens.n_features
    rows = np.array([0, M // 3, (2 * M) // 3, M - 1])
    ref = {}
    th = threading.Thread(target=lambda: ref.update(
        r=oracle.shap_interactions(ens, wl.X[rows], n=8)), daemon=True)
    th.start()
    e = q.Ensemble(ens, device=dev)
    X = torch.from_numpy(wl.X).to(dev)
    U = float(e.info["n_pair_updates"])
    res, got = {}, {}
    for prec, dt, steps in (("fp32", torch.float32, 2), ("fp64", torch.float64, 1)):
        if not args.no_autotune:
            e.autotune(1024, prec)
        e.set_graph_replay(not args.eager)
        Phi = torch.empty((M, F, F), dtype=dt, device=dev)
        res[prec] = time_steps(lambda: e.shap_interactions(X, prec, out=Phi), steps, 1, torch,
                               "interactions")
        got[prec] = Phi[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
        e.set_graph_replay(False)
        del Phi
        torch.cuda.empty_cache()
        log("interactions 50k %s: %.1f ms per call" % (prec, res[prec]["ms_per_step"]))
    th.join()
    _, Phi_o = ref["r"]

    def rel(g):
        return float((np.abs(g - Phi_o).reshape(len(rows), -1).max(1)
                      / np.abs(Phi_o).reshape(len(rows), -1).max(1)).max())
    t32 = res["fp32"]["kernel_ms"] * 1e-3
    out = {"workload": "c3_interactions at its stated size: 500 grown trees, depths 3..20, "
                       "leaf cap 4096, 200 features, all 50,000 explained samples; "
                       "Phi[50000, 200, 200]",
           "samples": M, "leaves": e.n_leaves,
           "value": M * e.n_leaves / (res["fp32"]["ms_per_step"] * 1e-3), "unit": "paths/s",
           "ms_per_call": res["fp32"]["ms_per_step"], "kernel_ms": res["fp32"]["kernel_ms"],
           "fp64_ms_per_call": res["fp64"]["ms_per_step"],
           "fp64_value": M * e.n_leaves / (res["fp64"]["ms_per_step"] * 1e-3),
           "speedup_fp32_over_fp64": res["fp64"]["ms_per_step"] / res["fp32"]["ms_per_step"],
           "pair_updates_per_sample": int(U),
           "pair_updates_per_s": M * U / t32,
           "frac_of_lds_f64_atomic_rate": M * U / t32 / LDS_F64_ATOMIC_RATE,
           "max_rel_err_fp32": rel(got["fp32"]), "max_rel_err_fp64": rel(got["fp64"]),
           "rows_checked": [int(r) for r in rows],
           "launch": "hipGraph replay" if not args.eager else "eager"}
    e.close()
    return out


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2605_04497_amd as q
    import synth
    from oracle import oracle

    q.set_tune_cache(args.tune_cache or None)
    if args.flop_call:
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        flop_call(args, torch, q, synth, dev)
        return
    if args.only:
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        fn = {"interactions": measure_interactions, "interactions_full": measure_interactions_full,
              "adjoint": measure_adjoint, "deep": measure_deep, "small": measure_small,
              "third_order": measure_third_order, "wide": measure_wide,
              "groups": measure_groups}[args.only]
        print(json.dumps({"leg": args.only, "result": fn(args, torch, q, synth, oracle, dev)}),
              flush=True)
        return

    over = {}
    if args.samples:
        over["M"] = args.samples
    if args.trees:
        over["T"] = args.trees
    t0 = time.perf_counter()
    wl = synth.make_workload("c2_values", **over)
    ens, Xh = wl.ensemble, wl.X
    log("workload generated in %.1f s: %d trees, %d leaves, M=%d" % (
        time.perf_counter() - t0, ens.n_trees, ens.n_leaves(), Xh.shape[0]))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration_mb > 0:
        n = args.copy_calibration_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of %d MB" % args.copy_calibration_mb)
        del src, dst
    e = q.Ensemble(ens, device=dev)
    X = torch.from_numpy(Xh).to(dev)
    M = X.shape[0]
    units = M * e.n_leaves
    n_el = e.info["n_elements"]
    # elements the first-order kernel walks: one row per pair of sibling
    # leaves (merged), one per other leaf
    n_vel = e.info["n_value_elements"] if not args.no_merge else n_el
    e.set_sibling_merge(not args.no_merge)
    tune_s = 0.0
    tune_hits = tune_misses = 0
    if not args.no_autotune:
        t0 = time.perf_counter()
        for prec in ("fp32", "fp64"):
            e.autotune(M, prec)
        tune_s = time.perf_counter() - t0
        tune_hits, tune_misses = q.tune_cache_stats()
        log("autotune: %.1f s (cache hits %d, misses %d); fp32 shape %s, fp64 shape %s" % (
            tune_s, tune_hits, tune_misses, e.launch_shape("values", "fp32", 0),
            e.launch_shape("values", "fp64", 0)))
    e.set_graph_replay(not args.eager)

    out32 = torch.empty((M, e.n_features), dtype=torch.float32, device=dev)
    out64 = torch.empty((M, e.n_features), dtype=torch.float64, device=dev)
    r32 = time_steps(lambda: e.shap_values(X, "fp32", out=out32), args.steps, args.warmup, torch)
    log("fp32: %.3f ms/step (kernel %.3f ms)" % (r32["ms_per_step"], r32["kernel_ms"]))
    r64 = time_steps(lambda: e.shap_values(X, "fp64", out=out64),
                     args.fp64_steps or args.steps, args.warmup, torch)
    log("fp64: %.3f ms/step (kernel %.3f ms)" % (r64["ms_per_step"], r64["kernel_ms"]))

    # accuracy on sampled rows against the FP64 oracle
    rows = np.random.default_rng(1).choice(M, min(args.check_rows, M), replace=False)
    want = oracle.shap_values(ens, Xh[rows], n=8)
    got32 = out32[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
    got64 = out64[torch.from_numpy(rows).to(dev)].cpu().numpy()

    def rel(g):
        return float((np.abs(g - want).max(1) / np.maximum(np.abs(want).max(1), 1e-30)).max())

    err32, err64 = rel(got32), rel(got64)
    abs32, abs64 = float(np.abs(got32 - want).max()), float(np.abs(got64 - want).max())
    log("row-normwise rel err vs oracle: fp32 %.2e fp64 %.2e" % (err32, err64))

    flops = FLOPS_PER_ELEMENT * float(M) * n_vel
    plain = None
    if not args.no_merge and not args.no_extras:
        # the same call walking every leaf's path (no sibling merging)
        e.set_sibling_merge(False)
        rp = time_steps(lambda: e.shap_values(X, "fp32", out=out32), max(2, args.steps // 2),
                        1, torch)
        e.set_sibling_merge(True)
        plain = {"value": units / (rp["ms_per_step"] * 1e-3), "ms_per_step": rp["ms_per_step"],
                 "kernel_ms": rp["kernel_ms"], "dtype": "f32",
                 "alu_tflops": float(M) * shared_kernel_flops(
                     float(e.info["n_paths"]), n_el, float(e.info["n_path_shared"]),
                     float(e.info["n_path_prefix_kept"]))
                 / (rp["kernel_ms"] * 1e-3) / 1e12}
        log("fp32 without sibling merging: %.3f ms/step" % rp["ms_per_step"])
    exact = None
    if not args.no_extras:
        # the optional node policy: 4 nodes for paths of at most 8 features
        # (exact there, Theorem 2), with launch shapes tuned for it
        e.set_node_policy("exact")
        if not args.no_autotune:
            e.autotune(M, "fp32")
        rx = time_steps(lambda: e.shap_values(X, "fp32", out=out32), max(2, args.steps // 2),
                        1, torch)
        e.set_node_policy("fixed8")
        gx = out32[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
        exact = {"value": units / (rx["ms_per_step"] * 1e-3), "ms_per_step": rx["ms_per_step"],
                 "dtype": "f32", "max_rel_err": rel(gx),
                 "note": "4-node rule for paths of at most 8 unique features (all of this "
                         "workload): exact for first order, same values up to rounding"}
        log("fp32 with the exact node policy: %.3f ms/step" % rx["ms_per_step"])
    # the arithmetic the kernel runs (every row of this workload has at most 8
    # features: one bucket, the shared-prefix walk); flops above is the
    # per-element count of the method without merging or reuse
    n_shared = float(e.info["n_value_shared"] if not args.no_merge else e.info["n_path_shared"])
    n_kept = float(e.info["n_value_prefix_kept"] if not args.no_merge
                   else e.info["n_path_prefix_kept"])
    n_rows = float(e.info["n_value_paths"] if not args.no_merge else e.info["n_paths"])
    assert e.info["max_unique"] <= 8
    kernel_flops = float(M) * shared_kernel_flops(n_rows, n_vel, n_shared, n_kept)
    achieved = kernel_flops / (r32["kernel_ms"] * 1e-3) / 1e12
    result = {
        "metric": METRIC,
        "value": units / (r32["ms_per_step"] * 1e-3),
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c2_values: 1000 random trees depth 8, 100 features (20 "
                               "integer-valued), covers from 100k rows, 100k explained samples",
                   "trees": ens.n_trees, "leaves": e.n_leaves, "features": e.n_features,
                   "samples": M, "unique_features_per_path": n_el / max(1, e.info["n_paths"]),
                   "sibling_merge": not args.no_merge,
                   "kernel_rows": e.info["n_value_paths"] if not args.no_merge
                   else e.info["n_paths"],
                   "kernel_elements": n_vel,
                   "max_unique": e.info["max_unique"]},
        "max_rel_err": {"fp32": err32, "fp64": err64, "max_abs_fp32": abs32,
                        "max_abs_fp64": abs64, "rows_checked": int(len(rows)),
                        "measure": "row-normwise vs FP64 oracle (8 nodes)"},
        "launch": {"mode": "hipGraph replay" if not args.eager else "eager",
                   "autotuned": not args.no_autotune, "autotune_s": tune_s,
                   "tune_cache": {"path": os.path.relpath(args.tune_cache, ROOT)
                                  if args.tune_cache else None,
                                  "hits": tune_hits, "misses": tune_misses},
                   "values_shape_fp32": list(e.launch_shape("values", "fp32", 0)),
                   "values_shape_fp64": list(e.launch_shape("values", "fp64", 0)),
                   "step_ms_median": r32["step_ms_median"], "step_ms_min": r32["step_ms_min"],
                   "step_ms_max": r32["step_ms_max"]},
        "fp32_without_sibling_merge": plain,
        "fp32_exact_node_policy": exact,
        "fp64": {"value": units / (r64["ms_per_step"] * 1e-3), "ms_per_step": r64["ms_per_step"],
                 "kernel_ms": r64["kernel_ms"], "dtype": "f64",
                 "speedup_fp32_over_fp64": r64["ms_per_step"] / r32["ms_per_step"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(e.launch_shape("values", "fp32", 0)),
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
                     "flops_per_launch": kernel_flops,
                     "flops_model": "executed FP32 flops per (sample, row) of d features with s "
                                    "reused slots: 224 + 16 d - 16 s - 8 min(s, 6) (8 nodes, "
                                    "FMA = 2 flops); matches SQ_INSTS_VALU_FLOPS_FP32 x 64",
                     "rows": n_rows, "elements_per_sample": n_vel,
                     "shared_slots_per_sample": n_shared,
                     "kept_prefix_levels_per_sample": n_kept,
                     "peak_note": "published MI355X FP32 vector peak; plain FP32 FMAs and "
                                  "multiplies on vector-register operands issue at up to 1.71 "
                                  "wave instructions per CU per clock in probes on this GPU "
                                  "(2 at this peak), so it applies without packed instructions",
                     "kernel": "values_kernel<float, 8, 8, true, 8>", "kernel_ms": r32["kernel_ms"],
                     "kernel_ms_scope": "event pair around each graph replay (zero-fill, "
                                        "values kernel, cast)" if not args.eager else
                                        "event pair around the values kernel launches",
                     "method_flops_per_launch": flops,
                     "method_flops_note": "51 flops per (sample, element) of the rows walked, "
                                          "without the slot reuse: a work count, not a "
                                          "roofline figure"},
    }
    if not args.no_extras:
        legs = [("interactions", measure_interactions), ("adjoint", measure_adjoint),
                ("deep", measure_deep), ("small", measure_small),
                ("third_order", measure_third_order), ("wide", measure_wide),
                ("groups", measure_groups)]
        if not args.no_full_interactions:
            legs.append(("interactions_full", measure_interactions_full))
        for key, fn in legs:
            try:
                result[key] = fn(args, torch, q, synth, oracle, dev)
                log("%s: %s" % (key, json.dumps(result[key])[:300]))
            except Exception as exc:  # report, keep the headline line
                result[key] = {"error": repr(exc)}
                log("%s failed: %r" % (key, exc))
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(ens, Xh, args.cpu_seconds, oracle)
        log("cpu baseline: %.3e paths/s on %d cores" % (result["cpu_baseline"]["value"],
                                                        result["cpu_baseline"]["cores"]))
    e.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
