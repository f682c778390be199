"""Benchmark of the VALMOD hot path on one MI355X.

A step is one valmod_run over one series: window statistics, the diagonal
pass(es), the per-length update, VALMP and the rankings for every length of the
workload. Inputs are resident in HBM before timing starts. Prints one JSON line.
The headline path is the FP32 recurrence with FP64 refresh; the FP64 path is
timed beside it on the same input and the two outputs are compared.

Metric (matrix-profile cells per second): sum over lengths L of N_L (N_L - 1) / 2,
N_L = n - L + 1, divided by the time of one step.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MP cells/s (pairs x lengths / s) FP32-refresh vs FP64 at <=1e-4 dist error"
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (packed)
FLOP_PER_CELL = 6         # 2 FMA co-moment update + 2 MUL normalisation


def kernel_code(path):
    """The source text without comments and blank lines: edits to comments do
    not make the profiled counters stale."""
    import re

    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in open(path).read().splitlines())
    return "\n".join(ln for ln in lines if ln)


def profiled_traffic(precision, workload):
    """HBM bytes per pass launch measured by rocprofv3 (FETCH_SIZE + WRITE_SIZE,
    scaled by a 1 GiB device-copy calibration) for the current kernel code on this
    workload; None when no summary was taken on this workload and kernel code."""
    import glob
    import hashlib

    src = os.path.join(ROOT, "paper_2008_13447_amd", "csrc", "valmod_pass.hip")
    sha = hashlib.sha256(kernel_code(src).encode()).hexdigest()[:16]
    for path in glob.glob(os.path.join(ROOT, "profiles", f"k_pass_{precision}_*.md")):
        fields = dict(line.split(": ", 1) for line in open(path) if ": " in line and not line.startswith(("-", "|")))
        if (fields.get("kernel_source_sha256_16", "").strip() == sha and fields.get("workload", "").strip() == workload
                and "traffic_bytes_per_launch" in fields):
            return float(fields["traffic_bytes_per_launch"])
    return None


def cells_total(n, lo, hi):
    return sum((n - L + 1) * (n - L) // 2 for L in range(lo, hi + 1))


def cpu_model():
    """Model name of the host CPU (first entry of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x, l_min, lengths, excl_den, gpu_prof_d, gpu_prof_i, rows_per_len, seed=0):
    """The oracle on a bounded sample: `rows_per_len` random owners (full distance
    profiles) at each of the given lengths, timed on the host cores; the same
    owners are compared with the GPU result."""
    import numpy as np

    import oracle
    from oracle import compare

    oracle.build(force=False)
    n = x.shape[0]
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or os.cpu_count() or 1
    oracle.profile(x, lengths[0], rows=np.arange(threads), excl_den=excl_den, nthreads=threads)  # warm
    cells = 0.0
    dt = 0.0
    worst = 0.0
    ties = 0
    for L in lengths:
        t = L - l_min
        N = n - L + 1
        sel = np.sort(compare.sample_rows(N, rows_per_len, seed + L))
        t0 = time.perf_counter()
        d, i = oracle.profile(x, L, rows=sel, excl_den=excl_den, nthreads=threads)
        dt += time.perf_counter() - t0
        rep = compare.check_profile_rows(x, L, sel, gpu_prof_d[t][sel], gpu_prof_i[t][sel].astype(np.int64), d, i,
                                         1e-9, excl_den)
        worst = max(worst, rep.get("max_dn_err", 0.0))
        ties += rep.get("idx_mismatch", 0)
        cells += len(sel) * (N - 1) / 2.0  # an owner row is half of its pairs' share of the N(N-1)/2 cells
    dt = max(dt, 1e-6)
    return dict(value=cells / dt, unit="cells/s", cores=threads, kind="oracle", cpu=cpu_model(),
                sample=f"{rows_per_len} random owners (full distance profiles) at each of L={list(lengths)}, "
                       f"{dt:.1f} s on {threads} threads",
                parity_rows=rows_per_len * len(lengths), parity_max_dn_err=worst, parity_idx_ties=ties)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4, 5],
                    help="workload; 4 is the batched one (--batch-count series in one plan)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--lanes", type=int, default=0, help="series run concurrently (0: library default)")
    ap.add_argument("--graph", action="store_true", help="capture the run in a HIP graph and replay it")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default pass geometry")
    ap.add_argument("--mode", default="exact", choices=["exact", "paper"],
                    help="paper: Alg. ComputeSubMP as published (motif per length exact, other entries may be "
                         "left uncomputed; the cells/s figure then counts cells not computed)")
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32"],
                    help="headline path (the other one is timed beside it unless --no-compare)")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-mode run beside an exact-mode headline")
    ap.add_argument("--compare-steps", type=int, default=1,
                    help="timed steps of the other precision (after its autotuning, no warm-up)")
    ap.add_argument("--k-motifs", type=int, default=0, help="top-k motif pairs (0: the workload's)")
    ap.add_argument("--mset", type=float, default=0.0, metavar="D",
                    help="also grow the motif sets of the global top-k pairs with radius factor D")
    ap.add_argument("--mset-cap", type=int, default=1024, help="members stored per motif set")
    ap.add_argument("--path", default="auto", choices=["auto", "full", "recompute"])
    ap.add_argument("--m-discords", type=int, default=1, metavar="M",
                    help="also rank the Top-k M-th discords (M > 1; exact mode)")
    ap.add_argument("--cpu-rows", type=int, default=256,
                    help="oracle owners per length (at l_min, the middle length and l_max)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; multi-GPU runs are not supported "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2008_13447_amd import gen, native

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes}))
        return

    dev = torch.device("cuda:0")
    if args.config == 4:
        batch = gen.config4(args.batch_count)
        w = batch[0]
        x = [torch.from_numpy(np.ascontiguousarray(b.x)).to(dev) for b in batch]
        lo, hi = [b.l_min for b in batch], [b.l_max for b in batch]
        cells = sum(cells_total(b.n, b.l_min, b.l_max) for b in batch)
        name = f"batched{args.batch_count}_rw_n4096-131072_lmin32-256"
    else:
        batch = None
        w = gen.WORKLOADS[args.config]()
        x = torch.from_numpy(np.ascontiguousarray(w.x)).to(dev)
        lo, hi = w.l_min, w.l_max
        cells = cells_total(w.n, w.l_min, w.l_max)
        name = w.name

    km = args.k_motifs or w.k_motifs

    def timed(precision, steps, warmup, mode=args.mode):
        graph = args.graph and precision == "fp64"
        v = native.Valmod(x, lo, hi, p=w.p, k_motifs=km, k_discords=w.k_discords,
                          excl_den=w.excl_den, precision=precision, path="full" if graph else args.path,
                          lanes=args.lanes, graph=graph, mode=mode, mset_radius=args.mset,
                          mset_cap=args.mset_cap, m_discords=args.m_discords)
        tune = None
        if not args.no_autotune:
            t0 = time.perf_counter()
            H, K, p_used = v.autotune()
            tune = {"segment_rows": H, "diagonals_per_lane": K, "p": p_used, "ms": (time.perf_counter() - t0) * 1e3}
            print(f"bench: {precision} autotune {tune}", file=sys.stderr, flush=True)
        for _ in range(warmup):
            v.run()
            print(f"bench: {precision} warm-up step done", file=sys.stderr, flush=True)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for k in range(steps):
            v.run()  # waits for the step (a line per step; the wait costs microseconds against seconds)
            print(f"bench: {precision} step {k + 1} of {steps} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize(dev)
        ms = (time.perf_counter() - t0) * 1e3 / steps
        print(f"bench: {precision} {ms:.1f} ms per step", file=sys.stderr, flush=True)
        timing = v.pass_timing()
        res = v.result(0)
        v.close()
        return ms, timing, res, tune

    ms, (pass_ms, launches, pass_cells), res, tune = timed(args.precision, args.steps, args.warmup)
    avg_ms = pass_ms / max(launches, 1)
    achieved = (pass_cells / max(launches, 1)) * FLOP_PER_CELL / (avg_ms * 1e-3) / 1e12
    peak = FP64_PEAK_TFLOPS if args.precision == "fp64" else FP32_PEAK_TFLOPS
    out = {
        "metric": METRIC, "value": cells / (ms * 1e-3), "unit": "cells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": name, "n": w.n if batch is None else sum(b.n for b in batch),
                   "l_min": lo if batch is None else min(lo), "l_max": hi if batch is None else max(hi),
                   "p": w.p, "k": km, "precision": args.precision, "path": args.path,
                   "lanes": args.lanes, "graph": bool(args.graph and args.precision == "fp64"),
                   "mode": args.mode, "mset_radius": args.mset, "m_discords": args.m_discords},
        "roofline": {"bound": "alu", "kernel": f"k_pass<{'double' if args.precision == 'fp64' else 'float'}> "
                     "(diagonal pass)", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": profiled_traffic(args.precision, name),
                     "avg_launch_ms": avg_ms, "launches_per_step": launches,
                     "cells_per_launch": pass_cells / max(launches, 1)},
    }
    out["autotune"] = tune
    if args.mset > 0:
        out["motif_sets"] = {"radius_factor": args.mset, "k": km,
                             "members": [int(c) for c in res["mset_count"]]}
    st = res["stats"].sum(axis=0)
    out["diagnostics"] = {name: int(st[c]) for c, name in enumerate(native.STAT_NAMES)}
    if not args.no_compare:
        # the other precision on the same input: throughput and output agreement (first series)
        other = "fp64" if args.precision == "fp32" else "fp32"
        ms2, _, res2, _ = timed(other, args.compare_steps, 0)
        L = np.arange(w.l_min, w.l_max + 1)[:, None]
        a, b = res["prof_dist"] / np.sqrt(L), res2["prof_dist"] / np.sqrt(L)
        fin = np.isfinite(a) & np.isfinite(b)
        out[f"{other}_path"] = {
            "value": cells / (ms2 * 1e-3), "ms_per_step": ms2, "steps": args.compare_steps, "warmup": 0,
            "speedup_of_headline": ms2 / ms,
            "max_abs_dn_diff": float(np.max(np.abs(a[fin] - b[fin]))) if fin.any() else 0.0,
            "idx_diff": int(np.sum(res["prof_idx"] != res2["prof_idx"])),
        }
    if not args.no_paper and args.mode == "exact" and batch is None and args.m_discords <= 1:
        # Alg. ComputeSubMP as published on the same input: its time, how much of
        # the profile it recomputes by row scans, and its per-length motifs (exact
        # by the method's guarantee) against the exact run's
        ms3, _, res3, tune3 = timed(args.precision, 1, 0, mode="paper")
        st3 = res3["stats"].sum(axis=0)
        nwin = sum(w.n - L + 1 for L in range(w.l_min, w.l_max + 1))
        Ls = np.arange(w.l_min, w.l_max + 1)
        out["paper_mode"] = {
            "ms_per_step": ms3, "steps": 1, "warmup": 0, "autotune": tune3,
            "full_passes": int(st3[3]), "recomputed_rows": int(st3[2]),
            "recomputed_fraction": float(st3[2]) / nwin, "certified_fraction": float(st3[0]) / nwin,
            "partial_entries": int(st3[10]),
            "max_motif_dn_diff": float(np.nanmax(np.abs(res3["motif_d"][:, 0] - res["motif_d"][:, 0]) / np.sqrt(Ls))),
        }
    if not args.no_cpu and batch is None:
        lengths = sorted({w.l_min, (w.l_min + w.l_max) // 2, w.l_max})
        out["cpu_baseline"] = cpu_baseline(w.x, w.l_min, lengths, w.excl_den, res["prof_dist"], res["prof_idx"],
                                           args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
