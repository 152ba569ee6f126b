"""Benchmark: H2-MG time-to-1e-8 relative residual (FP64 vs mixed) and H2
matvec throughput on one MI355X.

One step = build the H2 matrix from the points (tree, bases, couplings),
build the multigrid hierarchy (projected close blocks, coarsest Cholesky,
FP32 operator copies), solve A_H2 x = b in FP64, then solve again with FP32
operators inside FP64 iterative refinement.  Inputs are generated on the
host, copied to HBM before the timed region, and every numerical step runs
in libh2mg.so.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 1] [--warmup 0] [--workload matern3d_1m]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H2-MG time-to-1e-8 rel residual (FP64 vs mixed) + matvec GB/s, N=2^20"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="matern3d_1m")
    ap.add_argument("--n", type=int, default=0, help="override the number of points")
    ap.add_argument("--max-cycles", type=int, default=500)
    ap.add_argument("--mixed", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--matvec-reps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-leaves", type=int, default=3)
    ap.add_argument("--json-out", default="")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def block_gemv_roofline(g, kind, bytes_per_sec_peak=HBM_PEAK_GBS):
    st = g.kernel_stats(kind)
    if st["launches"] == 0 or st["ms"] == 0:
        return None
    avg_ms = st["ms"] / st["launches"]
    avg_bytes = st["work"] / st["launches"]
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": bytes_per_sec_peak,
            "unit": "GB/s", "frac": round(achieved / bytes_per_sec_peak, 4), "traffic": None,
            "kernel": f"k_bsr_gemv ({kind})", "launches": st["launches"],
            "avg_launch_ms": round(avg_ms, 4), "avg_bytes_per_launch": avg_bytes}


def cpu_baseline(w, P, x, leaves, gpu_matvec_s, gpu_solve_s):
    """Time the oracle's row-restricted H2 matvec on a few leaves of the same
    workload and scale to one full matvec, then to the solve by the GPU's
    solve/matvec time ratio."""
    from oracle.h2 import H2 as OracleH2
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    t0 = time.perf_counter()
    o = OracleH2(P, w.kernel, w.shift, w.leaf, w.eta, w.cheb_m, w.length_scale)
    t_setup = time.perf_counter() - t0
    nleaf = 2 ** o.L
    pick = np.linspace(0, nleaf - 1, leaves).astype(int)
    t0 = time.perf_counter()
    rows = 0
    for lf in pick:
        o.matvec_rows(x, int(lf))
        rows += o.tree.size(o.L, int(lf))
    t_rows = time.perf_counter() - t0
    matvec_s = t_rows / rows * w.n
    solve_s = matvec_s * (gpu_solve_s / gpu_matvec_s) if gpu_matvec_s > 0 else None
    return {"value": None if solve_s is None else round(solve_s, 1), "unit": "s",
            "cores": int(threads), "kind": "oracle",
            "sample": (f"oracle row-restricted H2 matvec on {leaves} of {nleaf} leaves "
                       f"({rows} rows) of the same N={w.n} workload in {t_rows:.1f} s "
                       f"(+{t_setup:.1f} s tree/partition); scaled to a full matvec "
                       f"({matvec_s:.0f} s) and to the solve by the GPU solve/matvec "
                       f"time ratio"),
            "oracle_matvec_s": round(matvec_s, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import synth
    from paper_2501_17656_amd import H2Matrix

    w = synth.workload(args.workload)
    if args.n:
        w = w.scaled(args.n)
    dev = torch.device("cuda:0")
    log(f"workload {w.name}: n={w.n} dim={w.dim} kernel={w.kernel} l={w.length_scale} "
        f"shift={w.shift} leaf={w.leaf} eta={w.eta} m={w.cheb_m}")
    P = w.make_points()
    b = w.make_rhs()
    x = w.make_x()
    pts_d = torch.from_numpy(P).to(dev)
    b_d = torch.from_numpy(b).to(dev)
    x_d = torch.from_numpy(x).to(dev)
    torch.cuda.synchronize()

    def step(record):
        t0 = time.perf_counter()
        g = H2Matrix(pts_d, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        log(f"build {t1 - t0:.2f} s, device memory {g.memory_bytes() / 1e9:.1f} GB")
        g.setup(("fp64", args.mixed))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        log(f"hierarchy setup {t2 - t1:.2f} s, {g.levels} levels, "
            f"memory {g.memory_bytes() / 1e9:.1f} GB")
        g.set_timing(True)
        x64, i64 = g.solve(b_d, rtol=1e-8, max_cycles=args.max_cycles, precision="fp64",
                           raise_on_error=False)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        log(f"fp64 solve {t3 - t2:.2f} s, cycles {i64['cycles']}, rel res {i64['rel_residual']:.2e}, "
            f"status {i64['status']}")
        rl64 = block_gemv_roofline(g, "gemv_fp64")
        near64 = g.kernel_stats("near_fp64")
        g.set_timing(True)
        xm, im = g.solve(b_d, rtol=1e-8, max_cycles=args.max_cycles, precision=args.mixed,
                         raise_on_error=False)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        log(f"{args.mixed}+fp64 refinement solve {t4 - t3:.2f} s, steps {im['cycles']}, "
            f"rel res {im['rel_residual']:.2e}, status {im['status']}")
        rlm = block_gemv_roofline(g, "gemv_" + args.mixed)
        g.set_timing(False)
        if record is not None:
            record.update(dict(g=g, build_s=t1 - t0, setup_s=t2 - t1, fp64_s=t3 - t2,
                               mixed_s=t4 - t3, i64=i64, im=im, rl64=rl64, rlm=rlm,
                               near64=near64, x64=x64, xm=xm))
        else:
            g.close()
        return t4 - t0

    for i in range(args.warmup):
        log(f"warmup step {i + 1}/{args.warmup}")
        step(None)
    torch.cuda.synchronize()
    rec = {}
    times = []
    for i in range(args.steps):
        log(f"timed step {i + 1}/{args.steps}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if rec.get("g") is not None:
            rec["g"].close()
        step(rec)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    g = rec["g"]

    # matvec throughput (outside the timed steps): algorithmic bytes of the
    # stored operator part of a fine matvec over its measured time
    g.set_timing(True)
    y = torch.empty_like(x_d)
    g.matvec(x_d, out=y)
    torch.cuda.synchronize()
    g.set_timing(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.matvec_reps):
        g.matvec(x_d, out=y)
    ev1.record()
    torch.cuda.synchronize()
    mv_ms = ev0.elapsed_time(ev1) / args.matvec_reps
    gst = g.kernel_stats("gemv_fp64")
    nst = g.kernel_stats("near_fp64")
    mv_bytes = gst["work"] / max(gst["launches"], 1)
    g.set_timing(False)

    res64 = rec["i64"]
    resm = rec["im"]
    mixed_ok = resm["converged"]
    out = {
        "metric": METRIC,
        "value": round(rec["mixed_s"] if mixed_ok else rec["fp64_s"], 3),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * float(np.mean(times)), 1),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": f"{args.mixed}+f64-refinement" if mixed_ok else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: N={w.n} points uniform in [0,1)^{w.dim}, {w.kernel} "
                         f"l={w.length_scale} + {w.shift}*I, leaf {w.leaf}, eta {w.eta}, "
                         f"Chebyshev {w.cheb_m}^{w.dim} (rank {w.rank}), b ~ N(0,1), rtol 1e-8, "
                         f"n_f=1 n_c=40"),
            "levels": g.levels,
        },
        "fp64_time_to_1e-8_s": round(rec["fp64_s"], 3),
        "fp64_cycles": res64["cycles"], "fp64_converged": res64["converged"],
        "fp64_rel_residual": res64["rel_residual"],
        "mixed_precision": args.mixed,
        "mixed_time_to_1e-8_s": round(rec["mixed_s"], 3),
        "mixed_refinement_steps": resm["cycles"], "mixed_converged": resm["converged"],
        "mixed_rel_residual": resm["rel_residual"],
        "speedup_mixed_vs_fp64": round(rec["fp64_s"] / rec["mixed_s"], 3) if rec["mixed_s"] > 0 else None,
        "build_s": round(rec["build_s"], 3),
        "setup_s": round(rec["setup_s"], 3),
        "device_memory_gb": round(g.memory_bytes() / 1e9, 1),
        "matvec_ms": round(mv_ms, 3),
        "matvec_stored_bytes_gb": round(mv_bytes / 1e9, 2),
        "matvec_stored_gbs": round(mv_bytes / (mv_ms * 1e-3) / 1e9, 1),
        "near_field_evals_per_s": (round(nst["work"] / (nst["ms"] * 1e-3), 0) if nst["ms"] else None),
        "roofline": rec["rlm"] if mixed_ok and rec["rlm"] else rec["rl64"],
        "roofline_fp64_gemv": rec["rl64"],
    }
    if not args.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(w, P, x, args.cpu_leaves, mv_ms * 1e-3,
                                               rec["mixed_s"] if mixed_ok else rec["fp64_s"])
        except Exception as e:  # the baseline must not hide the GPU result
            out["cpu_baseline"] = {"error": repr(e)}
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")
    g.close()


if __name__ == "__main__":
    main()
