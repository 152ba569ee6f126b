"""Benchmark: H2-MG time-to-1e-8 relative residual (FP64 vs mixed) and H2
matvec throughput on one MI355X at N = 2^20.

Default run (what `python bench.py --gpus 1 --steps K --warmup W` does):

1. Matvec on the specified 2^20-point Matern-3/2 matrix (shift 1e-3, leaf
   128, eta 0.7, rank 64): build, the near field stored as FP64 tiles, the
   fine H2 matvec timed, with its algorithmic bytes and GB/s.
2. The timed workload: the same points, kernel and H2 parameters with the
   diagonal shift of `--workload` (the rank-64 approximation of the 1e-3
   matrix is indefinite at this size).  Build and hierarchy setup are timed
   once and reported; one FP64 solve to 1e-8 is timed and reported.
3. The timed step: one solve A_H2 x = b from x0 = 0 to a 1e-8 relative
   residual with FP32 operators inside FP64 iterative refinement (Algorithm 1
   cycles, block smoother), cycles launched as captured graphs.  W warmup
   steps, then K timed steps; both stop early (at least one of each) when the
   next step would not fit in the wall-clock budget `--budget-s`, and the
   line reports the steps actually run.
4. One instrumented refinement step (HIP events around every block-GEMV
   launch) gives the roofline of the dominant kernel; the CPU oracle's rows
   of A_H2 x for the GPU's solutions give the residual check and the CPU
   baseline.  Then the JSON line is printed.

Everything else (the small configuration, the gradient run, boundary
elements, batched problems, cycles on the 1e-3 matrix, the paper's CG
smoother, 16 right-hand sides) runs only when its flag asks for it.

Inputs are generated on the host and copied to HBM before any timed region;
every numerical step runs in libh2mg.so.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5]
    python bench.py --copy-probe       # plain copy kernel for counter calibration
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

T_START = time.perf_counter()

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H2-MG time-to-1e-8 rel residual (FP64 vs mixed) + matvec GB/s, N=2^20"
HBM_PEAK_GBS = 8000.0

# opt-in parts of the default run: flag -> what it adds to the JSON line
EXTRAS = ("c1", "diff", "bem", "batched_first", "part_a", "cg_smoother", "sixteen_rhs")


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--budget-s", type=float, default=440.0,
                    help="wall-clock seconds from process start to the JSON line; warmup and "
                         "timed steps stop early (at least one of each) when the next one would "
                         "not fit")
    ap.add_argument("--workload", default="matern3d_1m_spd")
    ap.add_argument("--headline", default="matern3d_1m",
                    help="workload of the matvec measurement ('' to skip it)")
    ap.add_argument("--headline-cycles", type=int, default=4)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--spd-probe", default="",
                    help="n:cycles:shift,... run FP64 V-cycles of the headline shape and report "
                         "the Rayleigh quotient of the final iterate")
    ap.add_argument("--shift-scan", default="",
                    help="s1,s2,...: time-to-1e-8 of the headline shape at these diagonal shifts")
    ap.add_argument("--lanczos", default="",
                    help="n:steps,... Lanczos on the library's matvec of the headline matrix: "
                         "extreme Ritz values of A_H2")
    ap.add_argument("--growth", default="",
                    help="comma-separated N: iterations to 1e-8 of H2-MG and of plain CG against N")
    ap.add_argument("--sweep", default="",
                    help="comma-separated smoother:precision:n_f:n_c items on the shift-1 2^20 problem")
    ap.add_argument("--error-components", action="store_true",
                    help="the error analysis of the experiments (1D Gaussian, N = 1024)")
    ap.add_argument("--spd-probe-oracle", action="store_true",
                    help="also evaluate the Rayleigh quotient with the CPU oracle's matvec")
    ap.add_argument("--n", type=int, default=0, help="override the number of points")
    ap.add_argument("--max-cycles", type=int, default=500)
    ap.add_argument("--mixed", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--smoother", default="bj", choices=["bj", "cg"])
    ap.add_argument("--no-graphs", action="store_true", help="launch the timed cycles kernel by kernel")
    ap.add_argument("--matvec-reps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU seconds of sampled oracle rows in the CPU baseline")
    # opt-in parts (none runs by default)
    ap.add_argument("--c1", action="store_true", help="the small configuration's latency runs")
    ap.add_argument("--diff", action="store_true", help="the gradient run at N = 2^18")
    ap.add_argument("--bem", action="store_true", help="the boundary-element run at 10^6 panels")
    ap.add_argument("--batched-first", type=int, default=0,
                    help="solve the first problems of the batched configuration")
    ap.add_argument("--part-a", action="store_true",
                    help="cycles on the 1e-3 matrix (indefinite) and the 16-vector block product")
    ap.add_argument("--cg-smoother", action="store_true",
                    help="also solve the timed workload with the paper's plain CG smoother")
    ap.add_argument("--sixteen-rhs", action="store_true",
                    help="also solve 16 right-hand sides of the timed workload at once")
    ap.add_argument("--bem-one-point", action="store_true",
                    help="close boundary-element entries by the one-point rule (default: seven points)")
    ap.add_argument("--bem-grid", type=int, nargs=2, default=[1000, 500],
                    help="torus parameter grid (panels = 2 * a * b)")
    ap.add_argument("--json-out", default="")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only the requested extras that build matrices of their own "
                         "(--c1, --diff, --bem, --batched-first, --part-a), not the timed workload")
    ap.add_argument("--setup-only", action="store_true",
                    help="run only the build and hierarchy setup of the timed workload")
    ap.add_argument("--block-product", action="store_true",
                    help="run only the 16-vector block product on the headline matrix")
    ap.add_argument("--batched", action="store_true",
                    help="run only the batched solve of many uneven problems with 16 RHS each")
    ap.add_argument("--batch-problems", type=int, default=48)
    ap.add_argument("--batch-seed", type=int, default=3)
    ap.add_argument("--batch-shift", type=float, default=3.0)
    ap.add_argument("--batch-streams", type=int, default=4)
    ap.add_argument("--batch-budget-gb", type=float, default=200.0)
    ap.add_argument("--no-batch-autotune", dest="batch_autotune", action="store_false",
                    help="keep the default tile-run length instead of tuning it per task set")
    return ap.parse_args(argv)


def extras_requested(args):
    """The opt-in parts a run asked for (empty for the default run)."""
    on = {"c1": args.c1, "diff": args.diff, "bem": args.bem,
          "batched_first": args.batched_first > 0, "part_a": args.part_a,
          "cg_smoother": args.cg_smoother, "sixteen_rhs": args.sixteen_rhs}
    return [k for k in EXTRAS if on[k]]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def profiled_traffic(kind, avg_bytes):
    """HBM bytes (read + write) per launch of the block GEMV, from the
    rocprofv3 counters in profiles/gemv_counters_*.md: their ratio of HBM to
    algorithmic bytes applied to this run's algorithmic bytes per launch
    (the same kernels, another mix of launches).  None when the kernel source
    changed since the counters were taken."""
    import glob
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2501_17656_amd", "csrc")
    h = hashlib.sha256()
    for f in ("kernels_apply.hip", "device_common.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    cur = h.hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "gemv_counters_*.md"))):
        with open(path) as fh:
            for line in fh:
                m = re.match(r"\s*traffic (\S+) src=(\S+) per_launch_bytes=(\S+) alg_per_launch_bytes=(\S+)",
                             line)
                if m and m.group(1) == kind and m.group(2) == cur:
                    return round(avg_bytes * float(m.group(3)) / float(m.group(4)))
    return None


def block_gemv_roofline(g, kind, bytes_per_sec_peak=HBM_PEAK_GBS):
    st = g.kernel_stats(kind)
    if st["launches"] == 0 or st["ms"] == 0:
        return None
    avg_ms = st["ms"] / st["launches"]
    avg_bytes = st["work"] / st["launches"]
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": bytes_per_sec_peak,
            "unit": "GB/s", "frac": round(achieved / bytes_per_sec_peak, 4),
            "traffic": profiled_traffic(kind, avg_bytes),
            "kernel": "k_near_gemv" if kind.startswith("near") else f"k_bsr_gemv ({kind})",
            "launches": st["launches"],
            "avg_launch_ms": round(avg_ms, 4), "avg_bytes_per_launch": avg_bytes}


def cpu_threads():
    """Threads the oracle's BLAS may use: OMP_NUM_THREADS when set, else the
    CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_baseline(w, P, b, solutions, timed_key, seconds, gpu_matvec_ms):
    """The CPU oracle timed on the host cores, on a bounded sample of the same
    workload: its FP64 row-restricted H2 matvec (the blockwise sum restricted
    to the rows of one leaf) on leaves drawn in a seeded order, applied to the
    GPU's final solution `solutions[timed_key]`, until `seconds` of oracle
    time have run.  The rate is extrapolated linearly in rows to one full
    matvec (labelled as such).  The same rows give the oracle's residual
    b - A_H2 x of each GPU solution on the sampled leaves (the other solutions
    on the first three leaves only, untimed).  Also timed in full: the
    oracle's solve of the small configuration (N = 4096)."""
    from threadpoolctl import threadpool_limits

    from oracle.h2 import H2 as OracleH2
    threads = cpu_threads()
    out = {}
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        o = OracleH2(P, w.kernel, w.shift, w.leaf, w.eta, w.cheb_m, w.length_scale)
        t_setup = time.perf_counter() - t0
        nleaf = 2 ** o.L
        order = np.random.default_rng(5).permutation(nleaf)
        rows = 0
        t_rows = 0.0
        worst = {k: 0.0 for k in solutions}
        used = []
        for idx, leaf in enumerate(order):
            if t_rows >= seconds:
                break
            leaf = int(leaf)
            sel = o.tree.perm[o.rows(o.L, leaf)]
            nb = float(np.linalg.norm(b[sel]))
            for key, x in solutions.items():
                if key != timed_key and idx >= 3:
                    continue
                t1 = time.perf_counter()
                ax = o.matvec_rows(x, leaf)
                dt = time.perf_counter() - t1
                if key == timed_key:
                    t_rows += dt
                    rows += len(sel)
                worst[key] = max(worst[key], float(np.linalg.norm(b[sel] - ax)) / nb)
            used.append(leaf)
        matvec_s = t_rows / rows * w.n
        out["cpu_baseline"] = {
            "value": round(matvec_s, 1),
            "unit": f"s per H2 matvec at N={w.n} (extrapolated linearly from sampled rows)",
            "cores": threads, "kind": "oracle",
            "sample": (f"oracle FP64 row-restricted H2 matvec of the GPU's {timed_key} solution on "
                       f"{len(used)} of {nleaf} leaves ({rows} of {w.n} rows, seeded leaf order) of "
                       f"the timed workload: {t_rows:.1f} s measured, extrapolated x{w.n / rows:.0f} "
                       f"to one full matvec; oracle tree and partition {t_setup:.1f} s"),
            "measured_rows": rows, "measured_rows_s": round(t_rows, 2),
            "oracle_setup_s": round(t_setup, 2),
            "gpu_matvec_ms": gpu_matvec_ms,
        }
        out["oracle_residual_rows"] = {
            "leaves": len(used),
            "max_rel_residual_rows": {k: v for k, v in worst.items()},
            "note": "max over sampled leaves of ||b - A_H2 x|| / ||b|| on the leaf's rows, A_H2 x "
                    "by the oracle (other solutions than the timed one: first 3 leaves)"}
        # the small configuration's full oracle solve (N = 4096, 2D exponential kernel)
        import synth
        from oracle.galerkin import Hierarchy
        from oracle.vcycle import solve_user
        c1 = synth.workload("exp2d_4k")
        t0 = time.perf_counter()
        oc = OracleH2(c1.make_points(), c1.kernel, c1.shift, c1.leaf, c1.eta, c1.cheb_m, c1.length_scale)
        H = Hierarchy(oc)
        t1 = time.perf_counter()
        res = solve_user(oc, H, c1.make_rhs(), rtol=1e-8)
        t2 = time.perf_counter()
        out["cpu_baseline"]["small_config_oracle_solve"] = {
            "workload": f"{c1.name}: N={c1.n}, {c1.kernel} l={c1.length_scale} + {c1.shift}*I, "
                        f"leaf {c1.leaf}, rank {c1.rank}, paper CG smoother",
            "time_to_1e-8_s": round(t2 - t1, 3), "setup_s": round(t1 - t0, 3),
            "cycles": res.cycles, "converged": res.converged}
    return out


def copy_probe(gb: float = 8.0, reps: int = 5):
    """A plain device copy of known size (for FETCH_SIZE / WRITE_SIZE
    calibration): reads and writes gb GB per repetition."""
    import torch
    n = int(gb * 1e9 // 8)
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "reps": reps, "gbs_read_plus_write": round(2 * n * 8 / dt / 1e9, 1)}))


def spd_probe(args, torch, synth, H2Matrix):
    """Positive-definiteness probe of the H2 approximation of the headline
    shape: after `cycles` FP64 V-cycles on A_H2 x = b, report the residual
    history and x^T A_H2 x / x^T x (negative: A_H2 is indefinite)."""
    import dataclasses
    base = synth.workload(args.headline or "matern3d_1m")
    for item in args.spd_probe.split(","):
        n, cycles, shift = item.split(":")
        w = dataclasses.replace(base.scaled(int(n)), shift=float(shift))
        P = w.make_points()
        pts = torch.from_numpy(P).cuda()
        b = torch.from_numpy(w.make_rhs()).cuda()
        g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
        g.setup()
        x, info = g.solve(b, rtol=1e-8, max_cycles=int(cycles), raise_on_error=False)
        ax = g.matvec(x)
        torch.cuda.synchronize()
        rq = float((x @ ax) / (x @ x))
        out = {"spd_probe": w.name, "n": w.n, "shift": w.shift, "cycles": info["cycles"],
               "status": info["status"], "rel_residual": info["rel_residual"],
               "residual_history_every_10": [round(v, 4) for v in info["history"][::10]],
               "x_norm": float(x.norm()), "rayleigh_gpu": rq}
        if args.spd_probe_oracle:
            from oracle.h2 import H2 as OracleH2
            xh = x.cpu().numpy()
            o = OracleH2(P, w.kernel, w.shift, w.leaf, w.eta, w.cheb_m, w.length_scale)
            out["rayleigh_oracle"] = float(xh @ o.matvec(xh) / (xh @ xh))
        print(json.dumps(out), flush=True)
        g.close()
        del pts, b, x, ax
        torch.cuda.empty_cache()


def shift_scan(args, torch, synth, H2Matrix):
    """Time-to-1e-8 of the headline shape at other diagonal shifts: for each
    shift, build and hierarchy setup, then the mixed-precision and the FP64
    solve with the block smoother (at most --max-cycles cycles each), with
    status, cycles, time and, for an iterate that did not converge, its
    Rayleigh quotient (negative: A_H2 is indefinite at that shift)."""
    import dataclasses
    base = synth.workload(args.headline or "matern3d_1m")
    for shift in (float(v) for v in args.shift_scan.split(",")):
        w = dataclasses.replace(base, shift=shift)
        pts = torch.from_numpy(w.make_points()).cuda()
        b = torch.from_numpy(w.make_rhs()).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
        g.setup(("fp64", args.mixed))
        torch.cuda.synchronize()
        out = {"shift_scan": w.name, "n": w.n, "shift": shift,
               "build_and_setup_s": round(time.perf_counter() - t0, 2)}
        for prec in (args.mixed, "fp64"):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, info = g.solve(b, rtol=1e-8, max_cycles=args.max_cycles, precision=prec,
                              smoother="bj", raise_on_error=False)
            torch.cuda.synchronize()
            row = {"status": info["status"], "cycles": info["cycles"],
                   "rel_residual": info["rel_residual"], "s": round(time.perf_counter() - t1, 2),
                   "history_every_5": [round(v, 5) for v in info["history"][::5]]}
            if not info["converged"] and bool(torch.isfinite(x).all()) and float(x.norm()) > 0:
                ax = g.matvec(x)
                row["rayleigh"] = float((x @ ax) / (x @ x))
            out[prec] = row
            log(f"shift {shift} {prec}: {row['status']} {row['cycles']} cycles {row['s']} s")
        print(json.dumps(out), flush=True)
        g.close()
        del pts, b
        torch.cuda.empty_cache()


def lanczos_probe(args, torch, synth, H2Matrix):
    """Extreme eigenvalues of A_H2 for the headline shape (shift as specified)
    by Lanczos on the library's FP64 matvec, with full reorthogonalisation
    (the Lanczos vectors stay in device memory).  The shift only adds s * I,
    so lambda(A_H2 + (s' - s) I) = lambda(A_H2) + s' - s: one run gives the
    smallest eigenvalue for every shift.  A Ritz value is the Rayleigh
    quotient of its Ritz vector, so it bounds lambda_min from above (a
    negative one certifies that A_H2 is indefinite); the true residual
    ||A y - theta y|| (one more product) bounds the distance from theta to
    some eigenvalue.  Items
    n:steps[:cycles]: with cycles > 0 the start vector is the iterate of that
    many FP64 V-cycles (CG smoother) on A_H2 x = b from x0 = 0, which grows
    along the eigenvectors the cycle cannot reduce (a negative or near-zero
    eigenvalue); otherwise a random vector."""
    import scipy.linalg
    base = synth.workload(args.headline or "matern3d_1m")
    for item in args.lanczos.split(","):
        parts = [int(v) for v in item.split(":")]
        n, steps = parts[0], parts[1]
        cycles = parts[2] if len(parts) > 2 else 0
        w = base.scaled(n)
        P = w.make_points()
        pts = torch.from_numpy(P).cuda()
        g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
        start = {"kind": "random (seed 11)"}
        if cycles > 0:
            g.setup()
            b = torch.from_numpy(w.make_rhs()).cuda()
            v, info = g.solve(b, rtol=1e-8, max_cycles=cycles, raise_on_error=False)
            av = g.matvec(v)
            torch.cuda.synchronize()
            start = {"kind": f"iterate of {cycles} FP64 V-cycles (CG smoother) on A x = b",
                     "status": info["status"], "rel_residual": info["rel_residual"],
                     "rayleigh": float((v @ av) / (v @ v))}
            log(f"lanczos start: {start}")
            del b, av
        else:
            v = torch.from_numpy(synth.normal_vector(n, 11)).cuda()
        V = torch.empty((steps + 1, n), dtype=torch.float64, device="cuda")
        V[0] = v / v.norm()
        alpha, beta = [], []
        rows = []
        t0 = time.perf_counter()
        q = torch.empty(n, dtype=torch.float64, device="cuda")
        for k in range(steps):
            g.matvec(V[k], out=q)
            a_k = float(q @ V[k])
            alpha.append(a_k)
            q -= a_k * V[k]
            if k > 0:
                q -= beta[-1] * V[k - 1]
            # full reorthogonalisation (twice)
            for _ in range(2):
                q -= V[:k + 1].T @ (V[:k + 1] @ q)
            b_k = float(q.norm())
            beta.append(b_k)
            V[k + 1] = q / b_k
            if (k + 1) % 50 == 0 or k + 1 == steps:
                th, S = scipy.linalg.eigh_tridiagonal(np.array(alpha), np.array(beta[:-1]))
                est = np.abs(b_k * S[-1, :])
                rows.append({"step": k + 1, "ritz_min": [float(t) for t in th[:3]],
                             "ritz_min_resid_est": [float(e) for e in est[:3]],
                             "ritz_max": float(th[-1]), "s": round(time.perf_counter() - t0, 1)})
                log(f"lanczos n={n} step {k + 1}: ritz min {th[:3]}, est {est[:3]}, max {th[-1]:.4e}")
        th, S = scipy.linalg.eigh_tridiagonal(np.array(alpha), np.array(beta[:-1]))
        s0 = torch.from_numpy(np.ascontiguousarray(S[:, 0])).cuda()
        y = V[:steps].T @ s0
        y /= y.norm()
        ay = g.matvec(y)
        rq = float(y @ ay)
        resid = float((ay - rq * y).norm())
        ritz = []
        for k in range(min(4, steps)):
            sk = torch.from_numpy(np.ascontiguousarray(S[:, k])).cuda()
            yk = V[:steps].T @ sk
            yk /= yk.norm()
            ayk = g.matvec(yk)
            tk = float(yk @ ayk)
            ritz.append({"theta": tk, "residual": float((ayk - tk * yk).norm())})
        out = {"lanczos": w.name, "n": n, "steps": steps, "shift": w.shift, "start": start,
               "smallest_ritz_pairs": ritz,
               "ritz_min": float(th[0]), "ritz_max": float(th[-1]),
               "ritz_vector_rayleigh": rq, "ritz_vector_residual": resid,
               # a Rayleigh quotient bounds lambda_min from above: rq < 0 proves
               # an eigenvalue below zero; [rq - resid, rq + resid] holds one
               "certified_indefinite": bool(rq < 0),
               "eigenvalue_interval": [rq - resid, rq + resid],
               "smallest_shift_estimate": w.shift - rq,
               "history": rows, "seconds": round(time.perf_counter() - t0, 1)}
        print(json.dumps(out), flush=True)
        g.close()
        del V, pts, q, y, ay
        torch.cuda.empty_cache()


def block_product(args, torch, g, w, single_ms):
    """Y = A_H2 X for a block of 16 vectors (matrix-core tile products; each
    stored tile read once, its row and transposed products from the same
    staged copy; tile runs tuned on the first call): time per block product,
    the equivalent time per vector, the algorithmic GB/s of the near-field
    tiles (each stored tile counted once) and their matrix-core rate."""
    X = torch.from_numpy(synth_block(w, 16)).cuda()
    g.set_autotune(True)                                      # tile runs chosen on the first call
    try:
        Y = g.matvec_multi(X)
    except Exception as ex:
        return {"error": str(ex)}
    torch.cuda.synchronize()
    g.set_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.matvec_reps):
        g.matvec_multi(X, out=Y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.matvec_reps
    st = g.kernel_stats("near_gemm16_fp64")
    near_ms = st["ms"] / max(st["launches"], 1)
    tile_bytes = st["work"] / max(st["launches"], 1)          # each stored tile once (algorithmic)
    # every stored word serves the row product and, off the diagonal, the
    # transposed one: at most 2 x 2 flops per word and column
    flops = tile_bytes / 8.0 * 4.0 * 16.0
    g.set_timing(False)
    tuning = g.block_tuning()
    # every tile also reads its column's 64 x 16 operand block and, off the
    # diagonal, writes a 64 x 16 column contribution (FP64): the pass moves
    # tiles + 8 KiB per tile + 8 KiB per off-diagonal tile (the diagonal
    # tiles are those of a 64-point chunk with itself, n / 64 of them)
    ntiles = tile_bytes / 32768.0
    vec_bytes = 64 * 16 * 8.0 * (2.0 * ntiles - g.n / 64.0)
    return {"ms": round(ms, 3), "ms_per_vector": round(ms / 16, 3),
            "speedup_vs_16_single_products": round(16 * single_ms / ms, 2),
            "tile_runs": {k: v["run"] for k, v in tuning.items()},
            "near_tile_products_ms": round(near_ms, 3),
            "near_tiles_algorithmic_gbs": round(tile_bytes / (near_ms * 1e-3) / 1e9, 1),
            "near_tiles_frac_of_hbm_peak": round(tile_bytes / (near_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
            "near_pass_bytes_with_vectors_gb": round((tile_bytes + vec_bytes) / 1e9, 2),
            "near_pass_with_vectors_gbs": round((tile_bytes + vec_bytes) / (near_ms * 1e-3) / 1e9, 1),
            "near_pass_with_vectors_frac_of_hbm_peak":
                round((tile_bytes + vec_bytes) / (near_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
            "near_mfma_tflops": round(flops / (near_ms * 1e-3) / 1e12, 2),
            "near_mfma_frac_of_fp64_peak": round(flops / (near_ms * 1e-3) / 1e12 / 78.6, 3)}


def synth_block(w, nrhs):
    import synth
    return synth.normal_vector(w.n, w.x_seed, nrhs=nrhs)


def many_rhs_solve(args, torch, g, w, single_s):
    """16 right-hand sides of the timed workload solved at once
    (h2mg_solve_multi: every cycle on all columns, tile products on the
    matrix cores, the near field evaluated inside the products), with the
    same precision and smoother as the timed mixed solve."""
    B = torch.from_numpy(synth_block(w, 16)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        X, info = g.solve_multi(B, rtol=1e-8, precision=args.mixed, smoother=args.smoother,
                                max_cycles=args.max_cycles, raise_on_error=False)
    except Exception as ex:
        return {"error": str(ex)}
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"rhs": 16, "time_to_1e-8_s": round(dt, 3), "cycles": info["cycles"], "status": info["status"],
           "max_rel_residual": info["rel_residual"], "s_per_rhs": round(dt / 16, 3),
           "speedup_vs_16_single_solves": round(16 * single_s / dt, 2),
           "device_memory_gb": round(g.memory_bytes() / 1e9, 1)}
    log(f"16 right-hand sides at once ({args.mixed}+fp64 refinement): {dt:.2f} s, {info['cycles']} cycles, "
        f"{info['status']}, {16 * single_s / dt:.2f}x the throughput of single solves")
    del X, B
    return out


def galerkin_flops(P, leaf, eta, m, dim):
    """Algorithmic FP64 flops of the setup's Galerkin products on the tree of
    P (2 flops per multiply-add, zero padding not counted): the couplings
    R_s K R_t^T of the far pairs (4 r^3 each), the projected close leaf blocks
    Q_s^T K_st Q_t (2 r n_s n_t + 2 r^2 n_s), and the projected blocks above
    the leaves, [E_c]^T [M_cc'] [E_c'] over the 2 x 2 child blocks (12 r^3)."""
    from paper_2501_17656_amd.h2mg import Plan
    plan = Plan(P, leaf, eta, m)
    r = m ** dim
    L = plan.depth
    out = {"coupling": 0.0, "pi_leaf": 0.0, "pi_upper": 0.0, "far_blocks": 0, "leaf_blocks": 0,
           "upper_blocks": 0}
    for d in range(L + 1):
        far = plan.pairs(d, True)
        near = plan.pairs(d, False)
        far_u = int(np.sum(far[:, 0] < far[:, 1])) if len(far) else 0
        near_u = near[near[:, 0] <= near[:, 1]] if len(near) else near
        out["far_blocks"] += far_u
        out["coupling"] += far_u * 4.0 * r ** 3
        if d == L:
            sz = np.diff(plan.offsets(L)).astype(np.float64)
            ns, nt = sz[near_u[:, 0]], sz[near_u[:, 1]]
            out["pi_leaf"] = float(np.sum(2.0 * r * ns * nt + 2.0 * r * r * ns))
            out["leaf_blocks"] = int(len(near_u))
        elif plan.d_top >= 0 and d >= plan.d_top:
            out["upper_blocks"] += int(len(near_u))
            out["pi_upper"] += len(near_u) * 12.0 * r ** 3
    return out


def setup_only(args, torch, synth, H2Matrix):
    """Build and hierarchy setup of the timed workload, timed, with the
    algorithmic flops of the Galerkin products (for profiling the setup
    kernels)."""
    w = synth.workload(args.workload)
    P = w.make_points()
    pts = torch.from_numpy(P).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.setup(("fp64", args.mixed))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = {"workload": w.name, "n": w.n, "rank": w.rank, "build_s": round(t1 - t0, 3),
           "setup_s": round(t2 - t1, 3), "levels": g.levels,
           "galerkin_flops": galerkin_flops(P, w.leaf, w.eta, w.cheb_m, w.dim)}
    g.close()
    return out


def block_product_only(args, torch, synth, H2Matrix):
    """Only the 16-vector block product on the 2^20 headline matrix (near
    field stored, tile runs tuned), for profiling its kernels."""
    w = synth.workload(args.headline)
    g = H2Matrix(torch.from_numpy(w.make_points()).cuda(), w.kernel, w.length_scale, w.shift, w.leaf,
                 w.eta, w.cheb_m)
    g.store_near(True)
    single = torch.from_numpy(w.make_x()).cuda()
    y = g.matvec(single)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.matvec_reps):
        g.matvec(single, out=y)
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t0) / args.matvec_reps * 1e3
    out = block_product(args, torch, g, w, single_ms)
    out["single_product_ms"] = round(single_ms, 3)
    g.close()
    return out


def stored_near_matvec(args, torch, g, w, time_matvecs):
    """The fine H2 matvec with the close leaf blocks stored as FP64 tiles:
    time per product, algorithmic bytes (near tiles + couplings + the two
    leaf-basis copies + transfers + vectors) and the fraction of HBM peak.
    The tiles are released afterwards."""
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.store_near(True)
        torch.cuda.synchronize()
        t_store = time.perf_counter() - t0
    except Exception as ex:       # the tiles do not fit next to the operator
        return {"error": str(ex)}
    ms = time_matvecs()
    nst, gst = g.kernel_stats("near_gemv_fp64"), g.kernel_stats("gemv_fp64")
    launches = max(nst["launches"], 1)
    near_b = nst["work"] / launches
    coup_b = gst["work"] / max(gst["launches"], 1)
    r = w.rank
    L = (g.level_size(2) // r).bit_length() - 1 if g.levels > 1 else 0
    d_top = L - g.levels + 2
    transfer_b = 2 * ((1 << (L + 1)) - (1 << (d_top + 1))) * r * r * 8 if g.levels > 1 else 0
    basis_b = 2 * w.n * r * 8
    vec_b = 3 * w.n * 8
    total = near_b + coup_b + basis_b + transfer_b + vec_b
    near_ms = nst["ms"] / launches
    out = {
        "layout": "near field stored: 64x64 FP64 tiles over leaf chunks, upper triangle; "
                  "couplings stored upper triangle",
        "store_s": round(t_store, 3),
        "matvec_ms": round(ms, 3),
        "algorithmic_gb": round(total / 1e9, 2),
        "near_tiles_gb": round(near_b / 1e9, 2), "couplings_gb": round(coup_b / 1e9, 2),
        "bases_transfers_vectors_gb": round((basis_b + transfer_b + vec_b) / 1e9, 2),
        "matvec_gbs": round(total / (ms * 1e-3) / 1e9, 1),
        "matvec_frac_of_hbm_peak": round(total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
        "near_gemv_ms": round(near_ms, 3),
        "near_gemv_gbs": round(near_b / (near_ms * 1e-3) / 1e9, 1) if near_ms else None,
        "near_gemv_roofline": block_gemv_roofline(g, "near_gemv_fp64"),
        "device_memory_gb": round(g.memory_bytes() / 1e9, 1),
    }
    if args.part_a:
        out["block_of_16"] = block_product(args, torch, g, w, ms)
    g.store_near(False)
    torch.cuda.synchronize()
    log(f"stored-near matvec: {out['matvec_ms']} ms, {out['matvec_gbs']} GB/s "
        f"({out['matvec_frac_of_hbm_peak']:.0%} of peak), near GEMV {out['near_gemv_gbs']} GB/s")
    return out


def batched(args, torch, synth, H2Matrix, n_problems=None):
    """Many right-hand sides of many uneven problems: Gaussian-mixture point
    clouds in 3D (8 components, sigma 0.05), N log-uniform in [2^14, 2^18],
    Gaussian kernel l = 0.1, rank 27 (3^3 Chebyshev), leaf 64, eta 0.7, 16
    right-hand sides each, FP32 cycles (block smoother) inside FP64
    refinement to 1e-8 per column, cycles launched as captured graphs.  The
    problems are solved together (h2mg_solve_batch) in groups that fit in
    HBM (the near field is evaluated inside the products, so only the
    couplings, projected blocks and block vectors are stored); each group is
    then solved again problem by problem with the 16-column solve, and one
    column of every problem with the single-vector solve, for comparison."""
    from paper_2501_17656_amd import solve_batch
    rng = np.random.default_rng(args.batch_seed)
    sizes = np.exp(rng.uniform(np.log(16384), np.log(262144), args.batch_problems)).astype(int)
    if n_problems is not None:
        sizes = sizes[:n_problems]       # the first problems of the same sequence
    shift = args.batch_shift
    budget = args.batch_budget_gb * 1e9
    t_build = t_batch = t_seq = t_single = t_onelaunch = t_onelaunch_eager = 0.0
    group_equal = []
    per = []
    group = []

    def solve_group():
        nonlocal t_batch, t_seq, t_single, t_onelaunch, t_onelaunch_eager
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, infos = solve_batch([(g, B) for g, B, _ in group], rtol=1e-8, precision="fp32",
                                smoother="bj", nstreams=args.batch_streams, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_batch += dt
        log(f"batched: group of {len(group)} (N {sum(g.n for g, _, _ in group)}) solved together in "
            f"{dt:.2f} s, cycles {[i['cycles'] for i in infos]}")
        # the same problems with every tile-product step in one launch over all of them
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xg, infg = solve_batch([(g, B) for g, B, _ in group], rtol=1e-8, precision="fp32",
                               smoother="bj", raise_on_error=False, mode="group")
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t0
        t_onelaunch += dtg
        same = all(bool(torch.equal(a, b)) for a, b in zip(xs, xg))
        group_equal.append(same)
        log(f"batched: the same group with one launch per tile-product step: {dtg:.2f} s, "
            f"bitwise equal to the stream solves: {same}")
        # and launched kernel by kernel (no cycle graphs)
        for g, _, _ in group:
            g.set_graphs(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xe, _ = solve_batch([(g, B) for g, B, _ in group], rtol=1e-8, precision="fp32",
                            smoother="bj", raise_on_error=False, mode="group")
        torch.cuda.synchronize()
        dte = time.perf_counter() - t0
        t_onelaunch_eager += dte
        for g, _, _ in group:
            g.set_graphs(True)
        group_equal.append(all(bool(torch.equal(a, b)) for a, b in zip(xs, xe)))
        log(f"batched: the same, kernel by kernel: {dte:.2f} s")
        for (g, B, i), info in zip(group, infos):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, im = g.solve_multi(B, rtol=1e-8, precision="fp32", smoother="bj", raise_on_error=False)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, i1 = g.solve(B[:, 0].contiguous(), rtol=1e-8, precision="fp32", smoother="bj",
                            raise_on_error=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            t_seq += t1 - t0
            t_single += 16 * (t2 - t1)
            per.append({"n": g.n, "levels": g.levels, "tuning": g.block_tuning() if args.batch_autotune else None,
                        "batch_cycles": info["cycles"],
                        "batch_status": info["status"], "batch_max_rel_residual": info["rel_residual"],
                        "block_solve_s": round(t1 - t0, 3), "single_rhs_solve_s": round(t2 - t1, 3),
                        "single_rhs_cycles": i1["cycles"]})
            g.close()
        group.clear()

    mem = 0.0
    for i, n in enumerate(sizes):
        P = synth.gaussian_mixture_points(int(n), 3, seed=1000 + i)
        B = torch.from_numpy(synth.normal_vector(int(n), 2000 + i, nrhs=16)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = H2Matrix(torch.from_numpy(P).cuda(), "gauss", 0.1, shift, 64, 0.7, 3)
        g.setup(("fp64", "fp32"))
        torch.cuda.synchronize()
        t_build += time.perf_counter() - t0
        log(f"batched: problem {i}: N={int(n)}, built in {time.perf_counter() - t0:.2f} s, "
            f"{g.memory_bytes() / 1e9:.2f} GB")
        g.set_graphs(True)
        if args.batch_autotune:
            # block buffers and tile-run tuning in the precision of the cycles
            # (a solve stopped before its first cycle)
            g.set_autotune(True)
            g.solve_multi(B, rtol=1e-8, precision="fp32", smoother="bj", max_cycles=0, raise_on_error=False)
        # block buffers and vectors of the 16-column solve: about 50 vectors of n x 16
        need = g.memory_bytes() + 50 * 16 * 8 * int(n)
        if group and mem + need > budget:
            solve_group()
            mem = 0.0
        group.append((g, B, i))
        mem += need
    if group:
        solve_group()
    nrhs_total = 16 * len(sizes)
    ok = all(p["batch_status"] == "OK" for p in per)
    # tile-product rates of the largest problem (product + reduce, FP32, as tuned)
    rates = {}
    big = max(per, key=lambda p: p["n"])
    for key, v in (big["tuning"] or {}).items():
        if not v["ms"]:
            continue
        if key == "near":
            rates["near_evaluated_Gentries_per_s"] = round(v["tiles_read"] * 4096 / (v["ms"] * 1e-3) / 1e9, 1)
        else:
            rates[f"{key}_GB_per_s"] = round(v["tiles_read"] * 32 * 32 * 4 / (v["ms"] * 1e-3) / 1e9, 1)
    out = {
        "workload": (f"{len(sizes)} problems, N log-uniform in [16384, 262144] (total {int(sizes.sum())} points), "
                     f"Gaussian-mixture clouds in 3D (8 components, sigma 0.05), gauss l=0.1 + {shift}*I "
                     f"(shift raised from 1e-2: the rank-27 approximation is indefinite there), rank 27, "
                     f"leaf 64, eta 0.7, 16 RHS each ~ N(0,1), FP32 cycles + FP64 refinement to 1e-8 per "
                     f"column, block smoother, graph-launched cycles, {args.batch_streams} streams, tile runs "
                     f"{'tuned per task set' if args.batch_autotune else 'fixed at 8'}"),
        "all_converged": ok,
        "build_and_setup_s": round(t_build, 2),
        "batched_solve_s": round(t_batch, 3),
        "rhs_per_s_batched": round(nrhs_total / t_batch, 2),
        "one_launch_per_step_solve_s": round(t_onelaunch, 3),
        "one_launch_per_step_kernel_by_kernel_s": round(t_onelaunch_eager, 3),
        "rhs_per_s_one_launch_per_step": round(nrhs_total / t_onelaunch, 2),
        "one_launch_per_step_bitwise_equal": all(group_equal),
        "sequential_block_solves_s": round(t_seq, 3),
        "single_rhs_solves_s_extrapolated": round(t_single, 3),
        "speedup_batched_vs_single_rhs": round(t_single / t_batch, 2),
        "speedup_batched_vs_sequential_blocks": round(t_seq / t_batch, 3),
        "largest_problem_tile_rates": {"n": big["n"], **rates},
        "problems": per,
    }
    log(f"batched: {len(sizes)} problems x 16 RHS in {t_batch:.2f} s ({nrhs_total / t_batch:.1f} RHS/s), "
        f"sequential 16-column solves {t_seq:.2f} s, single-RHS solves (16 x one column) {t_single:.2f} s")
    return out


def c1_latency(args, torch, synth, H2Matrix):
    """The small configuration (exp kernel, N = 4096 in 2D, leaf 64, rank 16):
    cache-resident and launch-bound, so it measures latency, with the
    oracle's full solve of the same problem timed beside it."""
    w = synth.workload("exp2d_4k")
    P, b = w.make_points(), w.make_rhs()
    pts = torch.from_numpy(P).cuda()
    bd = torch.from_numpy(b).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
    g.setup(("fp64", "fp32"))
    torch.cuda.synchronize()
    out = {"workload": f"{w.name}: N={w.n}, {w.kernel} l={w.length_scale} + {w.shift}*I, "
                       f"leaf {w.leaf}, eta {w.eta}, rank {w.rank}, rtol 1e-8; each cycle launched "
                       f"as one captured HIP graph",
           "build_and_setup_s": round(time.perf_counter() - t0, 4)}
    g.set_graphs(True)
    runs = [(m, sm, pr) for sm in ("cg", "bj") for pr in ("fp64", "fp32") for m in ("v",)]
    runs += [(m, sm, "fp64") for sm in ("cg", "bj") for m in ("w", "f", "cg")]
    for method, smoother, prec in runs:
        kw = dict(rtol=1e-8, precision=prec, smoother=smoother, method=method, raise_on_error=False,
                  max_cycles=20000 if method == "cg" else 500)
        g.solve(bd, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = g.solve(bd, **kw)
        torch.cuda.synchronize()
        key = f"{smoother}_{prec}" if method == "v" else f"{method}-cycle_{smoother}_{prec}"
        if method == "cg":
            key = f"plain_{'pcg' if smoother == 'bj' else 'cg'}_fp64"
        out[key] = {"time_to_1e-8_s": round(time.perf_counter() - t0, 4),
                    ("iterations" if method == "cg" else "cycles"): info["cycles"],
                    "converged": info["converged"]}
    g.close()
    if not args.no_cpu:
        from oracle.galerkin import Hierarchy
        from oracle.h2 import H2 as OracleH2
        from oracle.vcycle import solve_user
        t0 = time.perf_counter()
        o = OracleH2(P, w.kernel, w.shift, w.leaf, w.eta, w.cheb_m, w.length_scale)
        H = Hierarchy(o)
        t1 = time.perf_counter()
        res = solve_user(o, H, b, rtol=1e-8)
        t2 = time.perf_counter()
        out["oracle_cg_fp64"] = {"time_to_1e-8_s": round(t2 - t1, 3), "setup_s": round(t1 - t0, 3),
                                 "cycles": res.cycles, "converged": res.converged,
                                 "threads": int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())}
    log(f"C1 {w.name}: " + ", ".join(f"{k} {v['time_to_1e-8_s']} s/{v.get('cycles', v.get('iterations'))}"
                                      for k, v in out.items() if isinstance(v, dict)))
    return out


def growth_scan(args, torch, synth, H2Matrix):
    """Iterations to 1e-8 against N on the shift-1 Matern problem: H2-MG
    V-cycles (paper CG smoother and block smoother) next to the comparison
    solver, CG (and block-Jacobi PCG) on A_H2 alone.  FP64; the near field is
    stored when it fits, which speeds up every fine-level product alike."""
    base = synth.workload("matern3d_1m_shift1")
    for n in [int(v) for v in args.growth.split(",")]:
        w = base.scaled(n)
        pts = torch.from_numpy(w.make_points()).cuda()
        b = torch.from_numpy(w.make_rhs()).cuda()
        g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
        try:
            g.store_near(True)
            stored = True
        except Exception:
            stored = False
        g.setup()
        out = {"growth": w.name, "n": n, "near_stored": stored}
        for label, kw in (("vcycle_cg_smoother", dict(method="v", smoother="cg")),
                          ("vcycle_block_smoother", dict(method="v", smoother="bj")),
                          ("plain_cg", dict(method="cg", smoother="cg", max_cycles=50000)),
                          ("plain_pcg_block_jacobi", dict(method="cg", smoother="bj", max_cycles=50000))):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = g.solve(b, rtol=1e-8, raise_on_error=False, **kw)
            torch.cuda.synchronize()
            out[label] = {"count": info["cycles"], "s": round(time.perf_counter() - t0, 3),
                          "converged": info["converged"], "rel_residual": info["rel_residual"]}
            log(f"growth n={n} {label}: {info['cycles']} in {out[label]['s']} s ({info['status']})")
        print(json.dumps(out), flush=True)
        g.close()
        del pts, b
        torch.cuda.empty_cache()


def differentiation(args, torch, synth, H2Matrix):
    """Gradient of L = b^T A^{-1} b in (l, s, points) on the exponential-
    kernel workload (N = 2^18): forward H2-MG solve, then the derivative-
    kernel H2 builds and their 1 + 1 + dim products."""
    w = synth.workload("exp3d_256k")
    pts = torch.from_numpy(w.make_points()).cuda()
    b = torch.from_numpy(w.make_rhs()).cuda()
    out = {"workload": f"{w.name}: N={w.n}, {w.kernel} l={w.length_scale} + {w.shift}*I, "
                       f"leaf {w.leaf}, eta {w.eta}, rank {w.rank}, solve rtol 1e-10, block smoother"}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
    g.setup()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, info = g.solve(b, rtol=1e-10, smoother="bj", raise_on_error=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out.update({"build_and_setup_s": round(t1 - t0, 3), "solve_s": round(t2 - t1, 3),
                "solve_cycles": info["cycles"], "solve_status": info["status"]})
    # the same forward solve with FP32 cycles inside FP64 refinement
    g.setup(("fp64", "fp32"))
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    xm, im = g.solve(b, rtol=1e-10, smoother="bj", precision="fp32", raise_on_error=False)
    torch.cuda.synchronize()
    out.update({"solve_fp32_refinement_s": round(time.perf_counter() - t5, 3),
                "solve_fp32_refinement_steps": im["cycles"], "solve_fp32_refinement_status": im["status"],
                "solutions_rel_diff": float((xm - x).norm() / x.norm())})
    del xm
    t2 = time.perf_counter()
    if info["converged"]:
        hl, hg = g.derivative("dl"), g.derivative("g")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        L, dl, ds, gp, _ = g.quadratic_gradient(hl, hg, b, x)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        out.update({"derivative_builds_s": round(t3 - t2, 3), "gradient_products_s": round(t4 - t3, 3),
                    "loss": L, "dL_dl": dl, "dL_ds": ds,
                    "grad_points_norm": float(gp.norm()),
                    "backward_total_s": round(t4 - t2, 3)})
        hl.close()
        hg.close()
    g.close()
    log(f"differentiation {w.name}: solve {out['solve_s']} s ({out['solve_status']}), FP32 refinement "
        f"{out['solve_fp32_refinement_s']} s, backward {out.get('backward_total_s')} s")
    return out


def smoothing_sweep(args, torch, synth, H2Matrix):
    """Time-to-1e-8 against the smoothing counts (n_f, n_c) on the shift-1
    Matern problem at 2^20: each item smoother:precision:n_f:n_c."""
    w = synth.workload("matern3d_1m_shift1")
    pts = torch.from_numpy(w.make_points()).cuda()
    b = torch.from_numpy(w.make_rhs()).cuda()
    g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
    g.setup(("fp64", "fp32"))
    for item in args.sweep.split(","):
        smoother, prec, nf, nc = item.split(":")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = g.solve(b, rtol=1e-8, precision=prec, smoother=smoother, n_fine=int(nf),
                          n_coarse=int(nc), raise_on_error=False, max_cycles=300)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out = {"sweep": w.name, "smoother": smoother, "precision": prec, "n_f": int(nf),
               "n_c": int(nc), "cycles": info["cycles"], "time_s": round(dt, 3),
               "status": info["status"], "rel_residual": info["rel_residual"]}
        print(json.dumps(out), flush=True)
        log(f"sweep {item}: {info['cycles']} cycles, {dt:.2f} s, {info['status']}")
    g.close()


def error_components(args, torch, synth, H2Matrix):
    """The error analysis of the experiments: 1D Gaussian kernel, N = 1024
    equally spaced points, sigma = 2 l^2 = 0.01, c = 1e-3; b = A x_true,
    x_0 = 0; after the first fine-level smoothing of cycles 1 and 2, the
    error split into U_1^T e (what restriction carries to the coarse levels)
    and its complement Q_1^T e.  Norms on the host from the library's
    smoother, level products, restriction and V-cycle."""
    import math
    pts = torch.from_numpy(synth.tensor_grid_points(1024, 1)).cuda()
    x_true = torch.from_numpy(synth.normal_vector(1024, 3)).cuda()
    for leaf, m in ((32, 8), (16, 6)):
        g = H2Matrix(pts, "gauss", math.sqrt(0.01 / 2), 1e-3, leaf, 0.7, m)
        b = g.matvec(x_true)
        for nc in (2, 40):
            x = torch.zeros_like(b)
            rows = []
            for _ in range(3):
                r = b - g.matvec(x)
                err = x + g.smooth(1, r, 1) - x_true
                ue = g.restrict(1, err)
                ue2 = float((ue @ ue).item())
                qn = math.sqrt(max(float((err @ err).item()) - ue2, 0.0))
                rows.append({"U1T_e_norm": math.sqrt(ue2), "U1T_e_max": float(ue.abs().max().item()),
                             "Q1T_e_norm": qn})
                x = g.vcycle(x, b, n_coarse=nc)
            print(json.dumps({"error_components": "gauss1d_1024", "leaf": leaf, "m": m, "n_c": nc,
                              "levels": g.levels, "after_first_smoothing": rows}), flush=True)
        g.close()


def boundary_elements(args, torch, synth, H2Matrix):
    """Laplace single layer on the bumpy torus (Section 4.3's problem, the
    symmetric scaled form): panels, H2 build (1/(4 pi r), leaf 128, rank 64),
    hierarchy, FP64 and FP32-refinement solves with the paper's CG smoother
    for Dirichlet data given by a random harmonic polynomial of degree 2,
    and the matvec."""
    from paper_2501_17656_amd import bem_density, bem_harmonic_rhs, bem_panels, bem_quadrature7
    nmaj, nmin = args.bem_grid
    V, T = synth.bumpy_torus_mesh(nmaj, nmin)
    Vd = torch.from_numpy(V).cuda()
    Td = torch.from_numpy(T).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y, sc, dg = bem_panels(Vd, Td)
    g = H2Matrix(y, "laplace", 1.0, 0.0, 128, 0.7, 4, scale=sc, diag=dg)
    if not args.bem_one_point:
        # the close entries by the seven-point rule on both triangles (stored tiles)
        qy, qu = bem_quadrature7(Vd, Td)
        g.set_near_quadrature(qy, qu)
        del qy, qu
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.setup(("fp64", "fp32"))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    coeffs = synth.harmonic_coefficients(7)
    f = bem_harmonic_rhs(y, sc, coeffs)
    out = {"workload": f"bumpy torus (R 1, r 0.35, 40 bumps of 0.05), {len(T)} panels, Laplace single "
                       f"layer 1/(4 pi r), closed-form self term, symmetric scaled form, close entries by "
                       f"{'the one-point rule' if args.bem_one_point else 'the seven-point rule on both triangles'}, leaf 128, "
                       f"eta 0.7, rank 64, right-hand side a random harmonic polynomial of degree 2 (seed 7), "
                       f"rtol 1e-8, CG smoother (the block "
                       f"smoother's FP32 PCG breaks down at 10^6 panels)",
           "panels_and_build_s": round(t1 - t0, 3), "setup_s": round(t2 - t1, 3),
           "levels": g.levels, "device_memory_gb": round(g.memory_bytes() / 1e9, 1)}
    x = torch.empty_like(f)
    g.matvec(f, out=x)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(3):
        g.matvec(f, out=x)
    torch.cuda.synchronize()
    out["matvec_ms"] = round((time.perf_counter() - t3) / 3 * 1e3, 3)
    for prec in ("fp64", "fp32"):
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        sol, info = g.solve(f, rtol=1e-8, precision=prec, smoother="cg", raise_on_error=False)
        torch.cuda.synchronize()
        out[prec] = {"time_to_1e-8_s": round(time.perf_counter() - t4, 3), "cycles": info["cycles"],
                     "status": info["status"], "rel_residual": info["rel_residual"]}
        if info["converged"]:
            sigma = bem_density(sol, sc)
            out[prec]["density_norm"] = float(sigma.norm())
        log(f"boundary elements {len(T)} panels {prec}: {out[prec]['time_to_1e-8_s']} s, "
            f"{info['cycles']} cycles, {info['status']}")
    if out["fp64"]["status"] == "OK" and out["fp32"]["status"] == "OK":
        out["speedup_mixed_vs_fp64"] = round(out["fp64"]["time_to_1e-8_s"] / out["fp32"]["time_to_1e-8_s"], 3)
    g.close()
    return out


def headline_matvec(args, torch, synth, H2Matrix):
    """The fine H2 matvec on the specified matrix (shift as given, here 1e-3):
    build, then y = A_H2 x timed with the near field evaluated from the
    points and with it stored as FP64 tiles.  Timings come from torch events
    around `matvec_reps` products launched without instrumentation; a second
    set with the library's per-launch HIP events gives the per-kernel rates."""
    w = synth.workload(args.headline)
    log(f"matvec workload {w.name}: n={w.n} shift={w.shift}")
    pts = torch.from_numpy(w.make_points()).cuda()
    x = torch.from_numpy(w.make_x()).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    y = torch.empty_like(x)

    def time_matvecs():
        g.set_timing(False)
        g.matvec(x, out=y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.matvec_reps):
            g.matvec(x, out=y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.matvec_reps
        g.set_timing(True)              # per-launch events, stats read by the caller
        for _ in range(args.matvec_reps):
            g.matvec(x, out=y)
        torch.cuda.synchronize()
        return ms

    ev_ms = time_matvecs()
    gst, nst = g.kernel_stats("gemv_fp64"), g.kernel_stats("near_fp64")
    gemv_bytes = gst["work"] / max(gst["launches"], 1)
    out = {
        "workload": f"{w.name}: N={w.n} uniform in [0,1)^{w.dim}, {w.kernel} l={w.length_scale} + "
                    f"{w.shift}*I, leaf {w.leaf}, eta {w.eta}, rank {w.rank}, x ~ N(0,1)",
        "build_s": round(t1 - t0, 3),
        "evaluated_near": {
            "matvec_ms": round(ev_ms, 3),
            "couplings_gb": round(gemv_bytes / 1e9, 2),
            "near_field_ms": round(nst["ms"] / max(nst["launches"], 1), 3),
            "near_field_evals_per_s": round(nst["work"] / (nst["ms"] * 1e-3), 0) if nst["ms"] else None,
        },
    }
    out["stored_near"] = stored_near_matvec(args, torch, g, w, time_matvecs)
    g.set_timing(False)
    g.close()
    del pts, x, y
    torch.cuda.empty_cache()
    return out


def part_a(args, torch, synth, H2Matrix):
    """Cycles on the specified 1e-3 matrix (indefinite at this size): hierarchy
    setup, a few FP64 V-cycles and mixed refinement steps with their residual
    history, the block smoother's first cycle, and the 16-vector block
    product with the near field stored."""
    w = synth.workload(args.headline)
    log(f"part A workload {w.name}: n={w.n} shift={w.shift}")
    pts = torch.from_numpy(w.make_points()).cuda()
    b = torch.from_numpy(w.make_rhs()).cuda()
    torch.cuda.synchronize()
    g = H2Matrix(pts, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
    torch.cuda.synchronize()
    t1b = time.perf_counter()
    g.setup(("fp64", args.mixed))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g.set_timing(True)
    _, i64 = g.solve(b, rtol=1e-8, max_cycles=args.headline_cycles, precision="fp64",
                     raise_on_error=False)
    rl64 = block_gemv_roofline(g, "gemv_fp64")
    g.set_timing(True)
    _, im = g.solve(b, rtol=1e-8, max_cycles=args.headline_cycles, precision=args.mixed,
                    raise_on_error=False)
    rlm = block_gemv_roofline(g, "gemv_" + args.mixed)
    g.set_timing(False)
    _, ibj = g.solve(b, rtol=1e-8, max_cycles=args.headline_cycles, precision="fp64",
                     smoother="bj", raise_on_error=False)
    out = {
        "workload": f"{w.name}: N={w.n}, {w.kernel} l={w.length_scale} + {w.shift}*I, leaf {w.leaf}, "
                    f"eta {w.eta}, rank {w.rank}",
        "setup_s": round(t2 - t1b, 3), "levels": g.levels,
        "device_memory_gb": round(g.memory_bytes() / 1e9, 1),
        "fp64_cycles_run": i64["cycles"], "fp64_s_per_cycle": round(i64["solve_seconds"] / max(i64["cycles"], 1), 3),
        "fp64_residual_history": [round(v, 4) for v in i64["history"]],
        "mixed_steps_run": im["cycles"], "mixed_s_per_step": round(im["solve_seconds"] / max(im["cycles"], 1), 3),
        "mixed_residual_history": [round(v, 4) for v in im["history"]],
        "block_smoother_fp64": {"cycles_run": ibj["cycles"], "status": ibj["status"],
                                "residual_history": [round(v, 4) for v in ibj["history"]]},
        "converges": False,
        "why": ("the rank-64 Chebyshev H2 approximation of this matrix is indefinite at this size "
                "(negative Rayleigh quotients of diverged V-cycle iterates from N = 65536 on)"),
        "gemv_fp64_roofline": rl64, "gemv_mixed_roofline": rlm,
    }
    try:
        g.store_near(True)
        single = torch.from_numpy(w.make_x()).cuda()
        y = g.matvec(single)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.matvec_reps):
            g.matvec(single, out=y)
        torch.cuda.synchronize()
        single_ms = (time.perf_counter() - t0) / args.matvec_reps * 1e3
        out["block_of_16"] = block_product(args, torch, g, w, single_ms)
    except Exception as ex:       # the tiles do not fit next to the hierarchy
        out["block_of_16"] = {"error": str(ex)}
    g.close()
    del pts, b
    torch.cuda.empty_cache()
    return out


def timed_solves(args, torch, g, b_d, deadline):
    """Warmup and timed mixed-precision solves from x0 = 0 on the built
    hierarchy.  Each stops early (after at least one solve) when the next
    solve, estimated by the slowest one so far, would end after `deadline`."""
    def one():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = g.solve(b_d, rtol=1e-8, max_cycles=args.max_cycles, precision=args.mixed,
                          smoother=args.smoother, raise_on_error=False)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, x, info

    slowest = 0.0
    warm = 0
    for i in range(args.warmup):
        # keep room for this warmup and one timed solve
        if warm > 0 and time.perf_counter() + 2 * slowest > deadline:
            break
        dt, x, info = one()
        slowest = max(slowest, dt)
        warm += 1
        log(f"warmup solve {i + 1}/{args.warmup}: {dt:.2f} s, {info['cycles']} steps, {info['status']}")
    times, infos = [], []
    x = None
    for i in range(args.steps):
        if times and time.perf_counter() + slowest > deadline:
            break
        dt, x, info = one()
        slowest = max(slowest, dt)
        times.append(dt)
        infos.append(info)
        log(f"timed solve {i + 1}/{args.steps}: {dt:.2f} s, {info['cycles']} steps, "
            f"rel res {info['rel_residual']:.2e}, {info['status']}")
    return warm, times, infos, x


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import synth
    from paper_2501_17656_amd import H2Matrix

    if args.copy_probe:
        copy_probe()
        return
    if args.spd_probe:
        spd_probe(args, torch, synth, H2Matrix)
        return
    if args.lanczos:
        lanczos_probe(args, torch, synth, H2Matrix)
        return
    if args.shift_scan:
        shift_scan(args, torch, synth, H2Matrix)
        return
    if args.growth:
        growth_scan(args, torch, synth, H2Matrix)
        return
    if args.sweep:
        smoothing_sweep(args, torch, synth, H2Matrix)
        return
    if args.error_components:
        error_components(args, torch, synth, H2Matrix)
        return
    if args.setup_only:
        print(json.dumps({"setup": setup_only(args, torch, synth, H2Matrix)}), flush=True)
        return
    if args.block_product:
        print(json.dumps({"block_product": block_product_only(args, torch, synth, H2Matrix)}), flush=True)
        return
    if args.batched:
        out = batched(args, torch, synth, H2Matrix)
        print(json.dumps({"batched": out}), flush=True)
        if args.json_out:
            with open(args.json_out, "w") as f:
                f.write(json.dumps({"batched": out}) + "\n")
        return

    extras = extras_requested(args)
    if args.extras_only:
        out = run_extras_alone(args, extras, torch, synth, H2Matrix)
        print(json.dumps(out), flush=True)
        if args.json_out:
            with open(args.json_out, "w") as f:
                f.write(json.dumps(out) + "\n")
        return
    deadline = T_START + args.budget_s
    # seconds kept after the timed solves: instrumented steps, oracle baseline
    reserve = 12.0 + (0.0 if args.no_cpu else args.cpu_seconds + 25.0)

    # 1. matvec GB/s on the specified matrix
    mv = headline_matvec(args, torch, synth, H2Matrix) if args.headline else None
    if mv:
        st = mv["stored_near"]
        log(f"matvec {mv['workload']}: evaluated near {mv['evaluated_near']['matvec_ms']} ms; "
            f"stored near {st.get('matvec_ms')} ms, {st.get('matvec_gbs')} GB/s")

    # 2. the timed workload: build and hierarchy once, one FP64 solve
    w = synth.workload(args.workload)
    if args.n:
        w = w.scaled(args.n)
    dev = torch.device("cuda:0")
    log(f"timed workload {w.name}: n={w.n} dim={w.dim} kernel={w.kernel} l={w.length_scale} "
        f"shift={w.shift} leaf={w.leaf} eta={w.eta} m={w.cheb_m}")
    P = w.make_points()
    b = w.make_rhs()
    pts_d = torch.from_numpy(P).to(dev)
    b_d = torch.from_numpy(b).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = H2Matrix(pts_d, w.kernel, w.length_scale, w.shift, w.leaf, w.eta, w.cheb_m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.setup(("fp64", args.mixed))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g.set_graphs(not args.no_graphs)
    log(f"build {t1 - t0:.2f} s, hierarchy {t2 - t1:.2f} s, {g.levels} levels, "
        f"{g.memory_bytes() / 1e9:.1f} GB")
    # block-GEMV launch of each level's product (grid sizes identify the
    # launches in a kernel trace)
    gemv_launches = {}
    for k in range(1, g.levels + 1):
        info = g.gemv_launch_info(k)
        info["depth"] = None if k == 1 else (g.level_size(k) // w.rank).bit_length() - 1
        gemv_launches[k] = info
    x64, i64 = g.solve(b_d, rtol=1e-8, max_cycles=args.max_cycles, precision="fp64",
                       smoother=args.smoother, raise_on_error=False)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    fp64_s = t3 - t2
    log(f"fp64 solve {fp64_s:.2f} s, {i64['cycles']} cycles, rel res {i64['rel_residual']:.2e}, "
        f"{i64['status']}")

    # 3. warmup and timed mixed-precision solves
    warm, times, infos, xm = timed_solves(args, torch, g, b_d, deadline - reserve)
    im = infos[-1]
    mixed_ok = all(i["converged"] for i in infos)
    mixed_s = float(np.mean(times))

    # 4. instrumented refinement step (per-launch HIP events) for the roofline,
    # and one instrumented FP64 cycle for the FP64 block GEMV
    g.set_timing(True)
    g.solve(b_d, rtol=1e-8, max_cycles=1, precision=args.mixed, smoother=args.smoother,
            raise_on_error=False)
    rlm = block_gemv_roofline(g, "gemv_" + args.mixed)
    g.set_timing(True)
    g.solve(b_d, rtol=1e-8, max_cycles=1, precision="fp64", smoother=args.smoother,
            raise_on_error=False)
    rl64 = block_gemv_roofline(g, "gemv_fp64")
    g.set_timing(False)
    log(f"instrumented steps: {args.mixed} GEMV {(rlm or {}).get('frac')}, "
        f"fp64 GEMV {(rl64 or {}).get('frac')} of HBM peak")

    extra = run_extras(args, extras, torch, synth, H2Matrix, g, w, b_d, mixed_s)
    dx = float((xm - x64).norm() / x64.norm())
    levels, mem_gb = g.levels, round(g.memory_bytes() / 1e9, 1)
    xm_h, x64_h = xm.cpu().numpy(), x64.cpu().numpy()
    g.close()
    del x64, xm
    torch.cuda.empty_cache()
    extra.update(run_extras_alone(args, extras, torch, synth, H2Matrix))
    st = (mv or {}).get("stored_near") or {}
    out = {
        "metric": METRIC,
        "value": round(mixed_s if mixed_ok else fp64_s, 3),
        "unit": "s",
        "n_gpus": 1,
        "steps": len(times),
        "warmup": warm,
        "ms_per_step": round(1e3 * mixed_s, 1),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": f"{args.mixed}+f64-refinement" if mixed_ok else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: N={w.n} points uniform in [0,1)^{w.dim} (seed {w.point_seed}), "
                         f"{w.kernel} l={w.length_scale} + {w.shift}*I (shift raised from 1e-3: the "
                         f"rank-64 Chebyshev approximation has eigenvalues down to -0.0936 at this size, "
                         f"so shifts below 0.095 are indefinite), leaf "
                         f"{w.leaf}, eta {w.eta}, Chebyshev {w.cheb_m}^{w.dim} (rank {w.rank}), "
                         f"b ~ N(0,1) (seed {w.rhs_seed}), x0 = 0, rtol 1e-8, n_f=1, n_c=40, smoother "
                         f"{args.smoother} ({'CG preconditioned by the diagonal blocks' if args.smoother == 'bj' else 'plain CG'}); "
                         f"step = one {args.mixed}-operator V-cycle solve inside FP64 refinement on the "
                         f"built hierarchy, cycles as captured graphs"),
            "levels": levels,
        },
        "steps_requested": args.steps, "warmup_requested": args.warmup,
        "budget_s": args.budget_s,
        "step_times_s": [round(t, 3) for t in times],
        "mixed_precision": args.mixed,
        "mixed_time_to_1e-8_s": round(mixed_s, 3),
        "mixed_refinement_steps": im["cycles"], "mixed_converged": mixed_ok,
        "mixed_rel_residual": im["rel_residual"],
        "fp64_time_to_1e-8_s": round(fp64_s, 3),
        "fp64_cycles": i64["cycles"], "fp64_converged": i64["converged"],
        "fp64_rel_residual": i64["rel_residual"],
        "speedup_mixed_vs_fp64": round(fp64_s / mixed_s, 3) if mixed_s > 0 else None,
        "mixed_vs_fp64_solution_rel_diff": dx,
        "build_s": round(t1 - t0, 3),
        "setup_s": round(t2 - t1, 3),
        "device_memory_gb": mem_gb,
        "matvec_ms": st.get("matvec_ms"),
        "matvec_gbs": st.get("matvec_gbs"),
        "matvec_frac_of_hbm_peak": st.get("matvec_frac_of_hbm_peak"),
        "matvec_algorithmic_gb": st.get("algorithmic_gb"),
        "matvec": mv,
        "roofline": rlm if mixed_ok and rlm else rl64,
        "roofline_fp64_gemv": rl64,
        "gemv_launches": gemv_launches,
    }
    out.update(extra)
    if not args.no_cpu:
        try:
            out.update(cpu_baseline(w, P, b, {args.mixed: xm_h, "fp64": x64_h}, args.mixed,
                                    args.cpu_seconds, st.get("matvec_ms")))
        except Exception as e:  # the baseline must not hide the GPU result
            out["cpu_baseline"] = {"error": repr(e)}
    out["wall_s"] = round(time.perf_counter() - T_START, 1)
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


def run_extras(args, extras, torch, synth, H2Matrix, g, w, b_d, mixed_s):
    """The opt-in parts that use the timed matrix (none in the default run)."""
    out = {}
    if "cg_smoother" in extras:
        runs = {}
        for prec in ("fp64", args.mixed):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = g.solve(b_d, rtol=1e-8, max_cycles=args.max_cycles, precision=prec,
                              smoother="cg", raise_on_error=False)
            torch.cuda.synchronize()
            runs[prec] = {"time_to_1e-8_s": round(time.perf_counter() - t0, 3), "cycles": info["cycles"],
                          "converged": info["converged"], "rel_residual": info["rel_residual"]}
        out["paper_cg_smoother"] = runs
    if "sixteen_rhs" in extras:
        out["sixteen_rhs_solve"] = many_rhs_solve(args, torch, g, w, mixed_s)
    return out


def run_extras_alone(args, extras, torch, synth, H2Matrix):
    """The opt-in parts that build matrices of their own (run after the timed
    matrix is released)."""
    out = {}
    if "c1" in extras:
        out["c1_small_config"] = c1_latency(args, torch, synth, H2Matrix)
    if "diff" in extras:
        out["differentiation"] = differentiation(args, torch, synth, H2Matrix)
    if "bem" in extras:
        out["boundary_elements"] = boundary_elements(args, torch, synth, H2Matrix)
    if "batched_first" in extras:
        out["batched_first_problems"] = batched(args, torch, synth, H2Matrix, args.batched_first)
    if "part_a" in extras:
        out["headline_shift_1e-3_cycles"] = part_a(args, torch, synth, H2Matrix)
    return out


if __name__ == "__main__":
    main()
