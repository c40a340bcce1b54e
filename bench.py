#!/usr/bin/env python3
"""Throughput of GenCD solves on one MI355X.

Workload: the tf-idf-like logistic problem (n = 100,000 samples, k = 500,000
features, Zipf(1.1) column popularity, ~50 nonzeros per row, lognormal values,
rows L2-normalised, labels from a 500-sparse w*), lambda = 0.05 lambda_max,
Shotgun with |J| = 4096.  One step = one full solve from w = 0 to FP64
KKT <= 1e-6 (inputs already resident in HBM).

Printed value: nnz-updates/s = sum over accepted proposals of nnz_j, divided
by the wall time of the timed solves.  Also reported: solves/s, coordinate
updates/s, the nonzeros actually scattered, the Thread-Greedy variant, the
roofline of Propose and of Update (each timed with HIP events around its own
dispatches on the solve's stream; `roofline` is the one with the larger
total time), the error of the result against the oracle's tight optimum,
and the FP64 oracle timed on the host as the CPU baseline.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of one Propose and one Update launch (headline), and of one
# fused epoch launch of the batched path, measured with rocprofv3 counters
# (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size) and kept
# as text summaries.  A figure is reported only while the kernel sources it
# was taken on are unchanged.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_propose_k_update_zipf1.1-logistic_n100k_k500k_pmc.md")
TRAFFIC_SOURCES = ["gencd_common.hpp", "gencd_kernels.hpp", "gencd_kernels.hip", "gencd_solver.hip"]
PATH_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_path_fused_binary_n50k_k200k_path64.md")
PATH_TRAFFIC_SOURCES = ["gencd_common.hpp", "gencd_kernels.hpp", "gencd_path.hip"]
# the autotuner's cache (JSON lines: one schedule per device, problem shape
# and column-length histogram, as gencd_autotune writes them); a key found
# there is answered without timing, so the headline's schedule is fixed
TUNE_CACHE = os.path.join(ROOT, "paper_1206_6409_amd", "tune_cache.jsonl")



def kernel_sources_sha256(sources=None):
    import hashlib
    h = hashlib.sha256()
    for name in sources or TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1206_6409_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel="k_propose", profile=None, sources=None, schedule=None):
    """Bytes per launch of `kernel` from a counter summary, or None when the
    summary is missing or was taken on other kernel sources (or, when
    `schedule` is given, under another launch schedule)."""
    try:
        text = open(profile or TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and " = " in line:
            k, v = line[2:].split(" = ", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_sources_sha256") != kernel_sources_sha256(sources):
        return None
    if schedule is not None and vals.get("schedule") != schedule:
        return None
    try:
        return float(vals[f"traffic_bytes_per_launch.{kernel}"])
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="shotgun",
                    choices=["shotgun", "coloring", "path", "serve", "sweep", "all"],
                    help="shotgun (default, the headline line) or an extra workload")
    ap.add_argument("--gpus", type=int, default=1)
    # a solve takes ~10 ms: enough warm-up and timed solves that clock and
    # cache state after the box comes up do not decide the figure
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink n and k (tests only)")
    ap.add_argument("--select", type=int, default=4096)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-thread-greedy", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time only the plain launch path")
    ap.add_argument("--no-tune", action="store_true",
                    help="headline: the default schedule instead of the autotuner's")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, metavar="PATH",
                    help="headline: the autotuner's cache file (read, appended to on a miss)")
    ap.add_argument("--schedule", type=int, nargs=3, metavar=("GROUP", "PIECE", "RESIDUAL"),
                    help="headline: this schedule instead of the autotuner's (profiling runs)")
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests in the stream")
    ap.add_argument("--calibration", type=int, default=200,
                    help="serve: warm-up requests, submitted at once, that set the rate")
    ap.add_argument("--plain-requests", type=int, default=100,
                    help="serve: prefix of the stream timed on the plain path")
    ap.add_argument("--oracle-sample", type=int, default=8,
                    help="serve: stratified requests checked against the oracle")
    ap.add_argument("--oracle-max-nnz", type=float, default=4e5,
                    help="serve: largest expected nnz of an oracle-checked request")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serve: arrival rate (skips the calibration run when > 0)")
    ap.add_argument("--slice", type=int, nargs=2, default=None, metavar=("FIRST", "END"),
                    help="serve: run only requests [FIRST, END) of the stream, arrivals "
                         "shifted to start at 0 (a long stream in several runs)")
    ap.add_argument("--merge", nargs="+", default=None, metavar="JSON",
                    help="serve: combine the lines of slice runs into one line")
    ap.add_argument("--lambdas", type=int, default=64, help="path: number of lambda values")
    ap.add_argument("--no-path-tight", action="store_true",
                    help="path: skip the KKT 1e-10 level (profiling runs)")
    ap.add_argument("--path-only", default=None, metavar="NAME",
                    help="path: run only the batched configuration NAME (e.g. B16_fused_epoch), "
                         "no plain path and no oracle leg (profiling runs)")
    ap.add_argument("--slots", type=int, default=16, help="serve: concurrent request slots")
    ap.add_argument("--serve-check", type=int, default=0, metavar="E",
                    help="serve: check_every of the requests (0: a tenth of the epochs run; "
                         "-m: an m-th)")
    ap.add_argument("--serve-fused", action="store_true",
                    help="serve: requests with GENCD_FUSED (server and plain path alike)")
    ap.add_argument("--sweep-scales", type=float, nargs="+", default=[1.0, 8.0],
                    help="sweep: scales of the logistic workload")
    ap.add_argument("--sweep-iters", type=int, default=10, help="sweep: Greedy iterations")
    ap.add_argument("--sweep-group", type=int, default=0, help="sweep: lanes per short column")
    ap.add_argument("--sweep-piece", type=int, default=0, help="sweep: nonzeros per long piece")
    ap.add_argument("--calibration-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (the reference "
                         "dispatch for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "row-sharded design is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serve" and args.merge:  # host only: combine slice lines
        print(json.dumps(merge_serve(args.merge)), flush=True)
        return

    import numpy as np
    import torch

    from paper_1206_6409_amd import gencd as G
    from paper_1206_6409_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    G.lib()  # fail loudly if the HIP library is missing
    torch.cuda.set_device(0)
    if args.calibration_copy > 0:
        nb = args.calibration_copy << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb} bytes read, {nb} bytes written")
        del src, dst
    if args.workload != "shotgun":
        names = ["coloring", "path", "serve"] if args.workload == "all" else [args.workload]
        for name in names:
            print(json.dumps(WORKLOADS[name](args)), flush=True)
        return

    t = time.time()
    P = synth.c2_zipf_logistic(scale=args.scale)
    log(f"generated {P.name}: nnz={P.nnz} in {time.time() - t:.1f}s")
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device="cuda")
    lam_max = G.lambda_max(X, y, P.loss)
    lam = 0.05 * lam_max
    base = dict(loss=P.loss, lam=lam, rule=G.SHOTGUN, select_size=args.select, seed=7,
                tol=args.tol, max_epochs=100000, check_every=1)
    ws = G.workspace(X, G.make_params(**base))
    # schedule of the Shotgun legs: the project's autotuner (lanes per short
    # column x piece size x captured graph x residual form), which times each
    # candidate on 3 epochs of this solve and keeps the fastest
    tuned, sched = {}, None
    if args.schedule:
        sched = {"from": "given on the command line"}
        tuned = dict(zip(("group", "piece", "residual"), args.schedule))
    elif not args.no_tune:
        sched = G.autotune(X, y, G.make_params(**base), epochs=3, cache_path=args.tune_cache)
        tuned = {"group": int(sched["group"]), "piece": int(sched["piece"]),
                 "residual": int(sched["residual"])}
        sched = {"from": "autotuner (3 epochs per candidate)"
                         + (", cached in " + os.path.relpath(args.tune_cache, ROOT)
                            if sched["from_cache"] else "")}
        log(f"autotuned schedule: {tuned}")
    if tuned:
        ws = G.workspace(X, G.make_params(**base, **tuned))
    sched_key = ",".join(str(tuned.get(f, d)) for f, d in (("group", 8), ("piece", 256),
                                                             ("residual", 0)))

    last_res = {}

    def run(rule, steps, warmup, flags=0, **kw):
        nonlocal ws
        pr = dict(base, rule=rule, **kw)
        need = G.workspace_bytes(X, G.make_params(flags=flags, **pr))
        if need > ws.numel():  # e.g. Block Shotgun's per-block vectors
            ws = G.workspace(X, G.make_params(flags=flags, **pr))
        for _ in range(warmup):
            G.solve(X, y, G.make_params(**pr), ws=ws)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for _ in range(steps):
            res = G.solve(X, y, G.make_params(flags=flags, **pr), ws=ws)
            stats.append(res.stats)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert all(s["converged"] == 1 for s in stats), stats[-1]
        last_res[(rule, flags)] = res
        return dt, stats, res

    log("timing Shotgun solves (plain launches)")
    dt_plain, stats_plain, _ = run(G.SHOTGUN, args.steps, args.warmup, **tuned)
    # kernel durations: HIP events around every Propose and Update launch
    # (GENCD_PROFILE; the library lets the host queue each epoch before it
    # starts, so no event pair spans a wait for the host), in solves of their
    # own, apart from the timed ones
    log("timing Propose and Update launches (kernel events)")
    _, stats_prof, _ = run(G.SHOTGUN, max(args.steps // 2, 1), 1, flags=G.PROFILE, **tuned)
    dt, stats = dt_plain, stats_plain
    path = "plain (per-iteration launches)"
    graph_info = None
    if not args.no_graph:
        log("timing Shotgun solves (captured epoch graphs)")
        dt_g, stats_g, _ = run(G.SHOTGUN, args.steps, args.warmup, flags=G.USE_GRAPH, **tuned)
        graph_info = {"solves_per_s": args.steps / dt_g,
                      "nnz_updates_per_s": sum(s["nnz_updates"] for s in stats_g) / dt_g}
        if dt_g < dt_plain:
            dt, stats, path = dt_g, stats_g, "graph (one captured HIP graph per epoch)"
    fused_info = None
    if not args.no_graph:
        # fused asynchronous Shotgun (Propose and Update in one launch; the
        # trajectory is not the Jacobi one, the optimum is the same)
        log("timing fused asynchronous Shotgun solves (captured epoch graphs)")
        dt_f, stats_f, _ = run(G.SHOTGUN, args.steps, args.warmup, flags=G.USE_GRAPH | G.FUSED,
                               **tuned)
        fused_info = {"solves_per_s": args.steps / dt_f,
                      "nnz_updates_per_s": sum(s["nnz_updates"] for s in stats_f) / dt_f,
                      "epochs_per_solve": stats_f[-1]["epochs"],
                      "objective": stats_f[-1]["objective"], "kkt_max": stats_f[-1]["kkt_max"]}
    prof_src = stats_prof
    nnz_upd = sum(s["nnz_updates"] for s in stats)
    coord_upd = sum(s["coord_updates"] for s in stats)
    value = nnz_upd / dt
    last = stats[-1]

    def kernel_roofline(name, what, ms, launches, nbytes, extra=None):
        achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        r = {"bound": "hbm", "kernel": f"{name} ({what})", "achieved": round(achieved, 3),
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
             "traffic": measured_traffic(name, schedule=sched_key),
             "avg_launch_us": round(ms * 1e3 / max(launches, 1), 3),
             "bytes_per_launch": round(nbytes / max(launches, 1), 1),
             "launches": launches, "total_ms": round(ms, 3)}
        if extra:
            r.update(extra)
        return r

    p_ms = sum(s["prof_kernel_ms"] for s in prof_src)
    u_ms = sum(s["prof_update_ms"] for s in prof_src)
    u_launch = sum(s["prof_update_launches"] for s in prof_src)
    scattered = sum(s["nnz_scattered"] for s in prof_src)
    coord_plain = sum(s["coord_updates"] for s in prof_src)
    # Update bytes counted over the columns whose increment was nonzero only
    # (the kernel skips the others): 24 B per scattered nonzero + 8 B per column
    u_bytes_nz = 24.0 * scattered + 8.0 * coord_plain
    rf_p = kernel_roofline(
        "k_propose", "Propose: gradient, step and proxy of every selected column; "
        "12 B per nonzero + 28 B per column", p_ms, sum(s["prof_launches"] for s in prof_src),
        sum(s["prof_bytes"] for s in prof_src))
    rf_u = kernel_roofline(
        "k_update", "Update: w_j += delta_j, z += delta_j X_j; 24 B per nonzero of every "
        "accepted column + 8 B per column", u_ms, u_launch,
        sum(s["prof_update_bytes"] for s in prof_src),
        {"achieved_nonzero_delta_only": round(u_bytes_nz / (u_ms * 1e-3) / 1e9, 3) if u_ms > 0 else 0.0,
         "bytes_per_launch_nonzero_delta_only": round(u_bytes_nz / max(u_launch, 1), 1)})
    dominant = rf_u if u_ms > p_ms else rf_p
    roofline = dict(dominant)
    out = {
        "metric": "nnz-updates/s of Shotgun solves to FP64 KKT 1e-6",
        "value": value,
        "unit": "nnz-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{P.name}: Zipf(1.1) ~50 nnz/row, lognormal row-normalised values, "
                        f"logistic, lambda=0.05*lambda_max, Shotgun |J|={args.select}",
            "n": P.n, "k": P.k, "nnz": P.nnz, "lambda": lam, "lambda_max": lam_max,
            "kkt_tol": args.tol, "path": path,
            "schedule": ({**sched, **tuned} if sched else "default (group 8, piece 256)"),
        },
        "plain_path": {"solves_per_s": args.steps / dt_plain,
                       "nnz_updates_per_s": sum(s["nnz_updates"] for s in stats_plain) / dt_plain},
        "graph_path": graph_info,
        "fused_async_path": fused_info,
        "solves_per_s": args.steps / dt,
        "coord_updates_per_s": coord_upd / dt,
        "epochs_per_solve": last["epochs"],
        "iters_per_solve": last["iters"],
        "objective": last["objective"],
        "kkt_max": last["kkt_max"],
        "duality_gap": last["gap"],
        "nnz_w": last["nnz_w"],
        # nonzeros the Update launches actually scattered (delta_j != 0), as a
        # fraction of the accepted nonzeros (profiled plain solves) and as a rate
        # on the headline path
        "nnz_scattered_fraction": scattered / max(sum(s["nnz_updates"] for s in prof_src), 1),
        "nnz_scattered_per_s": value * scattered / max(sum(s["nnz_updates"] for s in prof_src), 1),
        "z_drift_low_word_accumulation": max(s["z_drift"] for s in stats),
        "roofline": roofline,
        "kernels": {"k_propose": rf_p, "k_update": rf_u},
    }

    # the same solves with every atomic update of z TwoSum-compensated
    # (GENCD_EXACT_ACCUM) instead of the low-word accumulation renormalised
    # at each epoch end: throughput, and the drift of the FP32 pair from
    # X w measured at each FP64 check
    log("timing Shotgun solves with per-update compensated accumulation")
    dt_x, st_x, _ = run(G.SHOTGUN, args.steps, args.warmup, flags=G.EXACT_ACCUM, **tuned)
    out["exact_accum_path"] = {
        "solves_per_s": args.steps / dt_x,
        "nnz_updates_per_s": sum(s["nnz_updates"] for s in st_x) / dt_x,
        "z_drift": max(s["z_drift"] for s in st_x),
        "objective": st_x[-1]["objective"], "kkt_max": st_x[-1]["kkt_max"],
        "note": "plain launches; z drift = max_i |z_hi + z_lo - (Xw)_i| / rms(Xw) at the checks"}

    if not args.no_thread_greedy:
        kRuleSolves = 3  # after one untimed solve, on the captured-epoch path
        log("timing Thread-Greedy solves")
        dt2, st2, _ = run(G.THREAD_GREEDY, kRuleSolves, 1, flags=G.USE_GRAPH, block=64)
        out["thread_greedy"] = {
            "nnz_updates_per_s": kRuleSolves * st2[-1]["nnz_updates"] / dt2,
            "solves_per_s": kRuleSolves / dt2, "path": "graph",
            "epochs": st2[-1]["epochs"], "objective": st2[-1]["objective"],
            "kkt_max": st2[-1]["kkt_max"], "block": 64,
        }

        log("timing Top-Greedy solves")
        dt3, st3, _ = run(G.TOP_GREEDY, kRuleSolves, 1, flags=G.USE_GRAPH, block=256)
        out["top_greedy"] = {
            "nnz_updates_per_s": kRuleSolves * st3[-1]["nnz_updates"] / dt3,
            "solves_per_s": kRuleSolves / dt3, "path": "graph",
            "epochs": st3[-1]["epochs"], "objective": st3[-1]["objective"],
            "kkt_max": st3[-1]["kkt_max"], "accepted_per_iteration": 256,
        }

        log("timing Block Shotgun solves (64 preset blocks)")
        dt5, st5, _ = run(G.BLOCK_SHOTGUN, kRuleSolves, 1, flags=G.USE_GRAPH, block=64)
        out["block_shotgun"] = {
            "nnz_updates_per_s": kRuleSolves * st5[-1]["nnz_updates"] / dt5,
            "solves_per_s": kRuleSolves / dt5, "path": "graph",
            "epochs": st5[-1]["epochs"], "objective": st5[-1]["objective"],
            "kkt_max": st5[-1]["kkt_max"], "blocks": 64,
            "max_block_pstar": st5[-1]["select_size"], "max_block_rho": st5[-1]["rho"],
        }

        log("timing Shotgun solves with 500 improve-delta steps")
        dt4, st4, _ = run(G.SHOTGUN, 1, 0, improve=500)
        out["shotgun_improve500"] = {
            "nnz_updates_per_s": st4[-1]["nnz_updates"] / dt4,
            "solves_per_s": 1.0 / dt4,
            "epochs": st4[-1]["epochs"], "objective": st4[-1]["objective"],
            "kkt_max": st4[-1]["kkt_max"],
        }

    if not args.no_cpu_baseline:
        import oracle as O

        log("timing the FP64 oracle on the host")
        Xo = O.Matrix.of(P)
        yo = P.y.astype(np.float64)
        lam_o = 0.05 * O.lambda_max(Xo, yo, P.loss)
        t0 = time.perf_counter()
        r = O.solve(Xo, yo, P.loss, lam_o, O.SHOTGUN, select_size=args.select, seed=7,
                    tol=args.tol, max_epochs=100000)
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": r.nnz_updates / tc,
            "unit": "nnz-updates/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"one full Shotgun solve of the same workload to KKT {args.tol} "
                      f"({r.epochs} epochs, {tc:.1f} s) on 1 thread of {cpu_model()}",
            "objective": r.objective,
        }
        out["objective_rel_diff_vs_oracle"] = abs(last["objective"] - r.objective) / abs(r.objective)
        # the oracle's optimum to KKT 1e-10 (warm-started from its own solve),
        # against which every GPU result of this line is stated
        log("solving the oracle to KKT 1e-10 for the precision figures")
        ref = O.solve(Xo, yo, P.loss, float(lam), O.SHOTGUN, select_size=args.select, seed=7,
                      tol=1e-10, max_epochs=100000, w0=r.w)
        res_h = last_res[(G.SHOTGUN, G.USE_GRAPH)] if (G.SHOTGUN, G.USE_GRAPH) in last_res \
            else last_res[(G.SHOTGUN, G.PROFILE)]
        out["precision"] = precision_vs_oracle(O, Xo, yo, P.loss, float(lam), ref, res_h)

    print(json.dumps(out), flush=True)


def precision_vs_oracle(O, Xo, yo, loss, lam, ref, res):
    """Error of one GPU solve against the oracle's tight optimum: relative
    objective error, max_i |z_i - z*_i| / (|z*_i| + rms(z*)), and the KKT
    violation of the GPU's w evaluated independently by the oracle."""
    import numpy as np
    w = res.w.double().cpu().numpy()
    chk = O.check(Xo, yo, loss, lam, w)
    z = res.z.double().cpu().numpy() if res.z is not None else chk.z
    zs = ref.z
    scale = np.abs(zs) + np.sqrt(np.mean(zs ** 2)) + 1e-300
    return {"oracle_optimum_objective": ref.objective, "oracle_optimum_kkt": ref.kkt,
            "objective_rel_err": abs(chk.objective - ref.objective) / abs(ref.objective),
            "z_max_rel_err": float(np.max(np.abs(z - zs) / scale)),
            "kkt_max": chk.kkt, "gpu_reported_kkt_max": res.stats["kkt_max"]}


# ---------------------------------------------------------------------------
# Extra workloads (one JSON line each; not part of the default run)
# ---------------------------------------------------------------------------

def _timed(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def bench_coloring(args):
    """Lasso workload (n=2e5, k=1e6, Zipf(1.2), ~30 nnz/row): GPU colouring
    (bit-exact against the oracle) and Coloring solves to KKT 1e-6."""
    import numpy as np
    import torch

    import oracle as O
    from paper_1206_6409_amd import gencd as G
    from paper_1206_6409_amd import synth

    t = time.time()
    P = synth.c3_zipf_lasso(scale=args.scale)
    log(f"generated {P.name}: nnz={P.nnz} in {time.time() - t:.1f}s")
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device="cuda")
    G.color(X)  # warm-up
    t_col, (colors, nc) = _timed(lambda: G.color(X), reps=3)
    t0 = time.perf_counter()
    ocol, onc, _ = O.color(P.n, P.k, P.col_ptr, P.row_idx)
    t_ocol = time.perf_counter() - t0
    exact = bool(onc == nc and np.array_equal(colors.cpu().numpy(), ocol))
    sizes = np.bincount(colors.cpu().numpy()[np.diff(P.col_ptr) > 0], minlength=nc)
    lam = 0.1 * G.lambda_max(X, y, P.loss)
    params = dict(loss=P.loss, lam=lam, rule=G.COLORING, colors=colors, num_colors=nc, seed=3,
                  tol=args.tol, max_epochs=100000)
    G.solve(X, y, G.make_params(**params))
    t_plain, res = _timed(lambda: G.solve(X, y, G.make_params(**params)), reps=args.steps)
    t_graph, resg = _timed(lambda: G.solve(X, y, G.make_params(flags=G.USE_GRAPH, **params)),
                           reps=args.steps)
    best = min(t_plain, t_graph)
    st = (resg if t_graph <= t_plain else res).stats
    # balanced colouring: classes above the mean size split into parts
    t_bal, (bal, nbal) = _timed(lambda: G.balance_colors(X, colors, nc, 0), reps=3)
    bparams = dict(params, colors=bal, num_colors=nbal)
    G.solve(X, y, G.make_params(**bparams))
    t_bsolve, resb = _timed(lambda: G.solve(X, y, G.make_params(flags=G.USE_GRAPH, **bparams)),
                            reps=args.steps)
    bsizes = np.bincount(bal.cpu().numpy()[np.diff(P.col_ptr) > 0], minlength=nbal)
    Xo = O.Matrix.of(P)
    t0 = time.perf_counter()
    r = O.solve(Xo, P.y.astype(np.float64), P.loss, lam, O.COLORING, colors=ocol, seed=3,
                tol=args.tol, max_epochs=100000)
    t_or = time.perf_counter() - t0
    log("solving the oracle to KKT 1e-10 for the precision figures")
    ref = O.solve(Xo, P.y.astype(np.float64), P.loss, lam, O.COLORING, colors=ocol, seed=3,
                  tol=1e-10, max_epochs=100000, w0=r.w)
    prec = precision_vs_oracle(O, Xo, P.y.astype(np.float64), P.loss, lam, ref,
                               resg if t_graph <= t_plain else res)
    return {
        "metric": "nnz-updates/s of Coloring solves to FP64 KKT 1e-6; colouring time",
        "value": st["nnz_updates"] / best, "unit": "nnz-updates/s", "n_gpus": 1,
        "steps": args.steps, "ms_per_step": best * 1e3, "dtype": "f32", "data": "synthetic",
        "config": {"workload": P.name + ": Zipf(1.2) ~30 nnz/row, N(0,1), Lasso, lambda=0.1*lambda_max",
                   "n": P.n, "k": P.k, "nnz": P.nnz},
        "colouring": {"gpu_ms": t_col * 1e3, "oracle_cpu_ms": t_ocol * 1e3, "colors": int(nc),
                      "bit_exact": exact, "mean_class_size": float(sizes[sizes > 0].mean()),
                      "max_class_size": int(sizes.max())},
        "balanced": {"gpu_ms": t_bal * 1e3, "colors": int(nbal), "max_class_size": int(bsizes.max()),
                     "solve_ms": t_bsolve * 1e3, "epochs": resb.stats["epochs"],
                     "objective": resb.stats["objective"]},
        "solves_per_s": 1.0 / best, "plain_path_ms": t_plain * 1e3, "graph_path_ms": t_graph * 1e3,
        "epochs": st["epochs"], "iters": st["iters"], "objective": st["objective"],
        "kkt_max": st["kkt_max"],
        "objective_rel_diff_vs_oracle": abs(st["objective"] - r.objective) / abs(r.objective),
        "precision": prec,
        "z_drift_pair_update": st["z_drift"],
        "cpu_baseline": {"value": r.nnz_updates / t_or, "unit": "nnz-updates/s", "cores": 1,
                         "kind": "oracle", "sample": f"one full Coloring solve ({r.epochs} epochs, "
                                                     f"{t_or:.1f} s) on 1 thread of {cpu_model()}"},
    }


GOLDEN_PATH = os.path.join(ROOT, "tests", "golden", "c4_path_optima.txt")


def load_path_optima(lams):
    """Oracle optima of the 64-lambda path (tests/golden, written by an
    oracle-only script) as (objective, kkt, l1 norm) arrays, or None when
    absent or for another grid."""
    try:
        rows = [l.split() for l in open(GOLDEN_PATH) if l.strip() and not l.startswith("#")]
    except OSError:
        return None
    if len(rows) != len(lams):
        return None
    import numpy as np
    lam_g = np.array([float(r[1]) for r in rows])
    if np.max(np.abs(lam_g - lams) / lams) > 1e-12:
        return None
    return (np.array([float(r[2]) for r in rows]), np.array([float(r[3]) for r in rows]),
            np.array([float(r[5]) for r in rows]))


def bench_path(args):
    """64-lambda regularisation path (binary, n=5e4, k=2e5, density 0.05%),
    lambda geometric from lambda_max down to 1e-3 lambda_max: the batched
    solver (B slots sharing the selected sets, warm-started lambdas,
    adaptive FP64 checks; with and without the "improve delta_j" steps of
    Algorithm 3) against the plain path (one warm-started gencd_solve per
    lambda, with and without the steps; the speed-up is against its fastest
    form), at the metric's KKT 1e-6 and at KKT 1e-10, where every objective
    is compared with the oracle's optimum.  At the small lambdas of this path
    an absolute KKT 1e-6 exceeds lambda itself, and at KKT 1e-9 the
    objective is still up to ~8e-6 above the optimum there (the weights' l1
    norm reaches 4e4), so the tighter level is KKT 1e-10."""
    import numpy as np
    import torch

    import oracle as O
    from paper_1206_6409_amd import gencd as G
    from paper_1206_6409_amd import synth

    t = time.time()
    P = synth.c4_binary_path(scale=args.scale)
    log(f"generated {P.name}: nnz={P.nnz} in {time.time() - t:.1f}s")
    X = G.Matrix.of(P)
    y = torch.as_tensor(P.y, device="cuda")
    lm = G.lambda_max(X, y, P.loss)
    lams = synth.lambda_grid(lm, count=args.lambdas, ratio=1e-3)
    optima = load_path_optima(lams) if args.scale == 1.0 else None

    def prm(tol, flags=0, stagger=0, lam=0.0, improve=0):
        return G.make_params(P.loss, lam, rule=G.SHOTGUN, select_size=1024, seed=5, tol=tol,
                             max_epochs=60000, check_every=0, flags=flags, stagger=stagger,
                             improve=improve)

    def errors(objs, kkts, l1s):
        """Relative objective error against the oracle's optimum, and the
        convexity bound it must respect: for two points a, b of the same
        Eq. (1), |P(a) - P(b)| <= max(KKT(a), KKT(b)) (|a|_1 + |b|_1)."""
        if optima is None:
            return None
        obj_g, kkt_g, l1_g = optima
        e = np.abs(np.array(objs) - obj_g) / np.abs(obj_g)
        bound = np.maximum(np.array(kkts), kkt_g) * (np.array(l1s) + l1_g) / np.abs(obj_g)
        return {"max": float(e.max()), "median": float(np.median(e)),
                "lambdas_within_1e-6": int(np.sum(e <= 1e-6)),
                "lambdas_within_convexity_bound": int(np.sum(e <= np.maximum(bound, 1e-12))),
                "per_lambda": [float(x) for x in e],
                "convexity_bound_per_lambda": [float(x) for x in bound]}

    def plain(tol, improve):
        ws = G.workspace(X, prm(tol))
        w0, objs, kkts, l1s, epochs = None, [], [], [], 0
        for t, lam in enumerate(lams):
            if t % 8 == 0 or t >= 40:
                log(f"KKT {tol:g} plain path (improve {improve}): lambda {t} of {len(lams)}")
            r = G.solve(X, y, prm(tol, flags=G.USE_GRAPH, lam=float(lam), improve=improve), w0=w0,
                        ws=ws)
            assert r.stats["converged"], r.stats
            w0, epochs = r.w, epochs + r.stats["epochs"]
            objs.append(r.stats["objective"])
            kkts.append(r.stats["kkt_max"])
            l1s.append(float(r.w.double().abs().sum()))
        return objs, kkts, l1s, epochs

    out = {"metric": "solves/s of a 64-lambda path to FP64 KKT 1e-6, batched vs plain GPU path",
           "unit": "solves/s", "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": P.name + ": binary, logistic, 64 lambdas geometric to 1e-3 lambda_max",
                      "n": P.n, "k": P.k, "nnz": P.nnz, "select_size": 1024,
                      "check_every": "adaptive (a tenth of the epochs run, 1..64)"},
           "levels": {}}
    FE = G.FUSED | G.FUSED_EPOCH
    # (B, flags, stagger, improve-delta steps); the plain path's improve steps
    configs = {1e-6: [(16, 0, 0, 0), (16, G.FUSED, 0, 0), (16, FE, 0, 0), (32, 0, 0, 0),
                      (32, FE, 0, 0), (64, 0, 0, 0), (64, G.FUSED, 0, 0), (64, FE, 0, 0),
                      (64, FE, 20, 0), (16, FE, 0, 5), (16, FE, 0, 10), (16, FE, 0, 20),
                      (32, FE, 0, 10), (64, FE, 0, 10)],
               1e-10: [(16, FE, 0, 0), (16, FE, 0, 20), (16, FE, 0, 50), (16, FE, 0, 100),
                       (32, FE, 0, 50)]}
    plain_steps = {1e-6: (0, 10), 1e-10: (20,)}

    def leg_name(B, fl, stag, imp):
        return (f"B{B}" + ("_fused_epoch" if fl & G.FUSED_EPOCH else "_fused" if fl else "")
                + (f"_stagger{stag}" if stag else "") + (f"_improve{imp}" if imp else ""))

    cfg_of = {leg_name(*c): c for cs in configs.values() for c in cs}

    for tol in (args.tol,) if args.no_path_tight else (args.tol, 1e-10):
        lvl = {"batched": {}}
        best = None
        for B, fl, stag, imp in configs.get(tol, configs[1e-6]):
            name = leg_name(B, fl, stag, imp)
            if args.path_only and name != args.path_only:
                continue
            p_ = prm(tol, flags=G.USE_GRAPH | fl, stagger=stag, improve=imp)
            G.solve_path(X, y, p_, lams[:2], B=B)  # first-use costs out of the timing
            dt, res = _timed(lambda: G.solve_path(X, y, p_, lams, B=B))
            assert all(st["converged"] for st in res.stats)
            objs = [st["objective"] for st in res.stats]
            kkts = [st["kkt_max"] for st in res.stats]
            l1s = res.W.double().abs().sum(dim=1).tolist()
            lvl["batched"][name] = {
                "seconds": dt, "solves_per_s": len(lams) / dt,
                "max_epochs": max(st["epochs"] for st in res.stats),
                "nnz_updates_per_s": sum(st["nnz_updates"] for st in res.stats) / dt,
                "objective_rel_err_vs_oracle": errors(objs, kkts, l1s),
                "kkt_max": max(kkts)}
            log(f"KKT {tol:g} path {name}: {dt:.2f}s")
            if best is None or dt < lvl["batched"][best]["seconds"]:
                best = name
        lvl["best_batched"] = best
        if best is None:
            raise SystemExit(f"--path-only {args.path_only}: no such configuration")
        if not args.path_only:
            # the plain path (one warm-started gencd_solve per lambda) with the
            # same options; the speed-up is against its fastest form
            lvl["plain_paths"] = {}
            for imp in plain_steps.get(tol, (0,)):
                t_plain, (objs_p, kkts_p, l1s_p, ep_p) = _timed(lambda: plain(tol, imp))
                log(f"KKT {tol:g} plain path (improve {imp}): {t_plain:.2f}s")
                lvl["plain_paths"][f"improve{imp}"] = {
                    "seconds": t_plain, "solves_per_s": len(lams) / t_plain, "epochs_total": ep_p,
                    "objective_rel_err_vs_oracle": errors(objs_p, kkts_p, l1s_p),
                    "kkt_max": max(kkts_p)}
            pbest = min(lvl["plain_paths"], key=lambda k_: lvl["plain_paths"][k_]["seconds"])
            lvl["plain_path"] = dict(lvl["plain_paths"][pbest], form=pbest)
            lvl["speedup_vs_plain"] = lvl["plain_path"]["seconds"] / lvl["batched"][best]["seconds"]
        out["levels"][f"kkt_{tol:g}"] = lvl
    top = out["levels"][f"kkt_{args.tol:g}"]
    out["value"] = top["batched"][top["best_batched"]]["solves_per_s"]
    # roofline of the one-launch-per-epoch fused kernel: GENCD_PROFILE puts
    # HIP events around every k_path_fused launch on the call's stream (plain
    # launches); bytes per launch are the algorithmic count the library
    # reports (12 + 16 B per nonzero, 20 + 8 B per column at B slots)
    # and of its instance with the improve steps of the fastest configuration
    kern = {}
    top_cfg = cfg_of.get(top["best_batched"], (16, FE, 0, 0))
    profiled = [(16, 0), (64, 0)]
    if top_cfg[1] & G.FUSED_EPOCH and top_cfg[3] > 0:
        profiled.append((top_cfg[0], top_cfg[3]))
    for B, imp in profiled:
        p_ = prm(args.tol, flags=G.FUSED | G.FUSED_EPOCH | G.PROFILE, improve=imp)
        s0 = G.solve_path(X, y, p_, lams, B=B).stats[0]
        nl = max(s0["prof_launches"], 1)
        us = s0["prof_kernel_ms"] * 1e3 / nl
        bpl = s0["prof_bytes"] / nl
        kname = f"k_path_fused<{B}>" + (f" improve{imp}" if imp else "")
        kern[kname] = {
            "bound": "hbm",
            "kernel": f"k_path_fused<{B}> (the whole epoch in one launch: every slot's gradient, "
                      f"step and scatter; 12 + 16*{B} B per nonzero + 20 + 8*{B} B per column)"
                      + (f", up to {imp} improve-delta steps per slot and column (not counted; "
                         f"they make the launch arithmetic-bound, so the HBM fraction understates it)"
                         if imp else ""),
            "achieved": round(bpl / us / 1e3, 3), "peak": 8000.0, "unit": "GB/s",
            "frac": round(bpl / us / 1e3 / 8000.0, 6),
            "traffic": measured_traffic(kname, PATH_TRAFFIC_PROFILE, PATH_TRAFFIC_SOURCES),
            "avg_launch_us": round(us, 3), "bytes_per_launch": bpl, "launches": nl}
        log(f"{kname}: {us:.1f} us per epoch launch, {bpl / us / 1e3:.0f} GB/s")
    # the roofline names the kernel of the fastest configuration
    rname = f"k_path_fused<{top_cfg[0]}>" + (f" improve{top_cfg[3]}" if top_cfg[3] else "")
    out["roofline"] = kern.get(rname, kern["k_path_fused<16>"])
    out["kernels"] = kern
    out["oracle_optima"] = "tests/golden/c4_path_optima.txt (oracle, KKT 1e-10)" if optima is not None \
        else "absent: objectives not compared"
    if args.path_only:
        return out
    # oracle on the first lambdas (bounded sample), warm-started like the plain path
    Xo = O.Matrix.of(P)
    yo = P.y.astype(np.float64)
    t0 = time.perf_counter()
    w0, oupd, ocnt = None, 0, 0
    for lam in lams:
        r = O.solve(Xo, yo, P.loss, float(lam), O.SHOTGUN, select_size=1024, seed=5, tol=args.tol,
                    max_epochs=200000, w0=w0)
        w0, oupd, ocnt = r.w, oupd + r.nnz_updates, ocnt + 1
        if time.perf_counter() - t0 > 20.0:
            break
    t_or = time.perf_counter() - t0
    out["cpu_baseline"] = {"value": ocnt / t_or, "unit": "solves/s", "cores": 1, "kind": "oracle",
                           "nnz_updates_per_s": oupd / t_or,
                           "sample": f"the first {ocnt} lambdas of the path to KKT {args.tol:g}, "
                                     f"warm-started ({t_or:.1f} s) on 1 thread of {cpu_model()}"}
    return out


def bench_serve(args):
    """Serving: a Poisson stream of L1 solve requests, 50/50 Lasso and
    logistic, n ~ U{1k..50k}, k ~ U{1k..200k}, density U[0.1%, 2%], N(0, 1)
    values, lambda/lambda_max log-uniform [1e-3, 0.5], every request a
    distinct matrix generated on the device at its arrival.  The rate is 0.7x
    the saturated throughput of the server measured on a warm-up of
    --calibration requests submitted at once.  Reports p50/p99 latency
    (finish - arrival) and solves/s of the continuous-batching server; the
    plain path (one gencd_solve after another) on a prefix of the same
    stream, as a FIFO queue replayed with its measured solve times; and the
    error against the oracle's tight optimum on a stratified sample."""
    import numpy as np
    import torch

    import oracle as O
    from paper_1206_6409_amd import gencd as G
    from paper_1206_6409_amd import synth

    count, slots, tol = args.requests, args.slots, args.tol
    dev = torch.device("cuda", 0)
    stream = synth.c5_request_stream(count=count, rate=1.0)
    calib = synth.c5_request_stream(count=args.calibration, rate=1.0, seed=106, arrival_seed=1060)

    def make(r):
        X, y = G.generate_request(r.n, r.k, r.density, r.loss, r.seed)
        lam = r.lambda_ratio * G.lambda_max(X, y, r.loss)  # synchronises: X and y exist
        return X, y, lam

    def params(loss, lam):
        # |J| = P* = floor(k_live / (2 rho)) clamped to [1, k_live] (section 4.1);
        # adaptive FP64 check interval (a tenth of the epochs run, 1..64)
        return G.make_params(loss, lam, rule=G.SHOTGUN, select_size=0, seed=11, tol=tol,
                             max_epochs=100000, check_every=args.serve_check,
                             flags=G.FUSED if args.serve_fused else 0)

    # the largest request of the ranges fixes the per-slot arena share
    worst = G.Matrix(50000, 200000, torch.zeros(200001, dtype=torch.int64, device=dev),
                     torch.empty(0, dtype=torch.int32, device=dev),
                     torch.empty(0, dtype=torch.float32, device=dev))
    worst._s.nnz = int(50000 * 200000 * 0.02 * 1.01)
    per_slot = G.Server.request_bytes(worst, params(synth.LOGISTIC, 1.0))
    arena = G.Server.overhead_bytes(slots) + slots * per_slot
    log(f"serving: {slots} slots, arena {arena / 2**30:.1f} GiB")

    def run_stream(reqs, arrivals, keep=()):
        """Submit reqs[i] at arrivals[i] (seconds from the server's start) and
        collect every result; progress lines go to stderr."""
        srv = G.Server(arena_bytes=arena, max_slots=slots)
        t0 = time.perf_counter()  # the server's clock starts within microseconds of this
        live, results, kept = {}, {}, {}
        nxt, last_log = 0, t0
        saturated = None  # (seconds, results) when the last waiting request was admitted
        while len(results) < len(reqs):
            while nxt < len(reqs) and arrivals[nxt] <= time.perf_counter() - t0:
                r = reqs[nxt]
                X, y, lam = make(r)
                w = torch.empty(r.k, dtype=torch.float32, device=dev)
                z = torch.empty(r.n, dtype=torch.float32, device=dev)
                srv.submit(X, y, params(r.loss, lam), w, z, tag=nxt)
                live[nxt] = (X, y, lam, w, z)
                nxt += 1
            got = srv.poll(wait_for=0)
            if not got:
                time.sleep(0.0005)
            for g in got:
                i = g["user_tag"]
                X, y, lam, w, z = live.pop(i)
                g["latency_s"] = g["finish_s"] - arrivals[i]
                g["lambda"] = lam
                results[i] = g
                if i in keep:
                    kept[i] = (X, y, lam, w, z)
            if saturated is None and nxt == len(reqs) and srv.info()["waiting"] == 0:
                saturated = (time.perf_counter() - t0, len(results))
            if time.perf_counter() - last_log > 20.0:
                last_log = time.perf_counter()
                log(f"  {nxt} of {len(reqs)} submitted, {len(results)} done, "
                    f"{len(live)} in the server")
        info = srv.info()
        info["saturated_until"] = saturated
        srv.close()
        return [results[i] for i in range(len(reqs))], info, kept

    # saturated throughput on the calibration requests (all at time 0)
    if args.rate > 0:
        rate, sat, sat_makespan = args.rate, args.rate / 0.7, None
        log(f"rate {rate}/s given on the command line (no calibration run)")
    else:
        log(f"calibration: {len(calib)} requests submitted at once")
        res_c, info_c, _ = run_stream(calib, np.zeros(len(calib)))
        span_c = max(r["finish_s"] for r in res_c) - min(r["submit_s"] for r in res_c)
        sat_makespan = len(calib) / span_c
        # saturated = every slot busy and requests waiting: completions up to
        # the admission of the last waiting one (the tail after it is the
        # longest requests finishing alone)
        t_sat, n_sat = info_c["saturated_until"] or (span_c, len(calib))
        sat = n_sat / t_sat if n_sat > 0 else sat_makespan
        rate = 0.7 * sat
    gaps = np.random.default_rng(1050).exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    first, end = (0, count) if args.slice is None else (max(args.slice[0], 0), min(args.slice[1], count))
    if args.slice is not None:
        # a slice of the same stream: its own arrivals, shifted to start at 0
        stream = stream[first:end]
        arrivals = arrivals[first:end] - arrivals[first]
        count = len(stream)
        log(f"slice [{first}, {end}) of the stream")
    # stratified sample for the oracle: requests at nnz quantiles small enough
    # for the host (about 2 M nonzeros), both losses
    exp_nnz = np.array([r.n * r.k * r.density for r in stream])
    small = [i for i in np.argsort(exp_nnz) if exp_nnz[i] <= args.oracle_max_nnz]
    sample = sorted(set(small[int(q * (len(small) - 1))] for q in np.linspace(0, 1, args.oracle_sample)))
    log(f"stream: {count} requests at {rate:.2f}/s (0.7 x {sat:.2f} saturated)")
    t_main = time.perf_counter()
    res, info, kept = run_stream(stream, arrivals, keep=set(int(i) for i in sample))
    wall = time.perf_counter() - t_main
    # latency = finish - arrival: the client generates each request at its
    # arrival, so the generation time counts
    lat = np.array([r["latency_s"] for r in res])
    span = max(r["finish_s"] for r in res) - min(r["submit_s"] for r in res)
    statuses = {}
    for r in res:
        statuses[r["status"]] = statuses.get(r["status"], 0) + 1
    nnz_upd = sum(r["stats"]["nnz_updates"] for r in res)
    epochs = np.array([r["stats"]["epochs"] for r in res])
    # plain path: gencd_solve back to back on a prefix, queue replayed at the same arrivals
    nplain = min(args.plain_requests, count)
    service = []
    log(f"plain path: {nplain} requests one after another")
    for i in range(nplain):
        X, y, lam = make(stream[i])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        G.solve(X, y, params(stream[i].loss, lam))
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t1)
        del X, y
        if (i + 1) % 10 == 0:
            log(f"  plain {i + 1} of {nplain}: {sum(service):.1f} s so far")
    fin, t_free = [], 0.0
    for i in range(nplain):
        start = max(arrivals[i], t_free)
        t_free = start + service[i]
        fin.append(t_free - arrivals[i])
    fin = np.array(fin)
    # the server on the same requests, all submitted at once: its throughput
    # against the plain path's on identical work
    same = None
    if nplain:
        log(f"server on the plain path's {nplain} requests, submitted at once")
        res_s, _, _ = run_stream(stream[:nplain], np.zeros(nplain))
        span_s = max(r["finish_s"] for r in res_s) - min(r["submit_s"] for r in res_s)
        same = {"requests": nplain, "solves_per_s": nplain / span_s,
                "all_converged": all(r["status"] == 0 for r in res_s)}
    # error against the oracle's tight optimum, and the oracle's own speed
    prec, o_upd, o_time, o_solves = [], 0, 0.0, 0
    for i in sample:
        if i not in kept:
            continue
        X, y, lam, w, z = kept[i]
        r = stream[i]
        log(f"oracle on request {i}: n={r.n} k={r.k} nnz={X.nnz}")
        Xo = O.Matrix(X.n, X.k, X.col_ptr.cpu().numpy(), X.row_idx.cpu().numpy(),
                      X.val.cpu().numpy().astype(np.float64))
        yo = y.cpu().numpy().astype(np.float64)
        t1 = time.perf_counter()
        base = O.solve(Xo, yo, r.loss, lam, O.SHOTGUN, select_size=1024, seed=11, tol=tol,
                       max_epochs=100000)
        o_time += time.perf_counter() - t1
        o_upd += base.nnz_updates
        o_solves += 1
        ref = O.solve(Xo, yo, r.loss, lam, O.SHOTGUN, select_size=1024, seed=11, tol=1e-10,
                      max_epochs=20000, w0=base.w)
        chk = O.check(Xo, yo, r.loss, lam, w.double().cpu().numpy())
        zz = z.double().cpu().numpy()
        sc = np.abs(ref.z) + np.sqrt(np.mean(ref.z ** 2)) + 1e-300
        prec.append({"request": int(i), "n": r.n, "k": r.k, "nnz": X.nnz, "loss": r.loss,
                     "lambda_ratio": r.lambda_ratio,
                     "oracle_reference_kkt": ref.kkt,
                     "objective_rel_err": abs(chk.objective - ref.objective) / abs(ref.objective),
                     "z_max_rel_err": float(np.max(np.abs(zz - ref.z) / sc)), "kkt_max": chk.kkt})
    out = {
        "metric": "serving: solves/s and p50/p99 latency at 0.7x the saturated rate",
        "value": count / span, "unit": "solves/s", "n_gpus": 1, "dtype": "f32",
        "data": "synthetic, generated on the device per request",
        "config": {"workload": f"{count} Poisson requests, 50/50 Lasso/logistic, n U{{1k..50k}}, "
                               f"k U{{1k..200k}}, density U[0.1%,2%], N(0,1) values, "
                               f"lambda/lambda_max logU[1e-3,0.5], KKT {tol}, |J| = P*, "
                               + ("adaptive check interval" if args.serve_check == 0 else
                                  f"check_every {args.serve_check}")
                               + (", fused Propose+Update (GENCD_FUSED)" if args.serve_fused else ""),
                   "slots": slots, "rate_per_s": rate,
                   "mean_nnz": float(np.mean([r["stats"]["nnz_visits"] / max(r["stats"]["epochs"], 1)
                                              for r in res]))},
        "saturated_solves_per_s": sat, "calibration_requests": len(calib),
        "calibration_makespan_solves_per_s": sat_makespan,
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(lat.max()),
        "nnz_updates_per_s": nnz_upd / span, "wall_s": wall,
        "status_counts": {str(k): v for k, v in statuses.items()},
        "slice": [first, end],
        "latencies_s": [round(float(x), 6) for x in lat],
        "busy_span_s": span, "nnz_updates": nnz_upd,
        "epochs": {"p50": float(np.percentile(epochs, 50)), "p99": float(np.percentile(epochs, 99)),
                   "max": int(epochs.max())},
        "rounds": info["rounds"], "request_windows": info["slot_rounds"],
        "requests_per_round": info["slot_rounds"] / max(info["rounds"], 1),
        "rounds_with_several_requests": info["shared_rounds"],
        "plain_one_at_a_time": {"requests": nplain,
                                "solves_per_s": nplain / sum(service) if nplain else None,
                                "latency_p50_s": float(np.percentile(fin, 50)) if nplain else None,
                                "latency_p99_s": float(np.percentile(fin, 99)) if nplain else None,
                                "note": "FIFO replay of the same arrivals with measured gencd_solve times"},
        "server_saturated_on_plain_requests": same,
        "precision": {"sample": prec,
                      "objective_rel_err_max": max((p["objective_rel_err"] for p in prec), default=None),
                      "z_max_rel_err_max": max((p["z_max_rel_err"] for p in prec), default=None),
                      "kkt_max": max((p["kkt_max"] for p in prec), default=None)},
        "select_size_from_rho": {"min": int(min(r["stats"]["select_size"] for r in res)),
                                 "median": float(np.median([r["stats"]["select_size"] for r in res])),
                                 "max": int(max(r["stats"]["select_size"] for r in res))},
        "cpu_baseline": {"value": o_solves / o_time if o_time > 0 else None, "unit": "solves/s",
                         "cores": 1, "kind": "oracle",
                         "nnz_updates_per_s": o_upd / o_time if o_time > 0 else None,
                         "sample": f"{o_solves} requests of the stream at nnz quantiles up to {args.oracle_max_nnz:g} "
                                   f"(both losses), Shotgun |J|=1024 to KKT {tol}, {o_time:.1f} s "
                                   f"on 1 thread of {cpu_model()}"},
    }
    return out


def merge_serve(paths):
    """One serving line from the lines of slice runs of one stream (same rate):
    latency percentiles over every request, solves/s over the summed spans."""
    import numpy as np
    lines = [json.loads(open(p).read().strip().splitlines()[-1]) for p in paths]
    lat = np.concatenate([np.array(l["latencies_s"]) for l in lines])
    span = sum(l["busy_span_s"] for l in lines)
    out = dict(lines[0])
    out.pop("latencies_s", None)
    out["slices"] = [l["slice"] for l in lines]
    out["value"] = len(lat) / span
    out["latency_p50_s"] = float(np.percentile(lat, 50))
    out["latency_p99_s"] = float(np.percentile(lat, 99))
    out["latency_max_s"] = float(lat.max())
    out["nnz_updates_per_s"] = sum(l["nnz_updates"] for l in lines) / span
    out["wall_s"] = sum(l["wall_s"] for l in lines)
    sc = {}
    for l in lines:
        for k, v in l["status_counts"].items():
            sc[k] = sc.get(k, 0) + v
    out["status_counts"] = sc
    for key in ("rounds", "request_windows", "rounds_with_several_requests"):
        out[key] = sum(l[key] for l in lines)
    out["requests_per_round"] = out["request_windows"] / max(out["rounds"], 1)
    out["config"] = dict(out["config"])
    out["config"]["workload"] = out["config"]["workload"].replace(
        f"{lines[0]['slice'][1] - lines[0]['slice'][0]} Poisson", f"{len(lat)} Poisson")
    prec = [p for l in lines for p in l["precision"]["sample"]]
    out["precision"] = {"sample": prec,
                        "objective_rel_err_max": max((p["objective_rel_err"] for p in prec), default=None),
                        "z_max_rel_err_max": max((p["z_max_rel_err"] for p in prec), default=None),
                        "kkt_max": max((p["kkt_max"] for p in prec), default=None)}
    for key in ("plain_one_at_a_time", "server_saturated_on_plain_requests", "cpu_baseline"):
        for l in lines:  # the slice that ran the leg
            v = l.get(key)
            if v and (v.get("requests") or v.get("value")):
                out[key] = v
    out["note"] = ("one stream run as consecutive slices, each started empty; latencies and "
                   "rates combine every request of every slice")
    return out


def bench_sweep(args):
    """Propose over every live column (the Greedy rule's Propose, section
    2.3): the k_propose kernel at a work unit of the whole matrix instead of
    one |J| = 4096 window.  Runs on the logistic workload (X ~40 MB, held by
    the 256 MB last-level cache) and on its 8x scaled version (n = 8e5,
    k = 4e6, X ~320 MB, which does not fit), to show the kernel against the
    HBM roofline once launch and latency costs are amortised.  Windows this
    large read a refreshed residual vector (4 B per row gather); the bytes
    counted are 12 per nonzero and 28 per column."""
    import torch

    from paper_1206_6409_amd import gencd as G
    from paper_1206_6409_amd import synth

    out = {"metric": "Propose roofline over every live column (Greedy's proposal sweep)",
           "unit": "GB/s", "n_gpus": 1, "dtype": "f32", "data": "synthetic", "sweeps": {}}
    for scale in args.sweep_scales:
        t = time.time()
        P = synth.c2_zipf_logistic(scale=scale)
        log(f"generated {P.name}: nnz={P.nnz} in {time.time() - t:.1f}s")
        X = G.Matrix.of(P)
        y = torch.as_tensor(P.y, device="cuda")
        lam = 0.05 * G.lambda_max(X, y, P.loss)
        iters = args.sweep_iters

        def prm(flags, epochs):
            # one epoch of Greedy = one iteration over the whole live set;
            # one FP64 check, after the last epoch
            return G.make_params(P.loss, lam, rule=G.GREEDY, select_size=1, seed=7, tol=0.0,
                                 max_epochs=epochs, check_every=epochs, flags=flags,
                                 group=args.sweep_group, piece=args.sweep_piece)

        ws = G.workspace(X, prm(G.PROFILE, iters))
        G.solve(X, y, prm(0, 2), ws=ws)  # warm-up
        torch.cuda.synchronize()
        log(f"timing {iters} Greedy iterations (Propose over all live columns) on {P.name}")
        t0 = time.perf_counter()
        res = G.solve(X, y, prm(G.PROFILE, iters), ws=ws)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = res.stats
        ms, nl, nb = st["prof_kernel_ms"], st["prof_launches"], st["prof_bytes"]
        achieved = nb / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        out["sweeps"][P.name] = {
            "n": P.n, "k": P.k, "nnz": P.nnz, "k_live": st["select_size"],
            "matrix_bytes": 8 * P.nnz + 8 * (P.k + 1),
            "iterations": st["iters"], "wall_s": wall,
            "roofline": {"bound": "hbm", "kernel": "k_propose", "achieved": round(achieved, 3),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 6),
                         "avg_launch_us": round(ms * 1e3 / max(nl, 1), 3),
                         "bytes_per_launch": round(nb / max(nl, 1), 1), "launches": nl},
        }
        del X, y, ws, res
        torch.cuda.empty_cache()
    big = out["sweeps"][max(out["sweeps"], key=lambda k: out["sweeps"][k]["nnz"])]
    out["value"] = big["roofline"]["achieved"]
    out["config"] = {"workload": "Greedy Propose sweeps over the Zipf(1.1) logistic matrix at "
                                 f"scales {list(args.sweep_scales)}"}
    return out


WORKLOADS = {"coloring": bench_coloring, "path": bench_path, "serve": bench_serve,
             "sweep": bench_sweep}


if __name__ == "__main__":
    main()
