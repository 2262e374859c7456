"""Benchmark of the HOT hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input: every
pair of the batch is solved with Algorithm 2 (slab passes, structured solve,
KKT checks, restarts) to the relative KKT tolerance, then its transport plan
is recovered (Algorithm 1 + marginal repair) when --plan is on.  Inputs are
resident in HBM before the timed region starts.

Workloads (named by what they are):
  batched   256 pairs, side n uniform in {32,48,64,96,128}, half 1-5 Gaussian
            blob mixtures and half U(0,1) noise, FP32 streams, rel KKT 1e-4
            (the default; the headline "FP32 batched" figure)
  pair128   one 128 x 128 pair (5 blobs), FP32 streams, rel KKT 1e-4
  pair128nu the same pair on non-uniform bins (Gamma-spaced grid lines)
  pair64    one 64 x 64 pair (5 blobs)
  pair128noise  one 128 x 128 pair of U(0,1) noise
  pair512   one 512 x 512 pair (1-8 blobs + Cauchy blob), FP32, rel KKT 1e-4
  small     one 32 x 32 pair (3 blobs), FP64, rel KKT 1e-6
  serving   Poisson arrivals (200/s for --duration s), side in {64,96,128,192,256},
            1-5 blob mixtures, tolerance 1e-4 (70%, FP32 streams) or 1e-6 (30%,
            FP64), continuous batching; reports solves/s and p50/p99 latency

Prints one JSON line.
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

METRIC = "OT solves/sec to 1e-4 KKT (FP32 batched vs FP64 plain); HBM GB/s; p99 lat"
PEAK_HBM_GBS = 8000.0
TUNE_CACHE = os.path.join(ROOT, "paper_2408_00598_amd", "tuned", "gfx950.jsonl")


def cached_choice(path, fp32, total, npairs):
    """Last autotuner cache line for this precision, size class and pair-count
    class (the library keys its table by floor(log2) of the flow elements and
    of the pair count)."""
    if not path or not os.path.exists(path):
        return None
    cls, pcls = int(total).bit_length() - 1, int(npairs).bit_length() - 1
    found = None
    for line in open(path):
        try:
            e = json.loads(line)
        except ValueError:
            continue
        if (e.get("fp32"), e.get("size_class"), e.get("pairs_class")) == (fp32, cls, pcls):
            found = e
    return found


def launch_key(tuned):
    if not tuned:
        return "builtin"
    return "item_elems={},unroll={},vec_per_lane={}".format(
        tuned["item_elems"], tuned["unroll"], tuned["vec_per_lane"])


def make_workload(name, pairs):
    """(pairs, tol, precision, description without precision and tolerance)."""
    from paper_2408_00598_amd import hot, workloads
    if name == "batched":
        return (workloads.batch_pairs(pairs), 1e-4, hot.HOT_FP32_STREAM,
                f"batched {pairs} pairs, n~U{{32,48,64,96,128}}, 50% 1-5 Gaussian blobs / 50% "
                "U(0,1) noise")
    if name == "pair128":
        return ([workloads.pair_medium("blobs")], 1e-4, hot.HOT_FP32_STREAM,
                "one 128x128 pair, 5 Gaussian blobs + floor 1e-3")
    if name == "pair64":
        return ([workloads.pair_medium("blobs", n=64)], 1e-4, hot.HOT_FP32_STREAM,
                "one 64x64 pair, 5 Gaussian blobs + floor 1e-3")
    if name == "pair128nu":
        return ([workloads.pair_medium("blobs")], 1e-4, hot.HOT_FP32_STREAM,
                "one 128x128 pair, 5 Gaussian blobs + floor 1e-3, non-uniform bins "
                "(Gamma(0.7) line gaps)")
    if name == "pair128noise":
        return ([workloads.pair_medium("noise")], 1e-4, hot.HOT_FP32_STREAM,
                "one 128x128 pair, U(0,1) noise")
    if name == "pair512":
        return ([workloads.pair_large()], 1e-4, hot.HOT_FP32_STREAM,
                "one 512x512 pair, 1-8 Gaussian blobs + Cauchy blob, floor 1e-6")
    if name == "small":
        return ([workloads.pair_small()], 1e-6, hot.HOT_FP64,
                "one 32x32 pair, 3 Gaussian blobs + floor 1e-3")
    raise SystemExit(f"unknown workload {name}")


def describe(base, prec, tol, sigma_update):
    from paper_2408_00598_amd import hot
    p = "FP32 streams + FP64 reductions" if prec == hot.HOT_FP32_STREAM else "FP64"
    t = ("%.0e" % tol).replace("e-0", "e-").replace("e+0", "e") if tol > 0 else str(tol)
    return f"{base}, {p}, rel KKT {t}" + (", sigma re-balanced at restarts"
                                          if sigma_update else "")


def run_serving(args):
    """Replay a Poisson trace against the continuous-batching server."""
    import threading
    import torch
    from paper_2408_00598_amd import hot, workloads
    trace = workloads.serving_trace(rate=args.rate, duration=args.duration)
    dev = torch.device("cuda:0")
    # a pool of distinct pairs per side, resident in HBM before the clock starts
    pool = {}
    for n in workloads.SERVE_SIDES:
        pool[n] = []
        for q in range(args.pool):
            a, b = workloads.serving_pair(n, workloads.seed_for(4, 1000 * n + q))
            pool[n].append((torch.tensor(a, device=dev), torch.tensor(b, device=dev)))
    torch.cuda.synchronize()
    ctx = hot.Context(0)
    flags = hot.HOT_FLAG_RESTART | (hot.HOT_FLAG_SIGMA_UPDATE if args.sigma_update else 0)
    # warm the per-shape workspaces (or the shared groups) and graphs, then
    # replay the trace on the same server
    srv = hot.Server(ctx, max_slots=args.slots, shared=args.shared)
    for n in workloads.SERVE_SIDES:
        for prec, tol in ((hot.HOT_FP32_STREAM, 1e-4), (hot.HOT_FP64, 1e-6)):
            # (a few quanta only: this builds the workspaces and graphs)
            srv.submit(*pool[n][0], -1, tol=tol, prec=prec, max_iter=100, flags=flags)
    srv.drain(600.0)
    srv.poll(1024)
    results = []
    t0 = time.perf_counter()

    def feeder():
        for q, (t, n, tol, seed) in enumerate(trace):
            now = time.perf_counter() - t0
            if t > now:
                time.sleep(t - now)
            a, b = pool[n][seed % args.pool]
            if tol >= 1e-4:
                srv.submit(a, b, q, tol=tol, prec=hot.HOT_FP32_STREAM, max_iter=1000000,
                           flags=flags)
            elif args.fp32_first:  # FP32 streams until the KKT stalls, then FP64
                srv.submit(a, b, q, tol=tol, prec=hot.HOT_FP32_STREAM, max_iter=1000000,
                           flags=flags | hot.HOT_FLAG_ESCALATE)
            else:
                srv.submit(a, b, q, tol=tol, prec=hot.HOT_FP64, max_iter=1000000, flags=flags)

    th = threading.Thread(target=feeder)
    th.start()
    last = 0.0
    deadline = None
    while True:
        results += srv.poll(4096)
        now = time.perf_counter() - t0
        st = srv.stats()
        if now - last >= 1.0:
            last = now
            print(f"[serving] t={now:6.1f}s submitted={int(st['submitted'])} "
                  f"completed={int(st['completed'])} queued={int(st['queued'])} "
                  f"resident={int(st['resident'])}", file=sys.stderr, flush=True)
        if not th.is_alive():
            if deadline is None:
                deadline = now + args.drain
            if st["completed"] >= st["submitted"] or now >= deadline:
                break
        time.sleep(0.05)
    th.join()
    elapsed = time.perf_counter() - t0
    results += srv.poll(1 << 20)
    st = srv.stats()
    srv.close()  # drops requests still queued, stops the resident ones
    lat = np.array([r["latency"] for r in results])
    iters = np.array([r["iters"] for r in results])
    out = {
        "metric": METRIC, "value": len(results) / elapsed, "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": elapsed * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "stream_dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson {args.rate:g} req/s for {args.duration:g} s, "
                               "n~U{64,96,128,192,256}, 1-5 Gaussian blobs, tol 1e-4 (70%, FP32 "
                               "streams) / 1e-6 (30%, "
                               + ("FP32 streams widened to FP64 on a stall" if args.fp32_first
                                  else "FP64") + "), continuous batching"
                               + (", sigma re-balanced at restarts" if args.sigma_update else "")
                               + (", shared launches per class" if args.shared else ""),
                   "requests": len(trace), "slots": args.slots},
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "offered_rate": args.rate, "completed": len(results),
        "dropped_in_queue": int(st["queued"]), "stopped_resident": int(st["resident"]),
        "drain_cap_s": args.drain,
        "converged": int(sum(r["status"] == 0 for r in results)),
        "max_resident": st["max_resident"], "iters_mean": float(iters.mean()),
        "escalated": int(sum(r["escalated_at"] > 0 for r in results)),
        "max_shared": st["max_shared"],
    }
    tight = [r for r in results if trace[r["tag"]][2] < 1e-4]
    if tight:
        lt = np.array([r["latency"] for r in tight])
        out["tight_tol"] = {"count": len(tight), "latency_p50_s": float(np.percentile(lt, 50)),
                            "latency_p99_s": float(np.percentile(lt, 99)),
                            "converged": int(sum(r["status"] == 0 for r in tight))}
    print(json.dumps(out), flush=True)


# the slab kernels' source and the headers whose types and helpers they use
SLAB_SOURCES = ("hot_slab.hip", "hot_internal.h", "hot_device.h")


def slab_source_sha256(root=None):
    """One SHA-256 over the slab kernels' source files, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for f in SLAB_SOURCES:
        h.update(f.encode() + b"\0")
        h.update(open(os.path.join(root or ROOT, "paper_2408_00598_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, launch):
    """HBM traffic per slab-pass launch from the committed rocprofv3 counter
    summary of this workload, if it was taken on the current kernel sources
    and launch shape."""
    name = {"batched": "slab_pass_batched256_fp32_traffic.md",
            "pair512": "slab_pass_pair512_fp32_traffic.md"}.get(workload)
    if not name:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    sha = slab_source_sha256()
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", "`")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != sha or vals.get("launch_config") != launch:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"]) / 1e9
    except (KeyError, ValueError):
        return None


def cpu_baseline(pairs, iters, tol, budget_s=20.0, threads=False):
    """Oracle (FP64, single thread; threads: its OpenMP build, the same source
    on the host's cores) seconds per iteration measured per grid side on the
    first pair of that side, times the iterations each pair takes (iters),
    summed over the batch."""
    from oracle import oracle as O
    sides = sorted({a.shape for a, _ in pairs})
    per_side = {}
    share = budget_s / max(1, len(sides))
    for shp in sides:
        a, b = next((a, b) for a, b in pairs if a.shape == shp)
        k, t = 1, 0.0
        while True:
            t0 = time.perf_counter()
            O.hot(a, b, fixed_iters=k, restart=False, threads=threads)
            t = time.perf_counter() - t0
            if t >= share / 4 or k >= 4096:
                break
            k *= 4
        per_side[shp] = t / (k + 1)
    total = sum(per_side[a.shape] * max(1, k) for (a, _), k in zip(pairs, iters))
    sample = ("oracle s/iteration timed on one pair per grid side ("
              + ", ".join(f"{s[0]}x{s[1]}: {per_side[s]*1e3:.2f} ms/it" for s in sides)
              + ") x the iterations each pair took in the FP64 GPU solve (the oracle's "
              "decisions), summed over the batch")
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count()) if threads else 1
    return {"value": len(pairs) / total, "unit": "solves/s", "cores": cores,
            "kind": "oracle, OpenMP build of the same source" if threads else "oracle",
            "sample": sample, "estimated_seconds": total}


def solution_quality(ctx, dpairs, results, kw, ref_tol):
    """gap and feaserr of Sec. 4.1 for the timed solves: the objective gap
    |<c,x> - <c,x_ref>| / (|<c,x_ref>| + 1) against FP64 reference solves of
    the same pairs to rel KKT ref_tol (sigma re-balanced at restarts, which
    reaches tight tolerances in far fewer iterations), taken outside the
    timed region."""
    from paper_2408_00598_amd import hot
    import torch
    t0 = time.perf_counter()
    kref = dict(kw, tol=ref_tol, prec=hot.HOT_FP64, max_iter=2000000,
                flags=hot.HOT_FLAG_RESTART | hot.HOT_FLAG_SIGMA_UPDATE)
    kref.pop("coord_row", None)
    kref.pop("coord_col", None)
    if "coord_row" in kw:  # non-uniform bins: per-pair positions
        refs = [ctx.solve(a, b, coord_row=kw["coord_row"], coord_col=kw["coord_col"],
                          **kref)[0] for a, b in dpairs]
    elif len(dpairs) == 1:
        refs = [ctx.solve(*dpairs[0], **kref)[0]]
    else:
        refs = ctx.batch_solve(dpairs, **kref)
    torch.cuda.synchronize()
    gaps = np.array([abs(r["primal_obj"] - q["primal_obj"]) / (abs(q["primal_obj"]) + 1.0)
                     for r, q in zip(results, refs)])
    return {"gap_mean": float(gaps.mean()), "gap_max": float(gaps.max()),
            "feaserr_mean": float(np.mean([r["feaserr"] for r in results])),
            "gap_reference": f"FP64 hot solves of the same pairs to rel KKT {ref_tol:g}, sigma "
                             "re-balanced at restarts (Sec. 4.1 gap; not timed)",
            "reference_converged": int(sum(q["status"] == 0 for q in refs)),
            "reference_kkt_max": float(max(q["kkt"] for q in refs)),
            "reference_seconds": time.perf_counter() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched")
    ap.add_argument("--pairs", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the built-in launch-shape rule (no cache, no tuning)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="JSON-lines autotuner cache; a matching entry is loaded instead of "
                         "tuning live")
    ap.add_argument("--retune", action="store_true",
                    help="tune live before the warmup and append the choice to --tune-cache")
    ap.add_argument("--no-fp64-plain", action="store_true")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the reference solves behind gap_mean / gap_max")
    ap.add_argument("--ref-tol", type=float, default=1e-8,
                    help="relative KKT tolerance of the FP64 reference solves for the gap")
    ap.add_argument("--plan", action="store_true", help="recover plans inside each step")
    ap.add_argument("--duration", type=float, default=10.0, help="serving trace length (s)")
    ap.add_argument("--rate", type=float, default=200.0, help="serving arrival rate (1/s)")
    ap.add_argument("--slots", type=int, default=16, help="serving resident problems")
    ap.add_argument("--drain", type=float, default=20.0,
                    help="serving: seconds to keep draining after the last arrival")
    ap.add_argument("--pool", type=int, default=8, help="serving distinct pairs per side")
    ap.add_argument("--sigma-update", action="store_true",
                    help="solves re-balance sigma at restarts (HOT_FLAG_SIGMA_UPDATE)")
    ap.add_argument("--prec", choices=("fp32", "fp64"), default=None,
                    help="override the workload's precision (fp32: FP32 streams + FP64 "
                         "reductions; fp64: FP64 throughout)")
    ap.add_argument("--tol", type=float, default=None,
                    help="override the workload's relative KKT tolerance")
    ap.add_argument("--admm", action="store_true",
                    help="the generalized ADMM baseline (rho 1.7) instead of HOT")
    ap.add_argument("--escalate", action="store_true",
                    help="FP32 streams widened to FP64 when the KKT stalls (single pairs)")
    ap.add_argument("--shared", action="store_true",
                    help="serving: problems of one precision and side class share launches")
    ap.add_argument("--fp32-first", action="store_true",
                    help="serving: 1e-6 requests start on FP32 streams and widen to FP64 "
                         "on a stall")
    ap.add_argument("--abs-kkt", action="store_true",
                    help="stop on the absolute KKT residual ||R(w_bar)|| instead of the relative one")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (torch copy_) 5 times, for scaling "
                         "hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    if args.workload == "serving":
        run_serving(args)
        return

    import torch
    from paper_2408_00598_amd import hot

    pairs, tol, prec, base = make_workload(args.workload, args.pairs)
    default_run = (args.prec is None and args.tol is None and not args.sigma_update
                   and not args.admm and not args.abs_kkt and not args.escalate)
    if args.prec is not None:
        prec = hot.HOT_FP32_STREAM if args.prec == "fp32" else hot.HOT_FP64
    if args.tol is not None:
        tol = args.tol
    desc = describe(base, prec, tol, args.sigma_update)
    dev = torch.device("cuda:0")
    dpairs = [(torch.tensor(a, device=dev), torch.tensor(b, device=dev)) for a, b in pairs]
    torch.cuda.synchronize()
    ctx = hot.Context(0)
    flags = hot.HOT_FLAG_RESTART | (hot.HOT_FLAG_SIGMA_UPDATE if args.sigma_update else 0)
    if args.admm:
        flags = hot.HOT_FLAG_ADMM  # (relax <= 0 selects rho = 1.7)
    if args.abs_kkt:
        flags |= hot.HOT_FLAG_ABS_KKT
        desc = desc.replace("rel KKT", "abs KKT")
    if args.escalate:
        flags |= hot.HOT_FLAG_ESCALATE
        desc += ", widened to FP64 on a stall"
    if args.admm:
        desc += ", generalized ADMM (rho 1.7)"
    kw = dict(tol=tol, max_iter=1000000, prec=prec, flags=flags)
    if args.workload == "pair128nu":  # grid-line positions of the non-uniform bins
        from paper_2408_00598_amd import workloads
        rng = np.random.default_rng(workloads.seed_for(1, 900))
        m, n = pairs[0][0].shape
        kw["coord_row"] = torch.tensor(workloads.grid_lines(m, rng), device=dev)
        kw["coord_col"] = torch.tensor(workloads.grid_lines(n, rng), device=dev)

    plan_stats = []

    def step():
        if len(dpairs) == 1:
            res, sol = ctx.solve(*dpairs[0], keep=args.plan, **kw)
            out = [res]
            if args.plan:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                src, _, _, err = sol.recover_plan()
                torch.cuda.synchronize()
                plan_stats.append((time.perf_counter() - t1, int(src.numel()), err))
                sol.free()
            return out
        return ctx.batch_solve(dpairs, **kw)

    tuned = None
    if not args.no_autotune:
        fp32 = int(prec == hot.HOT_FP32_STREAM)
        total = sum(a.shape[0] ** 2 * a.shape[1] + a.shape[0] * a.shape[1] ** 2 for a, _ in pairs)
        hit = None if args.retune else cached_choice(args.tune_cache, fp32, total, len(pairs))
        if hit is not None and ctx.autotune_load(args.tune_cache):
            tuned = {k: hit.get(k) for k in ("item_elems", "unroll", "vec_per_lane",
                                             "us_per_iter", "default_us_per_iter")}
            tuned["source"] = "cache"
        else:
            tuned = ctx.autotune(dpairs, iters=30, prec=prec,
                                 cache_path=args.tune_cache if args.retune else None)
            tuned["source"] = "live"
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    value = len(dpairs) * args.steps / elapsed

    # roofline of the slab pass: same workload once more with event timing
    ctx.set_profiling(True)
    results_prof = step()
    prof = ctx.profile()
    ctx.set_profiling(False)
    achieved = prof["slab_bytes"] / prof["slab_seconds"] / 1e9 if prof["slab_seconds"] else 0.0
    # (the committed counter summaries cover the workloads' own precision and tolerance)
    traffic = measured_traffic(args.workload, launch_key(tuned)) if default_run else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS,
                "traffic": traffic,  # GB per launch (rocprofv3 FETCH/WRITE, copy-calibrated)
                "kernel": "k_slab_pass",
                "launches": prof["slab_launches"],
                "avg_launch_us": prof["slab_seconds"] / max(1, prof["slab_launches"]) * 1e6,
                "bytes_per_launch": prof["slab_bytes"] / max(1, prof["slab_launches"])}

    iters = [r["iters"] for r in results]
    quality = None
    if not args.no_quality:
        quality = solution_quality(ctx, dpairs, results, kw, args.ref_tol)
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "stream_dtype": "f32" if prec == hot.HOT_FP32_STREAM else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "pairs": len(dpairs), "tol": tol},
        "autotune": tuned,
        "launch_config": launch_key(tuned),
        "roofline": roofline,
        "solve_stats": {"iters_mean": float(np.mean(iters)), "iters_max": int(np.max(iters)),
                        "kkt_max": float(max(r["kkt"] for r in results)),
                        "kkt_abs_max": float(max(r["kkt_abs"] for r in results)),
                        "restarts_mean": float(np.mean([r["restarts"] for r in results])),
                        "feaserr_max": float(max(r["feaserr"] for r in results)),
                        "escalated": int(sum(r["escalated_at"] > 0 for r in results)),
                        "converged": int(sum(r["status"] == 0 for r in results))},
    }
    if quality is not None:
        out["solve_stats"].update(quality)
    if plan_stats:
        secs = [p[0] for p in plan_stats]
        out["plan"] = {"seconds_mean": float(np.mean(secs)), "seconds_min": float(np.min(secs)),
                       "nnz": plan_stats[-1][1], "marginal_l1_raw": plan_stats[-1][2][:2],
                       "marginal_l1_repaired": plan_stats[-1][2][2:],
                       "note": "Algorithm 1 + repair on the solved pair, inside each step"}
    fp64_iters = None
    if not args.no_fp64_plain and len(dpairs) > 1:
        # the same batch in FP64 throughout, batched (splits the headline gain
        # into its batching and precision parts), one warm-up and two timed runs
        kw64 = dict(kw, prec=hot.HOT_FP64)
        ctx.batch_solve(dpairs, **kw64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(2):
            r64 = ctx.batch_solve(dpairs, **kw64)
        torch.cuda.synchronize()
        t64 = (time.perf_counter() - t1) / 2
        fp64_iters = [r["iters"] for r in r64]
        out["batched_fp64"] = {"value": len(dpairs) / t64, "unit": "solves/s",
                               "ms_per_step": t64 * 1e3, "iters_mean": float(np.mean(fp64_iters)),
                               "converged": int(sum(r["status"] == 0 for r in r64))}
        # plain per-pair FP64 hot_solve on the same GPU, every pair of the
        # batch, after one warm-up solve per grid side
        for shp in sorted({tuple(a.shape) for a, _ in dpairs}):
            a, b = next((a, b) for a, b in dpairs if tuple(a.shape) == shp)
            ctx.solve(a, b, tol=tol, max_iter=1000000, prec=hot.HOT_FP64, flags=flags)
        torch.cuda.synchronize()
        ts = []
        for a, b in dpairs:
            t1 = time.perf_counter()
            ctx.solve(a, b, tol=tol, max_iter=1000000, prec=hot.HOT_FP64, flags=flags)
            ts.append(time.perf_counter() - t1)
        ts = np.array(ts)
        out["fp64_plain"] = {"value": len(dpairs) / ts.sum(), "unit": "solves/s",
                             "sample": f"hot_solve FP64, every one of the {len(dpairs)} pairs "
                                       "solved one after another (one warm-up solve per side "
                                       "first)",
                             "ms_per_pair_mean": float(ts.mean() * 1e3),
                             "ms_per_pair_p10_p50_p90": [float(np.percentile(ts, q) * 1e3)
                                                         for q in (10, 50, 90)]}
    if args.copy_calibration:
        n = 1 << 28  # 2^28 float32 = 1 GiB
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 5,
                                   "GB/s": 2 * 4 * n * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9}
    if not args.no_cpu_baseline:
        # the oracle is FP64: price it with the FP64 iteration counts when the
        # batch was also solved in FP64 (the oracle takes the same decisions)
        its = fp64_iters if fp64_iters is not None else iters
        out["cpu_baseline"] = cpu_baseline(pairs, its, tol)
        out["cpu_baseline_multicore"] = cpu_baseline(pairs, its, tol, threads=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
