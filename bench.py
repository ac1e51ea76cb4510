#!/usr/bin/env python3
"""Benchmark of the PRGD hot path on one MI355X.

Headline workload: order 14, n = 4 per mode, TT ranks min(8, 4^k, 4^{14-k})
(an MPS-shaped tensor), Gaussian cores N(0, 1/r_k), |Omega| = 2,000,000
distinct entries drawn uniformly, noiseless, float64.  Every iteration of a
solve from its start to relative error 1e-6 against the ground truth is timed.

A step is one full PRGD iteration on the device: sampled pass (evaluation,
residual, slice sums, gradient scatter), metric-weighted Grams, tangent
components, TT-SVD retraction, stopping-test reductions.  The observation set
and cores are resident in HBM before the timed region.  The iteration count to
tolerance l* comes from a first run with the truth cores; the timed run then
performs exactly l* iterations (or --steps) without any truth tracking.

Also measured: the same workload with the float32 sampled pass (mixed); the
n = 400 order-3 noisy workload, the 256 x 256 x 128 smooth-core workload and the
order-4 noiseless workload, each in both precisions; the sketched spectral
initialisation; the request server on a stream of independent problems; and the
float64 reference implementation on the host cores.

Prints one JSON line.  --gpus above 1 is not supported (one-GPU build).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
K1_STRIDE = 4   # the main sampled kernel of every 4th timed iteration is bracketed by events
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "|Ω|·iterations/s, time to 1e-6 rel. error; served solves/s + p99 latency"
HEADLINE = "c4"
# MI355X peaks (published): HBM 8 TB/s; FP64 vector and FP64 MFMA 78.6 TFLOP/s.
# Non-packed FP32 vector issue has the same rate as FP64 (packed FP32 is disabled
# in this build): 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s.
PEAK_ALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# How each workload is solved.  start: "spectral" = the device's sketched
# spectral initialisation of P_Omega(y)/p, "perturbed" = truth cores with 10%
# RMS noise per core (the sketched initialisation does not reach the basin of
# convergence on the order-14 and smooth-core workloads).  rule/tol: the
# stopping rule that defines "to tolerance"; the noisy workload floors near
# 3e-4 relative error, so its clock is relative change <= 1e-6.  The smooth-core
# cube is ill-conditioned: the theory step diverges on it for every constant
# tried (0.4 .. 1.001), the adaptive step converges.
LEGS = {
    "c4": dict(start="perturbed", rule="error", tol=1e-6, policy="theory", c=1.001, max_iter=500,
               desc="order-14 TT completion, n=4, TT ranks min(8,4^k,4^(14-k)), |Omega|=2,000,000 "
                    "(0.745%), noiseless, int32 indices"),
    "c2": dict(start="spectral", rule="change", tol=1e-6, policy="theory", c=0.9, max_iter=500,
               desc="order-3 TT completion, n=400, TT ranks (1,10,10,1), |Omega|=640,000 (1%), "
                    "noise 1e-3 RMS, int32 indices"),
    "c3": dict(start="perturbed", rule="error", tol=1e-6, policy="adaptive", c=1.0, max_iter=1500,
               desc="256x256x128 smooth-core cube, TT ranks (1,16,16,1), 5% observed, noiseless"),
    "hbm3": dict(start="perturbed", rule="error", tol=1e-6, policy="theory", c=1.001, max_iter=500,
                 desc="order-3 TT completion, n=1000, TT ranks (1,2,2,1), |Omega|=50,000,000 (5%), noiseless: "
                      "a memory-bound shape (20 bytes, ~36 flop per sample)"),
    "c1": dict(start="spectral", rule="residual", tol=1e-10, policy="theory", c=1.001, max_iter=500,
               desc="order-4 TT completion, n=10, TT ranks (1,2,2,2,1), 3,000 of 10^4 entries, noiseless"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sampled_pass_flops(shape, ranks, n_obs):
    """Algorithmic flops of the sampled pass: 2 x (3 S + r_1 + 2 r_{m-1}) per sample,
    S = sum_{k=2}^{m-1} r_{k-1} r_k (prefix chain, suffix chain, gradient outer products)."""
    m = len(shape)
    s = sum(ranks[k - 1] * ranks[k] for k in range(2, m))
    return 2.0 * (3 * s + ranks[1] + 2 * ranks[m - 1]) * n_obs


def sampled_pass_bytes(shape, n_obs, val_bytes):
    """Algorithmic HBM bytes of the sampled pass: the index/value stream (cores,
    gradients and slice sums are O(sum n r^2) and stay in cache)."""
    return float(n_obs) * (4 * len(shape) + val_bytes)


def observations(pb, L):
    return L.prgd_eval(pb.shape, pb.ranks, pb.truth, pb.indices) + pb.noise_std * pb.noise


def spectral_start(pb, L, vals):
    from paper_2501_13385_amd import workloads as wl
    sk = max(pb.ranks) + 4
    gauss = np.concatenate([a.ravel() for a in wl.sketch_gaussians(pb.shape, sk, wl.make_rng(1))])
    L.prgd_spectral_init(pb.shape, pb.ranks, pb.indices, vals, gauss, sk)     # warm-up
    t0 = time.perf_counter()
    init = L.prgd_spectral_init(pb.shape, pb.ranks, pb.indices, vals, gauss, sk)
    return init, time.perf_counter() - t0, sk


def solve_leg(pb, L, precision, steps, warmup, cfg, init, phases=True):
    """l* with the truth cores, then exactly K = steps (default l*) timed iterations of a
    fresh solve from the same start, without truth tracking."""
    vals = observations(pb, L)
    vals = vals.astype(np.float64 if precision == "fp64" else np.float32)
    kw = dict(precision=precision, step_policy=cfg["policy"], step=cfg["c"])
    out = {}
    # 1. iterations to tolerance (the error rule needs the truth cores)
    s = L.Solver(pb.shape, pb.ranks, pb.indices, vals, init, truth_cores=pb.truth, stop_rule=cfg["rule"],
                 tol=cfg["tol"], max_iter=cfg["max_iter"], **kw)
    try:
        r = s.run()
    finally:
        s.close()
    lstar = int(r["iterations"])
    out["iters_to_tol"] = lstar
    out["converged"] = r["status"] == 0
    out["rel_error_at_tol"] = r["rel_error"]
    out["rel_residual_at_tol"] = r["rel_residual"]
    K = steps if steps > 0 else max(1, lstar)
    # 2. warm-up on a separate solve of the same problem
    if warmup > 0:
        s = L.Solver(pb.shape, pb.ranks, pb.indices, vals, init, stop_rule="none", max_iter=warmup, **kw)
        try:
            s.iterate(warmup)
            s.sync()
        finally:
            s.close()

    def timed(iters):
        t_setup = time.perf_counter()
        s = L.Solver(pb.shape, pb.ranks, pb.indices, vals, init, stop_rule="none", max_iter=iters, **kw)
        setup = time.perf_counter() - t_setup
        try:
            s.sync()
            t0 = time.perf_counter()
            k1_ms, dev_ms = s.iterate_timed(iters, K1_STRIDE)   # waits for the stream
            t1 = time.perf_counter()
            rep = s.report()
        finally:
            s.close()
        if rep["iterations"] != iters:
            raise RuntimeError(f"expected {iters} completed iterations, got {rep['iterations']}")
        return t1 - t0, k1_ms, dev_ms, setup

    # 3. the timed window
    wall, k1_ms, dev_ms, setup = timed(K)
    out["steps"] = K
    out["setup_s"] = setup
    out["seconds"] = wall
    out["ms_per_step"] = 1e3 * wall / K
    out["device_ms_per_step"] = dev_ms / K
    out["value"] = pb.n_obs * K / wall
    out["k1_ms"] = k1_ms
    out["k1_launches_timed"] = -(-K // K1_STRIDE)
    out["time_to_tol_s"] = wall if K == lstar else timed(max(1, lstar))[0]
    if phases:
        # per-phase split from a short separate pass (seven events per iteration
        # would slow the timed loop itself)
        np_ = max(1, min(K, 20))
        s = L.Solver(pb.shape, pb.ranks, pb.indices, vals, init, stop_rule="none", max_iter=np_, **kw)
        try:
            ph = s.iterate_profiled(np_)
        finally:
            s.close()
        out["phase_ms_per_step"] = {k: v / np_ for k, v in ph.items()}
    return out


def workload_legs(name, L, precisions, steps, warmup, phases=True):
    from paper_2501_13385_amd import workloads as wl
    cfg = LEGS[name]
    pb = wl.named(name, seed=0)
    log(f"workload {name}: shape {pb.shape} ranks {pb.ranks} |Omega| {pb.n_obs} start {cfg['start']}")
    res = {"start": cfg["start"], "stop": f"{cfg['rule']} <= {cfg['tol']:g}", "step": f"{cfg['policy']} c={cfg['c']}"}
    if cfg["start"] == "spectral":
        init, t_init, sk = spectral_start(pb, L, observations(pb, L))
        res["spectral_init_s"] = t_init
        res["spectral_init_sketch"] = sk
    else:
        init = pb.init
    for prec in precisions:
        log(f"  {name} {prec}")
        res[prec] = solve_leg(pb, L, prec, steps, warmup, cfg, init, phases=phases)
        r = res[prec]
        log(f"    l*={r['iters_to_tol']} time_to_tol={r['time_to_tol_s']:.4g}s {r['ms_per_step']:.4f} ms/step "
            f"value={r['value']:.4g} k1={r['k1_ms']:.4g} ms err={r['rel_error_at_tol']:.3g}")
    return pb, res


def _serve_problem(q):
    """One request's random ingredients (numpy only; runs in a worker process)."""
    from paper_2501_13385_amd import workloads as wl
    return wl.problem(q["shape"], q["ranks"], q["n_obs"], q["seed"], name="serve", truth_kind="unit", init_rel=0.1)


def serving_leg(L, n_req, max_obs, pool, seed=0, max_iter=300, precisions=("fp64", "mixed")):
    """Request-server throughput and latency on a seeded stream of independent problems.

    Every request runs PRGD with the adaptive step (section 3.2.2): the theory
    step diverges on part of this mix (orders 8 with large mode sizes), the
    adaptive step recovers most of it.  Each request stops at relative error
    1e-6 against its ground truth (given to the server), so every precision is
    timed to the same recovery error; a request that reaches max_iter first
    counts as a failure and is listed."""
    from paper_2501_13385_amd import workloads as wl

    reqs = wl.serving_mix(n_req, seed, max_obs=max_obs)
    t_gen = time.perf_counter()
    pbs = []
    for i, pb in enumerate(pool.imap(_serve_problem, reqs, chunksize=1)):
        pbs.append(pb)
        if (i + 1) % 64 == 0 or i + 1 == n_req:
            log(f"serving: {i + 1}/{n_req} requests drawn")
    probs = [(pb, L.prgd_eval(pb.shape, pb.ranks, pb.truth, pb.indices)) for pb in pbs]
    log(f"serving: {n_req} requests generated in {time.perf_counter() - t_gen:.1f} s")
    kw = dict(step_policy="adaptive", stop_rule="error", tol=1e-6, max_iter=max_iter)

    def run(prec, arrivals=None):
        vals = [y if prec == "fp64" else y.astype(np.float32) for _, y in probs]
        with L.Server(max_slots=max(1, n_req), iters_per_tick=4) as sv:
            t0 = time.perf_counter()
            tickets = []
            for i, ((pb, _), v) in enumerate(zip(probs, vals)):
                if arrivals is not None:
                    dt = t0 + arrivals[i] - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                tickets.append(sv.submit(pb.shape, pb.ranks, pb.indices, v, pb.init, truth_cores=pb.truth,
                                         precision=prec, **kw))
            res = [sv.result(t) for t in tickets]
            t1 = time.perf_counter()
        lat = np.array([r[1]["finish_s"] - r[1]["submit_s"] for r in res])
        wait = np.array([r[1]["admit_s"] - r[1]["submit_s"] for r in res])
        errs = np.array([r[1]["rel_error"] for r in res])
        iters = np.array([r[1]["iterations"] for r in res])
        ok = np.array([r[0] == 0 and e <= 1e-6 for r, e in zip(res, errs)])
        fails = [{"order": len(pb.shape), "n": pb.shape[0], "rank": max(pb.ranks), "n_obs": pb.n_obs,
                  "status": int(r[0]), "iterations": int(r[1]["iterations"]), "rel_error": float(r[1]["rel_error"])}
                 for (pb, _), r, g in zip(probs, res, ok) if not g]
        return {"solves_per_s": n_req / (t1 - t0), "wall_s": t1 - t0,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "p50_admission_wait_s": float(np.percentile(wait, 50)),
                "success": int(ok.sum()), "success_rate": float(ok.mean()), "failures": fails,
                "max_rel_error": float(np.nanmax(errs)), "median_iterations": float(np.median(iters)),
                "samples_iterations_per_s": float(sum(pb.n_obs * it for (pb, _), it in zip(probs, iters)) / (t1 - t0))}

    out = {"requests": n_req, "max_obs": max_obs, "tol": "relative error <= 1e-6 (truth given)",
           "step": "adaptive", "max_iter": max_iter, "redraws": int(reqs[-1]["redraws"]) if reqs else 0,
           "orders": sorted({len(pb.shape) for pb, _ in probs}),
           "total_samples": int(sum(pb.n_obs for pb, _ in probs))}
    for prec in precisions:
        log(f"serving closed loop {prec}: {n_req} requests")
        out[f"closed_{prec}"] = run(prec)
        c = out[f"closed_{prec}"]
        log(f"  {prec}: {c['solves_per_s']:.3g} solves/s, p50 {c['p50_latency_s']:.3g} s, p99 {c['p99_latency_s']:.3g} s, "
            f"success {c['success']}/{n_req}")
    best = max(precisions, key=lambda p: out[f"closed_{p}"]["solves_per_s"])
    rate = 0.7 * out[f"closed_{best}"]["solves_per_s"]
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    log(f"serving open loop {best}: Poisson rate {rate:.3g}/s")
    out[f"open_{best}"] = run(best, arrivals)
    out[f"open_{best}"]["arrival_rate_per_s"] = rate
    c = out[f"open_{best}"]
    log(f"  open: p50 {c['p50_latency_s']:.3g} s, p99 {c['p99_latency_s']:.3g} s, success {c['success']}/{n_req}")
    return out


COPY_BYTES = 256 << 20     # bytes read and written by one calibration copy


def copy_calibration(reps=5):
    """A plain device copy of known size (COPY_BYTES read + written per launch), run
    under the same counters as the bench to scale FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    src_t = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst_t = torch.empty_like(src_t)
    for _ in range(reps):
        dst_t.copy_(src_t)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "reps": reps}), flush=True)


# The main sampled kernel of each workload and the source file it is built from;
# HBM traffic recorded under profiles/ is tied to that file's contents.
MAIN_KERNEL = {
    "c4": ("k_chain", "sampled_chain.hip"),
    "c2": ("k_sampled3", "sampled3.hip"),
    "hbm3": ("k_sampled3w", "sampled3.hip"),
}


def kernel_source_hash(workload=HEADLINE):
    src = MAIN_KERNEL[workload][1]
    with open(os.path.join(ROOT, "paper_2501_13385_amd", "csrc", src), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_path(workload=HEADLINE):
    return os.path.join(ROOT, "profiles", f"traffic_{MAIN_KERNEL[workload][0]}_{workload}.json")


def measured_traffic(precision, workload=HEADLINE):
    """HBM bytes per launch of the workload's main sampled kernel from the committed
    PMC summary, or None when the kernel source changed since the counters were taken."""
    try:
        with open(traffic_path(workload)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != kernel_source_hash(workload):
        return None
    leg = rec.get(precision)
    return None if leg is None else leg.get("bytes_per_launch")


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(pb, name, n_sample, threads):
    """The reference implementation, as it stands, on the host cores: one PRGD
    iteration of the workload restricted to its first n_sample observations."""
    from threadpoolctl import threadpool_limits

    from oracle import prgd, tt

    idx = np.ascontiguousarray(pb.indices[:, :n_sample])
    y = tt.tt_eval(pb.truth, idx) + pb.noise_std * pb.noise[:n_sample]
    pol = prgd.Policy(step_rule="theory", c=LEGS[name]["c"])
    cores = [c.copy() for c in pb.init]
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        prgd.prgd_step(cores, idx, y, pol, pb.ranks)
        t1 = time.perf_counter()
    return {"value": n_sample / (t1 - t0), "unit": "samples*iterations/s", "cores": threads, "kind": "oracle",
            "sample": f"1 PRGD iteration of the {name} workload restricted to its first {n_sample} of "
                      f"{pb.n_obs} observations (same start), float64 numpy, {t1 - t0:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed iterations (0: the iterations to tolerance)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workloads", default="c4,c2,c3,c1,hbm3", help="comma list; the first is the headline")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000, help="observations in the CPU baseline's sample")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-max-obs", type=int, default=4_194_304)
    ap.add_argument("--serving-only", action="store_true", help="run only the serving leg (prints its JSON)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the headline's timed iterations (for kernel profilers)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    pool = None
    if not args.no_serving and not args.profile_only:
        # workers that draw the serving problems (numpy only), forked before
        # anything in this process touches the GPU
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(max(1, min(16, host_cores())))

    from paper_2501_13385_amd import _lib as L

    L.load()
    if args.serving_only:
        print(json.dumps(serving_leg(L, args.serve_requests, args.serve_max_obs, pool)), flush=True)
        pool.close()
        return
    names = [w for w in args.workloads.split(",") if w]
    head_name = names[0]
    precs = ["fp64", "mixed"] if args.only == "both" else [args.only]
    if args.profile_only:
        pb, res = workload_legs(head_name, L, precs, args.steps, args.warmup, phases=False)
        print(json.dumps({p: {k: res[p][k] for k in ("ms_per_step", "k1_ms", "steps")} for p in precs}), flush=True)
        return
    pb, head = workload_legs(head_name, L, precs, args.steps, args.warmup)
    hp = "fp64" if "fp64" in head else "mixed"
    h = head[hp]
    flops = sampled_pass_flops(pb.shape, pb.ranks, pb.n_obs)
    t_k1 = h["k1_ms"] * 1e-3
    kname = MAIN_KERNEL.get(head_name, ("sampled pass",))[0]
    roof = {"kernel": f"sampled pass, main kernel ({kname})", "bound": "alu",
            "achieved": flops / t_k1 / 1e12, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
            "frac": flops / t_k1 / 1e12 / PEAK_ALU_TFLOPS,
            "traffic": measured_traffic(hp, head_name) if head_name in MAIN_KERNEL else None,
            "hbm_GBs": sampled_pass_bytes(pb.shape, pb.n_obs, 8 if hp == "fp64" else 4) / t_k1 / 1e9,
            "flops_per_launch": flops, "avg_launch_us": 1e6 * t_k1,
            "launches_timed": h["k1_launches_timed"], "timed_every": K1_STRIDE}
    line = {
        "metric": METRIC,
        "value": h["value"],
        "unit": "samples*iterations/s",
        "n_gpus": 1,
        "steps": h["steps"],
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if hp == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": LEGS[head_name]["desc"], "global_batch": pb.n_obs, "precision": hp,
                   "start": head["start"], "stop": head["stop"], "step": head["step"]},
        "time_to_tol_s": h["time_to_tol_s"],
        "iters_to_tol": h["iters_to_tol"],
        "rel_error_at_tol": h["rel_error_at_tol"],
        "converged": h["converged"],
        "setup_s": h["setup_s"],
        "device_ms_per_step": h["device_ms_per_step"],
        "phase_ms_per_step": h["phase_ms_per_step"],
        "roofline": roof,
    }
    if "mixed" in head and hp != "mixed":
        m = head["mixed"]
        line["mixed"] = {k: m[k] for k in ("value", "ms_per_step", "time_to_tol_s", "iters_to_tol",
                                           "rel_error_at_tol", "converged", "k1_ms", "phase_ms_per_step")}
        line["mixed"]["dtype"] = "f32+f64"
    others = {}
    for w in names[1:]:
        pbw = None
        try:
            pbw, res = workload_legs(w, L, precs, 0, args.warmup)
        except Exception as e:   # one workload's failure is reported, not fatal to the line
            log(f"workload {w} failed: {e}")
            res = {"error": str(e)}
        res["workload"] = LEGS[w]["desc"]
        if pbw is not None:   # the main sampled kernel against the HBM roofline
            for prec in ("fp64", "mixed"):
                if prec in res and res[prec].get("k1_ms"):
                    b = sampled_pass_bytes(pbw.shape, pbw.n_obs, 8 if prec == "fp64" else 4)
                    gbs = b / (res[prec]["k1_ms"] * 1e-3) / 1e9
                    res[prec]["hbm_roofline"] = {"kernel": MAIN_KERNEL[w][0] if w in MAIN_KERNEL else None,
                                                 "bytes_per_launch": b, "achieved_GBs": gbs, "peak_GBs": PEAK_HBM_GBS,
                                                 "frac": gbs / PEAK_HBM_GBS,
                                                 "traffic": measured_traffic(prec, w) if w in MAIN_KERNEL else None}
        others[w] = res
    line["workloads"] = others
    if not args.no_serving:
        line["serving"] = serving_leg(L, args.serve_requests, args.serve_max_obs, pool)
        pool.close()
    if not args.no_cpu_baseline:
        n_s = min(args.cpu_sample, pb.n_obs)
        nc = host_cores()
        log(f"cpu baseline: one reference iteration on {n_s} observations, {nc} threads")
        line["cpu_baseline"] = cpu_baseline(pb, head_name, n_s, nc)
        log(f"cpu baseline: one thread, {n_s // 4} observations")
        line["cpu_baseline_1thread"] = cpu_baseline(pb, head_name, n_s // 4, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
