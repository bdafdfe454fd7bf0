"""Benchmark: PoVar outer iterations per second on one MI355X.

A step is one PoVar outer iteration (linearisation after an accept, damping
and tangent projection, the order-m power series, retraction, closed-form
landmark re-solve, LM decision).  `value` is FP32-bulk iterations/s (FP32
Jacobians and series, FP64 landmark blocks, camera factorisation and cost) on
the mid-size synthetic workload: 250 cameras, 60,000 points, ~300k
observations, eta = 0.01, series order 20.  The same JSON line carries:

* the FP64 GPU path on the same problem;
* the roofline of the series (bytes per order of the algorithmic model:
  12 per observation, 36 per landmark, 800 per camera) at 250 cameras (cache
  resident) and at the roofline rows, 1,800 cameras / 5M observations and
  13,700 cameras / 29M observations, in both precisions, with the per-kernel
  durations and the HBM traffic measured by rocprofv3 counters;
* the time to the FP64 oracle's final cost: iterations and seconds each GPU
  path needs to reach f_ref (1 + 1e-6), f_ref the oracle's cost after the
  workload's 100 iterations, on five seeded problems;
* the serving stream: 512 requests, Poisson arrivals at a fixed rate,
  admission by HBM budget, p50/p99 latency per size bucket;
* the FP64 CPU oracle timed on the host (all cores and one core).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
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

from paper_2405_05079_amd import povar, synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
WORKLOAD = 2


_hip = None


def device_sync():
    """hipDeviceSynchronize (what torch.cuda.synchronize calls), without
    paying for a torch import."""
    global _hip
    if _hip is None:
        import ctypes
        _hip = ctypes.CDLL("libamdhip64.so")
    rc = _hip.hipDeviceSynchronize()
    if rc != 0:
        raise RuntimeError(f"hipDeviceSynchronize failed: {rc}")


def alg_bytes_per_order(n_obs: int, n_l: int, n_p: int) -> int:
    """Algorithmic bytes of one series order (the two passes together): per
    observation the camera index and the FP32 measurement once (12 B), per
    landmark x~_j and the symmetric V_j^+ in FP32 (36 B), per camera the
    series vector, the packed FP64 Cholesky factor and the partial sums
    (800 B).  What the method must move, whatever the kernels do."""
    return 12 * n_obs + 36 * n_l + 800 * n_p


def series_bytes(n_obs: int, n_l: int, n_p: int, fp32: bool):
    """This implementation's own per-launch byte model of the two series
    kernels (every input of the kernel read once, every output written once;
    s = 4 for FP32-bulk, 8 for FP64):
    landmark pass: per observation the packed camera index (4 B) and the
      measurement (2s); per landmark X_j (3s), V_j^+ (6 FP64 = 48 B) and z_j
      written (3s); per camera x_i (12s) and Pbar_i (9s);
    camera pass: per observation the landmark index (4 B) and the measurement
      (2s); per landmark z_j and X_j (6s); per camera the FP64 12x12 block K_i
      (1152 B), Pbar_i (9s), x_i written (12s) and the FP64 partial sum acc_i
      read and written (192 B).  Reported beside the algorithmic model."""
    s = 4 if fp32 else 8
    lpass = (4 + 2 * s) * n_obs + (6 * s + 48) * n_l + 21 * s * n_p
    cpass = (4 + 2 * s) * n_obs + 6 * s * n_l + (1344 + 21 * s) * n_p
    return lpass, cpass


def timed_iters(gp, steps: int) -> float:
    gp.report()
    device_sync()
    t0 = time.perf_counter()
    gp.enqueue(steps)
    device_sync()        # waits for every stream, the library's included
    return time.perf_counter() - t0


def series_kernel_names(prec: str, layout: dict, n_cams: int):
    """rocprofv3 names of the landmark pass, the camera pass and the combine
    kernel of a problem with this layout."""
    t = "float" if prec == "fp32_bulk" else "double"
    if layout["coop_gather"]:
        land = "k_series_landmark_coop" if prec == "fp32_bulk" else "k_series_landmark_coop64"
    else:
        land = f"k_series_landmark<{t}>"
    cam = f"k_series_camera_slots<{t}>" if layout["blocked"] else f"k_series_camera<{t}, 1024>"
    return land, cam, f"k_series_camera_combine<{t}>"


def series_leg(ctx, prob, prec: str, steps: int, warmup: int, workload: str):
    """Timed iterations of one problem and the roofline of its series orders:
    the durations of the landmark pass and of the camera pass (with its
    combine kernel) from HIP events recorded by the kernels' own dispatches,
    the algorithmic bytes per order over their sum, and the HBM traffic the
    committed rocprofv3 counters measured for these kernels (None when the
    kernels changed since)."""
    gp = povar.Problem.from_synth(ctx, prob, precision=prec, ftol=0.0, max_iters=10 ** 6)
    gp.step(warmup)
    secs = timed_iters(gp, steps)
    rep = gp.report()
    gp.kernel_timing(True)
    gp.step(max(3, min(steps // 4, 20)))
    kt = gp.kernel_times()
    gp.kernel_timing(False)
    layout = gp.layout()
    stage1 = (gp.cameras(), gp.points()) if prec == "fp64" else None
    gp.close()
    us_l = 1e3 * kt["ms_landmark_pass"] / max(1, kt["n_landmark_pass"])
    us_c = 1e3 * kt["ms_camera_pass"] / max(1, kt["n_camera_pass"])
    b_alg = alg_bytes_per_order(prob.n_obs, prob.n_pts, prob.n_cams)
    b_l, b_c = series_bytes(prob.n_obs, prob.n_pts, prob.n_cams, prec == "fp32_bulk")
    land, cam, comb = series_kernel_names(prec, layout, prob.n_cams)
    h = kernel_source_hash()
    tr = [traffic_from_profiles(k, workload, h) for k in (land, cam)]
    tr_comb = traffic_from_profiles(comb, workload, h)
    traffic = (tr[0] + tr[1] + (tr_comb or 0.0)) if None not in tr else None
    order_us = us_l + us_c
    dom, dom_us = (land, us_l) if us_l >= us_c else (cam, us_c)
    out = {
        "precision": prec, "iters_per_s": round(steps / secs, 3), "ms_per_iter": round(1e3 * secs / steps, 4),
        "steps": steps, "cost_after": rep["cost_final"], "layout": layout,
        "us_landmark_pass": round(us_l, 3), "us_camera_pass_with_combine": round(us_c, 3),
        "us_per_order": round(order_us, 3),
        "alg_bytes_per_order": b_alg,
        "alg_frac_per_order": round(b_alg / (order_us * 1e-6) / (HBM_PEAK_GBS * 1e9), 4),
        "dominant_kernel": {"name": dom, "avg_us": round(dom_us, 3),
                            "alg_frac": round(b_alg / (dom_us * 1e-6) / (HBM_PEAK_GBS * 1e9), 4)},
        "counter_bytes_per_order": traffic,
        "counter_over_alg": round(traffic / b_alg, 3) if traffic else None,
        "counter_rate_frac": round(traffic / (order_us * 1e-6) / (HBM_PEAK_GBS * 1e9), 4) if traffic else None,
        "kernel_counter_rate_frac": {k: round(t / (u * 1e-6) / (HBM_PEAK_GBS * 1e9), 4)
                                     for k, t, u in ((land, tr[0], us_l), (cam, tr[1], us_c)) if t},
        "builder_model_bytes_per_launch": {"landmark_pass": b_l, "camera_pass": b_c},
    }
    return out, stage1


def iters_to_reach(gp, n_iters: int, target: float):
    """Runs n_iters LM iterations; the first iteration (1-based) whose accepted
    cost is <= target, or None, and the accepted cost after each iteration."""
    gp.step(n_iters)
    cost, _, acc = gp.trace()
    best = np.minimum.accumulate(np.where(acc, cost, np.inf))
    hit = np.nonzero(best <= target)[0]
    return (int(hit[0]) + 1 if hit.size else None), best


def matched_cost(ctx, rates: dict, seeds: int):
    """Time to the oracle's final cost on `seeds` problems of the 250-camera
    workload: f_ref is the FP64 oracle's cost after the workload's 100
    iterations (stored by tests/golden/make_oracle_costs.py); each GPU path
    runs up to 200 iterations, and the first iteration whose accepted cost is
    within f_ref (1 + 1e-6) is converted to seconds at that path's measured
    iteration rate (`rates`, iterations/s)."""
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_costs.json")))
    rows = []
    for k in range(seeds):
        key = "2" if k == 0 else f"2.{k}"
        if key not in golden:
            continue
        g = golden[key]
        prob = synth.workload(WORKLOAD, k)
        target = g["cost_final"] * (1 + 1e-6)
        row = {"seed": k, "oracle_cost_final": g["cost_final"], "oracle_iters": g["iters"]}
        for prec in ("fp32_bulk", "fp64"):
            gp = povar.Problem.from_synth(ctx, prob, precision=prec, ftol=0.0, max_iters=2 * g["iters"])
            it, best = iters_to_reach(gp, 2 * g["iters"], target)
            gp.close()
            row[prec] = {"iters_to_match": it, "seconds_to_match": (it / rates[prec]) if it else None,
                         "cost_at_ref_iters": float(best[g["iters"] - 1]),
                         "rel_vs_oracle_at_ref_iters": float((best[g["iters"] - 1] - g["cost_final"])
                                                             / g["cost_final"])}
        rows.append(row)

    def med(prec, key):
        v = [r[prec][key] for r in rows if r[prec][key] is not None]
        return float(np.median(v)) if v else None
    out = {"f_ref": "FP64 oracle cost after 100 iterations (stored)", "target": "f_ref (1 + 1e-6)",
           "cap_iters": 200, "seeds": rows}
    for prec in ("fp32_bulk", "fp64"):
        out[prec] = {"matched": sum(r[prec]["iters_to_match"] is not None for r in rows),
                     "median_iters_to_match": med(prec, "iters_to_match"),
                     "median_seconds_to_match": med(prec, "seconds_to_match"),
                     "median_rel_vs_oracle_at_ref_iters": med(prec, "rel_vs_oracle_at_ref_iters")}
    both = [r for r in rows if r["fp32_bulk"]["seconds_to_match"] and r["fp64"]["seconds_to_match"]]
    out["speedup_fp32_over_fp64_at_matched_cost"] = (
        float(np.median([r["fp64"]["seconds_to_match"] / r["fp32_bulk"]["seconds_to_match"] for r in both]))
        if both else None)
    m32 = out["fp32_bulk"]["median_seconds_to_match"]
    out["fp32_bulk_iters_per_s_at_matched_cost"] = (out["fp32_bulk"]["median_iters_to_match"] / m32) if m32 else None
    return out


def matched_cost_row(ctx, prob, rates: dict):
    """Time to a matched final cost at a size the oracle cannot run for a
    whole trajectory: f_ref is the FP64 GPU path's accepted cost after the
    workload's iteration count (that path's steps match the stored oracle
    steps at this size to 1e-12, tests/test_gpu_full_size.py); FP32-bulk runs
    up to twice as many iterations, and the first whose accepted cost is
    within f_ref (1 + 1e-6) is converted to seconds at its measured rate."""
    n = prob.iters
    gp = povar.Problem.from_synth(ctx, prob, precision="fp64", ftol=0.0, max_iters=n)
    _, best64 = iters_to_reach(gp, n, -np.inf)
    gp.close()
    f_ref = float(best64[n - 1])
    if not np.isfinite(f_ref):
        return {"f_ref": f"FP64 GPU path's cost after {n} iterations", "f_ref_value": None,
                "note": "no accepted FP64 step"}
    target = f_ref * (1 + 1e-6)
    it64 = int(np.nonzero(best64 <= target)[0][0]) + 1
    gp = povar.Problem.from_synth(ctx, prob, precision="fp32_bulk", ftol=0.0, max_iters=2 * n)
    it32, best32 = iters_to_reach(gp, 2 * n, target)
    gp.close()
    out = {"f_ref": f"FP64 GPU path's cost after {n} iterations", "f_ref_value": f_ref,
           "target": "f_ref (1 + 1e-6)", "cap_iters": 2 * n,
           "fp64": {"iters_to_match": it64, "seconds_to_match": it64 / rates["fp64"]},
           "fp32_bulk": {"iters_to_match": it32, "seconds_to_match": (it32 / rates["fp32_bulk"]) if it32 else None,
                         "rel_vs_ref_at_ref_iters": float((best32[n - 1] - f_ref) / f_ref)}}
    s32 = out["fp32_bulk"]["seconds_to_match"]
    out["speedup_fp32_over_fp64_at_matched_cost"] = (out["fp64"]["seconds_to_match"] / s32) if s32 else None
    # the same target with both paths damped no lower than 1e-6 (the default
    # floor is 1e-12): below it the FP32 series' rounding makes steps fail
    floor = {"lambda_min": DAMPING_FLOOR_ALT}
    for prec in ("fp64", "fp32_bulk"):
        gp = povar.Problem.from_synth(ctx, prob, precision=prec, ftol=0.0, max_iters=2 * n,
                                      lambda_min=DAMPING_FLOOR_ALT)
        it, _ = iters_to_reach(gp, 2 * n, target)
        gp.close()
        floor[prec] = {"iters_to_match": it, "seconds_to_match": (it / rates[prec]) if it else None}
    a, b = floor["fp64"]["seconds_to_match"], floor["fp32_bulk"]["seconds_to_match"]
    floor["speedup_fp32_over_fp64_at_matched_cost"] = (a / b) if a and b else None
    out["both_with_lambda_min_1e-6"] = floor
    return out


# damping floor of the second matched-cost comparison at the large workloads
DAMPING_FLOOR_ALT = 1e-6

BUCKETS = [(20, 40), (40, 80), (80, 160), (160, 320), (320, 401)]
# Arrival rate of the serving leg: 0.8 x the closed-loop throughput of the
# 512-request stream (1 GiB budget, 64 slots), measured on one MI355X with the
# server that groups problems by size: 205.6 problems/s, the mean of seven
# runs (194-213), and kept fixed.
SERVING_RATE_PER_S = 164.5
SERVING_ARRIVAL_SEEDS = (4999, 5999)


def _serving_problem(args):
    nc, npt, seed = args
    return synth.serving_problem(nc, npt, seed)


def serving_problems(n_requests: int):
    from concurrent.futures import ProcessPoolExecutor
    sizes = synth.serving_stream(512)[:n_requests]
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(_serving_problem, sizes, chunksize=8))


def run_stream(ctx, probs, arrivals, budget, slots, opts):
    """Submit probs at the given arrival offsets (seconds; None = all at once)
    to a fresh server and wait for every result.  Submits (host layout
    builds, thread-safe, outside the GIL) run on a pool of threads, each at
    its request's arrival time, so one request's layout build does not delay
    the next arrival.  Returns (latencies from the submit call's entry,
    latencies from the scheduled arrival (None for all at once), submit lags
    (entry minus arrival), wall seconds, max resident, the server's worker
    profile); the server's clock starts just before this function's."""
    from concurrent.futures import ThreadPoolExecutor
    sv = povar.Server(ctx, hbm_budget_bytes=budget, max_slots=slots)
    t0 = time.perf_counter()

    def submit_at(i):
        if arrivals is not None:
            wait = arrivals[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        return sv.submit(probs[i], **opts)

    times = {}
    max_res = 0
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        futs = [ex.submit(submit_at, i) for i in range(len(probs))]
        pending = set(range(len(probs)))
        while pending:
            max_res = max(max_res, sv.stats()["active"])
            for i in [i for i in pending if futs[i].done()]:
                r = sv.poll(futs[i].result())
                if r is not None:
                    times[i] = r[3]
                    pending.discard(i)
            time.sleep(0.002)
    wall = time.perf_counter() - t0
    prof = sv.profile()
    sv.close()
    n = len(probs)
    lat = [times[i][2] - times[i][0] for i in range(n)]
    if arrivals is None:
        return lat, None, None, wall, max_res, prof
    lat_arr = [times[i][2] - arrivals[i] for i in range(n)]
    lag = [times[i][0] - arrivals[i] for i in range(n)]
    return lat, lat_arr, lag, wall, max_res, prof


def serving(ctx, n_requests: int, budget: int, slots: int, calibrate: bool):
    """Continuous-batching leg: the serving stream (cameras log-uniform in
    [20, 400], points = 250 x cameras, mean track 5, series order 20, 50
    iterations, FP32-bulk).  A closed-loop run (all requests queued at once,
    where the HBM budget limits admission) gives the throughput; the
    open-loop runs submit with Poisson arrivals at the fixed rate
    SERVING_RATE_PER_S (two arrival draws, latencies pooled per bucket)."""
    probs = serving_problems(n_requests)
    opts = dict(precision="fp32_bulk", order=20, max_iters=50, ftol=0.0)
    footprint = sum(povar.footprint(p.n_cams, p.n_pts, p.n_obs, "fp32_bulk") for p in probs)
    _, _, _, closed_wall, closed_res, closed_prof = run_stream(ctx, probs, None, budget, slots, opts)
    closed_rate = len(probs) / closed_wall
    rate = 0.8 * closed_rate if calibrate else SERVING_RATE_PER_S
    lat, lat_sub, lags, walls, max_res, profs = [], [], [], [], 0, []
    for seed in SERVING_ARRIVAL_SEEDS:
        rng = np.random.default_rng(seed)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(probs)))
        l_sub, l_arr, lag, wall, mr, prof = run_stream(ctx, probs, arrivals, budget, slots, opts)
        lat.append(np.asarray(l_arr))
        lat_sub.append(np.asarray(l_sub))
        lags.append(np.asarray(lag))
        walls.append(wall)
        max_res = max(max_res, mr)
        profs.append(prof)
    ncam = np.tile(np.array([p.n_cams for p in probs]), len(SERVING_ARRIVAL_SEEDS))
    # latency from the scheduled arrival (the submit's own layout build and any
    # wait for a submitting thread included)
    lat, lat_sub, lags = np.concatenate(lat), np.concatenate(lat_sub), np.concatenate(lags)
    per_bucket = {}
    for lo, hi in BUCKETS:
        sel = (ncam >= lo) & (ncam < hi)
        if sel.any():
            per_bucket[f"{lo}-{hi - 1}"] = {"n": int(sel.sum()),
                                            "p50_s": round(float(np.percentile(lat[sel], 50)), 4),
                                            "p99_s": round(float(np.percentile(lat[sel], 99)), 4)}
    obs = int(sum(p.n_obs for p in probs))
    return {"requests": len(probs), "of_stream": 512, "iters_per_request": 50, "order": 20,
            "precision": "fp32_bulk", "hbm_budget_bytes": budget, "max_slots": slots,
            "sum_footprint_bytes": int(footprint),
            "closed_loop_problems_per_s": round(closed_rate, 3),
            "closed_loop_obs_iters_per_s": round(obs * 50 / closed_wall, 1),
            "closed_loop_max_resident": closed_res, "closed_loop_worker": closed_prof,
            "arrival_rate_per_s": round(rate, 3), "arrival_rate_source": "calibrated now" if calibrate else
            "fixed (SERVING_RATE_PER_S)", "arrival_draws": len(SERVING_ARRIVAL_SEEDS),
            "open_loop_problems_per_s": round(len(probs) / float(np.mean(walls)), 3),
            "p50_s": round(float(np.percentile(lat, 50)), 4), "p99_s": round(float(np.percentile(lat, 99)), 4),
            "latency_from": "scheduled arrival",
            "p50_from_submit_s": round(float(np.percentile(lat_sub, 50)), 4),
            "p99_from_submit_s": round(float(np.percentile(lat_sub, 99)), 4),
            "submit_lag_p50_s": round(float(np.percentile(lags, 50)), 4),
            "submit_lag_p99_s": round(float(np.percentile(lags, 99)), 4),
            "max_resident": max_res, "open_loop_worker": profs[0], "obs_total": obs,
            "per_bucket_cameras": per_bucket}


def refine_leg(ctx, prob, P1, X1, steps: int, eta_handover: bool = True):
    """The second stage (projective refinement, RiPoBA, FP64) on the same
    problem.  The rate: `steps` graph-replayed LM iterations from the first
    stage's FP64 solution (the stratified pipeline).  The costs: before and
    after, against the noise floor of the measurements, from that solution and
    from the ground truth perturbed by N(0, 0.02^2) per coordinate (cameras
    and homogeneous landmarks, each then put back on its sphere), and (with
    eta_handover) from a first stage run at eta = 0.3.  From random cameras
    the first stage at the
    workload's eta = 0.01 can stop in a poor basin of its own objective, and
    the refinement then only improves the start it was given."""
    def unit(a):
        return a / np.linalg.norm(a, axis=1, keepdims=True)

    def make(P, Xh):
        return povar.Problem.refine(ctx, prob.n_cams, prob.n_pts, prob.cam_idx, prob.pt_idx, prob.meas,
                                    unit(P), unit(Xh), order=prob.order, ftol=0.0, max_iters=10 ** 6)

    gp = make(P1, np.concatenate([X1, np.ones((X1.shape[0], 1))], axis=1))
    c0 = gp.report()["cost_initial"]
    gp.step(5)
    secs = timed_iters(gp, steps)
    rep = gp.report()
    gp.close()
    rng = np.random.default_rng(77)
    Pg = prob.cams_gt.reshape(prob.n_cams, 12)
    Xg = np.concatenate([prob.pts_gt, np.ones((prob.n_pts, 1))], axis=1)
    gp = make(unit(Pg) + 0.02 * rng.standard_normal(Pg.shape), unit(Xg) + 0.02 * rng.standard_normal(Xg.shape))
    g0 = gp.report()["cost_initial"]
    gp.step(steps)
    grep_ = gp.report()
    gp.close()
    out = {"iters_per_s": round(steps / secs, 2), "steps": steps, "precision": "fp64", "order": prob.order,
           # sigma^2 per coordinate of every observation: reachable only
           # without outliers (the 1,800-camera workload holds 1%)
           "noise_floor": synth.SIGMA ** 2 * 2 * prob.n_obs,
           "outlier_frac": next(w["outlier_frac"] for w in synth.WORKLOADS.values() if w["name"] == prob.name),
           "from_first_stage": {"cost_initial": c0, "cost_after": rep["cost_final"], "iters": rep["iters"]},
           "from_perturbed_truth": {"sigma": 0.02, "cost_initial": g0, "cost_after": grep_["cost_final"],
                                    "iters": grep_["iters"]}}
    if not eta_handover:
        return out
    # the stratified pipeline with the first stage at eta = 0.3 (one of the
    # paper's ablation values): FP32-bulk, the workload's iteration count
    s1 = povar.Problem.from_synth(ctx, prob, precision="fp32_bulk", eta=0.3, ftol=0.0, max_iters=prob.iters)
    r1 = s1.solve()
    P3, X3 = s1.cameras(), s1.points()
    s1.close()
    gp = make(P3, np.concatenate([X3, np.ones((X3.shape[0], 1))], axis=1))
    e0 = gp.report()["cost_initial"]
    gp.step(steps)
    erep = gp.report()
    gp.close()
    out["from_first_stage_eta_0.3"] = {"first_stage_iters": r1["iters"], "first_stage_cost": r1["cost_final"],
                                       "cost_initial": e0, "cost_after": erep["cost_final"], "iters": erep["iters"]}
    return out


def eta_sweep(ctx, prob, iters: int):
    """The pOSE weight eta at the paper's main value (0.1) and its ablation
    values (0.2-0.4) on the same problem and kernels: FP32-bulk iterations
    per second and the cost after `iters` iterations from the same random
    cameras.  Costs of different eta are different objectives."""
    out = {}
    for eta in (0.1, 0.2, 0.3, 0.4):
        gp = povar.Problem.from_synth(ctx, prob, precision="fp32_bulk", eta=eta, ftol=0.0, max_iters=10 ** 6)
        gp.step(5)
        secs = timed_iters(gp, iters)
        rep = gp.report()
        gp.close()
        out[str(eta)] = {"iters_per_s": round(iters / secs, 1), "cost_initial": rep["cost_initial"],
                         "cost_after": rep["cost_final"], "iters": rep["iters"]}
    return out


def metric_leg(ctx, reps: int = 5):
    """The metric upgrade (App. D) at 250 and 13,700 cameras: calibrated
    cameras seen through a random projective frame, each with a random scale
    and sign and 1e-3 relative noise on every entry.  Wall time of the whole
    call (host inputs to host outputs, device allocation included), median of
    `reps`; the largest rotation error against the ground truth."""
    out = {}
    for n in (250, 13700):
        G, K = synth.calibrated_cameras(n, 7000 + n)
        rng = np.random.default_rng(7100 + n)
        Hp = np.eye(4) + 0.3 * rng.standard_normal((4, 4))
        s = rng.uniform(0.5, 2.0, n) * rng.choice([-1.0, 1.0], n)
        P = s[:, None, None] * (G @ Hp) * (1.0 + 1e-3 * rng.standard_normal((n, 3, 4)))
        povar.metric_upgrade(ctx, P, K, ftol=1e-10)
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            g = povar.metric_upgrade(ctx, P, K, ftol=1e-10)
            times.append(time.perf_counter() - t0)
        B = np.linalg.solve(K, G)
        Rg = B[:, :, :3] / np.cbrt(np.linalg.det(B[:, :, :3]))[:, None, None]
        cosang = (np.einsum("nab,nab->n", g["R"], Rg @ Rg[0].T) - 1.0) / 2.0
        ms = 1e3 * float(np.median(times))
        out[str(n)] = {"ms_per_call": round(ms, 3), "iters": int(g["iters"]),
                       "ms_per_iter": round(ms / max(1, g["iters"]), 4),
                       "cost_initial": g["cost_initial"], "cost_final": g["cost_final"],
                       "max_rotation_error_deg": float(np.degrees(np.arccos(np.clip(cosang, -1, 1))).max())}
    return out


def copy_calibration(nbytes: int):
    """A plain device-to-device copy of known size (HIP runs it as a blit
    kernel), for scaling the HBM byte counters."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(a), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(nbytes)) == 0
    for _ in range(3):
        assert hip.hipMemcpy(b, a, ctypes.c_size_t(nbytes), 3) == 0   # device to device
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(a)
    hip.hipFree(b)
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}))


def stream_copy_gbps(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Achievable HBM rate of a plain device-to-device copy (HIP's blit
    kernel): bytes read plus bytes written per second, timed with HIP events
    over `reps` copies of `nbytes` after three untimed ones."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    e0, e1 = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(a), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipEventCreate(ctypes.byref(e0)) == 0 and hip.hipEventCreate(ctypes.byref(e1)) == 0
    try:
        for _ in range(3):
            assert hip.hipMemcpyAsync(b, a, ctypes.c_size_t(nbytes), 3, None) == 0
        assert hip.hipEventRecord(e0, None) == 0
        for _ in range(reps):
            assert hip.hipMemcpyAsync(b, a, ctypes.c_size_t(nbytes), 3, None) == 0
        assert hip.hipEventRecord(e1, None) == 0
        assert hip.hipEventSynchronize(e1) == 0
        ms = ctypes.c_float()
        assert hip.hipEventElapsedTime(ctypes.byref(ms), e0, e1) == 0
        return 2.0 * nbytes * reps / (ms.value * 1e-3) / 1e9
    finally:
        hip.hipEventDestroy(e0)
        hip.hipEventDestroy(e1)
        hip.hipFree(a)
        hip.hipFree(b)


def summarize_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, workload, out_path):
    """Per-launch HBM bytes of the series kernels from rocprofv3 counter CSVs:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) averaged over the kernel's
    dispatches, each scaled by bytes / counter of a plain copy of copy_bytes."""
    import csv

    def per_kernel(path):
        acc = {}
        for row in csv.DictReader(open(path)):
            k = row["Kernel_Name"]
            acc.setdefault(k, []).append(float(row["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    def copy_value(path):
        vals = [v for k, v in per_kernel(path).items() if "copyBuffer" in k or "copy" in k.lower()]
        return max(vals)

    f, w = per_kernel(fetch_csv), per_kernel(write_csv)
    fs = copy_bytes / copy_value(copy_fetch_csv)     # bytes per FETCH_SIZE unit
    ws = copy_bytes / copy_value(copy_write_csv)
    data = json.load(open(out_path)) if os.path.exists(out_path) else {}
    entry = data.setdefault(workload, {})
    for k in f:
        if "k_series_" not in k:
            continue
        short = k.split("(")[0].replace("void povar::", "").replace("povar::", "")
        entry[short] = {"fetch_bytes_per_launch": f[k] * fs, "write_bytes_per_launch": w.get(k, 0.0) * ws,
                        "hbm_bytes_per_launch": f[k] * fs + w.get(k, 0.0) * ws,
                        "fetch_counter_kib": f[k], "write_counter_kib": w.get(k, 0.0),
                        "copy_scale_fetch": fs, "copy_scale_write": ws,
                        "kernel_source_sha256": kernel_source_hash()}
    json.dump(data, open(out_path, "w"), indent=1)
    print(json.dumps(entry))


def traffic_from_profiles(kernel: str, workload: str, kernel_hash: str):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy), if the committed summary matches this
    kernel build and workload; None otherwise."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path)).get(workload, {}).get(kernel)
    if not d or d.get("kernel_source_sha256") != kernel_hash:
        return None
    return d["hbm_bytes_per_launch"]


def strip_comments(src: str) -> str:
    """C++ source without comments and with whitespace collapsed (string
    literals in the kernel sources hold no comment markers)."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_hash() -> str:
    """Hash of the kernel code the counters were taken on (comments and
    layout of the text do not count)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("povar_kernels.hip", "povar_internal.h"):
        h.update(strip_comments(open(os.path.join(ROOT, "paper_2405_05079_amd", "csrc", name)).read()).encode())
    return h.hexdigest()


def host_info() -> dict:
    """CPU model, logical cores and memory of the host the oracle ran on."""
    info = {"cores": os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["mem_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    try:   # the CPUs this process may run on (a container or cgroup share)
        info["cores_available"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return info


def cpu_baseline(ctx, prob, iters: int):
    """The FP64 oracle timed on the host on a bounded sample of the workload
    (`iters` LM iterations, incl. its initial landmark solve), once with the
    BLAS thread pool on every available core and once on one core; then,
    untimed, the error of the GPU's FP64-critical parts against it at the
    shared initial linearisation."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import povar_oracle as O
    host = host_info()
    runs = {}
    for label, limit in (("all_cores", host.get("cores_available", host["cores"])), ("one_core", 1)):
        with threadpool_limits(limits=limit):
            threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
            t0 = time.perf_counter()
            O.lm_solve(prob, opts=O.Options(order=prob.order, max_iters=iters, ftol=0.0))
            secs = time.perf_counter() - t0
        runs[label] = {"iters_per_s": iters / secs, "seconds": round(secs, 2), "threads": threads}
    best = runs["all_cores"]
    base = {"value": best["iters_per_s"], "unit": "iters/s", "cores": best["threads"], "kind": "oracle",
            "sample": f"{iters} LM iterations of the FP64 oracle (NumPy/SciPy) on the same {prob.n_cams}-camera "
                      f"problem, incl. its initial landmark solve: {best['seconds']} s on "
                      f"{best['threads']} BLAS threads, {runs['one_core']['seconds']} s on one",
            "one_core": runs["one_core"], "host": host}
    return base, critical_errors(ctx, prob, O)


def critical_errors(ctx, prob, O, lam=1e-3):
    """Relative errors of the GPU against the oracle at the initial state:
    V_j^+ (per landmark, Frobenius), U_i and the damped camera block inverse
    K_i = B_i (B_i^T U_i,lambda B_i)^-1 B_i^T (per camera, Frobenius), the cost,
    one damped camera step of the workload's order (per camera, 2-norm) and
    the cost at its trial cameras; max and median over landmarks / cameras."""
    P, X, f = O.initial_state(prob, prob.cams0)
    lin = O.linearize(P, X, prob)
    ref_step = O.camera_step(P, lin, lam, prob.order)
    rs = O.reduced_system(P, lin, lam)
    ref_K = np.einsum("nik,nkl,njl->nij", rs.B, np.linalg.inv(rs.Ut), rs.B)
    Pn = O.retract(P, ref_step)
    Xn, _ = O.solve_landmarks(Pn, prob)
    f_trial = O.cost(Pn, Xn, prob)

    def rel_rows(a, b):
        a, b = a.reshape(len(a), -1), b.reshape(len(b), -1)
        r = np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)
        return {"max": float(r.max()), "median": float(np.median(r))}

    out = {"at": f"initial state of the {prob.n_cams}-camera problem; step at lambda {lam}, order {prob.order}"}
    for prec in ("fp32_bulk", "fp64"):
        gp = povar.Problem.from_synth(ctx, prob, precision=prec)
        d = gp.debug_linearize()
        K = gp.debug_camera_blocks(lam)
        dp, _, ct = gp.debug_step(lam, prob.order)
        gp.close()
        out[prec] = {"V_pinv": rel_rows(d["Vp"], lin.Vp), "U": rel_rows(d["U"], lin.U),
                     "K": rel_rows(K, ref_K), "cost": abs(d["cost"] - lin.cost) / lin.cost,
                     "step": rel_rows(dp, ref_step), "trial_cost": abs(ct - f_trial) / f_trial}
    return out


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    # about 12 s of oracle work per timing on the host of the GPU (all cores, then one)
    ap.add_argument("--cpu-iters", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-matched", action="store_true")
    ap.add_argument("--matched-seeds", type=int, default=5,
                    help="problems of the 250-camera workload for the time-to-oracle-cost comparison")
    ap.add_argument("--workload", type=int, default=WORKLOAD,
                    help="headline workload: 2 (default, 250 cameras); 3 or 5 time that one alone")
    ap.add_argument("--rows", default="3,5",
                    help="roofline-row workloads timed beside the headline (comma list; empty: none)")
    ap.add_argument("--no-refine", action="store_true",
                    help="skip the second-stage (projective refinement) leg")
    ap.add_argument("--no-metric", action="store_true", help="skip the metric-upgrade leg")
    ap.add_argument("--no-eta-sweep", action="store_true", help="skip the eta sweep (0.1-0.4)")
    ap.add_argument("--serve", type=int, default=512,
                    help="requests of the 512-request serving stream to run (0: skip)")
    ap.add_argument("--serve-budget", type=int, default=1 << 30)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--calibrate-serving", action="store_true",
                    help="set the serving arrival rate from this run's closed loop instead of the fixed rate")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                               "COPY_WRITE_CSV", "COPY_BYTES"),
                    help="write profiles/hbm_traffic.json from rocprofv3 counter CSVs")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.summarize_counters:
        a = args.summarize_counters
        summarize_counters(a[0], a[1], a[2], a[3], int(a[4]), f"workload{args.workload}",
                           os.path.join(ROOT, "profiles", "hbm_traffic.json"))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU here; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    rows = [int(r) for r in args.rows.split(",") if r.strip()]
    if args.workload != WORKLOAD:
        # one workload alone (profiling runs): no other legs
        rows = []
        args.no_matched = args.no_cpu_baseline = args.no_metric = args.no_eta_sweep = args.no_refine = True
        args.serve = 0
    prob = synth.workload(args.workload)
    log(f"workload {prob.name}: {prob.n_cams} cameras, {prob.n_pts} points, {prob.n_obs} observations, "
        f"order {prob.order}")
    ctx = povar.Context(0)
    wname = f"workload{args.workload}"
    legs, stage1 = {}, None
    for prec in ("fp32_bulk", "fp64"):
        legs[prec], s1 = series_leg(ctx, prob, prec, args.steps, args.warmup, wname)
        stage1 = s1 or stage1
        log(f"{prec}: {legs[prec]['iters_per_s']:.1f} iters/s, series order {legs[prec]['us_per_order']:.2f} us")
    fp32 = legs["fp32_bulk"]
    b_alg = fp32["alg_bytes_per_order"]
    achieved = b_alg / (fp32["us_per_order"] * 1e-6) / 1e9
    copy_gbps = stream_copy_gbps()
    log(f"plain device copy: {copy_gbps:.0f} GB/s (read + write)")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "achievable_copy_GBps": round(copy_gbps, 1),
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": fp32["counter_bytes_per_order"],
                "unit_of_work": "one series order (landmark pass + camera pass with its combine kernel)",
                "alg_bytes": b_alg, "us": fp32["us_per_order"],
                "dominant_kernel": fp32["dominant_kernel"],
                "traffic_over_alg": fp32["counter_over_alg"],
                "note": ("250 cameras: 5.9 MB per order stays in the 256 MB Infinity Cache, so HBM is not "
                         "what bounds it; the HBM rows are roofline_rows")}
    out = {
        "metric": "VarPro iters/s FP32-bulk vs FP64 at matched final cost; p50/p99 solve latency",
        "value": round(fp32["iters_per_s"], 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp32["ms_per_iter"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded; shapes of the paper's BAL workloads)",
        "config": {"workload": f"{prob.name}: {prob.n_cams} cameras, {prob.n_pts} points, "
                               f"{prob.n_obs} observations, eta {prob.eta}, series order {prob.order}, "
                               "FP32-bulk with FP64 V_j / U_i / cost",
                   "precision": "fp32_bulk"},
        "fp64_iters_per_s": legs["fp64"]["iters_per_s"],
        "fp32_over_fp64": round(fp32["iters_per_s"] / legs["fp64"]["iters_per_s"], 3),
        "roofline": roofline,
        "series": legs,
    }
    if rows:
        out["roofline_rows"] = {}
        for w in rows:
            pw = synth.workload(w)
            log(f"roofline row {pw.name}: {pw.n_obs} observations")
            row = {"workload": f"{pw.name}: {pw.n_cams} cameras, {pw.n_pts} points, {pw.n_obs} observations, "
                               f"series order {pw.order}"}
            for prec in ("fp32_bulk", "fp64"):
                row[prec], _ = series_leg(ctx, pw, prec, args.steps, min(args.warmup, 5), f"workload{w}")
                cb = row[prec]["counter_bytes_per_order"]
                row[prec]["counter_rate_of_copy"] = (
                    round(cb / (row[prec]["us_per_order"] * 1e-6) / (copy_gbps * 1e9), 4) if cb else None)
                log(f"  {prec}: {row[prec]['iters_per_s']:.2f} iters/s, order {row[prec]['us_per_order']:.1f} us, "
                    f"alg frac {row[prec]['alg_frac_per_order']}")
            if not args.no_matched:
                row["matched_cost"] = matched_cost_row(
                    ctx, pw, {p: row[p]["iters_per_s"] for p in ("fp32_bulk", "fp64")})
                mc = row["matched_cost"]
                log(f"  matched cost: FP64 {mc['fp64']['iters_to_match']} iterations, FP32-bulk "
                    f"{mc['fp32_bulk']['iters_to_match']}, speedup {mc['speedup_fp32_over_fp64_at_matched_cost']}")
                fl = mc["both_with_lambda_min_1e-6"]
                log(f"  both with lambda_min 1e-6: FP64 {fl['fp64']['iters_to_match']}, FP32-bulk "
                    f"{fl['fp32_bulk']['iters_to_match']}, speedup {fl['speedup_fp32_over_fp64_at_matched_cost']}")
            out["roofline_rows"][f"workload{w}"] = row
            del pw
    if not args.no_matched:
        rates = {p: legs[p]["iters_per_s"] for p in legs}
        out["matched_cost"] = matched_cost(ctx, rates, args.matched_seeds)
        log(f"matched cost: {out['matched_cost']['fp32_bulk']} {out['matched_cost']['fp64']}")
    if not args.no_refine:
        out["refine"] = refine_leg(ctx, prob, *stage1, min(args.steps, 50), eta_handover=True)
        log(f"refinement: {out['refine']['iters_per_s']} iters/s")
    if not args.no_eta_sweep:
        out["eta_sweep"] = eta_sweep(ctx, prob, min(args.steps, prob.iters))
        log(f"eta sweep: {out['eta_sweep']}")
    if not args.no_metric:
        out["metric_upgrade"] = metric_leg(ctx)
        log(f"metric upgrade: {out['metric_upgrade']}")
    if args.serve > 0:
        out["serving"] = serving(ctx, args.serve, args.serve_budget, args.serve_slots, args.calibrate_serving)
        log(f"serving: p50 {out['serving']['p50_s']} s, p99 {out['serving']['p99_s']} s, closed loop "
            f"{out['serving']['closed_loop_problems_per_s']} problems/s")
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["errors_vs_oracle"] = cpu_baseline(ctx, prob, args.cpu_iters)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
