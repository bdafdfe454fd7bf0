"""Continuous-batching server: each result equals the problem solved alone,
admission respects the slot cap and the device-memory budget, and requests
arriving while others run are admitted as capacity frees up (needs a GPU)."""
import time

import numpy as np
import pytest

from paper_2405_05079_amd import povar, synth

pytestmark = pytest.mark.gpu

OPTS = dict(precision="fp32_bulk", order=10, max_iters=8, ftol=0.0)


@pytest.fixture(scope="module")
def ctx():
    c = povar.Context(0)
    yield c
    c.close()


def requests():
    sizes = [(20, 2500), (45, 6000), (12, 900), (80, 9000), (30, 4000), (60, 7000), (25, 3000)]
    return [synth.make_problem(n_c, n_p, track=("geom", 0.25), seed=700 + i) for i, (n_c, n_p) in enumerate(sizes)]


def solve_alone(ctx, prob):
    gp = povar.Problem.from_synth(ctx, prob, **OPTS)
    rep = gp.solve()
    out = (rep, gp.cameras(), gp.points())
    gp.close()
    return out


def drain(sv, tickets, timeout=120.0):
    out, t0, max_active = {}, time.time(), 0
    while len(out) < len(tickets):
        max_active = max(max_active, sv.stats()["active"])
        for t in tickets:
            if t not in out:
                r = sv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return out, max_active


def test_results_equal_single_solves_and_mix_is_bitwise_independent(ctx):
    probs = requests()
    print("[case] server mix of", len(probs), flush=True)
    alone = [solve_alone(ctx, p) for p in probs]
    sv = povar.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=3)
    tickets = [sv.submit(p, **OPTS) for p in probs]
    res, max_active = drain(sv, tickets)
    assert max_active <= 3
    for p, t, (rep_a, cams_a, pts_a) in zip(probs, tickets, alone):
        rep, cams, pts, times = res[t]
        np.testing.assert_array_equal(cams, cams_a)
        np.testing.assert_array_equal(pts, pts_a)
        assert rep["cost_final"] == rep_a["cost_final"] and rep["iters"] == OPTS["max_iters"]
        assert times[0] <= times[1] <= times[2]
    # a request solved alone by the server equals the same request in the mix
    sv2 = povar.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=3)
    t_alone = sv2.submit(probs[3], **OPTS)
    r_alone, _ = drain(sv2, [t_alone])
    np.testing.assert_array_equal(r_alone[t_alone][1], res[tickets[3]][1])
    st = sv.stats()
    assert st["finished"] == len(probs) and st["active"] == 0 and st["queued"] == 0
    sv.close()
    sv2.close()


def test_admission_respects_budget_and_late_arrivals_join(ctx):
    probs = requests()
    print("[case] server budget", flush=True)
    fps = []
    for p in probs:                  # exact device bytes after layout
        gp = povar.Problem.from_synth(ctx, p, **OPTS)
        fps.append(gp.info()["device_bytes"])
        gp.close()
    assert all(f <= povar.footprint(p.n_cams, p.n_pts, p.n_obs, "fp32_bulk") for f, p in zip(fps, probs))
    budget = int(max(fps) * 1.6)     # at most ~one large problem plus small ones
    sv = povar.Server(ctx, hbm_budget_bytes=budget, max_slots=8)
    first = [sv.submit(p, **OPTS) for p in probs[:3]]
    time.sleep(0.05)                 # later arrivals while the first ones run
    later = [sv.submit(p, **OPTS) for p in probs[3:]]
    res, _ = drain(sv, first + later)
    admits = {t: res[t][3][1] for t in first + later}
    finishes = {t: res[t][3][2] for t in first + later}
    # some request was admitted only after another one had finished
    assert any(admits[t] >= min(finishes.values()) for t in later)
    for t, p in zip(first + later, probs):
        assert res[t][0]["iters"] == OPTS["max_iters"]
    # the worker's own account: the budget deferred an admission, every
    # batched iteration was counted once, read-backs cover up to four of them
    prof = sv.profile()
    assert prof["budget_waits"] >= 1
    assert prof["batch_iters"] == sv.stats()["batch_iters"] >= OPTS["max_iters"]
    assert 1 <= prof["readbacks"] <= prof["batch_iters"] <= 4 * prof["readbacks"]
    assert min(prof["admit_s"], prof["launch_s"], prof["retire_s"]) >= 0.0 and prof["wait_s"] > 0.0
    sv.close()


def test_budget_frees_a_large_problem_while_small_ones_run(ctx):
    """A large problem (above 250,000 observations: the large class, on a
    stream of its own) finishes while small ones are still iterating; the next
    large request fits only once that problem's memory is freed, which the
    worker does after the small group's iterations in flight (freeing
    synchronises the device), without waiting for the small problems to
    finish.  Every result equals its problem solved alone, bitwise."""
    large = [synth.make_problem(60, 60000, track=("geom", 0.25), seed=901 + i) for i in range(2)]
    small = requests()[:3]
    assert min(p.n_obs for p in large) > 250000 >= max(p.n_obs for p in small)
    o_large, o_small = dict(OPTS, max_iters=3), dict(OPTS, max_iters=60)
    print("[case] server budget across size classes", flush=True)
    fps, alone = [], []
    for p, o in [(large[0], o_large), (small[0], o_small), (small[1], o_small), (large[1], o_large),
                 (small[2], o_small)]:
        gp = povar.Problem.from_synth(ctx, p, **o)
        fps.append(gp.info()["device_bytes"])
        alone.append((gp.solve(), gp.cameras(), gp.points()))
        gp.close()
    budget = fps[0] + fps[1] + fps[2] + fps[4] + (1 << 20)
    assert fps[3] > fps[1] + fps[2] + fps[4] + (1 << 20)   # the second large one waits for the first
    sv = povar.Server(ctx, hbm_budget_bytes=budget, max_slots=8)
    try:
        order = [(large[0], o_large), (small[0], o_small), (small[1], o_small), (large[1], o_large),
                 (small[2], o_small)]
        tickets = [sv.submit(p, **o) for p, o in order]
        res, _ = drain(sv, tickets)
        prof = sv.profile()
    finally:
        sv.close()
    for t, (rep_a, cams_a, pts_a) in zip(tickets, alone):
        rep, cams, pts, _ = res[t]
        np.testing.assert_array_equal(cams, cams_a)
        np.testing.assert_array_equal(pts, pts_a)
        assert rep["cost_final"] == rep_a["cost_final"]
    times = [res[t][3] for t in tickets]
    assert prof["budget_waits"] >= 1
    # the second large request entered after the first finished, while the
    # small ones admitted with the first were still running
    assert times[0][2] <= times[3][1] < min(times[1][2], times[2][2])


def test_early_stops_in_the_mix_equal_single_solves(ctx):
    """Problems that stop before their iteration limit by ftol (inside a batch
    of up to four iterations, whose remaining kernels then return at once for
    them) and problems whose series stops early by series_rtol, in both size
    groups: each result equals the same request solved alone, bitwise, with
    the same iteration count."""
    probs = [synth.make_problem(52, 52000, track=("geom", 0.25), seed=911),
             synth.make_problem(20, 2500, track=("geom", 0.25), seed=912),
             synth.make_problem(45, 6000, track=("geom", 0.25), seed=913),
             synth.make_problem(30, 4000, track=("geom", 0.25), seed=914)]
    assert probs[0].n_obs > 250000 >= max(p.n_obs for p in probs[1:])
    opts = [dict(OPTS, max_iters=40, ftol=0.05), dict(OPTS, max_iters=40, ftol=0.05),
            dict(OPTS, max_iters=12, series_rtol=0.01), dict(OPTS, max_iters=40, ftol=0.02, series_rtol=0.01)]
    print("[case] server early stops", flush=True)
    alone = []
    for p, o in zip(probs, opts):
        gp = povar.Problem.from_synth(ctx, p, **o)
        alone.append((gp.solve(), gp.cameras(), gp.points()))
        gp.close()
    iters = [a[0]["iters"] for a in alone]
    assert [n < o["max_iters"] for n, o in zip(iters, opts)] == [True, True, False, True], iters
    sv = povar.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=4)
    try:
        tickets = [sv.submit(p, **o) for p, o in zip(probs, opts)]
        res, _ = drain(sv, tickets)
    finally:
        sv.close()
    for t, (rep_a, cams_a, pts_a) in zip(tickets, alone):
        rep, cams, pts, _ = res[t]
        np.testing.assert_array_equal(cams, cams_a)
        np.testing.assert_array_equal(pts, pts_a)
        assert rep["cost_final"] == rep_a["cost_final"] and rep["iters"] == rep_a["iters"]


def test_oversized_and_invalid_requests_are_rejected(ctx):
    prob = requests()[0]
    print("[case] server rejects", flush=True)
    sv = povar.Server(ctx, hbm_budget_bytes=1 << 20, max_slots=2)
    with pytest.raises(povar.PovarError) as e:
        sv.submit(prob, **OPTS)
    assert e.value.status == povar.ENOMEM
    sv.close()
    sv = povar.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=2)
    bad = synth.Problem(prob.n_cams, prob.n_pts, prob.cam_idx.copy(), prob.pt_idx, prob.meas, prob.cams0)
    bad.cam_idx[0] = -1
    with pytest.raises(povar.PovarError) as e:
        sv.submit(bad, **OPTS)
    assert e.value.status == povar.EINVAL
    sv.close()


@pytest.mark.parametrize("prec", ["fp32_bulk", "fp64"])
def test_blocked_problems_in_a_mix_equal_single_solves(ctx, prec):
    """Problems whose camera pass is landmark-blocked (camera slots per XCD,
    partials per run) batched with small chunked problems: each result is
    bitwise the same as the problem solved alone (alone, a large FP64 problem
    also stages cameras in LDS for its landmark pass; the 400-camera problem
    has 128-byte camera records, gathered cooperatively in FP32)."""
    opts = dict(OPTS, precision=prec, max_iters=4)
    probs = [synth.make_problem(30, 140000, track=("uniform", 2, 3), seed=801),
             synth.make_problem(20, 2500, track=("geom", 0.25), seed=802),
             synth.make_problem(400, 140000, track=("uniform", 2, 3), cam_choice="zipf", seed=803),
             synth.make_problem(45, 6000, track=("geom", 0.25), seed=804)]
    print("[case] blocked mix", prec, flush=True)
    alone = []
    for p in probs:
        gp = povar.Problem.from_synth(ctx, p, **opts)
        alone.append((gp.solve(), gp.cameras(), gp.points(), gp.layout()["blocked"]))
        gp.close()
    assert [a[3] for a in alone] == [True, False, True, False]
    sv = povar.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=4)
    try:
        tickets = [sv.submit(p, **opts) for p in probs]
        res, _ = drain(sv, tickets)
    finally:
        sv.close()
    for t, (rep_a, cams_a, pts_a, _) in zip(tickets, alone):
        rep, cams, pts, _ = res[t]
        np.testing.assert_array_equal(cams, cams_a)
        np.testing.assert_array_equal(pts, pts_a)
        assert rep["cost_final"] == rep_a["cost_final"]


def test_mixed_precisions_in_one_server(ctx):
    """FP32-bulk and FP64 requests interleaved on one server (one group, and
    stream, per precision): each result equals the same request solved alone
    in its precision, bitwise."""
    probs = requests()[:6]
    precs = ["fp32_bulk", "fp64"] * 3
    print("[case] server mixed precisions", flush=True)
    alone = []
    for p, prec in zip(probs, precs):
        gp = povar.Problem.from_synth(ctx, p, **dict(OPTS, precision=prec))
        rep = gp.solve()
        alone.append((rep, gp.cameras(), gp.points()))
        gp.close()
    sv = povar.Server(ctx, hbm_budget_bytes=8 << 30, max_slots=4)
    tickets = [sv.submit(p, **dict(OPTS, precision=prec)) for p, prec in zip(probs, precs)]
    res, _ = drain(sv, tickets)
    for t, (rep_a, cams_a, pts_a) in zip(tickets, alone):
        rep, cams, pts, _ = res[t]
        np.testing.assert_array_equal(cams, cams_a)
        np.testing.assert_array_equal(pts, pts_a)
        assert rep["cost_final"] == rep_a["cost_final"]
    sv.close()
