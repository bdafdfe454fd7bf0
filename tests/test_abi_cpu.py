"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-only calls behave as documented."""
import ctypes as C
import os
import re

import pytest

from paper_2405_05079_amd import povar

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "povar.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(povar_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(povar.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = povar.lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_options_default_values():
    o = povar.Options()
    assert povar.lib().povar_options_default(C.byref(o)) == povar.OK
    assert o.struct_size == C.sizeof(povar.Options)
    assert (o.eta, o.series_order, o.max_iters, o.ftol) == (0.01, 20, 50, 1e-6)
    assert (o.lambda0, o.lambda_min, o.lambda_max) == (1e-4, 1e-12, 1e12)
    assert (o.precision, o.manifold, o.use_graph) == (0, 0, 1)
    assert o.series_rtol == 0.0   # the series runs all its terms unless asked to stop early
    assert povar.lib().povar_options_default(None) == povar.EINVAL


def test_footprint_is_monotone_and_rejects_bad_sizes():
    small = povar.footprint(20, 500, 3000, "fp64")
    big = povar.footprint(250, 60000, 300000, "fp64")
    assert 0 < small < big
    assert povar.footprint(250, 60000, 400000, "fp64") > big
    # FP32-bulk adds FP32 copies of the streams and drops the FP64 camera-major one
    assert povar.footprint(250, 60000, 300000, "fp32_bulk") != big
    out = C.c_uint64()
    assert povar.lib().povar_problem_footprint(0, 10, 10, 0, C.byref(out)) == povar.EINVAL
    assert povar.lib().povar_problem_footprint(10, 10, 10, 7, C.byref(out)) == povar.EINVAL


def test_null_handles_are_rejected():
    lib = povar.lib()
    assert lib.povar_solve(None, None) == povar.EINVAL
    assert lib.povar_problem_destroy(None) == povar.EINVAL
    assert lib.povar_ctx_destroy(None) == povar.EINVAL
    assert isinstance(lib.povar_last_error(None), bytes)


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_context_without_gpu_reports_device_error():
    h = C.c_void_p()
    st = povar.lib().povar_ctx_create(0, None, C.byref(h))
    assert st == povar.EDEVICE
    assert b"device" in povar.lib().povar_last_error(None).lower()


# Layout shapes for the host-side layout check: small problems, landmarks with
# more than 64 observations (continuation packet slots), cameras with more than
# one chunk, and landmark-blocked camera passes in both precisions, with uniform
# and Zipf-weighted camera choice.
LAYOUT_CASES = [
    ("small", dict(n_cams=20, n_pts=500, track=("uniform", 4, 8)), "fp64", 0),
    ("long-tracks", dict(n_cams=150, n_pts=300, track=("uniform", 70, 140)), "fp64", 0),
    ("two-cameras", dict(n_cams=2, n_pts=3000, track=("uniform", 1, 2)), "fp32_bulk", 0),
    ("blocked-fp64", dict(n_cams=40, n_pts=70_000, track=("geom", 0.25)), "fp64", 1),
    ("blocked-fp64-zipf", dict(n_cams=1200, n_pts=70_000, track=("geom", 0.25), cam_choice="zipf"), "fp64", 1),
    ("blocked-fp32-6cam", dict(n_cams=6, n_pts=140_000, track=("uniform", 2, 3)), "fp32_bulk", 1),
    ("blocked-fp32-zipf", dict(n_cams=300, n_pts=140_000, track=("uniform", 2, 3), cam_choice="zipf"),
     "fp32_bulk", 1),
]


@pytest.mark.parametrize("name,kw,prec,blocked", LAYOUT_CASES, ids=[c[0] for c in LAYOUT_CASES])
def test_layout_invariants(name, kw, prec, blocked):
    from paper_2405_05079_amd import synth
    p = synth.make_problem(seed=7, **kw)
    r = povar.layout_check(p.cam_idx, p.pt_idx, p.meas, p.n_cams, p.n_pts, prec)
    assert r["blocked"] == blocked
    assert 0 < r["device_bytes"] <= r["footprint"]
    if blocked:
        assert r["n_slots"] % 32 == 0 and r["n_runs"] >= p.n_cams
        rec_bytes = 8 * (4 if prec == "fp32_bulk" else 8)
        assert r["lm_block"] * rec_bytes <= 2 << 20


@pytest.mark.parametrize("prec,limit", [("fp64", 65_536), ("fp32_bulk", 131_072)])
def test_blocking_starts_where_the_records_outgrow_half_the_l2(prec, limit):
    # landmark records of 8 values: the camera pass is blocked once they pass 4 MiB
    from paper_2405_05079_amd import synth
    for n_pts, want in ((limit, 0), (limit + 1, 1)):
        p = synth.make_problem(n_cams=8, n_pts=n_pts, track=("uniform", 2, 2), seed=3)
        assert povar.layout_check(p.cam_idx, p.pt_idx, p.meas, p.n_cams, p.n_pts, prec)["blocked"] == want


def test_layout_check_rejects_invalid_problems():
    import numpy as np
    cam = np.array([0, 1, 0], np.int32)
    pt = np.array([0, 0, 1], np.int32)
    meas = np.zeros((3, 2))
    with pytest.raises(povar.PovarError, match="camera 2 has no observation"):
        povar.layout_check(cam, pt, meas, 3, 2, "fp64")
    with pytest.raises(povar.PovarError, match="out of range"):
        povar.layout_check(cam, pt, meas, 2, 1, "fp64")
    bad = meas.copy()
    bad[1, 0] = np.nan
    with pytest.raises(povar.PovarError, match="non-finite"):
        povar.layout_check(cam, pt, bad, 2, 2, "fp64")
    assert povar.layout_check(cam, pt, meas, 2, 2, "fp64")["n_packets"] == 1


def test_layout_on_edge_shapes():
    """Cameras of exactly 2048, 2049 and 4096 observations and landmarks of
    exactly 64, 65 and 63: the host layout passes its invariant checks in
    both precisions, with one, two and two chunks for the first three
    cameras and one for each of the other 77."""
    from edge_shapes import boundary_problem
    p = boundary_problem()
    for prec in ("fp64", "fp32_bulk"):
        info = povar.layout_check(p.cam_idx, p.pt_idx, p.meas, p.n_cams, p.n_pts, prec)
        assert info["n_chunks"] == 1 + 2 + 2 + 77
        assert not info["blocked"]


def test_host_memory_exhaustion_is_an_error_status():
    """A host allocation that fails inside the library comes back as
    POVAR_ENOMEM with a message, not as an exception through the C ABI: a
    layout of two billion points under a 6 GiB address-space limit (in a
    child process)."""
    import subprocess
    import sys
    code = (
        "import resource, sys, ctypes\n"
        "resource.setrlimit(resource.RLIMIT_AS, (6 << 30, 6 << 30))\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import numpy as np\n"
        "from paper_2405_05079_amd import povar\n"
        "L = povar.lib()\n"
        "cam = np.zeros(1, np.int32); pt = np.zeros(1, np.int32); m = np.zeros(2)\n"
        "out = (ctypes.c_int64 * 8)()\n"
        "st = L.povar_debug_layout_check(1, 2_000_000_000, 1, cam.ctypes.data, pt.ctypes.data, m.ctypes.data, 1, out)\n"
        "print(st, L.povar_last_error(None).decode())\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    st, msg = r.stdout.strip().split(" ", 1)
    assert int(st) == povar.ENOMEM and "host resources exhausted" in msg
