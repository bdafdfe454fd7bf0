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
