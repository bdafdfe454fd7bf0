"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer,
then under ThreadSanitizer (no GPU): every source built host-only with the
sanitizers on the host pass, linked with tests/host_sanitize/driver.cpp, which
builds and checks device layouts of many shapes (some large enough for the
multi-threaded build), feeds invalid inputs and options to the C ABI and draws
seeded cameras.  Any sanitizer report fails the run."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_05079_amd", "csrc")
SOURCES = ["povar_kernels.hip", "povar_problem.hip", "povar_server.hip", "povar_metric.hip"]


def hipcc():
    p = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return p if os.path.exists(p) else shutil.which("hipcc")


def build_and_run(san, env_extra):
    """Builds every source (host-only where there are no kernels) and the
    driver with the given host sanitizer flags, runs the driver and returns
    its result."""
    common = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    with tempfile.TemporaryDirectory() as tmp:
        objs, procs = [], []
        for src in SOURCES + [os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp")]:
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            # the sources without kernels are built for the host only
            extra = ["-x", "hip", "--offload-host-only"] if src.endswith(".cpp") else \
                ([] if src in ("povar_kernels.hip", "povar_metric.hip") else ["--offload-host-only"])
            procs.append(subprocess.Popen([hipcc(), *common, *san, *extra, "-c", os.path.join(CSRC, src), "-o", obj]))
            objs.append(obj)
        for pr in procs:
            assert pr.wait(timeout=600) == 0
        exe = os.path.join(tmp, "host_checks")
        subprocess.run([hipcc(), "--offload-arch=gfx950", *san, *objs, "-o", exe, "-lpthread"], check=True,
                       timeout=300)
        return subprocess.run([exe], capture_output=True, text=True, timeout=600,
                              env=dict(os.environ, **env_extra))


@pytest.mark.skipif(hipcc() is None, reason="hipcc is needed to build the host code")
def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    r = build_and_run(san, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                            "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "0 failure(s)" in r.stdout


@pytest.mark.skipif(hipcc() is None, reason="hipcc is needed to build the host code")
def test_host_code_under_thread_sanitizer():
    """The layout build of problems above 131,072 observations runs on several
    threads (the driver builds and checks such layouts): no data race."""
    san = ["-Xarch_host", "-fsanitize=thread", "-Xarch_host", "-fno-omit-frame-pointer"]
    r = build_and_run(san, {"TSAN_OPTIONS": "halt_on_error=1"})
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "0 failure(s)" in r.stdout
