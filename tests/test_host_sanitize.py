"""The host library's CPU-only paths under AddressSanitizer (with leak
checking) and UndefinedBehaviorSanitizer: every library source is rebuilt
with the sanitizers on its host code only (the device code is built as
usual and never runs here) and linked with the checks in
`tests/host_sanitize/n2f_host_checks.cpp`: configuration checks, plans and
workspace sizes over many shapes, the initial weights, a 2000-request
simulated serving trace, and the argument checks of the entry points."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_10209_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["n2f_kernels.hip", "n2f_conv.hip", "n2f_api.cpp", "n2f_sched.cpp", "n2f_noalloc.hip", "n2f_generic.hip"]
# sanitizers for the host side of each translation unit only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{out[-4000:]}"
    return out


def test_host_library_under_address_and_undefined_sanitizers():
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    tmp = tempfile.mkdtemp(prefix="n2f_san_")
    try:
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN, *inc,
                  "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
        drv = os.path.join(tmp, "checks.o")
        _run([HIPCC, "-O1", "-g", "-std=c++17", *HOST_SAN, "-I", os.path.join(ROOT, "include"), "-c",
              os.path.join(ROOT, "tests", "host_sanitize", "n2f_host_checks.cpp"), "-o", drv])
        exe = os.path.join(tmp, "n2f_host_checks")
        _run([HIPCC, "--offload-arch=gfx950", *HOST_SAN, drv, *objs, "-o", exe])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        out = _run([exe], env=env, timeout=600)
        assert "host checks passed" in out
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
