"""The host code of the library (descriptor validation, line cover, band
packing, plan resolution, entry-point argument checks, autotuner cache) under
AddressSanitizer and UndefinedBehaviorSanitizer: a CPU-only build with the
host pass instrumented (libstencil_asan.so) runs the host ABI tests in a
child process with the sanitizer runtime preloaded; any report fails it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_abi_under_asan_and_ubsan(tmp_path):
    from paper_2310_16298_amd import build
    rt = build.asan_runtime()
    if not rt or not os.path.exists(rt):
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    lib = build.build_sanitized()
    env = dict(os.environ)
    env.update({
        "STENCIL_LIBRARY": lib,
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": f"detect_leaks=0:halt_on_error=1:log_path={tmp_path}/asan",
        "UBSAN_OPTIONS": f"halt_on_error=1:print_stacktrace=1:log_path={tmp_path}/ubsan",
    })
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                          os.path.join(ROOT, "tests", "test_host_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    reports = "".join(open(os.path.join(tmp_path, f)).read() for f in sorted(os.listdir(tmp_path))
                      if f.startswith(("asan", "ubsan")))
    assert res.returncode == 0 and not reports, (res.stdout[-3000:], res.stderr[-3000:], reports[:5000])
    assert " passed" in res.stdout
