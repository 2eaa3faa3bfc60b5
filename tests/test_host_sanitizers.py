"""The host-only sources of the library (options, phi tables, interpolative decompositions,
operator sets, the on-disk operator cache) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer, and driven through the C ABI by tests/native/host_sanitize_driver.cpp,
once without and once with the operator cache.  No GPU: the device sources are not part of
this build (the server's worker thread needs a GPU and is exercised by the GPU tests)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1105_3505_amd", "csrc")
HOST_SOURCES = ["api_host.cpp", "linalg_host.cpp", "operators_host.cpp", "opcache_host.cpp", "phi_host.cpp"]


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "native", "host_sanitize_driver.cpp")]
    cmd += [os.path.join(CSRC, s) for s in HOST_SOURCES] + ["-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    for cache in (None, str(tmp_path / "cache")):
        e = dict(env)
        if cache:
            os.makedirs(cache, exist_ok=True)
            e["LFMM_CACHE_DIR"] = cache
        else:
            e.pop("LFMM_CACHE_DIR", None)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=e)
        assert r.returncode == 0 and "host driver: ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
