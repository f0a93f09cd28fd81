"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/test_abi.py against a build of the library whose host code is
instrumented (device code is not), in a child process that preloads the
compiler's sanitizer runtime.  CPU only: no test in test_abi.py launches a
kernel."""

import os
import subprocess
import sys

from paper_2604_21645_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib: str) -> bool:
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = [os.path.join(build.CSRC, f) for f in os.listdir(build.CSRC)]
    srcs += [os.path.join(build.INCLUDE, f) for f in os.listdir(build.INCLUDE)]
    return any(os.path.getmtime(p) > t for p in srcs)


def test_abi_tests_pass_under_host_sanitizers():
    lib = build.SAN_LIB
    if _stale(lib):
        build.build(sanitize=True)
    rt = build.asan_runtime()
    assert os.path.exists(rt), rt
    env = dict(os.environ)
    env["MIPQ_SANITIZED_LIB"] = lib
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["LD_PRELOAD"] = rt + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert " passed" in r.stdout
