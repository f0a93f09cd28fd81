"""Build libmipq.so (gfx950) from csrc/*.hip with hipcc.

Usage:  python -m paper_2604_21645_amd.build [--verbose]

Each source is compiled to an object of its own (in parallel), then linked
into ``paper_2604_21645_amd/libmipq.so`` next to this file.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmipq.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("MIPQ_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # the exact float32 rule must not be fused into multiply-adds
    "-ffp-contract=off",
    # no packed float32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wno-unused-command-line-argument",
]
# extra flags per source file
EXTRA = {
    # min/max of matrix-core scores need no NaN quieting: inputs are finite
    # and matrix-core results go straight to VGPRs (no accumulator reads)
    "pq_mfma.hip": ["-fno-honor-nans", "-mno-amdgpu-ieee", "-mllvm", "-amdgpu-mfma-vgpr-form"],
    # matrix-core results straight to VGPRs
    "ivf.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    # minima of matrix-core estimates without NaN quieting; IEEE mode stays on
    # (with it off the device library's work-item queries become calls)
    "coarse.hip": ["-fno-honor-nans", "-mllvm", "-amdgpu-mfma-vgpr-form"],
    "adc.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    # the minimum chains of the issue-rate probe become v_min3_f32
    "peaks.hip": ["-fno-honor-nans", "-mno-amdgpu-ieee", "-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


# host-side AddressSanitizer + UndefinedBehaviorSanitizer (device code is not
# instrumented): the CPU tests of the C ABI run against this build
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_LIB = os.path.join(BUILD_DIR, "libmipq_sanitized.so")


def _compile(src: str, verbose: bool, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, src.replace(".hip", ".san.o" if sanitize else ".o"))
    cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + EXTRA.get(src, []) + (SANITIZE if sanitize else [])
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s%s" % (src, res.stdout, res.stderr))
    for line in res.stderr.splitlines():
        if "warning" in line and "packed-fp32-ops" not in line and verbose:
            print(line)
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source and link the shared library; returns its path.
    sanitize: the host-sanitized library at SAN_LIB instead (not loaded by
    the package; its users preload the sanitizer runtime, asan_runtime())."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, sanitize), sources()))
    out = SAN_LIB if sanitize else LIB
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + (SANITIZE if sanitize else [])
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (res.stdout, res.stderr))
    os.replace(tmp, out)
    return out


def asan_runtime() -> str:
    """Path of the compiler's AddressSanitizer runtime (to preload into a
    process that loads the sanitized library)."""
    res = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return res.stdout.strip()


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv, sanitize="--sanitize" in sys.argv))
