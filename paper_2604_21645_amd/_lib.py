"""ctypes loader for libmipq.so (argument marshalling only).

torch is imported before the library is opened so that the library binds to
the HIP runtime torch already mapped (one runtime per process: torch's
streams and device pointers are then valid inside the library).
"""

from __future__ import annotations

import ctypes
import os
import re

import torch  # noqa: F401  (must precede loading the library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmipq.so")
# the host-sanitized build (tests of the C ABI only; see build.py)
if os.environ.get("MIPQ_SANITIZED_LIB"):
    LIB_PATH = os.environ["MIPQ_SANITIZED_LIB"]
HEADER = os.path.join(os.path.dirname(HERE), "include", "mipq.h")

_P = ctypes.c_void_p
_I = ctypes.c_int
_L = ctypes.c_int64
_S = ctypes.c_size_t

SIGNATURES = {
    "mipq_abi_version": (_I, []),
    "mipq_last_error": (ctypes.c_char_p, []),
    "mipq_pq_fit_workspace_size": (_S, [_L, _I, _I, _I, _I, _I]),
    "mipq_pq_fit": (_I, [_P, _L, _P, _L, _I, _I, _I, _I, _P, _P, _I, _I, _P, _P, _P, _P, _P, _P, _S, _P]),
    "mipq_pq_encode_workspace_size": (_S, [_L, _I, _I, _I, _I]),
    "mipq_pq_encode": (_I, [_P, _L, _I, _I, _I, _P, _I, _I, _P, _P, _P, _P, _P, _S, _P]),
    "mipq_pq_encode_noalloc": (_I, [_P, _L, _I, _I, _I, _P, _I, _I, _P, _P, _P, _P, _P]),
    "mipq_pq_decode_rmse_workspace_size": (_S, [_L, _I, _I, _I]),
    "mipq_pq_decode_rmse": (_I, [_P, _L, _I, _I, _I, _P, _P, _P, _P, _P, _S, _P]),
    "mipq_pq_decode_centroids": (_I, [_P, _L, _I, _I, _I, _P, _P]),
    "mipq_recon_backward_workspace_size": (_S, [_L, _I, _I, _I]),
    "mipq_recon_backward": (_I, [_P, _P, _P, _L, _I, _I, _I, _P, _P, _P, _P, _P, _S, _P]),
    "mipq_kmeans_fit_workspace_size": (_S, [_L, _I, _I, _I, _I]),
    "mipq_kmeans_fit": (_I, [_P, _L, _P, _L, _I, _I, _I, _P, _I, _P, _P, _P, _P, _S, _P]),
    "mipq_coarse_assign_workspace_size": (_S, [_I, _I, _I]),
    "mipq_coarse_assign": (_I, [_P, _L, _I, _P, _I, _I, _P, _P, _P, _S, _P]),
    "mipq_ii_build_workspace_size": (_S, [_L, _I, _I, _L, _I, _I, _I, _I, _I]),
    "mipq_ii_build": (_I, [_P, _L, _I, _I, _I, _P, _L, _P, _I, _I, _I, _P, _I, _P, _P, _P, _P, _P, _P, _P,
                           _P, _S, _P]),
    "mipq_ii_add_workspace_size": (_S, [_L, _I, _I, _I, _I, _I]),
    "mipq_ii_add": (_I, [_P, _L, _I, _P, _I, _P, _I, _I, _I, _P, _P, _P, _P, _P, _S, _P]),
    "mipq_ii_merge_workspace_size": (_S, [_I, _I]),
    "mipq_ii_merge": (_I, [_P, _P, _P, _P, _I, _I, _I, _P, _P, _P, _P, _S, _P]),
    "mipq_adc_search_workspace_size": (_S, [_I, _I, _I, _I, _I]),
    "mipq_adc_search": (_I, [_P, _I, _I, _P, _I, _P, _I, _I, _P, _P, _P, _I, _I, _P, _P, _P, _P, _P, _S, _P]),
    "mipq_pq_fit_batched_workspace_size": (_S, [_P, _I, _I, _I, _I, _I, _I]),
    "mipq_pq_fit_batched": (_I, [_P, _I, _I, _I, _I, _I, _I, _P, _P, _P, _S, _P]),
    "mipq_plan_create": (_I, [_P, _P, _I, _I, _I, _I, _I, _I, _I, _P, _S, _P]),
    "mipq_plan_info": (_I, [_P, _P, _I]),
    "mipq_plan_destroy": (_I, [_P]),
    "mipq_rotate": (_I, [_P, _L, _I, _P, _P, _P]),
    "mipq_opq_procrustes_workspace_size": (_S, [_L, _I]),
    "mipq_opq_procrustes": (_I, [_P, _P, _L, _I, _P, _P, _P, _P, _P, _P, _S, _P]),
    "mipq_profile_enable": (_I, [_I]),
    "mipq_profile_collect": (_I, [_I, ctypes.POINTER(_L), ctypes.POINTER(ctypes.c_double)]),
    "mipq_peak_probe": (_I, [_I, _I, _P, _S, ctypes.POINTER(ctypes.c_double), _P]),
}

# kernel ids of mipq_profile_collect (enum mipq_kernel)
KERNELS = {"assign_fp32": 0, "assign_bf16": 1, "update": 2, "finalize": 3, "pack_bf16": 4, "decode": 5,
           "backward": 6, "coarse_pack": 7, "coarse_assign": 8, "sort": 9, "coarse_update": 10, "adc": 11,
           "assign_bf16_batched": 12, "assign_fp8": 13, "pack_fp8": 14, "rotate": 15, "cross": 16,
           "polar": 17, "adc_scan": 18, "fit_round_bf16": 19}


class MipqProblem(ctypes.Structure):
    """struct mipq_problem of include/mipq.h"""
    _fields_ = [("x", _P), ("n", _L), ("init_rows", _P), ("codebook", _P), ("codes", _P),
                ("sse_rmse", _P), ("objective", _P)]


PLAN_AUTOTUNE, PLAN_GRAPH, PLAN_DETERMINISTIC, PLAN_RETUNE = 1, 2, 4, 8
CHECK_FINITE, DETERMINISTIC = 1, 2   # call flags of pq_fit / pq_encode
ENONFINITE = -5

# kinds of mipq_peak_probe (enum mipq_probe)
PROBES = {"add_f32": 0, "fma_f32": 1, "min3_f32": 2, "fma_f64": 3, "mfma_bf16": 4, "mfma_f8": 5, "copy": 6,
          "add_vv": 7, "min_vv": 8, "min3_add": 9}

_lib = None


class MipqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("mipq error %d: %s" % (code, msg))
        self.code = code


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/mipq.h."""
    with open(path) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(mipq_\w+)\s*\(", text)))


def hip_runtimes_mapped():
    """Paths of every libamdhip64 mapped into this process."""
    with open("/proc/self/maps") as f:
        return sorted(set(re.findall(r"\S*libamdhip64\S*", f.read())))


def lib():
    """The loaded library; raises if it is not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmipq.so is not built; run `python -m paper_2604_21645_amd.build`")
    handle = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args
    runtimes = hip_runtimes_mapped()
    if len(runtimes) > 1:
        raise RuntimeError("more than one HIP runtime mapped: %s" % runtimes)
    _lib = handle
    return _lib


def check(rc: int) -> None:
    if rc != 0:
        raise MipqError(rc, lib().mipq_last_error().decode())
