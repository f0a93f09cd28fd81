"""The C ABI loads without a GPU, exports every declared symbol and rejects bad
arguments with the documented status codes before touching the device."""

import ctypes

import pytest

from paper_2604_21645_amd import _lib

EINVAL, ENOMEM, EUNSUPPORTED = -1, -2, -4


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_every_header_function_is_exported(L):
    names = _lib.header_functions()
    assert "mipq_pq_fit" in names and "mipq_pq_encode" in names
    for name in names:
        assert hasattr(L, name), name
        assert name in _lib.SIGNATURES, name


def test_the_configured_library_is_the_one_mapped(L):
    with open("/proc/self/maps") as f:
        assert _lib.LIB_PATH in f.read()


def test_single_hip_runtime_and_version(L):
    assert len(_lib.hip_runtimes_mapped()) == 1
    assert L.mipq_abi_version() == 2


def test_workspace_queries(L):
    small = L.mipq_pq_encode_workspace_size(1000, 128, 16, 256, 1)
    big = L.mipq_pq_encode_workspace_size(100000, 128, 16, 256, 1)
    assert 0 < small <= big
    assert L.mipq_pq_fit_workspace_size(1000, 128, 16, 256, 25, 1) < L.mipq_pq_fit_workspace_size(100000, 128, 16, 256, 25, 1)
    # FP32 needs only the error partials and the check flag
    assert 0 < L.mipq_pq_encode_workspace_size(1000, 128, 16, 256, 0) < small
    assert L.mipq_pq_encode_workspace_size(1000, 130, 16, 256, 1) == 0   # invalid shape
    assert L.mipq_pq_fit_workspace_size(1000, 128, 16, 256, 25, 1) > 0
    assert L.mipq_pq_decode_rmse_workspace_size(1000, 128, 16, 256) > 0


def _encode(L, n=10, d=128, m=16, ks=256, prec=1, ws=None, ws_bytes=0, x=1, cb=1, codes=1, flags=0):
    return L.mipq_pq_encode(x, n, d, m, ks, cb, prec, flags, codes, None, None, None, ws, ws_bytes, None)


@pytest.mark.parametrize("kw,code", [
    (dict(d=130), EINVAL),
    (dict(m=0), EINVAL),
    (dict(ks=0), EINVAL),
    (dict(ks=257), EINVAL),
    (dict(n=-1), EINVAL),
    (dict(prec=7), EINVAL),
    (dict(d=512, m=16), EUNSUPPORTED),
    (dict(x=None), EINVAL),
    (dict(ws=None), EINVAL),
    (dict(ws=256, ws_bytes=16), ENOMEM),
    (dict(flags=2), EINVAL),     # MIPQ_DETERMINISTIC is a fit flag
    (dict(flags=8), EINVAL),
    (dict(n=0, flags=1), EINVAL),   # the finite check needs the workspace even for no rows
])
def test_encode_rejects_bad_arguments(L, kw, code):
    assert _encode(L, **kw) == code
    assert len(L.mipq_last_error()) > 0


def test_fit_rejects_bad_arguments(L):
    def fit(init_rows=1, iters=5, ws=256, ws_bytes=1 << 30, flags=0):
        return L.mipq_pq_fit(1, 100, None, 0, 128, 16, 256, iters, init_rows, None, 1, flags, 1, None, None, None,
                             None, ws, ws_bytes, None)
    # no initial codebook or rows
    assert fit(init_rows=None) == EINVAL
    # negative iterations
    assert fit(iters=-1) == EINVAL
    # workspace too small
    assert fit(ws_bytes=64) == ENOMEM
    assert b"workspace" in L.mipq_last_error()
    # misaligned workspace
    assert fit(ws=257) == EINVAL
    # unknown flag
    assert fit(flags=4) == EINVAL
    assert b"flags" in L.mipq_last_error()


def test_decode_needs_x_for_the_error(L):
    rc = L.mipq_pq_decode_rmse(1, 10, 128, 16, 256, 1, None, None, 1, 256, 1 << 20, None)
    assert rc == EINVAL


def _table(ns, m=12, ks=256, ok_ptrs=True):
    t = (_lib.MipqProblem * len(ns))()
    for i, n in enumerate(ns):
        p = 4096 * (i + 1) if ok_ptrs else None
        t[i] = _lib.MipqProblem(p, n, p, p, p, None, None)
    return t


def test_batched_workspace_grows_with_problems(L):
    one = (ctypes.c_int64 * 1)(20000)
    two = (ctypes.c_int64 * 2)(20000, 500000)
    a = L.mipq_pq_fit_batched_workspace_size(one, 1, 96, 12, 256, 20, 1)
    b = L.mipq_pq_fit_batched_workspace_size(two, 2, 96, 12, 256, 20, 1)
    assert 0 < a < b
    assert L.mipq_pq_fit_batched_workspace_size(two, 2, 96, 12, 256, 20, 0) == 0   # FP32: not offered
    bad = (ctypes.c_int64 * 2)(20000, 0)
    assert L.mipq_pq_fit_batched_workspace_size(bad, 2, 96, 12, 256, 20, 1) == 0


@pytest.mark.parametrize("case,code", [
    (dict(nprob=0), EINVAL),
    (dict(prec=0), EUNSUPPORTED),
    (dict(d=97), EINVAL),
    (dict(d=384, m=12), EUNSUPPORTED),    # d/m = 32 > 16
    (dict(ns=[100, 0]), EINVAL),
    (dict(ok_ptrs=False), EINVAL),
    (dict(ws=None), EINVAL),
    (dict(ws_bytes=64), ENOMEM),
    (dict(ws=4096 + 8), EINVAL),           # misaligned
])
def test_batched_rejects_bad_arguments(L, case, code):
    ns = case.get("ns", [100, 3000])
    t = _table(ns, ok_ptrs=case.get("ok_ptrs", True))
    nprob = case.get("nprob", len(ns))
    rc = L.mipq_pq_fit_batched(t, nprob, case.get("d", 96), case.get("m", 12), 256, 5, case.get("prec", 1), None,
                               None, case.get("ws", 4096), case.get("ws_bytes", 1 << 30), None)
    assert rc == code
    assert len(L.mipq_last_error()) > 0


def test_plan_rejects_bad_arguments(L):
    plan = ctypes.c_void_p()
    t = _table([100, 3000])
    assert L.mipq_plan_create(None, t, 2, 96, 12, 256, 5, 1, 3, 4096, 1 << 30, None) == EINVAL
    assert L.mipq_plan_create(ctypes.byref(plan), t, 2, 96, 12, 256, 5, 1, 64, 4096, 1 << 30, None) == EINVAL
    assert L.mipq_plan_create(ctypes.byref(plan), t, 2, 96, 12, 256, 5, 1, 3, 4096, 64, None) == ENOMEM
    assert plan.value is None
    assert L.mipq_plan_destroy(None) == 0
    info = (ctypes.c_int64 * 4)()
    assert L.mipq_plan_info(None, info, 4) == EINVAL


def test_ii_add_rejects_bad_arguments(L):
    add = L.mipq_ii_add
    args = [4096, 100, 32, 4096, 64, 4096, 4, 16, 1, 4096, 4096, 4096, None, 4096, 1 << 30, None]
    a = list(args)
    a[8] = 2                                          # FP8: the coarse rule runs in FP32 or BF16
    assert add(*a) == EUNSUPPORTED
    a = list(args)
    a[6] = 5                                          # d % m != 0
    assert add(*a) == EINVAL
    a = list(args)
    a[5] = None                                       # no codebook
    assert add(*a) == EINVAL
    a = list(args)
    a[14] = 64                                        # workspace too small
    assert add(*a) == ENOMEM
    assert L.mipq_ii_add_workspace_size(100, 32, 64, 4, 16, 1) > 0
    assert L.mipq_ii_add_workspace_size(100, 32, 64, 4, 16, 2) == 0


def test_ii_merge_rejects_bad_arguments(L):
    P = ctypes.c_void_p * 2
    offs, ids, codes = P(4096, 8192), P(4096, 8192), P(4096, 8192)
    ns = (ctypes.c_int64 * 2)(10, 20)
    merge = L.mipq_ii_merge
    assert merge(offs, ids, codes, ns, 0, 8, 4, 4096, 4096, 4096, 4096, 1 << 20, None) == EINVAL
    assert merge(offs, ids, codes, ns, 2, 0, 4, 4096, 4096, 4096, 4096, 1 << 20, None) == EINVAL
    assert merge(offs, ids, codes, ns, 2, 8, 0, 4096, 4096, 4096, 4096, 1 << 20, None) == EINVAL
    bad = (ctypes.c_int64 * 2)(10, -1)
    assert merge(offs, ids, codes, bad, 2, 8, 4, 4096, 4096, 4096, 4096, 1 << 20, None) == EINVAL
    assert merge(offs, P(4096, None), codes, ns, 2, 8, 4, 4096, 4096, 4096, 4096, 1 << 20, None) == EINVAL
    assert merge(offs, ids, codes, ns, 2, 8, 4, 4096, 4096, 4096, 4096, 64, None) == ENOMEM
    assert merge(offs, ids, codes, ns, 2, 8, 4, 4096, 4096, 4096, 4096 + 8, 1 << 20, None) == EINVAL
    assert L.mipq_ii_merge_workspace_size(2, 8) > 0 and L.mipq_ii_merge_workspace_size(0, 8) == 0


def test_fit_width_limits(L):
    # FP32 fits take subspaces up to 48 wide (float64 sums of 256 centroids in LDS)
    assert L.mipq_pq_fit_workspace_size(1000, 48, 1, 256, 5, 0) > 0
    assert L.mipq_pq_fit_workspace_size(1000, 64, 1, 256, 5, 0) == 0
    assert L.mipq_pq_fit_workspace_size(1000, 48, 2, 256, 5, 1) == 0    # matrix-core paths: d/m <= 16
    assert L.mipq_recon_backward_workspace_size(1000, 48, 1, 256) > 0


def test_kmeans_fit_rejects_bad_arguments(L):
    km = L.mipq_kmeans_fit
    assert L.mipq_kmeans_fit_workspace_size(1000, 128, 64, 5, 1) > 0
    assert L.mipq_kmeans_fit_workspace_size(1000, 128, 64, 5, 2) == 0       # FP8: not offered
    assert km(4096, 100, None, 0, 128, 64, 5, None, 1, 4096, None, None, 4096, 1 << 30, None) == EINVAL   # no init
    assert km(4096, 100, None, 0, 128, 64, -1, 4096, 1, 4096, None, None, 4096, 1 << 30, None) == EINVAL
    assert km(4096, 100, None, 0, 128, 0, 5, 4096, 1, 4096, None, None, 4096, 1 << 30, None) == EINVAL
    assert km(4096, 100, None, 0, 100, 64, 5, 4096, 1, 4096, None, None, 4096, 1 << 30, None) == EUNSUPPORTED
    assert km(4096, 100, None, 0, 128, 64, 5, 4096, 1, 4096, None, None, 4096, 64, None) == ENOMEM


def test_adc_search_rejects_tables_beyond_lds(L):
    # d = 256, m = 256 (d/m = 1), ks = 256: a 256 KiB table per (query, list)
    adc = L.mipq_adc_search
    F = 4096
    assert adc(F, 10, 256, F, 64, F, 256, 256, F, F, F, 8, 10, F, F, None, None, F, 1 << 30, None) == EUNSUPPORTED
    # m * ks = 192 * 58 <= 11264 fits with topk = 1024: refused only for the too-small workspace
    assert adc(F, 10, 192, F, 64, F, 192, 58, F, F, F, 8, 1024, F, F, None, None, F, 64, None) == ENOMEM


def test_noalloc_encode_rejects_before_touching_the_device(L):
    enc = L.mipq_pq_encode_noalloc
    assert enc(1, (1 << 24) + 1, 128, 16, 256, 1, 1, 0, 1, None, None, None, None) == EINVAL
    assert b"noalloc" in L.mipq_last_error()
    assert enc(1, 100, 128, 16, 256, 1, 1, 1, 1, None, None, None, None) == EINVAL   # MIPQ_CHECK_FINITE
    assert enc(1, 100, 130, 16, 256, 1, 1, 0, 1, None, None, None, None) == EINVAL   # shape
    # more scratch than the fixed array: 2^23 rows of 256 one-dimensional subspaces
    assert enc(1, 1 << 23, 256, 256, 256, 1, 1, 0, 1, None, None, None, None) == ENOMEM
    assert b"scratch" in L.mipq_last_error()
