"""MI355X-native product quantisation and inverted-index hot path.

Thin Python layer over libmipq.so (include/mipq.h): every function checks
dtypes and devices, allocates outputs and workspaces with torch, passes raw
pointers and torch's current HIP stream to the C ABI, and returns tensors.
All arithmetic runs in the library's HIP kernels; there is no CPU fallback.
"""

from __future__ import annotations

import torch

import ctypes

from ._lib import (CHECK_FINITE, DETERMINISTIC, ENONFINITE, PLAN_AUTOTUNE, PLAN_DETERMINISTIC,  # noqa: F401
                   PLAN_GRAPH, PLAN_RETUNE, MipqError, MipqProblem, check, lib)

FP32, BF16, FP8 = 0, 1, 2
_PREC = {"fp32": FP32, "bf16": BF16, "fp8": FP8, FP32: FP32, BF16: BF16, FP8: FP8}


def _prec(p) -> int:
    try:
        return _PREC[p]
    except KeyError:
        raise ValueError("precision must be 'fp32', 'bf16' or 'fp8'") from None


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be on the GPU" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    return t.contiguous()


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def pq_fit(x: torch.Tensor, m: int, ks: int, iters: int, init_rows: torch.Tensor | None = None,
           init_codebook: torch.Tensor | None = None, train_rows: torch.Tensor | None = None,
           precision="bf16", labels: bool = True, codebook64: bool = False, objective: bool = True,
           out: torch.Tensor | None = None, rescored: bool = False, deterministic: bool = False,
           check_finite: bool = False):
    """Fit per-subspace k-means codebooks (Lloyd, ``iters`` rounds).

    Returns a dict with ``codebook`` float32 [m, ks, d/m] (written into
    ``out`` when given) and, on request, ``labels`` uint8 [n_train, m] (last
    assignment), ``codebook64``, ``objective`` float64 [iters] and
    ``rescored`` int64 [iters] (pairs re-decided by the float32 rule in each
    round).  ``deterministic``: float64 sums in a fixed order (bit-identical
    runs); ``check_finite``: raise MipqError (code ENONFINITE) on NaN or
    infinite inputs.
    """
    L = lib()
    x = _dev(x, torch.float32, "x")
    dev = x.device
    n, d = x.shape
    ds = d // m if m else 0
    tr = _dev(train_rows, torch.int64, "train_rows") if train_rows is not None else None
    n_train = tr.numel() if tr is not None else n
    ir = _dev(init_rows, torch.int64, "init_rows") if init_rows is not None else None
    ic = _dev(init_codebook, torch.float32, "init_codebook") if init_codebook is not None else None
    p = _prec(precision)
    if out is not None:
        if (out.dtype != torch.float32 or out.device != dev or tuple(out.shape) != (m, ks, ds)
                or not out.is_contiguous()):
            raise ValueError("out must be a contiguous float32 [m, ks, d/m] tensor on the device of x")
        res = {"codebook": out}
    else:
        res = {"codebook": torch.empty((m, ks, ds), dtype=torch.float32, device=dev)}
    if labels:
        res["labels"] = torch.empty((n_train, m), dtype=torch.uint8, device=dev)
    if codebook64:
        res["codebook64"] = torch.empty((m, ks, ds), dtype=torch.float64, device=dev)
    if objective:
        res["objective"] = torch.empty(max(iters, 0), dtype=torch.float64, device=dev)
    if rescored:
        res["rescored"] = torch.empty(max(iters, 0), dtype=torch.int64, device=dev)
    flags = (DETERMINISTIC if deterministic else 0) | (CHECK_FINITE if check_finite else 0)
    nbytes = L.mipq_pq_fit_workspace_size(n_train, d, m, ks, iters, p)
    ws = _ws(nbytes, dev)
    check(L.mipq_pq_fit(_ptr(x), n, _ptr(tr), n_train, d, m, ks, iters, _ptr(ir), _ptr(ic), p, flags,
                        _ptr(res["codebook"]), _ptr(res.get("codebook64")), _ptr(res.get("labels")),
                        _ptr(res.get("objective")), _ptr(res.get("rescored")), _ptr(ws), ws.numel(),
                        _stream(dev)))
    return res


def pq_encode_ex(x: torch.Tensor, codebook: torch.Tensor, precision="bf16", min_dist: bool = False,
                 sse_rmse: bool = False, rescored: bool = False, check_finite: bool = False) -> dict:
    """Encode (mipq_pq_encode) with every optional output: a dict with
    ``codes`` uint8 [n, m] and, on request, ``min_dist`` float32 [n, m] (the
    float32-rule distance to the chosen centroid), ``sse_rmse`` float64 [2]
    and ``rescored`` int64 [1]."""
    L = lib()
    x = _dev(x, torch.float32, "x")
    cb = _dev(codebook, torch.float32, "codebook")
    dev = x.device
    n, d = x.shape
    m, ks, ds = cb.shape
    if m * ds != d:
        raise ValueError("codebook shape %s does not match d=%d" % (tuple(cb.shape), d))
    p = _prec(precision)
    res = {"codes": torch.empty((n, m), dtype=torch.uint8, device=dev)}
    if min_dist:
        res["min_dist"] = torch.empty((n, m), dtype=torch.float32, device=dev)
    if sse_rmse:
        res["sse_rmse"] = torch.empty(2, dtype=torch.float64, device=dev)
    if rescored:
        res["rescored"] = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = _ws(L.mipq_pq_encode_workspace_size(n, d, m, ks, p), dev)
    check(L.mipq_pq_encode(_ptr(x), n, d, m, ks, _ptr(cb), p, CHECK_FINITE if check_finite else 0,
                           _ptr(res["codes"]), _ptr(res.get("min_dist")), _ptr(res.get("sse_rmse")),
                           _ptr(res.get("rescored")), _ptr(ws), ws.numel(), _stream(dev)))
    return res


def pq_encode_noalloc(x: torch.Tensor, codebook: torch.Tensor, precision="bf16", codes: torch.Tensor | None = None,
                      min_dist: torch.Tensor | None = None, sse_rmse: torch.Tensor | None = None,
                      rescored: torch.Tensor | None = None) -> torch.Tensor:
    """mipq_pq_encode_noalloc: encode with the library's fixed scratch array
    (no workspace).  Outputs may be passed in (then nothing is allocated
    here either); ``codes`` is returned."""
    L = lib()
    x = _dev(x, torch.float32, "x")
    cb = _dev(codebook, torch.float32, "codebook")
    dev = x.device
    n, d = x.shape
    m, ks, ds = cb.shape
    if m * ds != d:
        raise ValueError("codebook shape %s does not match d=%d" % (tuple(cb.shape), d))
    if codes is None:
        codes = torch.empty((n, m), dtype=torch.uint8, device=dev)
    for t, shape, dt, name in ((codes, (n, m), torch.uint8, "codes"), (min_dist, (n, m), torch.float32, "min_dist"),
                               (sse_rmse, (2,), torch.float64, "sse_rmse"), (rescored, (1,), torch.int64, "rescored")):
        if t is not None and (t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous() or t.device != dev):
            raise ValueError("%s must be a contiguous %s tensor of shape %s on %s" % (name, dt, shape, dev))
    check(L.mipq_pq_encode_noalloc(_ptr(x), n, d, m, ks, _ptr(cb), _prec(precision), 0, _ptr(codes), _ptr(min_dist),
                                   _ptr(sse_rmse), _ptr(rescored), _stream(dev)))
    return codes


def pq_encode(x: torch.Tensor, codebook: torch.Tensor, precision="bf16", rescored: bool = False):
    """Codes uint8 [n, m]; with ``rescored=True`` also the int64 count of
    (row, subspace) pairs the BF16 path re-decided in float32."""
    r = pq_encode_ex(x, codebook, precision, rescored=rescored)
    return (r["codes"], r["rescored"]) if rescored else r["codes"]


def pq_decode_rmse(codes: torch.Tensor, codebook: torch.Tensor, x: torch.Tensor | None = None,
                   x_hat: bool = False):
    """Decode codes; returns (x_hat or None, sse_rmse float64 [2] or None)."""
    L = lib()
    codes = _dev(codes, torch.uint8, "codes")
    cb = _dev(codebook, torch.float32, "codebook")
    dev = codes.device
    n, m = codes.shape
    m2, ks, ds = cb.shape
    if m2 != m:
        raise ValueError("codes have %d subspaces, codebook %d" % (m, m2))
    d = m * ds
    xx = _dev(x, torch.float32, "x") if x is not None else None
    xh = torch.empty((n, d), dtype=torch.float32, device=dev) if x_hat else None
    sr = torch.empty(2, dtype=torch.float64, device=dev) if xx is not None else None
    ws = _ws(L.mipq_pq_decode_rmse_workspace_size(n, d, m, ks), dev)
    check(L.mipq_pq_decode_rmse(_ptr(codes), n, d, m, ks, _ptr(cb), _ptr(xx), _ptr(xh), _ptr(sr),
                                _ptr(ws), ws.numel(), _stream(dev)))
    return xh, sr


def recon_backward(x: torch.Tensor, codebook: torch.Tensor, codes: torch.Tensor,
                   grad_out: torch.Tensor | None = None, grad_x: bool = True, grad_codebook: bool = True):
    """Reconstruction loss L = sum ||x - x_hat||^2 (codes fixed) and its gradients.

    Returns (loss float64 [1], dL/dx float32 [n, d] or None, dL/dC float32
    [m, ks, ds] or None), each gradient scaled by ``grad_out`` (float64 [1],
    default 1)."""
    L = lib()
    x = _dev(x, torch.float32, "x")
    cb = _dev(codebook, torch.float32, "codebook")
    codes = _dev(codes, torch.uint8, "codes")
    dev = x.device
    n, d = x.shape
    m, ks, ds = cb.shape
    if m * ds != d or codes.shape != (n, m):
        raise ValueError("shapes of x %s, codebook %s and codes %s disagree"
                         % (tuple(x.shape), tuple(cb.shape), tuple(codes.shape)))
    g = None
    if grad_out is not None:
        g = grad_out.detach().to(device=dev, dtype=torch.float64).reshape(1).contiguous()
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    gx = torch.empty((n, d), dtype=torch.float32, device=dev) if grad_x else None
    gc = torch.empty((m, ks, ds), dtype=torch.float32, device=dev) if grad_codebook else None
    ws = _ws(L.mipq_recon_backward_workspace_size(n, d, m, ks), dev)
    check(L.mipq_recon_backward(_ptr(x), _ptr(codes), _ptr(cb), n, d, m, ks, _ptr(g), _ptr(gx), _ptr(gc),
                                _ptr(loss), _ptr(ws), ws.numel(), _stream(dev)))
    return loss, gx, gc


class PQReconLoss(torch.autograd.Function):
    """L = sum over rows of ||x - decode(codes, codebook)||^2 with the codes held
    fixed; differentiable in x and codebook (float64 loss, float32 gradients).

        loss = PQReconLoss.apply(x, codebook, codes)
        loss = PQReconLoss.apply(x, codebook, codes, sse)

    sse (optional): a float64 device tensor whose first entry is already that
    sum, as the encode of the same x against the same codebook writes it
    (``pq_encode_ex(x, codebook, sse_rmse=True)["sse_rmse"]``, its fused
    error); the forward then returns it instead of decoding the rows again.
    """

    @staticmethod
    def forward(ctx, x, codebook, codes, sse=None):
        if sse is None:
            _, sse = pq_decode_rmse(codes, codebook, x)
        elif sse.dtype != torch.float64 or sse.device != x.device or sse.numel() < 1:
            raise ValueError("sse must be a float64 tensor on the rows' device")
        ctx.save_for_backward(x, codebook, codes)
        return sse[0].clone().reshape(())

    @staticmethod
    def backward(ctx, g):
        x, codebook, codes = ctx.saved_tensors
        need_x, need_c = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_x or need_c):
            return None, None, None, None
        _, gx, gc = recon_backward(x, codebook, codes, grad_out=g, grad_x=need_x, grad_codebook=need_c)
        return gx, gc, None, None


def coarse_assign(x: torch.Tensor, coarse: torch.Tensor, precision="bf16", rescored: bool = False):
    """Coarse list label (int32 [n]) of every row; optionally the int64 number
    of rows re-decided with the exact rule."""
    L = lib()
    x = _dev(x, torch.float32, "x")
    cc = _dev(coarse, torch.float32, "coarse")
    dev = x.device
    n, d = x.shape
    kc = cc.shape[0]
    p = _prec(precision)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    resc = torch.zeros(1, dtype=torch.int64, device=dev) if rescored else None
    ws = _ws(L.mipq_coarse_assign_workspace_size(d, kc, p), dev)
    check(L.mipq_coarse_assign(_ptr(x), n, d, _ptr(cc), kc, p, _ptr(labels), _ptr(resc), _ptr(ws), ws.numel(),
                               _stream(dev)))
    return (labels, resc) if rescored else labels


def kmeans_fit(x: torch.Tensor, k: int, iters: int, init_rows: torch.Tensor, train_rows: torch.Tensor | None = None,
               precision="bf16", labels: bool = True, objective: bool = True):
    """k-means over whole rows (``mipq_kmeans_fit``, the coarse quantiser):
    dict(centroids float32 [k, d], labels int32 [n_train] (last assignment),
    objective float64 [iters])."""
    L = lib()
    x = _dev(x, torch.float32, "x")
    dev = x.device
    n, d = x.shape
    tr = _dev(train_rows, torch.int64, "train_rows") if train_rows is not None else None
    n_train = tr.numel() if tr is not None else n
    ir = _dev(init_rows, torch.int64, "init_rows")
    if ir.numel() != k:
        raise ValueError("init_rows must hold k row indices")
    p = _prec(precision)
    out = {"centroids": torch.empty((k, d), dtype=torch.float32, device=dev)}
    if labels:
        out["labels"] = torch.empty(n_train, dtype=torch.int32, device=dev)
    if objective:
        out["objective"] = torch.empty(max(iters, 1), dtype=torch.float64, device=dev)
    ws = _ws(L.mipq_kmeans_fit_workspace_size(n_train, d, k, iters, p), dev)
    check(L.mipq_kmeans_fit(_ptr(x), n, _ptr(tr), n_train, d, k, iters, _ptr(ir), p, _ptr(out["centroids"]),
                            _ptr(out.get("labels")), _ptr(out.get("objective")), _ptr(ws), ws.numel(),
                            _stream(dev)))
    if objective:
        out["objective"] = out["objective"][:iters]
    return out


def ii_build(x: torch.Tensor, kc: int, coarse_iters: int, train_rows: torch.Tensor, coarse_init: torch.Tensor,
             m: int, ks: int, pq_iters: int, pq_init: torch.Tensor, precision="bf16", labels: bool = True,
             coarse_objective: bool = False):
    """Inverted file with residual PQ; returns a dict with coarse, pq_codebook,
    offsets, ids, codes_sorted (and labels, coarse_objective on request)."""
    L = lib()
    x = _dev(x, torch.float32, "x")
    tr = _dev(train_rows, torch.int64, "train_rows")
    ci = _dev(coarse_init, torch.int64, "coarse_init")
    pi = _dev(pq_init, torch.int64, "pq_init")
    dev = x.device
    n, d = x.shape
    n_train = tr.numel()
    p = _prec(precision)
    out = {
        "coarse": torch.empty((kc, d), dtype=torch.float32, device=dev),
        "pq_codebook": torch.empty((m, ks, d // m), dtype=torch.float32, device=dev),
        "offsets": torch.empty(kc + 1, dtype=torch.int64, device=dev),
        "ids": torch.empty(n, dtype=torch.int32, device=dev),
        "codes_sorted": torch.empty((n, m), dtype=torch.uint8, device=dev),
    }
    if labels:
        out["labels"] = torch.empty(n, dtype=torch.int32, device=dev)
    if coarse_objective:
        out["coarse_objective"] = torch.empty(max(coarse_iters, 1), dtype=torch.float64, device=dev)
    ws = _ws(L.mipq_ii_build_workspace_size(n, d, kc, n_train, m, ks, pq_iters, coarse_iters, p), dev)
    check(L.mipq_ii_build(_ptr(x), n, d, kc, coarse_iters, _ptr(tr), n_train, _ptr(ci), m, ks, pq_iters, _ptr(pi), p,
                          _ptr(out["coarse"]), _ptr(out["pq_codebook"]), _ptr(out["offsets"]), _ptr(out["ids"]),
                          _ptr(out["codes_sorted"]), _ptr(out.get("labels")), _ptr(out.get("coarse_objective")),
                          _ptr(ws), ws.numel(), _stream(dev)))
    return out


def ii_add(x: torch.Tensor, coarse: torch.Tensor, pq_codebook: torch.Tensor, precision="bf16",
           labels: bool = False):
    """Posting lists of the rows ``x`` under fixed quantisers (``mipq_ii_add``):
    dict with coarse, pq_codebook (the given ones), offsets, ids (0..n-1 of
    this ``x``), codes_sorted and, on request, labels."""
    L = lib()
    x = _dev(x, torch.float32, "x")
    cc = _dev(coarse, torch.float32, "coarse")
    pqc = _dev(pq_codebook, torch.float32, "pq_codebook")
    dev = x.device
    n, d = x.shape
    kc = cc.shape[0]
    m, ks, _ = pqc.shape
    p = _prec(precision)
    out = {
        "coarse": cc,
        "pq_codebook": pqc,
        "offsets": torch.empty(kc + 1, dtype=torch.int64, device=dev),
        "ids": torch.empty(n, dtype=torch.int32, device=dev),
        "codes_sorted": torch.empty((n, m), dtype=torch.uint8, device=dev),
    }
    if labels:
        out["labels"] = torch.empty(n, dtype=torch.int32, device=dev)
    ws = _ws(L.mipq_ii_add_workspace_size(n, d, kc, m, ks, p), dev)
    check(L.mipq_ii_add(_ptr(x), n, d, _ptr(cc), kc, _ptr(pqc), m, ks, p, _ptr(out["offsets"]), _ptr(out["ids"]),
                        _ptr(out["codes_sorted"]), _ptr(out.get("labels")), _ptr(ws), ws.numel(), _stream(dev)))
    return out


def ii_merge(parts):
    """One index from indexes over consecutive row ranges (``mipq_ii_merge``):
    list l is list l of every part in order, ids shifted by the rows of the
    parts before.  ``parts``: dicts from ``ii_add`` / ``ii_build`` sharing
    the quantisers of the first."""
    L = lib()
    if not parts:
        raise ValueError("need at least one part")
    first = parts[0]
    cc, pqc = first["coarse"], first["pq_codebook"]
    dev = cc.device
    kc = cc.shape[0]
    m = pqc.shape[0]
    offs = [_dev(p["offsets"], torch.int64, "offsets") for p in parts]
    ids = [_dev(p["ids"], torch.int32, "ids") for p in parts]
    codes = [_dev(p["codes_sorted"], torch.uint8, "codes_sorted") for p in parts]
    if any(o.numel() != kc + 1 for o in offs) or any(c.dim() != 2 or c.shape[1] != m for c in codes):
        raise ValueError("every part needs kc + 1 offsets and m codes per row")
    ns = [int(i.numel()) for i in ids]
    total = sum(ns)
    k = len(parts)
    out = {
        "coarse": cc,
        "pq_codebook": pqc,
        "offsets": torch.empty(kc + 1, dtype=torch.int64, device=dev),
        "ids": torch.empty(total, dtype=torch.int32, device=dev),
        "codes_sorted": torch.empty((total, m), dtype=torch.uint8, device=dev),
    }
    po = (ctypes.c_void_p * k)(*[_ptr(o) for o in offs])
    pi = (ctypes.c_void_p * k)(*[_ptr(i) for i in ids])
    pc = (ctypes.c_void_p * k)(*[_ptr(c) for c in codes])
    pn = (ctypes.c_int64 * k)(*ns)
    ws = _ws(L.mipq_ii_merge_workspace_size(k, kc), dev)
    check(L.mipq_ii_merge(po, pi, pc, pn, k, kc, m, _ptr(out["offsets"]), _ptr(out["ids"]),
                          _ptr(out["codes_sorted"]), _ptr(ws), ws.numel(), _stream(dev)))
    return out


def adc_search(q: torch.Tensor, index: dict, nprobe: int, topk: int, wide: bool = False, work: bool = False):
    """Top-k (ids int32 [nq, topk], distances float32 [nq, topk]) per query
    over an index from ``ii_build``; optionally (appended in this order) the
    int64 number of queries whose probe selection ranked every list exactly
    and the int64 [4] work counters of the list scans (table entries built,
    rows given the partial sum over their first 4 subspaces, rows summed in
    full -- a row that passed the partial sum counts in both -- and lists
    scanned)."""
    L = lib()
    q = _dev(q, torch.float32, "q")
    dev = q.device
    nq, d = q.shape
    cc = _dev(index["coarse"], torch.float32, "coarse")
    pqc = _dev(index["pq_codebook"], torch.float32, "pq_codebook")
    off = _dev(index["offsets"], torch.int64, "offsets")
    ids = _dev(index["ids"], torch.int32, "ids")
    codes = _dev(index["codes_sorted"], torch.uint8, "codes_sorted")
    kc = cc.shape[0]
    m, ks, _ = pqc.shape
    out_ids = torch.empty((nq, topk), dtype=torch.int32, device=dev)
    out_d = torch.empty((nq, topk), dtype=torch.float32, device=dev)
    w = torch.zeros(1, dtype=torch.int64, device=dev) if wide else None
    wk = torch.zeros(4, dtype=torch.int64, device=dev) if work else None
    ws = _ws(L.mipq_adc_search_workspace_size(nq, d, kc, nprobe, topk), dev)
    check(L.mipq_adc_search(_ptr(q), nq, d, _ptr(cc), kc, _ptr(pqc), m, ks, _ptr(off), _ptr(ids), _ptr(codes),
                            nprobe, topk, _ptr(out_ids), _ptr(out_d), _ptr(w), _ptr(wk), _ptr(ws), ws.numel(),
                            _stream(dev)))
    out = (out_ids, out_d)
    if wide:
        out += (w,)
    if work:
        out += (wk,)
    return out


def rotate(x: torch.Tensor, rotation: torch.Tensor) -> torch.Tensor:
    """y = x R (``mipq_rotate``): x float32 [n, d], R float64 [d, d]."""
    x = _dev(x, torch.float32, "x")
    r = _dev(rotation, torch.float64, "rotation")
    n, d = x.shape
    if tuple(r.shape) != (d, d):
        raise ValueError("rotation must be [d, d]")
    y = torch.empty((n, d), dtype=torch.float32, device=x.device)
    check(lib().mipq_rotate(_ptr(x), n, d, _ptr(r), _ptr(y), _stream(x.device)))
    return y


def procrustes(x: torch.Tensor, y_hat: torch.Tensor, v_init: torch.Tensor | None = None,
               return_v: bool = False):
    """Orthogonal R minimising ||x R - y_hat|| (``mipq_opq_procrustes``):
    returns (R float64 [d, d], M = x^T y_hat float64 [d, d], Jacobi sweeps
    int32 [1]) and, with ``return_v``, V float64 [d, d] to warm-start the
    next call through ``v_init``."""
    L = lib()
    x = _dev(x, torch.float32, "x")
    yh = _dev(y_hat, torch.float32, "y_hat")
    if x.shape != yh.shape:
        raise ValueError("x and y_hat must have the same shape")
    n, d = x.shape
    dev = x.device
    v0 = _dev(v_init, torch.float64, "v_init") if v_init is not None else None
    if v0 is not None and tuple(v0.shape) != (d, d):
        raise ValueError("v_init must be [d, d]")
    r = torch.empty((d, d), dtype=torch.float64, device=dev)
    m = torch.empty((d, d), dtype=torch.float64, device=dev)
    v = torch.empty((d, d), dtype=torch.float64, device=dev) if return_v else None
    sw = torch.empty(1, dtype=torch.int32, device=dev)
    ws = _ws(L.mipq_opq_procrustes_workspace_size(n, d), dev)
    check(L.mipq_opq_procrustes(_ptr(x), _ptr(yh), n, d, _ptr(v0), _ptr(r), _ptr(v), _ptr(m), _ptr(sw), _ptr(ws),
                                ws.numel(), _stream(dev)))
    return (r, m, sw, v) if return_v else (r, m, sw)


def opq_fit(x: torch.Tensor, m: int, ks: int, outer_iters: int, pq_iters: int, init_rows: torch.Tensor,
            precision="bf16", history: bool = False):
    """Optimized PQ (non-parametric): R = I and a codebook seeded from the
    rows ``init_rows`` of x, then ``outer_iters`` times: y = x R; ``pq_iters``
    Lloyd rounds on y from the current codebook; codes of y; R = the
    Procrustes rotation of x onto the decoded codes.  Composed from the
    boundary calls.

    Returns dict(R float64 [d, d], codebook float32 [m, ks, d/m], objective
    float64 [outer_iters] = SSE of x R (rounded to float32) against the
    decoded codes after each rotation update, sweeps (Jacobi sweeps of each
    Procrustes step, each warm-started from the previous step's V), and with
    ``history`` the lists ``rotations`` and ``codebooks`` of every outer
    iteration).
    """
    x = _dev(x, torch.float32, "x")
    dev = x.device
    n, d = x.shape
    r = torch.eye(d, dtype=torch.float64, device=dev)
    v = None      # V of the previous Procrustes step: warm start of the next
    sweeps = []
    cb = None
    obj = torch.empty(max(outer_iters, 0), dtype=torch.float64, device=dev)
    rots, books = [], []
    for it in range(outer_iters):
        y = rotate(x, r)
        if cb is None:
            cb = pq_fit(y, m, ks, pq_iters, init_rows=init_rows, precision=precision, labels=False,
                        objective=False)["codebook"]
        else:
            cb = pq_fit(y, m, ks, pq_iters, init_codebook=cb, precision=precision, labels=False,
                        objective=False)["codebook"]
        codes = pq_encode(y, cb, precision)
        yh, _ = pq_decode_rmse(codes, cb, x_hat=True)
        r, _, sw, v = procrustes(x, yh, v_init=v, return_v=True)
        sweeps.append(sw)
        _, sr = pq_decode_rmse(codes, cb, rotate(x, r))
        obj[it:it + 1].copy_(sr[0:1])
        if history:
            rots.append(r)
            books.append(cb)
    if cb is None:
        raise ValueError("outer_iters must be >= 1")
    out = {"R": r, "codebook": cb, "objective": obj, "sweeps": sweeps}
    if history:
        out["rotations"] = rots
        out["codebooks"] = books
    return out


def opq_encode(x: torch.Tensor, rotation: torch.Tensor, codebook: torch.Tensor, precision="bf16"):
    """Codes of the rotated rows x R."""
    return pq_encode(rotate(x, rotation), codebook, precision)


class BatchedFit:
    """Fit + encode of many independent problems sharing d, m and ks, every
    phase one launch over all problems (``mipq_pq_fit_batched``).

    ``xs``: list of float32 [n_i, d] device tensors; ``init_rows``: list of
    int64 [m, ks] device tensors (rows of the matching x).  With ``plan`` the
    grid and kernel variant are fixed once (``autotune``: looked up in the
    tuning cache, else timed on the problems and stored; ``retune`` ignores
    the cache) and, with ``graph``, the launches are replayed from HIP graphs;
    ``deterministic`` forms the float64 centroid sums in a fixed order (needs
    a plan).
    ``run()`` fills ``results[i]`` = dict(codebook, codes, sse_rmse,
    objective).
    """

    def __init__(self, xs, init_rows, m: int, ks: int, iters: int, precision="bf16", plan: bool = True,
                 autotune: bool = True, graph: bool = True, objective: bool = True, sse: bool = True,
                 codebooks: torch.Tensor | None = None, deterministic: bool = False, retune: bool = False):
        L = lib()
        if len(xs) != len(init_rows) or not xs:
            raise ValueError("need one init_rows tensor per problem (and at least one problem)")
        self.xs = [_dev(x, torch.float32, "xs[%d]" % i) for i, x in enumerate(xs)]
        self.init_rows = [_dev(r, torch.int64, "init_rows[%d]" % i) for i, r in enumerate(init_rows)]
        dev = self.xs[0].device
        d = self.xs[0].shape[1]
        if any(x.dim() != 2 or x.shape[1] != d for x in self.xs):
            raise ValueError("every problem needs rows of the same width")
        if any(r.shape != (m, ks) for r in self.init_rows):
            raise ValueError("init_rows must be [m, ks] per problem")
        self.device, self.d, self.m, self.ks, self.iters = dev, d, m, ks, iters
        self.precision = _prec(precision)
        ds = d // m if m else 0
        self.results = []
        table = (MipqProblem * len(self.xs))()
        if codebooks is not None:   # caller's contiguous [nprob, m, ks, ds] storage
            if codebooks.shape != (len(self.xs), m, ks, ds) or not codebooks.is_contiguous():
                raise ValueError("codebooks must be a contiguous [nprob, m, ks, d/m] tensor")
            codebooks = _dev(codebooks, torch.float32, "codebooks")
        self.codebooks = codebooks
        for i, (x, r) in enumerate(zip(self.xs, self.init_rows)):
            res = {"codebook": codebooks[i] if codebooks is not None else
                   torch.empty((m, ks, ds), dtype=torch.float32, device=dev),
                   "codes": torch.empty((x.shape[0], m), dtype=torch.uint8, device=dev)}
            if sse:
                res["sse_rmse"] = torch.empty(2, dtype=torch.float64, device=dev)
            if objective:
                res["objective"] = torch.empty(max(iters, 1), dtype=torch.float64, device=dev)
            self.results.append(res)
            table[i] = MipqProblem(x.data_ptr(), x.shape[0], r.data_ptr(), res["codebook"].data_ptr(),
                                   res["codes"].data_ptr(), _ptr(res.get("sse_rmse")), _ptr(res.get("objective")))
        self._table = table
        sizes = (ctypes.c_int64 * len(self.xs))(*[x.shape[0] for x in self.xs])
        nbytes = L.mipq_pq_fit_batched_workspace_size(sizes, len(self.xs), d, m, ks, iters, self.precision)
        if nbytes == 0:
            check(L.mipq_pq_fit_batched(table, len(self.xs), d, m, ks, iters, self.precision, None, None, None, 0,
                                        _stream(dev)))
        self.ws = _ws(nbytes, dev)
        self._plan = ctypes.c_void_p()
        if deterministic and not plan:
            raise ValueError("deterministic batched fits need a plan (plan=True)")
        if plan:
            flags = ((PLAN_AUTOTUNE if autotune else 0) | (PLAN_GRAPH if graph else 0) |
                     (PLAN_DETERMINISTIC if deterministic else 0) | (PLAN_RETUNE if retune else 0))
            check(L.mipq_plan_create(ctypes.byref(self._plan), table, len(self.xs), d, m, ks, iters, self.precision,
                                     flags, _ptr(self.ws), self.ws.numel(), _stream(dev)))

    def run(self, rescored: bool = False):
        """Enqueue the whole batched fit + encode on torch's current stream."""
        resc = torch.zeros(1, dtype=torch.int64, device=self.device) if rescored else None
        check(lib().mipq_pq_fit_batched(self._table, len(self.xs), self.d, self.m, self.ks, self.iters,
                                        self.precision, self._plan if self._plan.value else None, _ptr(resc),
                                        _ptr(self.ws), self.ws.numel(), _stream(self.device)))
        return resc

    def info(self) -> dict:
        """Plan choices: assignment grid and variant, resident blocks, graphs,
        whether the choice came from the tuning cache, and the candidates this
        plan timed as (grid, variant, nanoseconds per launch)."""
        if not self._plan.value:
            return {}
        n = 6 + 3 * 16
        buf = (ctypes.c_int64 * n)()
        check(lib().mipq_plan_info(self._plan, buf, n))
        k = min(int(buf[5]), 16)
        return {"grid": int(buf[0]), "resident": int(buf[1]), "graph": bool(buf[2]), "variant": int(buf[3]),
                "cached": bool(buf[4]),
                "candidates": [tuple(int(buf[6 + 3 * i + j]) for j in range(3)) for i in range(k)]}

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            lib().mipq_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pq_fit_batched(xs, init_rows, m: int, ks: int, iters: int, precision="bf16", plan: bool = False,
                   autotune: bool = False, graph: bool = False):
    """One-shot batched fit + encode; returns the list of per-problem result dicts."""
    b = BatchedFit(xs, init_rows, m, ks, iters, precision, plan=plan, autotune=autotune, graph=graph)
    b.run()
    torch.cuda.current_stream(b.device).synchronize()
    b.close()
    return b.results


def two_level_fit(xs, chunk_inits, global_init, m: int, ks: int, iters: int, precision="bf16"):
    """The paper's two-level chunked fit (Section 3), composed from the
    boundary calls: every chunk is fitted on its own rows, each chunk's
    codebook is decoded into its Ks centroid rows (the decode of the code rows
    (k, k, ..., k)), the rows of all chunks are pooled, and one global
    codebook is fitted on the pool from ``global_init`` (int64 [m, ks], rows
    of the pool).  The chunk fits are one batched fit of all chunks in BF16
    when d/m <= 16 and ``precision`` is not FP32; otherwise one ``pq_fit`` per
    chunk in ``precision`` (FP32 for wider subspaces).

    Returns dict(pool float32 [chunks*ks, d], codebook float32 [m, ks, d/m],
    chunk_codebooks list).
    """
    dev = xs[0].device
    d = xs[0].shape[1]
    ds = d // m
    books = torch.empty((len(xs), m, ks, ds), dtype=torch.float32, device=dev)
    if ds > 16 or _prec(precision) == FP32:
        cp = FP32 if ds > 16 else _prec(precision)
        for i, (x, ini) in enumerate(zip(xs, chunk_inits)):
            pq_fit(x, m, ks, iters, init_rows=ini, precision=cp, labels=False, objective=False, out=books[i])
        chunk_books = list(books.unbind(0))
    else:
        b = BatchedFit(xs, chunk_inits, m, ks, iters, precision="bf16", plan=False, objective=False, sse=False,
                       codebooks=books)
        b.run()
        chunk_books = [r["codebook"] for r in b.results]
    pool = decode_centroids(books)
    gp = FP32 if ds > 16 else precision
    g = pq_fit(pool, m, ks, iters, init_rows=global_init, precision=gp, labels=False, objective=False)
    return {"pool": pool, "codebook": g["codebook"], "chunk_codebooks": chunk_books}


def decode_centroids(codebooks: torch.Tensor) -> torch.Tensor:
    """[nbooks, m, ks, ds] codebooks -> float32 [nbooks*ks, m*ds]: row b*ks + k
    is the decode of the code row (k, ..., k) with codebook b."""
    cb = _dev(codebooks, torch.float32, "codebooks")
    nb, m, ks, ds = cb.shape
    out = torch.empty((nb * ks, m * ds), dtype=torch.float32, device=cb.device)
    check(lib().mipq_pq_decode_centroids(_ptr(cb), nb, m * ds, m, ks, _ptr(out), _stream(cb.device)))
    return out


def peak_probe(kind: str, blocks: int, buf: torch.Tensor) -> float:
    """Enqueue one probe launch (mipq_peak_probe) on the current stream of
    buf's device; returns the work of the launch (lane instructions, flops or
    bytes moved)."""
    from ._lib import PROBES
    if kind not in PROBES:
        raise ValueError("unknown probe %r" % kind)
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("probe buffer must be a contiguous device tensor")
    w = ctypes.c_double(0)
    check(lib().mipq_peak_probe(PROBES[kind], int(blocks), _ptr(buf), buf.numel() * buf.element_size(),
                                ctypes.byref(w), _stream(buf.device)))
    return w.value
