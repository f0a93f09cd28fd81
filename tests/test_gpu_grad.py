"""GPU parity of the reconstruction-loss backward (codes fixed) and its
torch.autograd.Function: against the oracle's analytic gradient, against
central finite differences of the GPU loss (h = 1e-3 on the float32 value,
realised step), and the k-means identity dL/dC = 0 right after an update."""

import numpy as np
import pytest
import torch

import paper_2604_21645_amd as mipq
from oracle import grad as ograd
from oracle import pq
from synth import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _setup(n=20011, d=256, m=32, ks=256, seed=5):
    x = wl.gaussian_mixture(seed, n, d, 300, sigma=0.1)
    rng = np.random.default_rng(seed)
    rows = np.stack([rng.choice(n, size=ks, replace=False) for _ in range(m)])
    cb = (pq.init_codebook(x, rows, m) + rng.standard_normal((m, ks, d // m)) * 0.01).astype(np.float32)
    codes = mipq.pq_encode(_t(x), _t(cb), "bf16")
    return x, cb, codes


def _check_grads(x, cb, codes_np, g, loss, gx, gc):
    lref, gxr, gcr = ograd.grads(x, codes_np, cb.astype(np.float64), g=g)
    assert float(loss) == pytest.approx(lref, rel=1e-12)
    # dL/dx: both sides form 2g(x - x_hat) in float64 and round once to float32
    np.testing.assert_array_equal(gx, gxr.astype(np.float32))
    # dL/dC: float64 sums in different orders; bound by the size of the terms
    m, ks, ds = cb.shape
    scale = np.zeros_like(gcr)
    for j in range(m):
        cnt = np.bincount(codes_np[:, j], minlength=ks).astype(np.float64)
        absx = np.abs(x[:, j * ds:(j + 1) * ds]).astype(np.float64)
        sabs = np.stack([np.bincount(codes_np[:, j], weights=absx[:, t], minlength=ks) for t in range(ds)], 1)
        scale[j] = 2 * abs(g) * (cnt[:, None] * np.abs(cb[j]) + sabs)
    err = np.abs(gc.astype(np.float64) - gcr)
    assert np.all(err <= 1e-12 * scale + 2.0 ** -23 * np.abs(gcr) + 1e-30)


@pytest.mark.parametrize("g", [1.0, -0.37])
def test_backward_matches_oracle_gradient(g):
    x, cb, codes = _setup()
    loss, gx, gc = mipq.recon_backward(_t(x), _t(cb), codes, grad_out=torch.tensor([g], dtype=torch.float64))
    _check_grads(x, cb, codes.cpu().numpy().astype(np.int64), g, loss.item(), gx.cpu().numpy(),
                 gc.cpu().numpy())


def test_autograd_function_and_upstream_scaling():
    x, cb, codes = _setup(n=5003, d=64, m=8, ks=64)
    xt = _t(x).requires_grad_(True)
    ct = _t(cb).requires_grad_(True)
    loss = mipq.PQReconLoss.apply(xt, ct, codes)
    (3.0 * loss).backward()
    _, gx, gc = mipq.recon_backward(_t(x), _t(cb), codes, grad_out=torch.tensor([3.0], dtype=torch.float64))
    assert torch.equal(xt.grad, gx) and torch.equal(ct.grad, gc)
    ref, _, _ = ograd.grads(x, codes.cpu().numpy().astype(np.int64), cb.astype(np.float64))
    assert loss.item() == pytest.approx(ref, rel=1e-12)


def test_loss_from_the_encodes_fused_error():
    # the encode's fused error as the forward: the same loss (float64 sums in
    # another order) and the same gradients
    x, cb, _ = _setup(n=20011, d=256, m=32, ks=256, seed=8)
    r = mipq.pq_encode_ex(_t(x), _t(cb), "bf16", sse_rmse=True)
    codes = r["codes"]
    xt = _t(x).requires_grad_(True)
    ct = _t(cb).requires_grad_(True)
    loss = mipq.PQReconLoss.apply(xt, ct, codes, r["sse_rmse"])
    loss.backward()
    x2 = _t(x).requires_grad_(True)
    c2 = _t(cb).requires_grad_(True)
    ref = mipq.PQReconLoss.apply(x2, c2, codes)
    ref.backward()
    assert loss.item() == pytest.approx(ref.item(), rel=1e-12)
    assert torch.equal(xt.grad, x2.grad) and torch.equal(ct.grad, c2.grad)
    lref, _, _ = ograd.grads(x, codes.cpu().numpy().astype(np.int64), cb.astype(np.float64))
    assert loss.item() == pytest.approx(lref, rel=1e-12)


def test_central_finite_differences_on_1000_entries():
    x, cb, codes = _setup(n=20011, d=256, m=32, ks=256, seed=6)
    xt, ct = _t(x), _t(cb)
    _, gx, gc = mipq.recon_backward(xt, ct, codes)
    gx, gc = gx.cpu().numpy().astype(np.float64), gc.cpu().numpy().astype(np.float64)
    cbe, xe = wl.fd_entries(6, x.shape[0], x.shape[1], 32, 256, 8, count=1000)
    h = 1e-3

    def loss_at(xx, cc):
        _, sr = mipq.pq_decode_rmse(codes, cc, xx)
        return sr[0].item()

    worst = 0.0
    for j, k, t in cbe:
        c0 = cb[j, k, t]
        cp, cm = np.float32(c0 + h), np.float32(c0 - h)
        ct[j, k, t] = float(cp)
        lp = loss_at(xt, ct)
        ct[j, k, t] = float(cm)
        lm = loss_at(xt, ct)
        ct[j, k, t] = float(c0)
        fd = (lp - lm) / (float(cp) - float(cm))
        worst = max(worst, abs(fd - gc[j, k, t]) / max(abs(gc[j, k, t]), 1.0))
    for r, c in xe:
        v0 = x[r, c]
        vp, vm = np.float32(v0 + h), np.float32(v0 - h)
        xt[r, c] = float(vp)
        lp = loss_at(xt, ct)
        xt[r, c] = float(vm)
        lm = loss_at(xt, ct)
        xt[r, c] = float(v0)
        fd = (lp - lm) / (float(vp) - float(vm))
        worst = max(worst, abs(fd - gx[r, c]) / max(abs(gx[r, c]), 1.0))
    print("worst relative FD error", worst, flush=True)
    assert worst < 1e-4


def test_codebook_gradient_vanishes_after_an_update():
    w = wl.plain_pq(seed=8, n=6000, m=8, ks=64, iters=3)
    fit = mipq.pq_fit(_t(w.x), w.m, w.ks, 1, init_rows=_t(w.init_rows), precision="bf16", codebook64=True)
    codes = fit["labels"]           # the assignment the update averaged
    cb32 = fit["codebook"]
    _, _, gc = mipq.recon_backward(_t(w.x), cb32, codes, grad_x=False)
    # cnt*C32 - S = cnt*(C32 - C64): only the float32 rounding of the means remains
    cnt = np.stack([np.bincount(codes.cpu().numpy()[:, j], minlength=64) for j in range(8)]).astype(np.float64)
    bound = 2 * cnt[:, :, None] * np.abs(cb32.cpu().numpy().astype(np.float64)) * 2.0 ** -23 + 1e-9
    assert np.all(np.abs(gc.cpu().numpy()) <= bound)


def test_full_size_differentiable_codebooks():
    """2M x 256 rows, M=32, Ks=256: fit 20 rounds on a 200k sample (BF16),
    encode all rows (BF16), loss and backward.  The loss and 1,000 seeded
    gradient entries (500 codebook, 500 input) against the oracle's analytic
    gradient on all rows, and the same entries against central finite
    differences (h = 1e-3, realised float32 step) of the GPU loss of all 2M
    rows."""
    w = wl.diff_codebooks()
    xt = _t(w.x)
    print("full-size differentiable codebooks: fit", flush=True)
    fit = mipq.pq_fit(xt, w.m, w.ks, w.iters, init_rows=_t(w.init_rows), train_rows=_t(w.train_rows),
                      precision="bf16", labels=False)
    cb = fit["codebook"]
    codes = mipq.pq_encode(xt, cb, "bf16")
    loss, gx, gc = mipq.recon_backward(xt, cb, codes)
    cbn = cb.cpu().numpy().astype(np.float64)
    cn = codes.cpu().numpy().astype(np.int64)
    print("oracle gradient on all rows", flush=True)
    lref, gxr, gcr = ograd.grads(w.x, cn, cbn)
    assert loss.item() == pytest.approx(lref, rel=1e-11)
    ds = w.x.shape[1] // w.m
    cbe, xe = wl.fd_entries(5, w.x.shape[0], w.x.shape[1], w.m, w.ks, ds, count=1000)
    gxn = gx.cpu().numpy()
    np.testing.assert_array_equal(gxn[xe[:, 0], xe[:, 1]], gxr[xe[:, 0], xe[:, 1]].astype(np.float32))
    gcn = gc.cpu().numpy().astype(np.float64)
    for j in np.unique(cbe[:, 0]):
        sel = cbe[cbe[:, 0] == j]
        lab = cn[:, j]
        cnt = np.bincount(lab, minlength=w.ks).astype(np.float64)
        absx = np.abs(w.x[:, j * ds:(j + 1) * ds]).astype(np.float64)
        sabs = np.stack([np.bincount(lab, weights=absx[:, t], minlength=w.ks) for t in range(ds)], 1)
        scale = 2.0 * (cnt[:, None] * np.abs(cbn[j]) + sabs)   # float64 sums in different orders
        for _, k, t in sel:
            assert abs(gcn[j, k, t] - gcr[j, k, t]) <= 1e-12 * scale[k, t] + 2.0 ** -23 * abs(gcr[j, k, t]) + 1e-30
    del gxr
    print("finite differences on 1,000 entries of the 2M-row loss", flush=True)
    h = 1e-3
    ct = cb.clone()

    def loss_at(xx, cc):
        _, sr = mipq.pq_decode_rmse(codes, cc, xx)
        return sr[0].item()

    worst = 0.0
    for j, k, t in cbe:
        c0 = float(ct[j, k, t].item())
        cp, cm = np.float32(c0 + h), np.float32(c0 - h)
        ct[j, k, t] = float(cp)
        lp = loss_at(xt, ct)
        ct[j, k, t] = float(cm)
        lm = loss_at(xt, ct)
        ct[j, k, t] = c0
        fd = (lp - lm) / (float(cp) - float(cm))
        worst = max(worst, abs(fd - gcn[j, k, t]) / max(abs(gcn[j, k, t]), 1.0))
    for r, c in xe:
        v0 = float(w.x[r, c])
        vp, vm = np.float32(v0 + h), np.float32(v0 - h)
        xt[r, c] = float(vp)
        lp = loss_at(xt, ct)
        xt[r, c] = float(vm)
        lm = loss_at(xt, ct)
        xt[r, c] = v0
        fd = (lp - lm) / (float(vp) - float(vm))
        worst = max(worst, abs(fd - float(gxn[r, c])) / max(abs(float(gxn[r, c])), 1.0))
    print("worst relative FD error on the 2M-row loss", worst, flush=True)
    assert worst < 1e-4
