"""Accuracy sweep of the trade-off between the number of subspaces M and the
code size Ks (paper Section 2.1 and its Figure 1: RMSE falls as either
grows; the chunked fit stays close to the single one) on rows shaped like the
paper's data (d = 48, so d/m = 48, 24, 12, 6, 3: the wide subspaces run in
FP32, the others in BF16 with padded subspace blocks).

Every sweep point is first checked round by round against the oracle on a
small sample (labels bit for bit, float64 centroids to 1e-12), then the full
grid runs on 24 chunks of 16,750 rows with sampled codes against the oracle.
"""

import numpy as np
import pytest
import torch

import paper_2604_21645_amd as mipq
from oracle import pq
from synth import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
D = 48
SWEEP_M = [1, 2, 4, 8, 16]
SWEEP_KS = [16, 32, 64, 128, 256]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _prec(m):
    return "fp32" if D // m > 16 else "bf16"


@pytest.mark.parametrize("ks", [16, 256])
@pytest.mark.parametrize("m", SWEEP_M)
def test_sweep_point_lockstep_with_oracle(m, ks):
    x = wl.gaussian_mixture(60 + m, 3000, D, 50, sigma=0.08)
    init = wl.init_rows_per_subspace(60 + m, x.shape[0], m, ks, key=ks)
    prec = _prec(m)
    print("sweep point", m, ks, prec, flush=True)
    xt = _t(x)
    cb = pq.init_codebook(x, init, m).astype(np.float32)
    for _ in range(4):
        step = mipq.pq_fit(xt, m, ks, 1, init_codebook=_t(cb), precision=prec, codebook64=True)
        codes, _, _ = pq.assign(x, cb.astype(np.float64), "fp32")
        np.testing.assert_array_equal(step["labels"].cpu().numpy().astype(np.int64), codes)
        upd, _, _ = pq.update(x, codes, cb.astype(np.float64))
        np.testing.assert_allclose(step["codebook64"].cpu().numpy(), upd, rtol=1e-12, atol=1e-12)
        cb = step["codebook"].cpu().numpy()
    codes = mipq.pq_encode(xt, _t(cb), prec)
    ref, _ = pq.encode(x, cb.astype(np.float64), decide="fp32")
    np.testing.assert_array_equal(codes.cpu().numpy().astype(np.int64), ref)
    _, sr = mipq.pq_decode_rmse(codes, _t(cb), xt)
    sse, rmse = pq.sse_rmse(x, ref, cb.astype(np.float64))
    assert sr[0].item() == pytest.approx(sse, rel=1e-12) and sr[1].item() == pytest.approx(rmse, rel=1e-12)


def test_rmse_grid_single_and_two_level():
    """24 chunks x 16,750 rows x 48 from the soil-shaped mixture, 10 rounds:
    RMSE of one global fit and of the two-level fit at every (M, Ks) of the
    grid.  RMSE falls along both axes (1% slack for k-means local optima) and
    the two-level fit stays within 25% of the single fit."""
    n_chunks, rows, iters = 24, 16_750, 10
    x = wl.gaussian_mixture(6, n_chunks * rows, D, 500, sigma=0.08)
    xt = _t(x)
    xs = list(torch.split(xt, rows))
    sample = np.random.default_rng(5).choice(x.shape[0], 500, replace=False)
    single = np.zeros((len(SWEEP_M), len(SWEEP_KS)))
    two = np.zeros_like(single)
    for a, m in enumerate(SWEEP_M):
        prec = _prec(m)
        for b, ks in enumerate(SWEEP_KS):
            print("grid", m, ks, prec, flush=True)
            init = wl.init_rows_per_subspace(6, x.shape[0], m, ks, key=1000 + m * 1000 + ks)
            one = mipq.pq_fit(xt, m, ks, iters, init_rows=_t(init), precision=prec, labels=False, objective=False)
            codes = mipq.pq_encode(xt, one["codebook"], prec)
            _, sr = mipq.pq_decode_rmse(codes, one["codebook"], xt)
            single[a, b] = sr[1].item()
            cb = one["codebook"].cpu().numpy().astype(np.float64)
            ref, _ = pq.encode(x[sample], cb, decide="fp32")
            np.testing.assert_array_equal(codes.cpu().numpy()[sample].astype(np.int64), ref)
            inits = [_t(wl.init_rows_per_subspace(6, rows, m, ks, key=c)) for c in range(n_chunks)]
            ginit = wl.init_rows_per_subspace(6, n_chunks * ks, m, ks, key=n_chunks + 1)
            out = mipq.two_level_fit(xs, inits, _t(ginit), m, ks, iters, precision=prec)
            codes2 = mipq.pq_encode(xt, out["codebook"], prec)
            _, sr2 = mipq.pq_decode_rmse(codes2, out["codebook"], xt)
            two[a, b] = sr2[1].item()
            cb2 = out["codebook"].cpu().numpy().astype(np.float64)
            ref2, _ = pq.encode(x[sample], cb2, decide="fp32")
            np.testing.assert_array_equal(codes2.cpu().numpy()[sample].astype(np.int64), ref2)
    print("RMSE single fit (rows M = %s, columns Ks = %s)" % (SWEEP_M, SWEEP_KS), flush=True)
    print(np.array2string(single, precision=5), flush=True)
    print("RMSE two-level fit", flush=True)
    print(np.array2string(two, precision=5), flush=True)
    print("relative gap", flush=True)
    print(np.array2string((two - single) / single, precision=4), flush=True)
    assert np.all(np.isfinite(single)) and np.all(np.isfinite(two))
    for r in (single, two):
        assert np.all(r[:, 1:] <= r[:, :-1] * 1.01), "RMSE must fall with Ks"
        assert np.all(r[1:, :] <= r[:-1, :] * 1.01), "RMSE must fall with M"
    assert np.all(np.abs(two - single) / single < 0.25)
