"""GPU parity of the paper's two-level chunked fit (Section 3): per-chunk
fits (batched), pooled decoded centroids, a global fit on the pool; and the
RMSE of the two-level codebook beside a single global fit."""

import numpy as np
import pytest
import torch

import paper_2604_21645_amd as mipq
from oracle import chunked, pq
from synth import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _chunks(sizes, d, m, ks, seed):
    total = int(sum(sizes))
    allx = wl.gaussian_mixture(seed, total, d, 40, mean_hi=255.0, sigma=20.0, integer_clip=(0, 255))
    xs, inits, off = [], [], 0
    for i, n in enumerate(sizes):
        xs.append(allx[off:off + n])
        off += n
        inits.append(wl.init_rows_per_subspace(seed, n, m, ks, key=i))
    return allx, xs, inits


def test_two_level_fit_matches_oracle():
    m, ks, iters, d = 8, 32, 5, 64
    allx, xs, inits = _chunks([500, 1203, 777, 2048, 64], d, m, ks, seed=41)
    ginit = wl.init_rows_per_subspace(41, len(xs) * ks, m, ks, key=99)
    out = mipq.two_level_fit([_t(x) for x in xs], [_t(i) for i in inits], _t(ginit), m, ks, iters)
    ref = chunked.two_level_fit(xs, inits, ginit, m, iters, decide="fp32")
    # integer rows: every chunk fit is exact, so the pool is bit-identical
    np.testing.assert_array_equal(out["pool"].cpu().numpy(), ref["pool"])
    cb = out["codebook"].cpu().numpy()
    np.testing.assert_allclose(cb, ref["codebook"], rtol=1e-6, atol=1e-6)
    # lockstep: all rows encoded with the GPU codebook equal the oracle's codes
    codes = mipq.pq_encode(_t(allx), out["codebook"], "bf16").cpu().numpy().astype(np.int64)
    cref, _ = pq.encode(allx, cb.astype(np.float64), decide="fp32")
    np.testing.assert_array_equal(codes, cref)


def test_two_level_rmse_beside_a_single_global_fit():
    """The paper reports a negligible RMSE difference between the chunked
    and the single fit; print the relative gap on a 16-chunk workload."""
    m, ks, iters, d = 16, 256, 10, 128
    sizes = [20000 + 997 * i for i in range(16)]
    allx, xs, inits = _chunks(sizes, d, m, ks, seed=42)
    ginit = wl.init_rows_per_subspace(42, len(xs) * ks, m, ks, key=99)
    out = mipq.two_level_fit([_t(x) for x in xs], [_t(i) for i in inits], _t(ginit), m, ks, iters)
    xt = _t(allx)
    codes = mipq.pq_encode(xt, out["codebook"], "bf16")
    _, sr2 = mipq.pq_decode_rmse(codes, out["codebook"], xt)
    init1 = wl.init_rows_per_subspace(42, allx.shape[0], m, ks, key=98)
    one = mipq.pq_fit(xt, m, ks, iters, init_rows=_t(init1), precision="bf16", labels=False)
    _, sr1 = mipq.pq_decode_rmse(mipq.pq_encode(xt, one["codebook"], "bf16"), one["codebook"], xt)
    r2, r1 = sr2[1].item(), sr1[1].item()
    print("RMSE two-level %.4f single %.4f relative gap %.4f" % (r2, r1, (r2 - r1) / r1), flush=True)
    assert np.isfinite(r2) and r2 > 0 and abs(r2 - r1) / r1 < 0.25


def test_decode_centroids_is_the_transposed_codebooks():
    rng = np.random.default_rng(3)
    books = rng.standard_normal((5, 6, 37, 8)).astype(np.float32)
    out = mipq.decode_centroids(_t(books)).cpu().numpy()
    ref = np.concatenate([chunked.decoded_centroids(b) for b in books])
    np.testing.assert_array_equal(out, ref)


def test_soil_shaped_two_level_pipeline_sampled():
    """400 chunks x 16,750 rows x 48 (ds = 6): two-level fit, encode all rows,
    RMSE; sampled codes and the pool against the oracle."""
    w = wl.soil_chunks()
    xt = _t(w.x)
    xs = list(torch.split(xt, w.chunk_rows))
    out = mipq.two_level_fit(xs, [_t(i) for i in w.chunk_inits], _t(w.global_init), w.m, w.ks, w.iters)
    pool = out["pool"].cpu().numpy()
    books = [b.cpu().numpy() for b in out["chunk_codebooks"]]
    for c in (0, 199, 399):
        np.testing.assert_array_equal(pool[c * w.ks:(c + 1) * w.ks], chunked.decoded_centroids(books[c]))
        rows = np.random.default_rng(c).choice(w.chunk_rows, 200, replace=False)
        # encoding a chunk with its own codebook follows the exact rule
        xc = w.chunks[c]
        codes = mipq.pq_encode(_t(xc), out["chunk_codebooks"][c], "bf16").cpu().numpy().astype(np.int64)
        ref, _ = pq.encode(xc[rows], books[c].astype(np.float64), decide="fp32")
        np.testing.assert_array_equal(codes[rows], ref)
    cb = out["codebook"]
    codes = mipq.pq_encode(xt, cb, "bf16")
    _, sr = mipq.pq_decode_rmse(codes, cb, xt)
    rows = np.random.default_rng(9).choice(w.x.shape[0], 3000, replace=False)
    ref, _ = pq.encode(w.x[rows], cb.cpu().numpy().astype(np.float64), decide="fp32")
    np.testing.assert_array_equal(codes.cpu().numpy()[rows].astype(np.int64), ref)
    print("soil-shaped two-level RMSE %.5f" % sr[1].item(), flush=True)
    assert np.isfinite(sr[1].item())
