"""GPU parity of the PQ hot path (fit, encode, decode + RMSE) against the CPU oracle.

Every call goes through the C ABI (paper_2604_21645_amd -> libmipq.so).  Codes
must equal the oracle's float32-decision codes bit for bit in every precision,
and the float64 oracle's codes outside its near-ties; centroids, objective and
RMSE are compared with tolerances derived from float64 summation order.
"""

import os

import numpy as np
import pytest
import torch

import paper_2604_21645_amd as mipq
from oracle import pq
from synth import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _data(kind, n, d, seed):
    if kind == "integer":
        return wl.gaussian_mixture(seed, n, d, 50, mean_hi=255.0, sigma=20.0, integer_clip=(0, 255))
    return wl.gaussian_mixture(seed, n, d, 40, sigma=0.05)


def _codebook(x, m, ks, seed):
    """float32 codebook from seeded rows, jittered so equal rows do not tie."""
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    rows = np.stack([rng.choice(n, size=ks, replace=ks > n) for _ in range(m)])
    cb = pq.init_codebook(x, rows, m)
    cb = cb + rng.standard_normal(cb.shape) * (np.abs(cb).mean() * 1e-3)
    return cb.astype(np.float32)


ENCODE_CASES = [
    dict(n=3001, d=128, m=16, ks=256, kind="integer"),   # ds=8, ragged tail
    dict(n=2077, d=128, m=8, ks=256, kind="float"),      # ds=16
    dict(n=1000, d=64, m=16, ks=100, kind="float"),      # ds=4, partial tile
    dict(n=513, d=36, m=12, ks=16, kind="float"),        # ds=3, one tile
    dict(n=700, d=96, m=8, ks=200, kind="float"),        # ds=12, two 8-dim blocks
    dict(n=77, d=40, m=8, ks=1, kind="float"),           # ks=1, ds=5
    dict(n=1, d=96, m=12, ks=256, kind="float"),         # single row
    dict(n=33, d=128, m=16, ks=64, kind="integer"),      # one row past a tile
]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("case", ENCODE_CASES, ids=lambda c: "n%(n)d_d%(d)d_m%(m)d_ks%(ks)d" % c)
def test_encode_matches_oracle(prec, case):
    print("encode", prec, case, flush=True)
    x = _data(case["kind"], case["n"], case["d"], seed=case["n"])
    cb = _codebook(x, case["m"], case["ks"], seed=case["d"])
    codes = mipq.pq_encode(_t(x), _t(cb), prec).cpu().numpy().astype(np.int64)
    ref32, _, _ = pq.assign(x, cb.astype(np.float64), "fp32")
    np.testing.assert_array_equal(codes, ref32)
    ref64, _, tie = pq.assign(x, cb.astype(np.float64), "fp64")
    assert np.all(codes[~tie] == ref64[~tie])


def test_encode_empty_input():
    x = torch.empty((0, 128), dtype=torch.float32, device=DEV)
    cb = torch.zeros((16, 256, 8), dtype=torch.float32, device=DEV)
    for prec in ("fp32", "bf16"):
        assert mipq.pq_encode(x, cb, prec).shape == (0, 16)


def test_bf16_and_fp32_agree_on_duplicate_rows_and_ties():
    # duplicated centroids and rows equidistant from several centroids: every
    # such pair is ambiguous for the matrix cores and decided by the exact rule
    rng = np.random.default_rng(3)
    cb = rng.integers(0, 4, size=(16, 64, 8)).astype(np.float32)
    cb[:, 32:] = cb[:, :32]
    x = rng.integers(0, 4, size=(2000, 128)).astype(np.float32)
    a = mipq.pq_encode(_t(x), _t(cb), "fp32").cpu().numpy()
    b, resc = mipq.pq_encode(_t(x), _t(cb), "bf16", rescored=True)
    np.testing.assert_array_equal(a, b.cpu().numpy())
    ref32, _, _ = pq.assign(x, cb.astype(np.float64), "fp32")
    np.testing.assert_array_equal(a.astype(np.int64), ref32)
    assert int(resc.item()) > 0


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_fit_end_to_end_and_lockstep(prec):
    w = wl.plain_pq(seed=1, n=4000, m=8, ks=64, iters=6)
    print("fit", prec, flush=True)
    out = mipq.pq_fit(_t(w.x), w.m, w.ks, w.iters, init_rows=_t(w.init_rows), precision=prec,
                      codebook64=True)
    ref = pq.lloyd(w.x, w.init_rows, w.m, w.iters, decide="fp32")
    np.testing.assert_array_equal(out["labels"].cpu().numpy().astype(np.int64), ref["codes"])
    np.testing.assert_allclose(out["codebook64"].cpu().numpy(), ref["codebook"], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(out["codebook"].cpu().numpy(), ref["codebook"].astype(np.float32))
    np.testing.assert_allclose(out["objective"].cpu().numpy(), ref["objective"], rtol=1e-12)
    # lockstep: one round at a time from the GPU's own centroids
    cb = pq.init_codebook(w.x, w.init_rows, w.m).astype(np.float32)
    for _ in range(3):
        step = mipq.pq_fit(_t(w.x), w.m, w.ks, 1, init_codebook=_t(cb), precision=prec, codebook64=True)
        codes, _, _ = pq.assign(w.x, cb.astype(np.float64), "fp32")
        np.testing.assert_array_equal(step["labels"].cpu().numpy().astype(np.int64), codes)
        upd, _, _ = pq.update(w.x, codes, cb.astype(np.float64))
        np.testing.assert_allclose(step["codebook64"].cpu().numpy(), upd, rtol=1e-12, atol=1e-12)
        cb = step["codebook"].cpu().numpy()


def test_fp8_outlier_rows_and_rescoring_counts():
    # rows far outside the centroid range saturate the fp8 operands; their
    # residuals widen the bound and the exact rule decides them
    x = _data("float", 4000, 128, seed=21)
    cb = _codebook(x, 16, 256, seed=22)
    x[::97] *= 1e4
    x[5::131] = -3e6
    codes, resc = mipq.pq_encode(_t(x), _t(cb), "fp8", rescored=True)
    ref32, _, _ = pq.assign(x, cb.astype(np.float64), "fp32")
    np.testing.assert_array_equal(codes.cpu().numpy().astype(np.int64), ref32)
    _, resc16 = mipq.pq_encode(_t(x), _t(cb), "bf16", rescored=True)
    print("rescored pairs fp8", int(resc.item()), "bf16", int(resc16.item()), "of", x.shape[0] * 16, flush=True)
    assert int(resc.item()) >= int(resc16.item())


def test_fit_on_a_row_sample_with_empty_clusters():
    w = wl.integer_pq(seed=2, n=20000, n_comp=30, m=16, ks=256, iters=4, n_train=5000)
    # duplicate init rows force empty clusters (the later duplicate never wins)
    init = w.init_rows.copy()
    init[:, 200:] = init[:, :56]
    out = mipq.pq_fit(_t(w.x), w.m, w.ks, w.iters, init_rows=_t(init), train_rows=_t(w.train_rows),
                      precision="bf16", codebook64=True)
    ref = pq.lloyd(w.train, init, w.m, w.iters, decide="fp32")
    np.testing.assert_array_equal(out["labels"].cpu().numpy().astype(np.int64), ref["codes"])
    # integer rows: float64 sums are exact in any order, centroids are identical
    np.testing.assert_array_equal(out["codebook64"].cpu().numpy(), ref["codebook"])


@pytest.mark.parametrize("m,ks", [(16, 256), (8, 37)])
def test_decode_rmse_matches_oracle(m, ks):
    x = _data("float", 5003, 128, seed=9)
    cb = _codebook(x, m, ks, seed=10)
    codes = mipq.pq_encode(_t(x), _t(cb), "bf16")
    xh, sr = mipq.pq_decode_rmse(codes, _t(cb), _t(x), x_hat=True)
    c = codes.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(xh.cpu().numpy(), pq.decode(c, cb.astype(np.float64)).astype(np.float32))
    sse, rmse = pq.sse_rmse(x, c, cb.astype(np.float64))
    got = sr.cpu().numpy()
    assert got[0] == pytest.approx(sse, rel=1e-12)
    assert got[1] == pytest.approx(rmse, rel=1e-12)


def test_full_size_integer_workload_sampled_parity():
    """1M x 128 integer rows, 100k-row sample, M=16, Ks=256, 25 rounds: the
    bench workload.  BF16 and FP32 produce identical codes on all 1M rows;
    sampled rows equal the oracle's."""
    w = wl.integer_pq()
    xt = _t(w.x)
    fit = mipq.pq_fit(xt, w.m, w.ks, w.iters, init_rows=_t(w.init_rows), train_rows=_t(w.train_rows),
                      precision="bf16")
    cb = fit["codebook"]
    obj = fit["objective"].cpu().numpy()
    assert np.all(np.diff(obj) <= 1e-9 * obj[:-1])
    cb16, resc = mipq.pq_encode(xt, cb, "bf16", rescored=True)
    c32 = mipq.pq_encode(xt, cb, "fp32")
    assert torch.equal(cb16, c32)
    print("rescored pairs", int(resc.item()), "of", w.x.shape[0] * w.m, flush=True)
    rows = np.random.default_rng(0).choice(w.x.shape[0], 4000, replace=False)
    ref32, _, _ = pq.assign(w.x[rows], cb.cpu().numpy().astype(np.float64), "fp32")
    np.testing.assert_array_equal(cb16.cpu().numpy()[rows].astype(np.int64), ref32)


ENCODE_OUT_CASES = [
    dict(n=3001, d=128, m=16, ks=256, kind="integer"),   # ds=8, ragged tail
    dict(n=1500, d=96, m=8, ks=200, kind="float"),       # ds=12
    dict(n=257, d=48, m=16, ks=32, kind="float"),        # ds=3
]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("case", ENCODE_OUT_CASES, ids=lambda c: "n%(n)d_d%(d)d_m%(m)d_ks%(ks)d" % c)
def test_encode_min_dist_and_error(prec, case):
    """The distance of every (row, subspace) to its chosen centroid (the value
    the code minimises under the float32 rule) and the float64 squared error
    of the codes, from the encode call itself."""
    print("encode outputs", prec, case, flush=True)
    x = _data(case["kind"], case["n"], case["d"], seed=case["n"] + 5)
    cb = _codebook(x, case["m"], case["ks"], seed=case["d"] + 5)
    m, ds = case["m"], case["d"] // case["m"]
    r = mipq.pq_encode_ex(_t(x), _t(cb), prec, min_dist=True, sse_rmse=True, rescored=True)
    codes = r["codes"].cpu().numpy().astype(np.int64)
    ref32, _, _ = pq.assign(x, cb.astype(np.float64), "fp32")
    np.testing.assert_array_equal(codes, ref32)
    want = np.stack([pq.dist32(pq.block(x, j, ds), cb[j]).min(axis=1) for j in range(m)], axis=1)
    np.testing.assert_array_equal(r["min_dist"].cpu().numpy(), want)
    sse, rmse = pq.sse_rmse(x, codes, cb.astype(np.float64))
    got = r["sse_rmse"].cpu().numpy()
    assert got[0] == pytest.approx(sse, rel=1e-12)
    assert got[1] == pytest.approx(rmse, rel=1e-12)
    _, sr = mipq.pq_decode_rmse(r["codes"], _t(cb), _t(x))
    assert sr.cpu().numpy()[0] == pytest.approx(got[0], rel=1e-13)


def test_encode_outputs_on_empty_input():
    x = torch.empty((0, 128), dtype=torch.float32, device=DEV)
    cb = torch.zeros((16, 256, 8), dtype=torch.float32, device=DEV)
    for prec in ("fp32", "bf16"):
        r = mipq.pq_encode_ex(x, cb, prec, min_dist=True, sse_rmse=True)
        assert r["min_dist"].shape == (0, 16)
        assert r["sse_rmse"].cpu().numpy().tolist() == [0.0, 0.0]


def test_fit_reports_rescored_pairs_per_round():
    w = wl.plain_pq(seed=4, n=3000, m=8, ks=64, iters=4)
    out32 = mipq.pq_fit(_t(w.x), w.m, w.ks, w.iters, init_rows=_t(w.init_rows), precision="fp32", rescored=True)
    assert out32["rescored"].cpu().numpy().tolist() == [0] * w.iters
    out = mipq.pq_fit(_t(w.x), w.m, w.ks, w.iters, init_rows=_t(w.init_rows), precision="bf16", rescored=True)
    r = out["rescored"].cpu().numpy()
    assert r.shape == (w.iters,) and np.all(r >= 0)
    # round 0 assigns against the initial codebook: the same pairs as an encode with it
    cb0 = pq.init_codebook(w.x, w.init_rows, w.m).astype(np.float32)
    _, resc0 = mipq.pq_encode(_t(w.x), _t(cb0), "bf16", rescored=True)
    assert int(r[0]) == int(resc0.item())
    print("rescored per round", r.tolist(), flush=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_check_finite_rejects_nan_and_inf(prec):
    x = _data("float", 700, 64, seed=5)
    cb = _codebook(x, 8, 32, seed=6)
    init = wl.init_rows_per_subspace(5, x.shape[0], 8, 32)
    clean = mipq.pq_encode_ex(_t(x), _t(cb), prec, check_finite=True)["codes"]
    assert torch.equal(clean, mipq.pq_encode(_t(x), _t(cb), prec))
    mipq.pq_fit(_t(x), 8, 32, 2, init_rows=_t(init), precision=prec, check_finite=True)
    for bad in (np.nan, np.inf, -np.inf):
        xb = x.copy()
        xb[123, 7] = bad
        cbb = cb.copy()
        cbb[3, 5, 1] = bad
        for call in (lambda: mipq.pq_encode_ex(_t(xb), _t(cb), prec, check_finite=True),
                     lambda: mipq.pq_encode_ex(_t(x), _t(cbb), prec, check_finite=True),
                     lambda: mipq.pq_fit(_t(xb), 8, 32, 2, init_rows=_t(init), precision=prec,
                                         check_finite=True)):
            with pytest.raises(mipq.MipqError) as e:
                call()
            assert e.value.code == mipq.ENONFINITE
    # with a training sample, only the sampled rows are checked
    xb = x.copy()
    xb[1] = np.nan
    sample = np.arange(2, x.shape[0], dtype=np.int64)
    init_s = wl.init_rows_per_subspace(6, len(sample), 8, 32)
    mipq.pq_fit(_t(xb), 8, 32, 2, init_rows=_t(init_s), train_rows=_t(sample), precision=prec, check_finite=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_deterministic_fit_repeats_bit_for_bit(prec):
    """Real-valued rows in 5 row chunks: the fixed-order float64 sums give the
    same codebook, labels and objective on every run, equal to the default
    mode's to float64 rounding and to the oracle's."""
    w = wl.plain_pq(seed=7, n=20000, m=8, ks=256, iters=4)
    print("deterministic fit", prec, flush=True)
    runs = [mipq.pq_fit(_t(w.x), w.m, w.ks, w.iters, init_rows=_t(w.init_rows), precision=prec, codebook64=True,
                        deterministic=True) for _ in range(3)]
    for r in runs[1:]:
        assert torch.equal(r["codebook64"], runs[0]["codebook64"])
        assert torch.equal(r["labels"], runs[0]["labels"])
        assert torch.equal(r["objective"], runs[0]["objective"])
    default = mipq.pq_fit(_t(w.x), w.m, w.ks, w.iters, init_rows=_t(w.init_rows), precision=prec, codebook64=True)
    np.testing.assert_allclose(runs[0]["codebook64"].cpu().numpy(), default["codebook64"].cpu().numpy(),
                               rtol=1e-12, atol=1e-12)
    ref = pq.lloyd(w.x, w.init_rows, w.m, w.iters, decide="fp32")
    np.testing.assert_allclose(runs[0]["codebook64"].cpu().numpy(), ref["codebook"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(runs[0]["objective"].cpu().numpy(), ref["objective"], rtol=1e-12)


def test_deterministic_fit_on_integer_rows_equals_the_oracle():
    # integer rows: every float64 sum is exact, so both modes equal the oracle bit for bit
    w = wl.integer_pq(seed=3, n=30000, n_comp=30, m=16, ks=256, iters=3, n_train=9000)
    out = mipq.pq_fit(_t(w.x), w.m, w.ks, w.iters, init_rows=_t(w.init_rows), train_rows=_t(w.train_rows),
                      precision="bf16", codebook64=True, deterministic=True)
    ref = pq.lloyd(w.train, w.init_rows, w.m, w.iters, decide="fp32")
    np.testing.assert_array_equal(out["labels"].cpu().numpy().astype(np.int64), ref["codes"])
    np.testing.assert_array_equal(out["codebook64"].cpu().numpy(), ref["codebook"])


@pytest.fixture(scope="module")
def plain_golden():
    return np.load(os.path.join(os.path.dirname(__file__), "golden", "plain_pq_fit.npz"), allow_pickle=False)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_plain_pq_full_shape(prec, plain_golden):
    """The plain PQ configuration at its stated shape: 10,000 x 128 rows from a
    64-component mixture (sigma 0.05), M=8 subspaces of 16 dimensions, Ks=256,
    20 Lloyd rounds from 256 seeded rows per subspace, all rows encoded, RMSE.
    Against the oracle's stored run (tests/golden/make_plain_pq_fit.py)."""
    g = plain_golden
    w = wl.plain_pq()
    assert (w.x.shape, w.m, w.ks, w.iters) == ((10000, 128), 8, 256, 20)
    xt = _t(w.x)
    print("plain_pq full shape", prec, flush=True)
    fit = mipq.pq_fit(xt, w.m, w.ks, w.iters, init_rows=_t(w.init_rows), precision=prec, codebook64=True,
                      rescored=True)
    np.testing.assert_array_equal(fit["labels"].cpu().numpy(), g["labels"])
    np.testing.assert_allclose(fit["codebook64"].cpu().numpy(), g["codebook"], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(fit["codebook"].cpu().numpy(), g["codebook"].astype(np.float32))
    np.testing.assert_allclose(fit["objective"].cpu().numpy(), g["objective"], rtol=1e-12)
    enc = mipq.pq_encode_ex(xt, fit["codebook"], prec, sse_rmse=True, rescored=True)
    codes = enc["codes"].cpu().numpy()
    np.testing.assert_array_equal(codes, g["codes"])
    tie = np.unpackbits(g["codes_near_tie"])[:codes.size].reshape(codes.shape).astype(bool)
    assert np.all(codes[~tie] == g["codes_fp64_decision"][~tie])
    sr = enc["sse_rmse"].cpu().numpy()
    assert sr[0] == pytest.approx(g["sse_rmse"][0], rel=1e-12)
    assert sr[1] == pytest.approx(g["sse_rmse"][1], rel=1e-12)
    # against a fit that decides in float64 throughout: RMSE within 1e-4 relative
    assert sr[1] == pytest.approx(g["rmse_fp64_fit"][0], rel=1e-4)
    print("near-ties per round", g["near_ties"].tolist(), "final", int(tie.sum()),
          "re-decided per round", fit["rescored"].cpu().numpy().tolist(), flush=True)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fit_encode_step_replays_from_a_graph(prec):
    """A fit + encode-with-error step captured once in a HIP graph: every
    replay, with other eager work and synchronisations between the replays and
    the outputs cleared before each, equals the eager step bit for bit."""
    w = wl.plain_pq(seed=9, n=3000, m=8, ks=256, iters=5)
    x, init = _t(w.x), _t(w.init_rows)

    def step():
        fit = mipq.pq_fit(x, w.m, w.ks, w.iters, init_rows=init, precision=prec, labels=False, objective=False)
        enc = mipq.pq_encode_ex(x, fit["codebook"], prec, sse_rmse=True, min_dist=True)
        return fit["codebook"], enc["codes"], enc["sse_rmse"], enc["min_dist"]

    ref = [t.clone() for t in step()]
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        step()
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=cs):
        out = step()
    other = _t(np.ascontiguousarray(w.x[::-1]))
    for rep in range(3):
        mipq.pq_encode_ex(other, ref[0], prec, sse_rmse=True)   # eager work between replays
        for t in out:
            t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert torch.equal(a, b), rep


FUSED_CASES = [
    dict(kind="integer", n=20000, d=128, m=16, ks=256, iters=4),   # ds=8, 8 tiles
    dict(kind="float", n=4000, d=128, m=8, ks=64, iters=6),        # ds=16: two 8-dim blocks
    dict(kind="float", n=3001, d=48, m=16, ks=100, iters=5),       # ds=3, partial tile, padded rows
    dict(kind="integer", n=130, d=64, m=8, ks=32, iters=3),        # fewer rows than one step per wave
]


@pytest.mark.parametrize("case", FUSED_CASES, ids=lambda c: "%(kind)s_n%(n)d_d%(d)d_m%(m)d_ks%(ks)d" % c)
def test_fused_rounds_match_the_oracle(case):
    """BF16 fits without the objective run each Lloyd round as one launch
    (assignment fused with the float64 sums) plus the finalize.  Labels and
    codebooks equal the oracle's float32-decision Lloyd; on integer rows the
    codebooks equal the two-pass rounds' (objective on) bit for bit."""
    x = _data(case["kind"], case["n"], case["d"], seed=case["n"] + 11)
    m, ks, iters = case["m"], case["ks"], case["iters"]
    rng = np.random.default_rng(case["n"])
    init = np.stack([rng.choice(case["n"], size=ks, replace=False) for _ in range(m)])
    print("fused rounds", case, flush=True)
    fused = mipq.pq_fit(_t(x), m, ks, iters, init_rows=_t(init), precision="bf16", codebook64=True,
                        objective=False, rescored=True)
    ref = pq.lloyd(x, init, m, iters, decide="fp32")
    np.testing.assert_array_equal(fused["labels"].cpu().numpy().astype(np.int64), ref["codes"])
    np.testing.assert_allclose(fused["codebook64"].cpu().numpy(), ref["codebook"], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(fused["codebook"].cpu().numpy(), ref["codebook"].astype(np.float32))
    two = mipq.pq_fit(_t(x), m, ks, iters, init_rows=_t(init), precision="bf16", codebook64=True,
                      objective=True, rescored=True)
    assert torch.equal(fused["rescored"], two["rescored"])
    assert torch.equal(fused["labels"], two["labels"])
    if case["kind"] == "integer":
        assert torch.equal(fused["codebook64"], two["codebook64"])


@pytest.mark.parametrize("n_train,iters", [(100_000, 25), (1_000_000, 2)])
def test_fused_rounds_at_full_size_equal_the_two_pass_rounds(n_train, iters):
    """The 1M x 128 integer workload (M=16, Ks=256): a 100k-row sample for 25
    rounds (one block round) and all 1M rows for 2 rounds (rows per wave at
    their cap, 123 chunks): fused and two-pass rounds give the same codebook
    bit for bit (integer rows: exact float64 sums in any order), the same
    labels and the same re-decided pairs per round."""
    w = wl.integer_pq(n_train=n_train)
    xt = _t(w.x)
    init = wl.init_rows_per_subspace(w.meta["seed"], n_train, w.m, w.ks)
    tr = _t(w.train_rows) if n_train < w.x.shape[0] else None
    print("fused full size", n_train, iters, flush=True)
    kw = dict(init_rows=_t(init), train_rows=tr, precision="bf16", codebook64=True, rescored=True)
    fused = mipq.pq_fit(xt, w.m, w.ks, iters, objective=False, **kw)
    two = mipq.pq_fit(xt, w.m, w.ks, iters, objective=True, **kw)
    assert torch.equal(fused["codebook64"], two["codebook64"])
    assert torch.equal(fused["labels"], two["labels"])
    assert torch.equal(fused["rescored"], two["rescored"])
    print("re-decided per round", fused["rescored"].cpu().numpy().tolist(), flush=True)
