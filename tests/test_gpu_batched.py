"""GPU parity of the batched fit + encode (many independent problems, one
launch per phase, optional plan with autotuned grid and HIP graphs).

Each problem's results must equal the single-problem calls on that problem
(pq_fit + pq_encode + pq_decode_rmse): the same code rule, the same row
chunks and reduction orders.  Integer-valued rows make every float64 sum
exact, so there the comparison is bit for bit end to end; on real-valued
rows the codes and errors are compared in lockstep (same codebook).
"""

import json
import os

import numpy as np
import pytest
import torch

import paper_2604_21645_amd as mipq
from oracle import pq
from synth import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(autouse=True, scope="module")
def _private_tune_cache(tmp_path_factory):
    """Plans of this module read and write a tuning cache of their own."""
    old = os.environ.get("MIPQ_TUNE_CACHE")
    os.environ["MIPQ_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "autotune.json")
    yield
    if old is None:
        del os.environ["MIPQ_TUNE_CACHE"]
    else:
        os.environ["MIPQ_TUNE_CACHE"] = old


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _problems(sizes, d, m, ks, kind, seed):
    total = int(sum(sizes))
    if kind == "integer":
        allx = wl.gaussian_mixture(seed, total, d, 40, mean_hi=255.0, sigma=20.0, integer_clip=(0, 255))
    else:
        allx = wl.gaussian_mixture(seed, total, d, 60, sphere_kappa=50.0)
    xs, inits, off = [], [], 0
    for i, n in enumerate(sizes):
        xs.append(allx[off:off + n])
        off += n
        inits.append(wl.init_rows_per_subspace(seed, n, m, ks, key=i))
    return xs, inits


def _single(x, init, m, ks, iters):
    xt = _t(x)
    fit = mipq.pq_fit(xt, m, ks, iters, init_rows=_t(init), precision="bf16", labels=False)
    codes = mipq.pq_encode(xt, fit["codebook"], "bf16")
    _, sr = mipq.pq_decode_rmse(codes, fit["codebook"], xt)
    return fit["codebook"], codes, sr, fit["objective"]


def _run(xs, inits, m, ks, iters, mode):
    xt = [_t(x) for x in xs]
    it = [_t(i) for i in inits]
    if mode == "eager":
        b = mipq.BatchedFit(xt, it, m, ks, iters, plan=False)
    elif mode == "plan":
        b = mipq.BatchedFit(xt, it, m, ks, iters, plan=True, autotune=False, graph=False)
    else:
        b = mipq.BatchedFit(xt, it, m, ks, iters, plan=True, autotune=True, graph=True)
    resc = b.run(rescored=True)
    torch.cuda.synchronize()
    return b, resc


SIZES = [64, 65, 97, 1000, 4097, 20011, 333]


@pytest.mark.parametrize("mode", ["eager", "plan", "graph"])
def test_integer_rows_equal_single_calls_bit_for_bit(mode):
    m, ks, iters, d = 12, 64, 5, 96
    xs, inits = _problems(SIZES, d, m, ks, "integer", seed=31)
    print("batched", mode, flush=True)
    b, resc = _run(xs, inits, m, ks, iters, mode)
    for i, (x, init) in enumerate(zip(xs, inits)):
        cb, codes, sr, obj = _single(x, init, m, ks, iters)
        r = b.results[i]
        assert torch.equal(r["codebook"], cb), i
        assert torch.equal(r["codes"], codes), i
        assert torch.equal(r["sse_rmse"], sr), i
        assert torch.equal(r["objective"], obj), i
    assert int(resc.item()) >= 0
    if mode == "graph":
        info = b.info()
        print("plan", info, flush=True)
        assert info["graph"] and info["grid"] % 8 == 0 and info["variant"] in (0, 1)
        assert info["cached"] or len(info["candidates"]) == 10
    b.close()


@pytest.mark.parametrize("mode", ["eager", "graph"])
@pytest.mark.parametrize("d,m,ks", [(96, 12, 256), (48, 6, 100), (48, 16, 16), (96, 8, 256), (64, 4, 100)])
def test_plans_without_objective_equal_single_calls(mode, d, m, ks):
    """Plans that return no objective (the benchmarked form, one fused launch
    per round; ds = 8, 8, 3, 12, 16 and Ks = 256, 100, 16, 256, 100 cover
    whole and partial 8-dimension blocks, one and two of them, and 1 to 8
    centroid tiles): on integer rows the codebooks, codes and errors equal
    the single calls bit for bit (float64 sums of integers are exact in any
    order)."""
    iters = 4
    # 300,001 rows: more chunks than the 256-block cap allows (8,192 rows at most)
    xs, inits = _problems([ks, 4097, 20011, 333, 9000, 300001], d, m, ks, "integer", seed=35)
    xt = [_t(x) for x in xs]
    it = [_t(i) for i in inits]
    print("no objective", mode, d, m, ks, flush=True)
    b = mipq.BatchedFit(xt, it, m, ks, iters, plan=mode == "graph", autotune=False, graph=mode == "graph",
                        objective=False)
    b.run()
    torch.cuda.synchronize()
    for i, (x, init) in enumerate(zip(xs, inits)):
        cb, codes, sr, _ = _single(x, init, m, ks, iters)
        r = b.results[i]
        assert "objective" not in r
        assert torch.equal(r["codebook"], cb), i
        assert torch.equal(r["codes"], codes), i
        assert torch.equal(r["sse_rmse"], sr), i
    b.close()


def test_plans_without_objective_match_the_oracle_on_real_rows():
    """Real-valued rows, plans without objectives: codes in lockstep with
    the oracle's fp32-decision encode on the batched codebooks (sampled), and
    codebooks equal to a plan with objectives up to float64 summation order."""
    d, m, ks, iters = 96, 12, 256, 5
    xs, inits = _problems([3001, 40000, 777], d, m, ks, "sphere", seed=36)
    xt = [_t(x) for x in xs]
    it = [_t(i) for i in inits]
    a = mipq.BatchedFit(xt, it, m, ks, iters, plan=True, autotune=False, graph=True, objective=False)
    a.run()
    c = mipq.BatchedFit(xt, it, m, ks, iters, plan=True, autotune=False, graph=True, objective=True)
    c.run()
    torch.cuda.synchronize()
    for i, x in enumerate(xs):
        ra, rc = a.results[i], c.results[i]
        np.testing.assert_allclose(ra["codebook"].cpu().numpy(), rc["codebook"].cpu().numpy(), rtol=1e-5, atol=1e-6)
        rows = np.random.default_rng(i).choice(x.shape[0], min(500, x.shape[0]), replace=False)
        ref, _ = pq.encode(x[rows], ra["codebook"].cpu().numpy().astype(np.float64), decide="fp32")
        np.testing.assert_array_equal(ra["codes"].cpu().numpy()[rows].astype(np.int64), ref)
    a.close()
    c.close()


def test_integer_rows_match_the_oracle():
    m, ks, iters, d = 12, 64, 4, 96
    xs, inits = _problems([64, 700, 2001], d, m, ks, "integer", seed=32)
    b, _ = _run(xs, inits, m, ks, iters, "graph")
    for i, (x, init) in enumerate(zip(xs, inits)):
        ref = pq.lloyd(x, init, m, iters, decide="fp32")
        r = b.results[i]
        # integer rows: float64 sums exact in any order
        np.testing.assert_array_equal(r["codebook"].cpu().numpy(), ref["codebook"].astype(np.float32))
        np.testing.assert_allclose(r["objective"].cpu().numpy(), ref["objective"], rtol=1e-12)
        codes_ref, _ = pq.encode(x, ref["codebook"].astype(np.float32).astype(np.float64), decide="fp32")
        np.testing.assert_array_equal(r["codes"].cpu().numpy().astype(np.int64), codes_ref)
        sse, rmse = pq.sse_rmse(x, codes_ref, ref["codebook"].astype(np.float32).astype(np.float64))
        got = r["sse_rmse"].cpu().numpy()
        assert got[0] == pytest.approx(sse, rel=1e-12) and got[1] == pytest.approx(rmse, rel=1e-12)
    b.close()


@pytest.mark.parametrize("d,m,ks", [(96, 12, 256), (64, 4, 100), (48, 16, 16)])
def test_unit_sphere_rows_lockstep(d, m, ks):
    """Real-valued rows (ds = 8, 16, 3; ks = 256, 100, 16): codes and errors
    in lockstep with the single calls on the batched codebooks; codebooks
    equal to the single fits up to float64 summation order."""
    iters = 6
    sizes = [ks, 3001, 777, 12345]
    xs, inits = _problems(sizes, d, m, ks, "sphere", seed=33)
    b, _ = _run(xs, inits, m, ks, iters, "graph")
    for i, (x, init) in enumerate(zip(xs, inits)):
        r = b.results[i]
        xt = _t(x)
        codes = mipq.pq_encode(xt, r["codebook"], "bf16")
        assert torch.equal(codes, r["codes"]), i
        _, sr = mipq.pq_decode_rmse(codes, r["codebook"], xt)
        assert torch.equal(sr, r["sse_rmse"]), i
        cb, _, _, obj = _single(x, init, m, ks, iters)
        np.testing.assert_allclose(r["codebook"].cpu().numpy(), cb.cpu().numpy(), rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(r["objective"].cpu().numpy(), obj.cpu().numpy(), rtol=1e-6)
        rows = np.random.default_rng(i).choice(x.shape[0], min(500, x.shape[0]), replace=False)
        ref, _ = pq.encode(x[rows], r["codebook"].cpu().numpy().astype(np.float64), decide="fp32")
        np.testing.assert_array_equal(r["codes"].cpu().numpy()[rows].astype(np.int64), ref)
    b.close()


def test_plan_replays_and_zero_rounds():
    m, ks, d = 12, 64, 96
    xs, inits = _problems([100, 2000], d, m, ks, "integer", seed=34)
    b, _ = _run(xs, inits, m, ks, 3, "graph")
    first = [{k: v.clone() for k, v in r.items()} for r in b.results]
    for r in b.results:
        for v in r.values():
            v.zero_()
    b.run()
    torch.cuda.synchronize()
    for r0, r1 in zip(first, b.results):
        for k in r0:
            assert torch.equal(r0[k], r1[k]), k
    b.close()
    # zero rounds: the initial rows are the codebook
    b0, _ = _run(xs, inits, m, ks, 0, "graph")
    for x, init, r in zip(xs, inits, b0.results):
        np.testing.assert_array_equal(r["codebook"].cpu().numpy(), pq.init_codebook(x, init, m).astype(np.float32))
    b0.close()


def test_full_size_uneven_batch_sampled():
    """64 problems, N_i log-uniform in [20k, 500k] (about 9.5M rows), D=96,
    M=12, Ks=256, 20 rounds on all rows of each problem, autotuned plan with
    graphs: sampled codes against the oracle on the final codebooks, objective
    non-increasing, errors against the oracle on four problems."""
    w = wl.batched_uneven()
    xs = [p.x for p in w.problems]
    inits = [p.init_rows for p in w.problems]
    print("problems", len(xs), "rows", sum(x.shape[0] for x in xs), flush=True)
    b, resc = _run(xs, inits, w.m, w.ks, w.iters, "graph")
    print("plan", b.info(), "rescored", int(resc.item()), flush=True)
    rng = np.random.default_rng(7)
    for i, x in enumerate(xs):
        r = b.results[i]
        obj = r["objective"].cpu().numpy()
        assert np.all(np.diff(obj) <= 1e-9 * obj[:-1]), i
        cb = r["codebook"].cpu().numpy().astype(np.float64)
        rows = rng.choice(x.shape[0], 300, replace=False)
        ref, _ = pq.encode(x[rows], cb, decide="fp32")
        np.testing.assert_array_equal(r["codes"].cpu().numpy()[rows].astype(np.int64), ref)
    for i in np.argsort([x.shape[0] for x in xs])[:4]:
        r = b.results[i]
        sse, _ = pq.sse_rmse(xs[i], r["codes"].cpu().numpy().astype(np.int64),
                             r["codebook"].cpu().numpy().astype(np.float64))
        assert r["sse_rmse"][0].item() == pytest.approx(sse, rel=1e-12)
    b.close()
    # the benchmarked form: no objectives, one fused launch per round
    f = mipq.BatchedFit([_t(x) for x in xs], [_t(i) for i in inits], w.m, w.ks, w.iters, plan=True, autotune=True,
                        graph=True, objective=False)
    f.run()
    torch.cuda.synchronize()
    print("fused plan", f.info(), flush=True)
    for i, x in enumerate(xs):
        r = f.results[i]
        cb = r["codebook"].cpu().numpy().astype(np.float64)
        rows = rng.choice(x.shape[0], 300, replace=False)
        ref, _ = pq.encode(x[rows], cb, decide="fp32")
        np.testing.assert_array_equal(r["codes"].cpu().numpy()[rows].astype(np.int64), ref)
    for i in np.argsort([x.shape[0] for x in xs])[:4]:
        r = f.results[i]
        sse, _ = pq.sse_rmse(xs[i], r["codes"].cpu().numpy().astype(np.int64),
                             r["codebook"].cpu().numpy().astype(np.float64))
        assert r["sse_rmse"][0].item() == pytest.approx(sse, rel=1e-12)
    f.close()


def test_deterministic_plan_repeats_and_equals_single_deterministic_fits():
    m, ks, iters, d = 12, 64, 4, 96
    xs, inits = _problems([3000, 9001, 5000, 700], d, m, ks, "float", seed=41)
    xt = [_t(x) for x in xs]
    it = [_t(i) for i in inits]
    b = mipq.BatchedFit(xt, it, m, ks, iters, plan=True, autotune=False, graph=True, deterministic=True)
    b.run()
    first = [{k: v.clone() for k, v in r.items()} for r in b.results]
    b.run()
    torch.cuda.synchronize()
    for i, (x, init) in enumerate(zip(xs, inits)):
        r = b.results[i]
        for k in ("codebook", "codes", "sse_rmse", "objective"):
            assert torch.equal(r[k], first[i][k]), (i, k)
        fit = mipq.pq_fit(xt[i], m, ks, iters, init_rows=it[i], precision="bf16", labels=False, deterministic=True)
        assert torch.equal(r["codebook"], fit["codebook"]), i
        assert torch.equal(r["objective"], fit["objective"]), i


def _outputs(b):
    return [{k: v.clone() for k, v in r.items()} for r in b.results]


@pytest.mark.parametrize("kind", ["integer", "float"])
def test_every_tuner_choice_gives_the_same_outputs(kind, tmp_path):
    """The tuner times both kernel variants at 1, 2, 4, 8 and 16 times their
    resident blocks and stores the fastest in the cache; a second plan takes
    it from there.  Every (variant, grid) forced through the cache gives the
    same codebooks, codes, errors and objectives bit for bit (integer rows:
    exact float64 sums in any order; float rows: deterministic sums)."""
    cache = tmp_path / "tune.json"
    os.environ["MIPQ_TUNE_CACHE"] = str(cache)
    m, ks, iters, d = 12, 256, 3, 96
    det = kind == "float"
    xs, inits = _problems([700, 20011, 4097, 256, 9000], d, m, ks, kind, seed=43)
    xt = [_t(x) for x in xs]
    it = [_t(i) for i in inits]

    def plan(**kw):
        b = mipq.BatchedFit(xt, it, m, ks, iters, plan=True, graph=True, deterministic=det, **kw)
        b.run()
        torch.cuda.synchronize()
        return b

    b = plan(autotune=True, retune=True)
    info = b.info()
    print("tuned", info, flush=True)
    assert not info["cached"] and len(info["candidates"]) == 10
    assert {(c[1]) for c in info["candidates"]} == {0, 1}
    fastest = min(info["candidates"], key=lambda c: c[2])
    assert (info["grid"], info["variant"]) == fastest[:2]
    ref = _outputs(b)
    b.close()
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    key, val = next(iter(entries.items()))
    assert key.startswith(torch.cuda.get_device_properties(0).gcnArchName)
    assert "|ds=8|ks=256|m=12|" in key and val["variant"] == info["variant"]

    b = plan(autotune=True)   # a cache hit: nothing timed
    hit = b.info()
    assert hit["cached"] and not hit["candidates"]
    assert (hit["grid"], hit["variant"]) == (info["grid"], info["variant"])
    b.close()

    for variant in (0, 1):
        for mult in (1, 2, 4, 8, 16):
            cache.write_text(json.dumps({key: {"grid_mult": mult, "variant": variant, "ns": 1}}, indent=0))
            b = plan(autotune=True)
            got = b.info()
            print("forced", variant, mult, got, flush=True)
            assert got["cached"] and got["variant"] == variant and got["grid"] == mult * got["resident"]
            for i, (r0, r1) in enumerate(zip(ref, b.results)):
                for k in r0:
                    assert torch.equal(r0[k], r1[k]), (variant, mult, i, k)
            b.close()

    cache.write_text("not json {")   # unreadable: ignored, retuned, rewritten
    b = plan(autotune=True)
    assert not b.info()["cached"]
    b.close()
    assert key in json.loads(cache.read_text())
