"""GPU parity of the inverted file: coarse assignment, stable bucketing, the
full index build and ADC top-k search, against the oracle in its
kernel-decision mode (bit for bit) and the float64 oracle outside near-ties."""

import dataclasses

import numpy as np
import pytest
import torch

import paper_2604_21645_amd as mipq
from oracle import ivf, pq
from synth import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,d,kc", [(3001, 128, 100), (777, 64, 33), (1000, 32, 300), (64, 16, 7),
                                    (1500, 96, 257), (1200, 192, 300), (900, 256, 161), (1000, 128, 2048)])
def test_coarse_assign_matches_oracle(prec, n, d, kc):
    print("coarse", prec, n, d, kc, flush=True)
    x = wl.gaussian_mixture(n + d, n, d, 50, sigma=0.05)
    cc = wl.gaussian_mixture(kc, kc, d, 50, sigma=0.05)
    lab, resc = mipq.coarse_assign(_t(x), _t(cc), prec, rescored=True)
    ref, tie = ivf.coarse_assign(x, cc, "kernel")
    np.testing.assert_array_equal(lab.cpu().numpy().astype(np.int64), ref)
    r64, _ = ivf.coarse_assign(x, cc, "fp64")
    got = lab.cpu().numpy()
    assert np.all(got[~tie] == r64[~tie])


def test_coarse_assign_duplicate_centroids_are_decided_exactly():
    rng = np.random.default_rng(4)
    cc = rng.integers(0, 3, size=(40, 32)).astype(np.float32)
    cc[20:] = cc[:20]
    x = rng.integers(0, 3, size=(500, 32)).astype(np.float32)
    lab, resc = mipq.coarse_assign(_t(x), _t(cc), "bf16", rescored=True)
    ref, _ = ivf.coarse_assign(x, cc, "kernel")
    np.testing.assert_array_equal(lab.cpu().numpy().astype(np.int64), ref)
    assert int(resc.item()) > 0


def test_coarse_assign_split_clusters_use_the_candidate_path():
    # every mixture component carries two centroids a hair apart (as k-means
    # leaves split clusters): most rows have two nearly equal best distances
    rng = np.random.default_rng(11)
    means = rng.uniform(0, 1, size=(60, 128))
    cc = np.concatenate([means + 1e-3 * rng.standard_normal(means.shape),
                         means + 1e-3 * rng.standard_normal(means.shape)]).astype(np.float32)
    x = wl.gaussian_mixture(12, 5000, 128, 60, sigma=0.05, means=means)
    lab, resc = mipq.coarse_assign(_t(x), _t(cc), "bf16", rescored=True)
    ref, tie = ivf.coarse_assign(x, cc, "kernel")
    np.testing.assert_array_equal(lab.cpu().numpy().astype(np.int64), ref)
    print("rescored rows", int(resc.item()), "of", x.shape[0], flush=True)
    assert int(resc.item()) > 50


def _small():
    return wl.ivf_adc(seed=21, n=20000, d=32, n_comp=64, kc=64, n_query=40, m=4, ks=16, coarse_iters=5,
                      pq_iters=5, n_train=4000, nprobe=6, topk=25)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_index_build_matches_oracle(prec):
    w = _small()
    idx = mipq.ii_build(_t(w.x), w.kc, w.coarse_iters, _t(w.coarse_train), _t(w.coarse_init), w.m, w.ks,
                        w.pq_iters, _t(w.pq_init), precision=prec, coarse_objective=True)
    ref = ivf.build(w.x, w.coarse_train, w.coarse_init, w.coarse_iters, w.m, w.pq_init, w.pq_iters)
    # coarse centroids: same decisions, same float64 sums in id order
    np.testing.assert_array_equal(idx["coarse"].cpu().numpy(), ref["coarse"].astype(np.float32))
    np.testing.assert_array_equal(idx["labels"].cpu().numpy().astype(np.int64), ref["labels"])
    np.testing.assert_array_equal(idx["offsets"].cpu().numpy(), ref["offsets"])
    np.testing.assert_array_equal(idx["ids"].cpu().numpy().astype(np.int64), ref["ids"])
    pqc = idx["pq_codebook"].cpu().numpy()
    np.testing.assert_allclose(pqc, ref["pq"], rtol=1e-6, atol=1e-7)
    # residual codes in list order, against the oracle's encode with the GPU codebook
    r = ivf.residuals(w.x, ref["labels"], ref["coarse"].astype(np.float32))
    codes_ref, _ = pq.encode(r, pqc.astype(np.float64), decide="fp32")
    np.testing.assert_array_equal(idx["codes_sorted"].cpu().numpy().astype(np.int64), codes_ref[ref["ids"]])
    obj = idx["coarse_objective"].cpu().numpy()
    assert np.all(np.diff(obj) <= 1e-9 * obj[:-1])


@pytest.mark.parametrize("n", [262144, 262145, 300001])
def test_posting_lists_at_sort_tile_boundaries(n):
    # the radix sort's tile grows past 256 elements above 262,144 keys (at most
    # 1,024 blocks): the k-means sample and all rows sorted at such sizes
    print("posting lists, n =", n, flush=True)
    w = wl.ivf_adc(seed=23, n=n, d=16, n_comp=64, kc=64, n_query=1, m=4, ks=16, coarse_iters=3, pq_iters=2,
                   n_train=n)
    idx = mipq.ii_build(_t(w.x), w.kc, w.coarse_iters, _t(w.coarse_train), _t(w.coarse_init), w.m, w.ks,
                        w.pq_iters, _t(w.pq_init))
    ref = ivf.build(w.x, w.coarse_train, w.coarse_init, w.coarse_iters, w.m, w.pq_init, w.pq_iters)
    np.testing.assert_array_equal(idx["coarse"].cpu().numpy(), ref["coarse"].astype(np.float32))
    np.testing.assert_array_equal(idx["offsets"].cpu().numpy(), ref["offsets"])
    np.testing.assert_array_equal(idx["ids"].cpu().numpy().astype(np.int64), ref["ids"])


def _gpu_index_np(idx):
    return (idx["coarse"].cpu().numpy(), idx["pq_codebook"].cpu().numpy(), idx["offsets"].cpu().numpy(),
            idx["ids"].cpu().numpy().astype(np.int64))


@pytest.mark.parametrize("nprobe,topk", [(6, 25), (1, 300), (64, 10)])
def test_adc_search_matches_oracle(nprobe, topk):
    w = _small()
    idx = mipq.ii_build(_t(w.x), w.kc, w.coarse_iters, _t(w.coarse_train), _t(w.coarse_init), w.m, w.ks,
                        w.pq_iters, _t(w.pq_init))
    cc, pqc, off, ids = _gpu_index_np(idx)
    codes_sorted = idx["codes_sorted"].cpu().numpy().astype(np.int64)
    codes_by_id = np.empty_like(codes_sorted)
    codes_by_id[ids] = codes_sorted
    gi, gd = mipq.adc_search(_t(w.queries), idx, nprobe, topk)
    ri, rd = ivf.adc_search(w.queries, cc, pqc, off, ids, codes_by_id, nprobe, topk, decide="kernel")
    np.testing.assert_array_equal(gi.cpu().numpy().astype(np.int64), ri)
    np.testing.assert_array_equal(gd.cpu().numpy(), rd.astype(np.float32))


@pytest.mark.parametrize("case", ["mixture", "integer_ties"])
@pytest.mark.parametrize("nprobe,topk", [(4, 10), (3, 100)])
def test_adc_search_m16_long_lists_matches_oracle(case, nprobe, topk):
    """M = 16 rows (the partial-sum pruned scan) over lists of several scan
    steps, so the bounds tighten inside a list and across lists; the
    integer-valued case puts many candidates at exactly the bound's score."""
    if case == "mixture":
        w = wl.ivf_adc(seed=31, n=60000, d=64, n_comp=40, kc=16, n_query=30, m=16, ks=64, coarse_iters=4,
                       pq_iters=4, n_train=6000, nprobe=nprobe, topk=topk)
    else:
        w = wl.ivf_adc(seed=32, n=40000, d=32, n_comp=8, kc=8, n_query=30, m=16, ks=16, coarse_iters=3,
                       pq_iters=3, n_train=4000, nprobe=nprobe, topk=topk)
        # rows repeat 200 prototypes, so equal codes in one list give equal scores
        rng = np.random.default_rng(33)
        protos = rng.integers(0, 3, size=(200, w.x.shape[1])).astype(np.float32)
        w = dataclasses.replace(w, x=protos[rng.integers(0, 200, w.x.shape[0])],
                                queries=rng.integers(0, 3, size=w.queries.shape).astype(np.float32))
    print("adc m16", case, nprobe, topk, flush=True)
    idx = mipq.ii_build(_t(w.x), w.kc, w.coarse_iters, _t(w.coarse_train), _t(w.coarse_init), w.m, w.ks,
                        w.pq_iters, _t(w.pq_init))
    cc, pqc, off, ids = _gpu_index_np(idx)
    assert np.diff(off).max() > 3 * 1024
    codes_sorted = idx["codes_sorted"].cpu().numpy().astype(np.int64)
    codes_by_id = np.empty_like(codes_sorted)
    codes_by_id[ids] = codes_sorted
    gi, gd = mipq.adc_search(_t(w.queries), idx, w.nprobe, w.topk)
    ri, rd = ivf.adc_search(w.queries, cc, pqc, off, ids, codes_by_id, w.nprobe, w.topk, decide="kernel")
    np.testing.assert_array_equal(gi.cpu().numpy().astype(np.int64), ri)
    np.testing.assert_array_equal(gd.cpu().numpy(), rd.astype(np.float32))
    if case == "integer_ties":   # the top-k ends inside a run of equal distances
        assert np.mean(rd[:, -1] == rd[:, -2]) > 0.5
    # the work counters leave the results unchanged and count within the method's work
    wi, wd, wk = mipq.adc_search(_t(w.queries), idx, w.nprobe, w.topk, work=True)
    assert torch.equal(wi, gi) and torch.equal(wd, gd)
    lut, part, full, lists = wk.cpu().numpy().tolist()
    pairs = w.queries.shape[0] * w.nprobe
    probed = off[1:] - off[:-1]
    assert 0 < lists <= pairs
    # a scanned list built at least its first 8 table rows; no pair builds more than M
    assert lut % w.ks == 0 and w.ks * 8 * lists <= lut <= w.ks * w.m * pairs
    # every row of a scanned list is summed partially, in full, or both
    assert 0 < full <= int(probed.max()) * pairs and part <= int(probed.max()) * pairs
    print("adc work", case, dict(lut=lut, part=part, full=full, lists=lists, pairs=pairs), flush=True)


def test_adc_search_many_lists_matches_oracle():
    """Kc above the LDS counters of the per-rank pair ordering: the scan
    order comes from the radix-sort path instead; results are the same."""
    w = wl.ivf_adc(seed=34, n=40000, d=32, n_comp=200, kc=9000, n_query=20, m=8, ks=16, coarse_iters=2,
                   pq_iters=2, n_train=20000, nprobe=40, topk=20)
    print("adc kc", w.kc, flush=True)
    idx = mipq.ii_build(_t(w.x), w.kc, w.coarse_iters, _t(w.coarse_train), _t(w.coarse_init), w.m, w.ks,
                        w.pq_iters, _t(w.pq_init))
    cc, pqc, off, ids = _gpu_index_np(idx)
    codes_sorted = idx["codes_sorted"].cpu().numpy().astype(np.int64)
    codes_by_id = np.empty_like(codes_sorted)
    codes_by_id[ids] = codes_sorted
    gi, gd = mipq.adc_search(_t(w.queries), idx, w.nprobe, w.topk)
    ri, rd = ivf.adc_search(w.queries, cc, pqc, off, ids, codes_by_id, w.nprobe, w.topk, decide="kernel")
    np.testing.assert_array_equal(gi.cpu().numpy().astype(np.int64), ri)
    np.testing.assert_array_equal(gd.cpu().numpy(), rd.astype(np.float32))


def test_full_size_index_and_search_sampled():
    """10M x 128 rows, Kc = 4096, residual PQ M=16 Ks=256, 10k queries,
    nprobe 32, top-100: bucket invariants on every row, sampled labels and
    codes, and 100 sampled queries against the oracle."""
    w = wl.ivf_adc()
    xt = _t(w.x)
    print("build", flush=True)
    idx = mipq.ii_build(xt, w.kc, w.coarse_iters, _t(w.coarse_train), _t(w.coarse_init), w.m, w.ks, w.pq_iters,
                        _t(w.pq_init))
    n = w.x.shape[0]
    cc, pqc, off, ids = _gpu_index_np(idx)
    lab = idx["labels"].cpu().numpy()
    assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) >= 0)
    np.testing.assert_array_equal(np.diff(off), np.bincount(lab, minlength=w.kc))
    assert np.array_equal(np.sort(ids), np.arange(n))
    for l in np.random.default_rng(1).choice(w.kc, 64, replace=False):
        seg = ids[off[l]:off[l + 1]]
        assert np.all(np.diff(seg) > 0) and np.all(lab[seg] == l)
    rows = np.random.default_rng(2).choice(n, 3000, replace=False)
    ref_lab, _ = ivf.coarse_assign(w.x[rows], cc, "kernel")
    np.testing.assert_array_equal(lab[rows].astype(np.int64), ref_lab)
    codes_sorted = idx["codes_sorted"].cpu().numpy()
    pos = np.empty(n, dtype=np.int64)
    pos[ids] = np.arange(n)
    r = ivf.residuals(w.x[rows], ref_lab, cc)
    cref, _ = pq.encode(r, pqc.astype(np.float64), decide="fp32")
    np.testing.assert_array_equal(codes_sorted[pos[rows]].astype(np.int64), cref)
    print("search", flush=True)
    gi, gd, wide = mipq.adc_search(_t(w.queries), idx, w.nprobe, w.topk, wide=True)
    print("wide probe selections", int(wide.item()), flush=True)
    codes_by_id = np.empty_like(codes_sorted)
    codes_by_id[ids] = codes_sorted
    qs = np.random.default_rng(3).choice(w.queries.shape[0], 100, replace=False)
    ri, rd = ivf.adc_search(w.queries[qs], cc, pqc, off, ids, codes_by_id, w.nprobe, w.topk, decide="kernel")
    np.testing.assert_array_equal(gi.cpu().numpy()[qs].astype(np.int64), ri)
    np.testing.assert_array_equal(gd.cpu().numpy()[qs], rd.astype(np.float32))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_chunk_adds_merged_equal_the_global_build(prec):
    """Index built chunk by chunk with the global quantisers, then merged:
    offsets, ids and codes equal one build over all rows bit for bit, and the
    oracle's add + merge on the same quantisers."""
    w = _small()
    print("add/merge", prec, flush=True)
    xt = _t(w.x)
    idx = mipq.ii_build(xt, w.kc, w.coarse_iters, _t(w.coarse_train), _t(w.coarse_init), w.m, w.ks,
                        w.pq_iters, _t(w.pq_init), precision=prec)
    whole = mipq.ii_add(xt, idx["coarse"], idx["pq_codebook"], prec, labels=True)
    for k in ("offsets", "ids", "codes_sorted", "labels"):
        assert torch.equal(whole[k], idx[k]), k
    cuts = [0, 1, 5000, 5000, 12345, 19999, 20000]
    parts = [mipq.ii_add(xt[a:b], idx["coarse"], idx["pq_codebook"], prec) for a, b in zip(cuts[:-1], cuts[1:])]
    merged = mipq.ii_merge(parts)
    for k in ("offsets", "ids", "codes_sorted"):
        assert torch.equal(merged[k], idx[k]), k
    cc = idx["coarse"].cpu().numpy()
    pcb = idx["pq_codebook"].cpu().numpy().astype(np.float64)
    ref = ivf.merge([ivf.add(w.x[a:b], cc, pcb) for a, b in zip(cuts[:-1], cuts[1:])])
    np.testing.assert_array_equal(merged["offsets"].cpu().numpy(), ref["offsets"])
    ids = merged["ids"].cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(ids, ref["ids"])
    np.testing.assert_array_equal(merged["codes_sorted"].cpu().numpy().astype(np.int64), ref["codes"][ids])


@pytest.mark.parametrize("kc,m,nparts", [(1, 16, 3), (300, 5, 37), (5000, 32, 9), (64, 16, 1)])
def test_merge_of_synthetic_parts_matches_oracle(kc, m, nparts):
    """Merge alone on part indexes with random labels (empty parts, empty and
    crowded lists, 16-byte and byte-wise code rows) against the oracle."""
    rng = np.random.default_rng(kc + m + nparts)
    parts_np, parts = [], []
    for p in range(nparts):
        n = 0 if p % 4 == 1 else int(rng.integers(1, 3000))
        lab = np.minimum(rng.geometric(0.02, size=n) - 1, kc - 1) if n else np.zeros(0, np.int64)
        off, ids = ivf.posting_lists(lab, kc)
        codes = rng.integers(0, 256, size=(n, m))
        parts_np.append(dict(offsets=off, ids=ids, codes=codes))
        parts.append(dict(coarse=torch.zeros((kc, 4), device=DEV), pq_codebook=torch.zeros((m, 1, 1), device=DEV),
                          offsets=_t(off), ids=_t(ids.astype(np.int32)),
                          codes_sorted=_t(codes[ids].astype(np.uint8).reshape(n, m))))
    print("merge", kc, m, nparts, flush=True)
    got = mipq.ii_merge(parts)
    ref = ivf.merge(parts_np)
    np.testing.assert_array_equal(got["offsets"].cpu().numpy(), ref["offsets"])
    ids = got["ids"].cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(ids, ref["ids"])
    np.testing.assert_array_equal(got["codes_sorted"].cpu().numpy().astype(np.int64), ref["codes"][ids])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_kmeans_fit_matches_oracle(prec):
    """The coarse quantiser on its own: centroids (float64 means in id order,
    rounded) and last labels bit for bit, objective to float64 rounding."""
    w = _small()
    xt = _t(w.x)
    print("kmeans", prec, flush=True)
    got = mipq.kmeans_fit(xt, w.kc, w.coarse_iters, _t(w.coarse_init), train_rows=_t(w.coarse_train), precision=prec)
    ref = ivf.coarse_fit(w.x[w.coarse_train], w.coarse_init, w.coarse_iters)
    np.testing.assert_array_equal(got["centroids"].cpu().numpy(), ref["codebook"].astype(np.float32))
    np.testing.assert_array_equal(got["labels"].cpu().numpy().astype(np.int64), ref["labels"])
    np.testing.assert_allclose(got["objective"].cpu().numpy(), ref["objective"], rtol=1e-12)
    # all rows as the training set, and zero rounds
    init = np.arange(0, 20000, 20000 // w.kc)[:w.kc]
    g2 = mipq.kmeans_fit(xt, w.kc, 3, _t(init), precision=prec)
    r2 = ivf.coarse_fit(w.x, init, 3)
    np.testing.assert_array_equal(g2["centroids"].cpu().numpy(), r2["codebook"].astype(np.float32))
    g0 = mipq.kmeans_fit(xt, w.kc, 0, _t(init), precision=prec, labels=False, objective=False)
    np.testing.assert_array_equal(g0["centroids"].cpu().numpy(), w.x[init])
