"""Pins for the CPU oracle: each function is checked against something other than
itself -- brute force on tiny inputs, scipy's vq/kmeans2, closed forms, exact
integer arithmetic and invariants -- chosen so that a dropped term, a wrong
sign, a wrong index or a transposed operand fails at least one of them.
"""

import os
import warnings

import numpy as np
import pytest
import scipy.cluster.vq as scv

from oracle import chunked, grad, ivf, opq, pq
from synth import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(seed, n, d, scale=1.0):
    return (np.random.default_rng(seed).standard_normal((n, d)) * scale).astype(np.float32)


# ---------------------------------------------------------------- assignment

def _brute_codes(x, cb, fp32):
    m, ks, ds = cb.shape
    out = np.zeros((x.shape[0], m), dtype=np.int64)
    for n in range(x.shape[0]):
        for j in range(m):
            best, bi = None, -1
            for k in range(ks):
                if fp32:
                    acc = None
                    for t in range(ds):
                        diff = np.float32(x[n, j * ds + t]) - np.float32(cb[j, k, t])
                        sq = np.float32(diff * diff)
                        acc = sq if acc is None else np.float32(acc + sq)
                    dist = acc
                else:
                    dist = 0.0
                    for t in range(ds):
                        diff = float(x[n, j * ds + t]) - float(cb[j, k, t])
                        dist += diff * diff
                if best is None or dist < best:
                    best, bi = dist, k
            out[n, j] = bi
    return out


@pytest.mark.parametrize("fp32", [False, True])
def test_assign_matches_brute_force(fp32):
    x = _rand(0, 37, 12)
    cb = _rand(1, 3 * 9, 4).reshape(3, 9, 4).astype(np.float64)
    codes, dmin, _ = pq.assign(x, cb, "fp32" if fp32 else "fp64")
    np.testing.assert_array_equal(codes, _brute_codes(x, cb.astype(np.float32) if fp32 else cb, fp32))
    # the reported distance is the float64 distance of the chosen centroid
    for n in range(5):
        for j in range(3):
            ref = sum((float(x[n, j * 4 + t]) - float(np.float32(cb[j, codes[n, j], t]) if fp32
                       else cb[j, codes[n, j], t])) ** 2 for t in range(4))
            assert dmin[n, j] == pytest.approx(ref, rel=1e-12)


def test_assign_ties_go_to_lowest_index():
    cb = np.zeros((1, 4, 2))
    cb[0, 1] = [1.0, 0.0]
    cb[0, 3] = [1.0, 0.0]          # duplicate of centroid 1
    cb[0, 0] = [5.0, 5.0]
    cb[0, 2] = [-1.0, 0.0]         # same distance to x as centroid 1
    x = np.array([[0.0, 0.0], [1.0, 0.0]], dtype=np.float32)
    for mode in ("fp64", "fp32"):
        codes, _, tie = pq.assign(x, cb, mode)
        assert codes[:, 0].tolist() == [1, 1]
        assert tie[:, 0].tolist() == [True, True]



def test_near_tie_threshold_is_relative_to_the_best_distance():
    # tie iff d2 - d1 <= 1e-5 * d1 for the two smallest distances d1 <= d2,
    # wherever they sit in the row
    d1 = 1024.0
    rows = [
        ([5.0e3, d1 * (1 + 0.9e-5), 9.0e3, d1], True),    # inside the band
        ([d1, 7.0e3, d1 * (1 + 1.1e-5)], False),           # outside the band
        ([d1 * (1 - 0.9e-5), d1], True),                   # runner-up first, best second
        ([d1, d1 * (1 - 1.1e-5)], False),
        # relative to d1, not d2: a gap of 1.000005e-5 d1 is within 1e-5 d2
        ([d1, d1 * (1 + 1.000005e-5)], False),
        # relative, not absolute: a gap of 5e-6 relative is 0.005 absolute
        ([1000.0, 1000.005], True),
        ([1e-3, 1e-3 + 2e-8], False),
        ([0.0, 0.0, 4.0], True),                            # duplicate zero distances
        ([3.0, 0.0, 1e-300], False),                        # d1 = 0 < d2
        ([2.0, 2.0], True),                                 # exact tie
    ]
    for vals, want in rows:
        got = pq.near_tie_mask(np.array([vals], np.float64))[0]
        assert bool(got) == want, (vals, want)
    # one candidate has no runner-up
    assert not pq.near_tie_mask(np.array([[1.0]]))[0]

def test_assign_matches_scipy_vq():
    x = _rand(2, 300, 16)
    cb = _rand(3, 4 * 20, 4).reshape(4, 20, 4).astype(np.float64)
    codes, _, _ = pq.assign(x, cb, "fp64")
    for j in range(4):
        lab, _ = scv.vq(x[:, j * 4:(j + 1) * 4].astype(np.float64), cb[j])
        np.testing.assert_array_equal(codes[:, j], lab)


def test_fp32_decision_equals_fp64_outside_near_ties():
    w = wl.plain_pq(seed=7, n=3000, m=8, ks=64, iters=1)
    cb = pq.init_codebook(w.x, w.init_rows, w.m) + 0.01
    c64, _, tie = pq.assign(w.x, cb, "fp64")
    c32, _, _ = pq.assign(w.x, cb.astype(np.float32).astype(np.float64), "fp32")
    c64b, _, _ = pq.assign(w.x, cb.astype(np.float32).astype(np.float64), "fp64")
    assert np.all(c32[~tie] == c64b[~tie])
    assert (c32 != c64).mean() < 1e-3


def test_integer_rows_decide_exactly_in_fp32():
    # integer rows in [0, 255], integer initial centroids: all distances are
    # integers below 2^24, exact in float32 and float64, so the two decision
    # modes agree everywhere, ties included.
    w = wl.integer_pq(seed=11, n=4000, n_comp=50, m=16, ks=64, n_train=4000)
    cb = pq.init_codebook(w.train, w.init_rows, w.m)
    assert np.all(cb == np.rint(cb))
    a64, d64, _ = pq.assign(w.x, cb, "fp64")
    a32, _, _ = pq.assign(w.x, cb, "fp32")
    np.testing.assert_array_equal(a64, a32)
    for j in range(w.m):
        xs = pq.block(w.x[:200], j, 8)
        np.testing.assert_array_equal(pq.dist32(xs, cb[j]).astype(np.float64), pq.dist64(xs, cb[j]))


# ---------------------------------------------------------------- Lloyd fit

def test_lloyd_matches_scipy_kmeans2():
    w = wl.plain_pq(seed=3, n=1500, m=4, ks=16, iters=6)
    fit = pq.lloyd(w.x, w.init_rows, w.m, w.iters, decide="fp64")
    c0 = pq.init_codebook(w.x, w.init_rows, w.m)
    ds = w.x.shape[1] // w.m
    for j in range(w.m):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            cbj, lab = scv.kmeans2(w.x[:, j * ds:(j + 1) * ds].astype(np.float64), c0[j].copy(),
                                   iter=w.iters, minit="matrix", missing="warn")
        np.testing.assert_allclose(fit["codebook"][j], cbj, rtol=1e-12, atol=1e-12)
        np.testing.assert_array_equal(fit["codes"][:, j], lab)


def test_lloyd_objective_never_increases_and_fixed_point():
    w = wl.plain_pq(seed=4, n=2000, m=8, ks=32, iters=12)
    fit = pq.lloyd(w.x, w.init_rows, w.m, w.iters, decide="fp64")
    j = fit["objective"]
    assert np.all(np.diff(j) <= 1e-12 * j[:-1])
    # more rounds from a converged codebook leave it unchanged
    more = pq.lloyd(w.x, w.init_rows, w.m, 40, decide="fp64")
    again = pq.lloyd(w.x, w.init_rows, w.m, 2, decide="fp64", init_codebook_value=more["codebook"])
    if np.all(np.diff(more["objective"][-3:]) == 0):
        np.testing.assert_array_equal(again["codebook"], more["codebook"])


def test_lloyd_resume_equals_longer_run():
    w = wl.plain_pq(seed=5, n=1200, m=4, ks=16, iters=9)
    full = pq.lloyd(w.x, w.init_rows, w.m, 9, decide="fp32")
    first = pq.lloyd(w.x, w.init_rows, w.m, 4, decide="fp32")
    rest = pq.lloyd(w.x, w.init_rows, w.m, 5, decide="fp32", init_codebook_value=first["codebook"])
    np.testing.assert_array_equal(full["codebook"], rest["codebook"])


def test_empty_cluster_keeps_previous_centroid():
    x = np.array([[0.0], [0.1], [0.2], [10.0]], dtype=np.float32)
    init = np.array([[0, 1, 1]])     # centroids 1 and 2 start equal: 2 never wins (lowest index)
    fit = pq.lloyd(x, init, 1, 1, decide="fp64")
    c = fit["codebook"][0, :, 0]
    assert c[2] == pytest.approx(0.1)                      # untouched
    assert c[0] == pytest.approx(0.0)
    assert c[1] == pytest.approx((0.1 + 0.2 + 10.0) / 3)


# ---------------------------------------------------------------- closed forms

def test_single_centroid_is_block_mean_and_sse_is_total_scatter():
    x = _rand(8, 500, 12, scale=3.0)
    init = np.zeros((3, 1), dtype=np.int64)
    fit = pq.lloyd(x, init, 3, 1, decide="fp64")
    np.testing.assert_allclose(fit["codebook"][:, 0, :].reshape(-1), x.astype(np.float64).mean(0),
                               rtol=1e-12, atol=1e-12)
    codes, _ = pq.encode(x, fit["codebook"])
    sse, rmse = pq.sse_rmse(x, codes, fit["codebook"])
    assert sse == pytest.approx(x.astype(np.float64).var(0).sum() * x.shape[0], rel=1e-10)
    assert rmse == pytest.approx(np.sqrt(sse / x.size), rel=1e-12)


def test_one_dimensional_subspaces_follow_midpoints():
    rng = np.random.default_rng(9)
    x = rng.uniform(-5, 5, size=(400, 3)).astype(np.float32)
    cb = rng.uniform(-5, 5, size=(3, 7, 1))
    codes, _, _ = pq.assign(x, cb, "fp64")
    for j in range(3):
        order = np.argsort(cb[j, :, 0])
        srt = cb[j, order, 0]
        mids = (srt[1:] + srt[:-1]) / 2
        expect = order[np.searchsorted(mids, x[:, j].astype(np.float64))]
        np.testing.assert_array_equal(codes[:, j], expect)


def test_identity_permutation_codes_and_zero_rmse():
    x = _rand(10, 64, 8)
    perm = np.stack([np.random.default_rng(s).permutation(64) for s in range(4)])
    cb = pq.init_codebook(x, perm, 4)
    codes, _ = pq.encode(x, cb)
    for j in range(4):
        inv = np.empty(64, dtype=np.int64)
        inv[perm[j]] = np.arange(64)
        np.testing.assert_array_equal(codes[:, j], inv)
    assert pq.sse_rmse(x, codes, cb)[1] == 0.0


def test_rmse_falls_with_more_subspaces_and_centroids():
    w = wl.plain_pq(seed=12, n=4000, iters=8, m=1, ks=16)
    res_m = []
    for m in (1, 2, 4, 8, 16):
        init = wl.init_rows_per_subspace(12, w.x.shape[0], m, 32)
        fit = pq.lloyd(w.x, init, m, 8)
        codes, _ = pq.encode(w.x, fit["codebook"])
        res_m.append(pq.sse_rmse(w.x, codes, fit["codebook"])[1])
    res_k = []
    for ks in (16, 32, 64, 128, 256):
        init = wl.init_rows_per_subspace(12, w.x.shape[0], 8, ks)
        fit = pq.lloyd(w.x, init, 8, 8)
        codes, _ = pq.encode(w.x, fit["codebook"])
        res_k.append(pq.sse_rmse(w.x, codes, fit["codebook"])[1])
    assert all(b < a for a, b in zip(res_m, res_m[1:])), res_m
    assert all(b < a for a, b in zip(res_k, res_k[1:])), res_k


def test_every_row_has_one_code_per_subspace():
    w = wl.plain_pq(seed=13, n=500, m=8, ks=32, iters=2)
    fit = pq.lloyd(w.x, w.init_rows, 8, 2)
    codes, _ = pq.encode(w.x, fit["codebook"])
    assert codes.shape == (500, 8)
    assert codes.min() >= 0 and codes.max() < 32


# ---------------------------------------------------------------- gradient

def test_gradient_matches_central_differences_and_vanishes_after_update():
    w = wl.plain_pq(seed=14, n=300, m=4, ks=8, iters=3)
    fit = pq.lloyd(w.x, w.init_rows, 4, 3)
    cb = fit["codebook"] + 0.003
    codes, _ = pq.encode(w.x, cb)
    lval, gx, gc = grad.grads(w.x, codes, cb, g=1.0)
    assert lval == pytest.approx(pq.sse_rmse(w.x, codes, cb)[0], rel=1e-12)
    rng = np.random.default_rng(0)
    h = 1e-3
    for _ in range(20):
        j, k, t = rng.integers(4), rng.integers(8), rng.integers(32 // 4)
        cp, cm = cb.copy(), cb.copy()
        cp[j, k, t] += h
        cm[j, k, t] -= h
        fd = (grad.loss(w.x, codes, cp) - grad.loss(w.x, codes, cm)) / (2 * h)
        assert fd == pytest.approx(gc[j, k, t], rel=1e-6, abs=1e-7)
    for _ in range(20):
        n, d = rng.integers(300), rng.integers(32)
        xp, xm = w.x.astype(np.float64), w.x.astype(np.float64).copy()
        xp = xp.copy()
        xp[n, d] += h
        xm[n, d] -= h
        fd = (grad.loss(xp, codes, cb) - grad.loss(xm, codes, cb)) / (2 * h)
        assert fd == pytest.approx(gx[n, d], rel=1e-6, abs=1e-7)
    # right after an update, the codebook gradient for the codes used in it is 0
    codes2, _, _ = pq.assign(w.x, cb, "fp64")
    upd, cnt, _ = pq.update(w.x, codes2, cb)
    _, _, g0 = grad.grads(w.x, codes2, upd)
    assert np.abs(g0).max() < 1e-9
    _, _, g3 = grad.grads(w.x, codes2, upd, g=3.0)
    assert np.abs(g3).max() < 1e-9


# ---------------------------------------------------------------- inverted index

def test_posting_lists_partition_and_match_stable_sort():
    rng = np.random.default_rng(15)
    lab = rng.integers(0, 37, size=2000)
    off, ids = ivf.posting_lists(lab, 40)
    assert off[0] == 0 and off[-1] == 2000 and np.all(np.diff(off) >= 0)
    np.testing.assert_array_equal(np.diff(off), np.bincount(lab, minlength=40))
    np.testing.assert_array_equal(ids, np.argsort(lab, kind="stable"))
    lists = [[] for _ in range(40)]
    for i, l in enumerate(lab[:300].tolist()):
        lists[l].append(i)
    off2, ids2 = ivf.posting_lists(lab[:300], 40)
    assert ids2.tolist() == [i for l in lists for i in l]


def test_coarse_fit_matches_kmeans2_on_full_rows():
    x = _rand(16, 800, 6)
    init = np.arange(0, 800, 80)[:10]
    fit = ivf.coarse_fit(x, init, 5, decide="fp64")
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        cb, lab = scv.kmeans2(x.astype(np.float64), x[init].astype(np.float64), iter=5,
                              minit="matrix", missing="warn")
    np.testing.assert_allclose(fit["codebook"], cb, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(fit["labels"], lab)


def test_coarse_kernel_decisions_match_fp64_outside_near_ties():
    x = _rand(17, 600, 128)
    cc = _rand(18, 50, 128)
    lk, tie = ivf.coarse_assign(x, cc, "kernel")
    l64, _ = ivf.coarse_assign(x, cc, "fp64")
    assert np.all(lk[~tie] == l64[~tie])


def _small_index(seed=19):
    w = wl.ivf_adc(seed=seed, n=3000, d=32, n_comp=40, kc=16, n_query=12, m=4, ks=16,
                   coarse_iters=4, pq_iters=4, n_train=1500, nprobe=4, topk=20)
    idx = ivf.build(w.x, w.coarse_train, w.coarse_init, w.coarse_iters, w.m, w.pq_init, w.pq_iters)
    return w, idx


def test_adc_table_sum_is_distance_to_decoded_vector():
    w, idx = _small_index()
    cc32 = idx["coarse"].astype(np.float32)
    pcb = idx["pq"].astype(np.float32)
    q = w.queries[0]
    for i in range(0, 3000, 97):
        l = idx["labels"][i]
        lut = ivf.adc_lut(q, cc32[l], pcb)
        s = sum(float(lut[j][idx["codes"][i, j]]) for j in range(w.m))
        xhat = cc32[l].astype(np.float64) + pq.decode(idx["codes"][i:i + 1], pcb)[0]
        ref = float(((q.astype(np.float64) - xhat) ** 2).sum())
        assert s == pytest.approx(ref, rel=2e-5, abs=1e-6)


def test_adc_exhaustive_probe_equals_brute_force_topk():
    w, idx = _small_index()
    cc32 = idx["coarse"].astype(np.float32)
    pcb = idx["pq"].astype(np.float32)
    ids, dist = ivf.adc_search(w.queries, cc32, pcb, idx["offsets"], idx["ids"], idx["codes"],
                               nprobe=16, topk=20, decide="fp64")
    xhat = cc32.astype(np.float64)[idx["labels"]] + pq.decode(idx["codes"], pcb)
    for qi in range(w.queries.shape[0]):
        d = ((w.queries[qi].astype(np.float64)[None, :] - xhat) ** 2).sum(1)
        order = np.lexsort((np.arange(len(d)), d))[:20]
        srt = np.sort(d)
        gap_ok = np.all(np.diff(srt[:21]) > 1e-9 * srt[1:21])
        if gap_ok:
            np.testing.assert_array_equal(ids[qi], order)
        np.testing.assert_allclose(dist[qi], d[order], rtol=1e-9)
        assert np.all(np.diff(dist[qi]) >= 0)



def _line_index():
    """Six lists with centroids at x = 0, 10, ..., 50 on the first axis; list l
    holds rows 2l (residual code 0 = (0, 0)) and 2l + 1 (code 1 = (0, 1))."""
    cc = np.array([[10.0 * l, 0.0] for l in range(6)], np.float32)
    pcb = np.array([[[0.0, 0.0], [0.0, 1.0]]], np.float32)     # m = 1, ks = 2, ds = 2
    offsets = np.arange(0, 13, 2, dtype=np.int64)
    ids = np.arange(12, dtype=np.int64)
    codes = (ids % 2).reshape(12, 1)
    return cc, pcb, offsets, ids, codes


@pytest.mark.parametrize("decide", ["kernel", "fp64"])
def test_adc_probes_the_nearest_lists_with_ties_to_the_lower_list(decide):
    cc, pcb, off, ids, codes = _line_index()
    q = np.array([[30.0, 0.0], [25.0, 0.0]], np.float32)
    # query 0: list distances 900, 400, 100, 0, 100, 400 -> lists 3 then 2
    # (2 and 4 tie at the boundary; the lower list wins)
    # query 1: 625, 225, 25, 25, 225, 625 -> list 2 alone at nprobe = 1
    got_ids, got_d = ivf.adc_search(q, cc, pcb, off, ids, codes, nprobe=2, topk=6, decide=decide)
    np.testing.assert_array_equal(got_ids[0], [6, 7, 4, 5, -1, -1])
    np.testing.assert_array_equal(got_d[0], [0.0, 1.0, 100.0, 101.0, np.inf, np.inf])
    np.testing.assert_array_equal(got_ids[1], [4, 6, 5, 7, -1, -1])
    np.testing.assert_array_equal(got_d[1], [25.0, 25.0, 26.0, 26.0, np.inf, np.inf])
    got_ids, got_d = ivf.adc_search(q, cc, pcb, off, ids, codes, nprobe=1, topk=3, decide=decide)
    np.testing.assert_array_equal(got_ids, [[6, 7, -1], [4, 5, -1]])
    # query 0 at nprobe = 3 takes lists 3, 2 and 4: equal scores order by id
    got_ids, got_d = ivf.adc_search(q[:1], cc, pcb, off, ids, codes, nprobe=3, topk=6, decide=decide)
    np.testing.assert_array_equal(got_ids[0], [6, 7, 4, 8, 5, 9])
    np.testing.assert_array_equal(got_d[0], [0.0, 1.0, 100.0, 100.0, 101.0, 101.0])
    # query 1 at nprobe = 3: lists 2 and 3 (tied), then 1 (1 and 4 tie)
    got_ids, _ = ivf.adc_search(q[1:], cc, pcb, off, ids, codes, nprobe=3, topk=12, decide=decide)
    assert set(got_ids[0][got_ids[0] >= 0]) == {2, 3, 4, 5, 6, 7}


def test_adc_probe_selection_matches_brute_force_below_full_probing():
    # nprobe < Kc on a real index: the probed lists are the nprobe smallest
    # (distance, list) pairs of a plain Python sort, and the results are the
    # brute-force top-k over the decoded rows of exactly those lists
    w, idx = _small_index()
    cc32 = idx["coarse"].astype(np.float32)
    pcb = idx["pq"].astype(np.float32)
    kc, nprobe, topk = cc32.shape[0], 5, 20
    got_ids, got_d = ivf.adc_search(w.queries, cc32, pcb, idx["offsets"], idx["ids"], idx["codes"],
                                    nprobe=nprobe, topk=topk, decide="fp64")
    xhat = cc32.astype(np.float64)[idx["labels"]] + pq.decode(idx["codes"], pcb)
    checked = 0
    for qi in range(w.queries.shape[0]):
        qv = [float(v) for v in w.queries[qi]]
        dl = []
        for l in range(kc):
            acc = 0.0
            for t in range(len(qv)):
                diff = qv[t] - float(cc32[l, t])
                acc += diff * diff
            dl.append((acc, l))
        dl.sort()
        if dl[nprobe][0] - dl[nprobe - 1][0] <= 1e-9 * dl[nprobe][0]:
            continue   # a near-tie at the probe boundary
        probed = {l for _, l in dl[:nprobe]}
        rows = [i for i in range(len(idx["labels"])) if idx["labels"][i] in probed]
        assert set(got_ids[qi][got_ids[qi] >= 0]) <= set(rows)
        score = {i: float(((w.queries[qi].astype(np.float64) - xhat[i]) ** 2).sum()) for i in rows}
        want = sorted((score[i], i) for i in rows)[:topk]
        gi = got_ids[qi][:len(want)]
        np.testing.assert_allclose(got_d[qi][:len(want)], [v for v, _ in want], rtol=1e-9)
        # every returned id carries its own brute-force score ...
        np.testing.assert_allclose([score[int(i)] for i in gi], got_d[qi][:len(want)], rtol=1e-9)
        # ... and the ids clearly inside the top-k are exactly the brute-force ones
        edge = want[-1][0] * (1 - 1e-9)
        assert {i for v, i in want if v < edge} == {int(i) for i in gi if score[int(i)] < edge}
        checked += 1
    assert checked >= 8

def test_adc_kernel_mode_sorted_and_close_to_fp64():
    w, idx = _small_index()
    cc32 = idx["coarse"].astype(np.float32)
    pcb = idx["pq"].astype(np.float32)
    a = ivf.adc_search(w.queries, cc32, pcb, idx["offsets"], idx["ids"], idx["codes"], 4, 20, "kernel")
    b = ivf.adc_search(w.queries, cc32, pcb, idx["offsets"], idx["ids"], idx["codes"], 4, 20, "fp64")
    np.testing.assert_allclose(a[1], b[1], rtol=2e-5)
    for qi in range(a[0].shape[0]):
        assert np.all(np.diff(a[1][qi]) >= 0)
        if np.all(np.diff(b[1][qi]) > 1e-5 * b[1][qi][1:]):
            np.testing.assert_array_equal(a[0][qi], b[0][qi])


def test_adc_pads_when_lists_are_short():
    w, idx = _small_index()
    cc32 = idx["coarse"].astype(np.float32)
    pcb = idx["pq"].astype(np.float32)
    ids, dist = ivf.adc_search(w.queries[:2], cc32, pcb, idx["offsets"], idx["ids"], idx["codes"],
                               nprobe=1, topk=3000, decide="kernel")
    for qi in range(2):
        n_real = int((ids[qi] >= 0).sum())
        assert n_real < 3000
        assert np.all(ids[qi, n_real:] == -1) and np.all(np.isinf(dist[qi, n_real:]))


def test_merge_hand_worked_two_parts():
    # part 0: rows 0..2 with labels (1, 0, 1); part 1: rows 0..1 with labels (0, 0)
    p0 = dict(offsets=np.array([0, 1, 3]), ids=np.array([1, 0, 2]), codes=np.array([[5], [6], [7]]))
    p1 = dict(offsets=np.array([0, 2, 2]), ids=np.array([0, 1]), codes=np.array([[8], [9]]))
    r = ivf.merge([p0, p1])
    assert r["offsets"].tolist() == [0, 3, 5]
    assert r["ids"].tolist() == [1, 3, 4, 0, 2]
    assert r["codes"][:, 0].tolist() == [5, 6, 7, 8, 9]
    # an empty part changes nothing
    pe = dict(offsets=np.zeros(3, np.int64), ids=np.zeros(0, np.int64), codes=np.zeros((0, 1), np.int64))
    r2 = ivf.merge([pe, p0, pe, p1, pe])
    assert r2["offsets"].tolist() == r["offsets"].tolist() and r2["ids"].tolist() == r["ids"].tolist()


def test_merge_of_chunk_adds_equals_the_index_of_all_rows():
    w, idx = _small_index()
    cc32 = idx["coarse"].astype(np.float32)
    pcb = idx["pq"].astype(np.float32).astype(np.float64)
    whole = ivf.add(w.x, cc32, pcb)
    np.testing.assert_array_equal(whole["labels"], idx["labels"])
    np.testing.assert_array_equal(whole["offsets"], idx["offsets"])
    np.testing.assert_array_equal(whole["ids"], idx["ids"])
    cuts = [0, 1, 700, 700, 1999, 3000]
    parts = [ivf.add(w.x[a:b], cc32, pcb) for a, b in zip(cuts[:-1], cuts[1:])]
    r = ivf.merge(parts)
    np.testing.assert_array_equal(r["offsets"], whole["offsets"])
    np.testing.assert_array_equal(r["ids"], whole["ids"])
    np.testing.assert_array_equal(r["codes"], whole["codes"])
    # the merged lists are the definition: list l = ascending ids with label l
    for l in range(len(r["offsets"]) - 1):
        got = r["ids"][r["offsets"][l]:r["offsets"][l + 1]]
        np.testing.assert_array_equal(got, np.flatnonzero(idx["labels"] == l))


# ---------------------------------------------------------------- the paper's chunked fit

def test_single_chunk_two_level_fit_reproduces_direct_fit():
    w = wl.plain_pq(seed=20, n=800, m=4, ks=16, iters=5)
    direct = pq.lloyd(w.x, w.init_rows, 4, 5)
    ident = np.tile(np.arange(16), (4, 1))
    two = chunked.two_level_fit([w.x], [w.init_rows], ident, 4, 5)
    np.testing.assert_allclose(two["codebook"], direct["codebook"].astype(np.float32), rtol=0, atol=0)


def test_paper_sizing_examples():
    vals = {}
    with open(os.path.join(GOLDEN, "paper_sizes.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                vals[k] = int(v)
    assert 10_000_000 // vals["rows_10m_chunks"] == vals["rows_per_chunk_10m"]
    assert vals["soilgrids_rows"] // vals["soilgrids_chunks"] == vals["soilgrids_rows_per_chunk"]
    x = _rand(21, 10, 48)
    init = np.tile(np.arange(4), (vals["subspaces_example"], 1))
    cb = pq.init_codebook(x, init, vals["subspaces_example"])
    codes, _ = pq.encode(x, cb)
    assert codes.shape[1] == vals["codes_per_row_example"]


# ---------------------------------------------------------------- optimized PQ

def _orthogonal(seed, d):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((d, d)))
    return q * np.sign(np.diag(r))[None, :]


def test_rotation_by_a_permutation_and_identity_is_exact():
    x = _rand(30, 200, 24)
    perm = np.random.default_rng(31).permutation(24)
    p = np.eye(24)[perm].T          # (x P)[:, j] = x[:, perm[j]]
    np.testing.assert_array_equal(opq.rotate(x, p), x[:, perm])
    np.testing.assert_array_equal(opq.rotate(x, np.eye(24)), x)



def test_rotation_sums_products_in_ascending_order_without_fusion():
    # Hand-worked values where the summation order and fusion change the
    # result.  Order: 1 + 2^-60 rounds to 1, so ascending t gives
    # ((1 + 2^-60) - 1) + 2^-60 = 2^-60, while descending t or pairwise
    # sums give 0.
    x = np.array([[1.0, 2.0 ** -60, -1.0, 2.0 ** -60]], np.float32)
    assert opq.rotate(x, np.ones((4, 1)))[0, 0] == np.float32(2.0 ** -60)
    # Fusion: with a = 1 + 2^-23 and r = 1 + 2^-52, fl64(a r) = 1 + 2^-23 + 2^-52
    # (the 2^-75 term is lost), so the separately rounded a r - a r is exactly
    # 0; a fused multiply-add of the second term would leave -2^-75.
    a = np.float32(1.0 + 2.0 ** -23)
    r = 1.0 + 2.0 ** -52
    y = opq.rotate(np.array([[a, -a]], np.float32), np.array([[r, 1.0], [r, 1.0]]))
    assert y[0, 0] == 0.0 and not np.signbit(y[0, 0])
    assert y[0, 1] == 0.0
    # One rounding to float32 at the end: 1 + 3 * 2^-25 (exact in float64)
    # rounds to 1 + 2^-23, whereas float32 partial sums would stay at 1.
    z = opq.rotate(np.array([[1.0, 2.0 ** -25, 2.0 ** -25, 2.0 ** -25]], np.float32), np.ones((4, 1)))
    assert z[0, 0] == np.float32(1.0 + 2.0 ** -23)

def test_procrustes_recovers_a_known_rotation():
    x = _rand(32, 500, 16).astype(np.float64)
    q = _orthogonal(33, 16)
    r, m = opq.procrustes(x, x @ q)
    np.testing.assert_allclose(r, q, atol=1e-10)
    np.testing.assert_allclose(m, x.T @ x @ q, rtol=1e-12, atol=1e-9)


def test_procrustes_is_orthogonal_and_beats_other_rotations():
    x = _rand(34, 300, 12).astype(np.float64)
    y = _rand(35, 300, 12).astype(np.float64)
    r, _ = opq.procrustes(x, y)
    np.testing.assert_allclose(r.T @ r, np.eye(12), atol=1e-12)
    best = np.linalg.norm(x @ r - y)
    for s in range(100):
        assert best <= np.linalg.norm(x @ _orthogonal(100 + s, 12) - y) + 1e-12
    # and every small rotation away from R (Cayley transform of a small skew matrix)
    rng = np.random.default_rng(36)
    for _ in range(50):
        a = 1e-3 * rng.standard_normal((12, 12))
        k = a - a.T
        c = np.linalg.solve(np.eye(12) + k, np.eye(12) - k)
        assert best <= np.linalg.norm(x @ (r @ c) - y) + 1e-12


def test_first_outer_iteration_is_plain_pq_and_objective_falls():
    x = wl.gaussian_mixture(37, 2000, 16, 30, sigma=0.1)
    x = (x.astype(np.float64) @ _orthogonal(38, 16)).astype(np.float32)   # correlated dimensions
    init = wl.init_rows_per_subspace(37, 2000, 4, 16)
    fit1 = opq.opq_fit(x, init, 4, 1, 3)
    ref = pq.lloyd(x, init, 4, 3, decide="fp32")
    np.testing.assert_array_equal(fit1["codebook"], ref["codebook"].astype(np.float32).astype(np.float64))
    # the first Procrustes step cannot raise the distortion of plain PQ (R = I)
    codes, _ = pq.encode(x, fit1["codebook"], decide="fp32")
    e_pq = opq.distortion(x, np.eye(16), codes, fit1["codebook"])
    assert fit1["objective"][0] <= e_pq * (1 + 1e-6)
    fit = opq.opq_fit(x, init, 4, 6, 2)
    obj = fit["objective"]
    assert np.all(np.diff(obj) <= 1e-5 * obj[:-1])
    assert obj[-1] < 0.97 * e_pq
    np.testing.assert_allclose(fit["R"].T @ fit["R"], np.eye(16), atol=1e-12)


def test_plain_pq_golden_file_is_the_oracles():
    """The stored results of the 10,000-row plain PQ workload (written by
    tests/golden/make_plain_pq_fit.py from the oracle) agree with a fresh oracle
    run on its first two rounds and on a sample of the final codes."""
    g = np.load(os.path.join(GOLDEN, "plain_pq_fit.npz"), allow_pickle=False)
    w = wl.plain_pq()
    two = pq.lloyd(w.x, w.init_rows, w.m, 2, decide="fp32")
    np.testing.assert_array_equal(two["objective"], g["objective"][:2])
    np.testing.assert_array_equal(two["near_ties"], g["near_ties"][:2])
    obj = g["objective"]
    assert np.all(np.diff(obj) <= 1e-12 * obj[:-1])
    rows = np.arange(0, w.x.shape[0], 97)
    c32, _, tie = pq.assign(w.x[rows], g["codebook"], "fp32")
    c64, _, _ = pq.assign(w.x[rows], g["codebook"], "fp64")
    np.testing.assert_array_equal(c32, g["codes"][rows])
    np.testing.assert_array_equal(c64, g["codes_fp64_decision"][rows])
    full_tie = np.unpackbits(g["codes_near_tie"])[:w.x.shape[0] * w.m].reshape(w.x.shape[0], w.m).astype(bool)
    np.testing.assert_array_equal(tie, full_tie[rows])
    cb32 = g["codebook"].astype(np.float32).astype(np.float64)
    sse, rmse = pq.sse_rmse(w.x, g["codes"].astype(np.int64), cb32)
    assert (sse, rmse) == tuple(g["sse_rmse"])
