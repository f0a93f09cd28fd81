"""Inverted-file oracle: coarse quantiser, residual PQ, posting lists, ADC top-k.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.2 of the paper describes an inverted index built from the PQ codes:
each row's id is stored under a bucket, and a query returns its first, second,
... k-th nearest neighbours.  The bucket here is a coarse k-means list (an
IVF-PQ index, the structure of the Rii library named in Section 3.1), and the
stored codes are PQ codes of the residual x - c_list.  The query scores every
row of its nearest ``nprobe`` lists with a per-(query, list) distance table
(asymmetric distance computation) and keeps the ``topk`` smallest.

Decision arithmetic (what the GPU library uses to turn distances into
integers, and what ``decide="kernel"`` reproduces bit for bit):
  * coarse distance  ||x - c||^2: float32 differences, squared and summed in
    float64 in ascending dimension order;
  * residual         r = x - c_label, rounded to float32 per element;
  * table entry      LUT[j][k] = subspace distance of (q - c_l) to C_j[k],
                     computed like ``pq.dist32``;
  * candidate score  s = sum over j ascending of LUT[j][code_j], float32;
  * ordering         by (distance, index), ascending.
``decide="fp64"`` uses float64 distances everywhere instead.
"""

from __future__ import annotations

import numpy as np

from . import pq


def coarse_dist(x: np.ndarray, cc: np.ndarray, decide: str = "kernel") -> np.ndarray:
    """[n, Kc] squared distances to the coarse centroids."""
    if decide == "fp64":
        return pq.dist64(x, cc)
    x32 = np.asarray(x, dtype=np.float32)
    c32 = np.asarray(cc, dtype=np.float32)
    acc = np.zeros((x32.shape[0], c32.shape[0]), dtype=np.float64)
    for t in range(x32.shape[1]):
        diff = (x32[:, None, t] - c32[None, :, t]).astype(np.float64)
        acc = acc + diff * diff
    return acc


def coarse_assign(x: np.ndarray, cc: np.ndarray, decide: str = "kernel", chunk: int = 2048):
    """Nearest coarse centroid (lowest index on ties) and the near-tie mask."""
    n = x.shape[0]
    lab = np.empty(n, dtype=np.int64)
    tie = np.empty(n, dtype=bool)
    for r0 in range(0, n, chunk):
        d = coarse_dist(x[r0:r0 + chunk], cc, decide)
        lab[r0:r0 + chunk] = np.argmin(d, axis=1)
        d64 = d if decide == "fp64" else pq.dist64(x[r0:r0 + chunk], np.asarray(cc, np.float32))
        tie[r0:r0 + chunk] = pq.near_tie_mask(d64)
    return lab, tie


def coarse_fit(train: np.ndarray, init_idx: np.ndarray, iters: int, decide: str = "kernel"):
    """k-means with Kc = len(init_idx) centroids over full rows (Lloyd, as in ``pq.lloyd``).

    In ``kernel`` mode each assignment is taken against the float32-rounded
    centroids with ``coarse_dist``; centroids are float64 means.
    """
    c = train[init_idx].astype(np.float64)
    kc = c.shape[0]
    objective = []
    lab = None
    for _ in range(iters):
        lab, _ = coarse_assign(train, c if decide == "fp64" else c.astype(np.float32), decide)
        diff = train.astype(np.float64) - c[lab] if decide == "fp64" else \
            train.astype(np.float64) - c.astype(np.float32).astype(np.float64)[lab]
        objective.append(float(np.einsum("nd,nd->", diff, diff)))
        cnt = np.bincount(lab, minlength=kc)
        sums = np.stack([np.bincount(lab, weights=train[:, t].astype(np.float64), minlength=kc)
                         for t in range(train.shape[1])], axis=1)
        filled = cnt > 0
        c = c.copy()
        c[filled] = sums[filled] / cnt[filled, None]
    return dict(codebook=c, labels=lab, objective=np.array(objective))


def residuals(x: np.ndarray, labels: np.ndarray, cc32: np.ndarray) -> np.ndarray:
    """r = x - c_label, float32 per element."""
    return np.asarray(x, np.float32) - np.asarray(cc32, np.float32)[labels]


def posting_lists(labels: np.ndarray, kc: int):
    """Bucket the ids by list: offsets [Kc+1] (exclusive prefix sum of the list
    sizes) and ids, ascending inside each list.  Written as its definition: list l
    holds exactly the ids whose label is l, in increasing order."""
    labels = np.asarray(labels)
    parts = [np.flatnonzero(labels == l) for l in range(kc)]
    counts = np.array([len(p) for p in parts], dtype=np.int64)
    offsets = np.zeros(kc + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    ids = np.concatenate(parts) if parts else np.zeros(0, np.int64)
    return offsets, ids.astype(np.int64)


def build(x: np.ndarray, train_rows: np.ndarray, coarse_init: np.ndarray, coarse_iters: int,
          m: int, pq_init: np.ndarray, pq_iters: int, decide: str = "kernel"):
    """Full index build: coarse fit on the sample, labels for all rows, residual
    PQ fitted on the sample's residuals, residual codes for all rows, posting lists."""
    train = x[train_rows]
    cf = coarse_fit(train, coarse_init, coarse_iters, decide)
    cc = cf["codebook"]
    cc32 = cc.astype(np.float32)
    labels, ltie = coarse_assign(x, cc32 if decide != "fp64" else cc, decide)
    tl, _ = coarse_assign(train, cc32 if decide != "fp64" else cc, decide)
    pdec = "fp32" if decide != "fp64" else "fp64"
    rtrain = residuals(train, tl, cc32)
    pf = pq.lloyd(rtrain, pq_init, m, pq_iters, decide=pdec)
    r = residuals(x, labels, cc32)
    codes, ctie = pq.encode(r, pf["codebook"], decide=pdec)
    offsets, ids = posting_lists(labels, cc.shape[0])
    return dict(coarse=cc, labels=labels, label_ties=ltie, pq=pf["codebook"], codes=codes,
                code_ties=ctie, offsets=offsets, ids=ids)


def add(x: np.ndarray, cc: np.ndarray, pq_cb: np.ndarray, decide: str = "kernel"):
    """Index of the rows ``x`` under fixed quantisers (the library's "add codes"
    step of Section 3.1.2): labels, residual codes and posting lists, with the
    row ids 0..n-1 of this ``x``."""
    cc32 = np.asarray(cc, np.float32)
    labels, _ = coarse_assign(x, cc32 if decide != "fp64" else cc, decide)
    codes, _ = pq.encode(residuals(x, labels, cc32), pq_cb, decide="fp32" if decide != "fp64" else "fp64")
    offsets, ids = posting_lists(labels, cc32.shape[0])
    return dict(labels=labels, codes=codes, offsets=offsets, ids=ids)


def merge(parts):
    """One index from indexes over consecutive row ranges (the library's
    "merge" step of Section 3.1.2).  ``parts``: dicts with offsets, ids and
    codes (codes by the part's own row id).  List l of the result is list l
    of part 0, then of part 1, ..., every id shifted by the number of rows in
    the parts before its own."""
    kc = len(parts[0]["offsets"]) - 1
    base, lists, codes = 0, [[] for _ in range(kc)], []
    for p in parts:
        off, ids = p["offsets"], p["ids"]
        for l in range(kc):
            lists[l].append(np.asarray(ids[off[l]:off[l + 1]], np.int64) + base)
        codes.append(p["codes"])
        base += len(p["ids"])
    flat = [np.concatenate(ls) for ls in lists]
    offsets = np.zeros(kc + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(f) for f in flat])
    return dict(offsets=offsets, ids=np.concatenate(flat), codes=np.concatenate(codes))


def adc_lut(q: np.ndarray, c_list: np.ndarray, pq_cb: np.ndarray) -> np.ndarray:
    """LUT[j][k] for one (query, list): subspace distance of (q - c_list) to C_j[k]."""
    m, ks, ds = pq_cb.shape
    r = np.asarray(q, np.float32) - np.asarray(c_list, np.float32)
    return np.stack([pq.dist32(r[None, j * ds:(j + 1) * ds], pq_cb[j])[0] for j in range(m)])


def adc_search(q: np.ndarray, cc: np.ndarray, pq_cb: np.ndarray, offsets: np.ndarray, ids: np.ndarray,
               codes_by_id: np.ndarray, nprobe: int, topk: int, decide: str = "kernel"):
    """Top-k (ids, distances) per query, sorted by (distance, id); padded with
    (-1, +inf) when fewer than topk candidates exist.

    ``codes_by_id[i]`` are the residual codes of row i.  In ``kernel`` mode the
    table and the sums are float32 as described in the module docstring; in
    ``fp64`` mode the score is ||(q - c_l) - r_hat||^2 in float64.
    """
    nq = q.shape[0]
    m, ks, ds = pq_cb.shape
    cc32 = np.asarray(cc, np.float32)
    out_ids = np.full((nq, topk), -1, dtype=np.int64)
    out_d = np.full((nq, topk), np.inf, dtype=np.float64)
    for i in range(nq):
        dq = coarse_dist(q[i:i + 1], cc32, "kernel" if decide != "fp64" else "fp64")[0]
        probes = np.lexsort((np.arange(len(dq)), dq))[:nprobe]
        cand_s, cand_id = [], []
        for l in probes:
            members = ids[offsets[l]:offsets[l + 1]]
            if len(members) == 0:
                continue
            cm = codes_by_id[members]
            if decide == "fp64":
                rq = q[i].astype(np.float64) - cc32[l].astype(np.float64)
                rhat = np.concatenate([pq_cb[j].astype(np.float64)[cm[:, j]] for j in range(m)], axis=1)
                diff = rq[None, :] - rhat
                s = np.einsum("nd,nd->n", diff, diff)
            else:
                lut = adc_lut(q[i], cc32[l], np.asarray(pq_cb, np.float32))
                s = lut[0][cm[:, 0]].astype(np.float32)
                for j in range(1, m):
                    s = s + lut[j][cm[:, j]]
            cand_s.append(np.asarray(s, np.float64))
            cand_id.append(members)
        if not cand_s:
            continue
        s = np.concatenate(cand_s)
        idv = np.concatenate(cand_id)
        order = np.lexsort((idv, s))[:topk]
        out_ids[i, :len(order)] = idv[order]
        out_d[i, :len(order)] = s[order]
    return out_ids, out_d
