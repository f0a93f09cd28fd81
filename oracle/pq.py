"""Product quantisation oracle: split, k-means codebooks, encode, decode, RMSE.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2.1 of the paper (fitting: split the dimensions into ``M``
subspaces and run k-means with ``Ks`` centroids in each; encoding: represent
each row of each subspace by its nearest subspace centroid, so a row becomes
``M`` codes) and Section 3 (encode, decode and report the reconstruction RMSE).

Readings taken where the paper is silent:
  * subspace j is the contiguous column block [j*ds, (j+1)*ds), ds = D / M;
  * k-means is Lloyd's iteration: a fixed number of (assign, update) rounds,
    no tolerance test; the initial centroids are given rows of the training
    set (one row list per subspace);
  * the distance is the squared Euclidean distance; equal distances go to
    the lowest centroid index;
  * an empty cluster keeps its previous centroid;
  * RMSE = sqrt(SSE / (N * D)) with SSE = sum of squared reconstruction errors.

Parity pins: brute force, scipy's vq/kmeans2 and closed forms in
``tests/test_oracle.py``.
"""

from __future__ import annotations

import numpy as np

NEAR_TIE_REL = 1e-5      # two best float64 distances within this relative gap
_CHUNK_ELEMS = 1 << 23   # bound on rows * Ks * ds elements per broadcast block


def subspace_width(d: int, m: int) -> int:
    """ds = D / M; the paper's split needs M to divide D."""
    if m <= 0 or d % m != 0:
        raise ValueError("D=%d is not divisible by M=%d" % (d, m))
    return d // m


def block(x: np.ndarray, j: int, ds: int) -> np.ndarray:
    """Columns of subspace j."""
    return x[:, j * ds:(j + 1) * ds]


def init_codebook(train: np.ndarray, init_rows: np.ndarray, m: int) -> np.ndarray:
    """Initial centroids: C[j, k] = the subspace-j block of training row init_rows[j, k]."""
    ds = subspace_width(train.shape[1], m)
    return np.stack([block(train, j, ds)[init_rows[j]].astype(np.float64) for j in range(m)])


def dist64(xs: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances [n, Ks] in float64 from the difference form."""
    diff = xs.astype(np.float64)[:, None, :] - np.asarray(c, dtype=np.float64)[None, :, :]
    return np.einsum("nkt,nkt->nk", diff, diff)


def dist32(xs: np.ndarray, c: np.ndarray) -> np.ndarray:
    """The GPU library's final-decision arithmetic for a subspace distance.

    float32 throughout, no fused multiply-add: each difference, each square
    and each running sum is rounded to float32, dimensions summed in
    ascending order starting from the first square.
    """
    xs = np.asarray(xs, dtype=np.float32)
    c = np.asarray(c, dtype=np.float32)
    acc = None
    for t in range(xs.shape[1]):
        diff = xs[:, None, t] - c[None, :, t]
        sq = diff * diff
        acc = sq if acc is None else acc + sq
    return acc


def _rows_per_chunk(ks: int, ds: int) -> int:
    return max(1, _CHUNK_ELEMS // max(1, ks * ds))


def near_tie_mask(d64: np.ndarray) -> np.ndarray:
    """True where the two smallest float64 distances are within NEAR_TIE_REL relative."""
    if d64.shape[1] < 2:
        return np.zeros(d64.shape[0], dtype=bool)
    two = np.partition(d64, 1, axis=1)[:, :2]
    d1, d2 = two[:, 0], two[:, 1]
    return (d2 - d1) <= NEAR_TIE_REL * d1


def assign(x: np.ndarray, codebook: np.ndarray, decide: str = "fp64"):
    """Nearest centroid per (row, subspace).

    ``codebook`` is [M, Ks, ds].  ``decide="fp64"`` takes the argmin of the
    float64 distances; ``decide="fp32"`` takes it from ``dist32`` against the
    float32-rounded codebook (what the GPU computes).  Ties go to the lowest
    index (numpy's argmin returns the first minimum).

    Returns (codes [N, M] int64, dmin [N, M] float64 distance of the chosen
    centroid, near_tie [N, M] bool).
    """
    m, ks, ds = codebook.shape
    n = x.shape[0]
    codes = np.empty((n, m), dtype=np.int64)
    dmin = np.empty((n, m), dtype=np.float64)
    tie = np.empty((n, m), dtype=bool)
    c32 = codebook.astype(np.float32)
    step = _rows_per_chunk(ks, ds)
    for j in range(m):
        cj = codebook[j] if decide == "fp64" else c32[j].astype(np.float64)
        for r0 in range(0, n, step):
            xs = block(x[r0:r0 + step], j, ds)
            d64 = dist64(xs, cj)
            if decide == "fp64":
                a = np.argmin(d64, axis=1)
            elif decide == "fp32":
                a = np.argmin(dist32(xs, c32[j]), axis=1)
            else:
                raise ValueError(decide)
            codes[r0:r0 + step, j] = a
            dmin[r0:r0 + step, j] = d64[np.arange(len(a)), a]
            tie[r0:r0 + step, j] = near_tie_mask(d64)
    return codes, dmin, tie


def update(train: np.ndarray, codes: np.ndarray, old: np.ndarray):
    """Lloyd update: centroid = mean of its rows (float64); empty keeps ``old``.

    Returns (new codebook [M, Ks, ds], counts [M, Ks] int64, sums [M, Ks, ds]).
    """
    m, ks, ds = old.shape
    new = np.empty_like(old, dtype=np.float64)
    cnt = np.empty((m, ks), dtype=np.int64)
    sums = np.empty((m, ks, ds), dtype=np.float64)
    for j in range(m):
        lab = codes[:, j]
        cnt[j] = np.bincount(lab, minlength=ks)
        xs = block(train, j, ds).astype(np.float64)
        for t in range(ds):
            sums[j, :, t] = np.bincount(lab, weights=xs[:, t], minlength=ks)
        filled = cnt[j] > 0
        new[j] = old[j]
        new[j, filled] = sums[j, filled] / cnt[j, filled, None]
    return new, cnt, sums


def lloyd(train: np.ndarray, init_rows: np.ndarray, m: int, iters: int, decide: str = "fp64",
          init_codebook_value: np.ndarray | None = None):
    """Fit M per-subspace k-means codebooks with ``iters`` Lloyd rounds.

    Each round assigns every training row against the current codebook, then
    replaces every non-empty centroid with the mean of its rows.  Returns a
    dict with the final float64 codebook, the codes of the last assignment,
    the objective J_t (sum of float64 distances of the chosen centroids) of
    every round and the near-tie count of every round.
    """
    c = (init_codebook(train, init_rows, m) if init_codebook_value is None
         else np.asarray(init_codebook_value, dtype=np.float64).copy())
    objective, ties = [], []
    codes = None
    for _ in range(iters):
        codes, dmin, tie = assign(train, c, decide)
        objective.append(float(dmin.sum()))
        ties.append(int(tie.sum()))
        c, _, _ = update(train, codes, c)
    return dict(codebook=c, codes=codes, objective=np.array(objective), near_ties=np.array(ties))


def encode(x: np.ndarray, codebook: np.ndarray, decide: str = "fp64"):
    """Codes [N, M] (int64) plus the near-tie mask, against a fixed codebook."""
    codes, _, tie = assign(x, codebook, decide)
    return codes, tie


def decode(codes: np.ndarray, codebook: np.ndarray) -> np.ndarray:
    """x_hat = concatenation over subspaces of the coded centroids, float64 [N, D]."""
    m = codebook.shape[0]
    cb = np.asarray(codebook, dtype=np.float64)
    return np.concatenate([cb[j][codes[:, j]] for j in range(m)], axis=1)


def sse_rmse(x: np.ndarray, codes: np.ndarray, codebook: np.ndarray):
    """(SSE, RMSE) of the reconstruction, float64, RMSE = sqrt(SSE / (N * D))."""
    diff = x.astype(np.float64) - decode(codes, codebook)
    sse = float(np.einsum("nd,nd->", diff, diff))
    n, d = x.shape
    return sse, float(np.sqrt(sse / (n * d))) if n * d else 0.0
