"""The paper's two-level chunked PQ fit (Section 3), as a CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3 splits the rows into chunks and fits PQ on each chunk independently.
Codes fitted per chunk only make sense inside that chunk, so each chunk
returns its decoded centroids instead (Ks rows of D values: centroid k of
every subspace, concatenated); the centroids of all chunks are pooled into a
"centroid dataset", a global PQ is fitted on it, and the original rows are
encoded and decoded with the global model to measure the RMSE.

Reading: "decoded centroids" of a chunk are the Ks vectors whose subspace-j
block is C_j[k], k = 0..Ks-1 (the decode of the code row (k, k, ..., k)).
"""

from __future__ import annotations

import numpy as np

from . import pq


def decoded_centroids(codebook: np.ndarray) -> np.ndarray:
    """[Ks, D]: row k is the concatenation of C_j[k] over the subspaces."""
    m, ks, ds = codebook.shape
    return np.concatenate([codebook[j] for j in range(m)], axis=1)


def two_level_fit(chunks, chunk_inits, global_init, m: int, iters: int, decide: str = "fp64"):
    """Fit each chunk, pool decoded centroids, fit the global codebook on the pool."""
    pooled = []
    for xc, ic in zip(chunks, chunk_inits):
        fit = pq.lloyd(xc, ic, m, iters, decide=decide)
        pooled.append(decoded_centroids(fit["codebook"]))
    pool = np.concatenate(pooled, axis=0).astype(np.float32)
    gfit = pq.lloyd(pool, global_init, m, iters, decide=decide)
    return dict(pool=pool, codebook=gfit["codebook"])
