"""Seeded synthetic inputs with the shapes of the paper's PQ and inverted-index runs.

The paper evaluates on a 6.7M x 48 sample of the SoilGrids 250 m product
(Section 3), which is not available here; the workloads below are Gaussian
mixtures (and one unit-sphere mixture) with the sizes used for the
measurements of this project.  Every array is reproducible from an integer
seed: each logical stream (means, labels, noise, training sample, initial
rows, queries) and each 1M-row chunk of a large array draws from its own
``numpy.random.SeedSequence(seed, spawn_key=(stream, chunk))``, so a chunk can
be regenerated on its own and the result never depends on chunk scheduling.

Nothing here computes a distance, an assignment or a centroid.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# stream identifiers for SeedSequence spawn keys
S_MEANS, S_LABELS, S_NOISE, S_TRAIN, S_INIT, S_QUERY, S_SIZES, S_PICK = range(8)
CHUNK_ROWS = 1 << 20


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=tuple(key))))


def gaussian_mixture(seed: int, n: int, d: int, n_comp: int, *, mean_lo: float = 0.0,
                     mean_hi: float = 1.0, sigma: float = 0.05, integer_clip: Optional[tuple] = None,
                     sphere_kappa: Optional[float] = None, stream_offset: int = 0,
                     means: Optional[np.ndarray] = None) -> np.ndarray:
    """Draw ``n`` float32 rows from a uniform-weight mixture of ``n_comp`` components.

    * means ~ U[mean_lo, mean_hi)^d, or unit Gaussian directions when
      ``sphere_kappa`` is given (von Mises-like: x = normalise(mu + g / sqrt(kappa)));
    * x = mu[label] + sigma * g, g ~ N(0, I);
    * ``integer_clip=(lo, hi)`` rounds half-to-even and clips, giving
      non-negative integer-valued float32 rows.
    ``stream_offset`` separates a second draw from the same mixture (queries).
    """
    if means is None:
        rm = _rng(seed, S_MEANS)
        if sphere_kappa is not None:
            means = rm.standard_normal((n_comp, d))
            means /= np.linalg.norm(means, axis=1, keepdims=True)
        else:
            means = rm.uniform(mean_lo, mean_hi, size=(n_comp, d))
    out = np.empty((n, d), dtype=np.float32)
    for c0 in range(0, n, CHUNK_ROWS):
        c1 = min(n, c0 + CHUNK_ROWS)
        ci = c0 // CHUNK_ROWS
        lab = _rng(seed, S_LABELS + stream_offset, ci).integers(0, n_comp, size=c1 - c0)
        g = _rng(seed, S_NOISE + stream_offset, ci).standard_normal((c1 - c0, d))
        if sphere_kappa is not None:
            v = means[lab] + g / np.sqrt(sphere_kappa)
            v /= np.linalg.norm(v, axis=1, keepdims=True)
        else:
            v = means[lab] + sigma * g
            if integer_clip is not None:
                v = np.clip(np.rint(v), integer_clip[0], integer_clip[1])
        out[c0:c1] = v
    return out


def choose_rows(seed: int, n: int, k: int, stream: int = S_TRAIN, key: int = 0) -> np.ndarray:
    """``k`` distinct row indices of ``range(n)`` (ascending), int64."""
    if k > n:
        raise ValueError("cannot choose %d distinct rows out of %d" % (k, n))
    idx = _rng(seed, stream, key).choice(n, size=k, replace=False)
    return np.sort(idx).astype(np.int64)


def init_rows_per_subspace(seed: int, n_train: int, m: int, ks: int, key: int = 0) -> np.ndarray:
    """Initial rows for each subspace: ``[m, ks]`` int64, distinct within a subspace.

    Drawn in subspace order from one generator, without replacement, in draw
    order (not sorted: row k of subspace j seeds centroid k of subspace j).
    """
    rng = _rng(seed, S_INIT, key)
    return np.stack([rng.choice(n_train, size=ks, replace=False) for _ in range(m)]).astype(np.int64)


@dataclass
class Workload:
    """One PQ fit+encode problem.

    ``x`` is encoded; the codebook is fitted on ``x[train_rows]`` (all of
    ``x`` when ``train_rows`` is None); ``init_rows[j, k]`` indexes the
    training set and seeds centroid k of subspace j.
    """
    name: str
    x: np.ndarray
    m: int
    ks: int
    iters: int
    init_rows: np.ndarray
    train_rows: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def train(self) -> np.ndarray:
        return self.x if self.train_rows is None else self.x[self.train_rows]


def plain_pq(seed: int = 1, n: int = 10_000, d: int = 128, n_comp: int = 64, m: int = 8,
             ks: int = 256, iters: int = 20, sigma: float = 0.05) -> Workload:
    """Plain PQ fit+encode: mixture of ``n_comp`` components, means U[0,1)^d."""
    x = gaussian_mixture(seed, n, d, n_comp, sigma=sigma)
    init = init_rows_per_subspace(seed, n, m, ks)
    return Workload("plain_pq", x, m, ks, iters, init,
                    meta=dict(seed=seed, n=n, d=d, n_comp=n_comp, sigma=sigma))


def integer_pq(seed: int = 2, n: int = 1_000_000, d: int = 128, n_comp: int = 1000, m: int = 16,
               ks: int = 256, iters: int = 25, n_train: int = 100_000, sigma: float = 20.0) -> Workload:
    """Integer-valued rows in [0, 255]: clip(rint(mu + sigma g)), means U[0,255)^d.

    Fit on a seeded ``n_train``-row sample, encode all ``n`` rows.
    """
    x = gaussian_mixture(seed, n, d, n_comp, mean_lo=0.0, mean_hi=255.0, sigma=sigma,
                         integer_clip=(0.0, 255.0))
    train = choose_rows(seed, n, min(n_train, n))
    init = init_rows_per_subspace(seed, len(train), m, ks)
    return Workload("integer_pq", x, m, ks, iters, init, train_rows=train,
                    meta=dict(seed=seed, n=n, d=d, n_comp=n_comp, sigma=sigma, n_train=len(train)))


@dataclass
class BatchedWorkload:
    """Many independent PQ problems of uneven size drawn from one mixture."""
    problems: list
    m: int
    ks: int
    iters: int
    meta: dict = field(default_factory=dict)


def batched_uneven(seed: int = 3, n_prob: int = 64, n_lo: int = 20_000, n_hi: int = 500_000,
                   d: int = 96, n_comp: int = 2000, kappa: float = 50.0, m: int = 12, ks: int = 256,
                   iters: int = 20) -> BatchedWorkload:
    """Uneven chunks: N_i = floor(exp(U(ln n_lo, ln n_hi))), unit-norm rows.

    All problems come from one unit-sphere mixture (like row chunks of one
    dataset); each is fitted on all its rows from its own initial rows.
    """
    sizes = np.floor(np.exp(_rng(seed, S_SIZES).uniform(np.log(n_lo), np.log(n_hi), size=n_prob)))
    sizes = np.maximum(sizes.astype(np.int64), ks)
    total = int(sizes.sum())
    allx = gaussian_mixture(seed, total, d, n_comp, sphere_kappa=kappa)
    probs = []
    off = 0
    for i, ni in enumerate(sizes):
        xi = allx[off:off + ni]
        off += ni
        init = init_rows_per_subspace(seed, int(ni), m, ks, key=i)
        probs.append(Workload("batched_%d" % i, xi, m, ks, iters, init))
    return BatchedWorkload(probs, m, ks, iters, meta=dict(seed=seed, total=total, d=d, kappa=kappa))


@dataclass
class ChunkedWorkload:
    """Rows split into equal chunks (the paper's chunked layout), for the
    two-level fit: per-chunk init rows and init rows of the pooled centroids."""
    x: np.ndarray
    chunk_rows: int
    chunk_inits: list
    global_init: np.ndarray
    m: int
    ks: int
    iters: int
    meta: dict = field(default_factory=dict)

    @property
    def chunks(self):
        return [self.x[i:i + self.chunk_rows] for i in range(0, self.x.shape[0], self.chunk_rows)]


def soil_chunks(seed: int = 6, n_chunks: int = 400, chunk_rows: int = 16_750, d: int = 48, n_comp: int = 500,
                m: int = 8, ks: int = 256, iters: int = 20, sigma: float = 0.08) -> ChunkedWorkload:
    """Stand-in with the shape of the paper's data: 6.7M x 48 rows in 400
    chunks of 16,750 rows (Section 3's SoilGrids sample, which is not
    available).  A Gaussian mixture of ``n_comp`` components, means
    U[0,1)^48; M=8 gives 6-dimensional subspaces."""
    x = gaussian_mixture(seed, n_chunks * chunk_rows, d, n_comp, sigma=sigma)
    inits = [init_rows_per_subspace(seed, chunk_rows, m, ks, key=i) for i in range(n_chunks)]
    ginit = init_rows_per_subspace(seed, n_chunks * ks, m, ks, key=n_chunks + 1)
    return ChunkedWorkload(x, chunk_rows, inits, ginit, m, ks, iters,
                           meta=dict(seed=seed, n_chunks=n_chunks, chunk_rows=chunk_rows, d=d, n_comp=n_comp,
                                     sigma=sigma))


@dataclass
class IvfWorkload:
    """Inverted index with residual PQ, plus queries from the same mixture."""
    x: np.ndarray
    queries: np.ndarray
    kc: int
    coarse_iters: int
    coarse_train: np.ndarray       # rows of x used to fit the coarse quantiser (and residual PQ)
    coarse_init: np.ndarray        # [kc] indices into coarse_train
    m: int
    ks: int
    pq_iters: int
    pq_init: np.ndarray            # [m, ks] indices into coarse_train
    nprobe: int
    topk: int
    meta: dict = field(default_factory=dict)


def ivf_adc(seed: int = 4, n: int = 10_000_000, d: int = 128, n_comp: int = 4096, kc: int = 4096,
            n_query: int = 10_000, m: int = 16, ks: int = 256, coarse_iters: int = 20,
            pq_iters: int = 20, n_train: Optional[int] = None, nprobe: int = 32, topk: int = 100,
            sigma: float = 0.05) -> IvfWorkload:
    """IVF + ADC workload; the coarse training sample defaults to 64 * kc rows."""
    if n_train is None:
        n_train = min(n, 64 * kc)
    x = gaussian_mixture(seed, n, d, n_comp, sigma=sigma)
    q = gaussian_mixture(seed, n_query, d, n_comp, sigma=sigma, stream_offset=S_QUERY)
    train = choose_rows(seed, n, n_train)
    cinit = _rng(seed, S_INIT, 1).choice(n_train, size=kc, replace=False).astype(np.int64)
    pinit = init_rows_per_subspace(seed, n_train, m, ks, key=2)
    return IvfWorkload(x, q, kc, coarse_iters, train, cinit, m, ks, pq_iters, pinit, nprobe, topk,
                       meta=dict(seed=seed, n=n, d=d, n_comp=n_comp, sigma=sigma))


def diff_codebooks(seed: int = 5, n: int = 2_000_000, d: int = 256, n_comp: int = 8192, m: int = 32,
                   ks: int = 256, iters: int = 20, n_train: int = 200_000, sigma: float = 0.1) -> Workload:
    """Differentiable-codebook workload: fit on a sample, encode all rows."""
    x = gaussian_mixture(seed, n, d, n_comp, sigma=sigma)
    train = choose_rows(seed, n, min(n_train, n))
    init = init_rows_per_subspace(seed, len(train), m, ks)
    return Workload("diff_codebooks", x, m, ks, iters, init, train_rows=train,
                    meta=dict(seed=seed, n=n, d=d, n_comp=n_comp, sigma=sigma, n_train=len(train)))


def fd_entries(seed: int, n_rows: int, d: int, m: int, ks: int, ds: int, count: int = 1000):
    """Seeded entries for finite-difference checks: half codebook, half input."""
    rng = _rng(seed, S_PICK)
    half = count // 2
    cb = np.stack([rng.integers(0, m, half), rng.integers(0, ks, half), rng.integers(0, ds, half)], 1)
    xi = np.stack([rng.integers(0, n_rows, count - half), rng.integers(0, d, count - half)], 1)
    return cb.astype(np.int64), xi.astype(np.int64)
