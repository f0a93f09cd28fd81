"""Optimized product quantisation oracle: an orthogonal rotation learnt before PQ.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.1.1 of the paper names the two algorithms of its PQ library: PQ and
optimized PQ.  Optimized PQ (the non-parametric form of Ge, He, Ke and Sun,
"Optimized Product Quantization", 2013/2014) quantises y = x R with an
orthogonal D x D matrix R and alternates two minimisations of the distortion
E(R, C, codes) = sum_n || x_n R - y_hat_n ||^2, y_hat_n = decode(codes_n, C):

  * R fixed: Lloyd rounds of the subspace k-means on the rotated rows
    (``pq.lloyd``), continuing from the current codebook, then the codes of
    the rotated rows against the new codebook;
  * C and codes fixed: the orthogonal Procrustes problem
    min over orthogonal R of || X R - Y_hat ||_F, whose solution is R = U V^T
    for the singular value decomposition U S V^T = X^T Y_hat.

Neither step can raise E, so E is non-increasing over the outer iterations
(up to the float32 rounding of the rotated rows).  R starts at the identity.

Arithmetic of the GPU path that the oracle reproduces:
  * rotation     y[n][j] = float32( sum over t ascending of x[n][t] * R[t][j] )
                 with x promoted to float64, R float64, every product and
                 partial sum rounded to float64, one final rounding to
                 float32 (``rotate``, bit for bit);
  * cross matrix M = X^T Y_hat in float64 (any summation order: compared with
                 a tolerance);
  * Procrustes   R = U V^T from M, float64.
"""

from __future__ import annotations

import numpy as np

from . import pq


def rotate(x: np.ndarray, r: np.ndarray) -> np.ndarray:
    """y = x R: y_j = sum over t ascending of x_t * R[t][j], every product and
    every partial sum rounded to float64, the result rounded once to float32."""
    x64 = np.asarray(x, np.float64)
    r64 = np.asarray(r, np.float64)
    acc = np.zeros((x64.shape[0], r64.shape[1]), dtype=np.float64)
    for t in range(x64.shape[1]):
        acc = acc + x64[:, t:t + 1] * r64[t:t + 1, :]
    return acc.astype(np.float32)


def cross(x: np.ndarray, y_hat: np.ndarray) -> np.ndarray:
    """M = X^T Y_hat in float64."""
    return np.asarray(x, np.float64).T @ np.asarray(y_hat, np.float64)


def procrustes(x: np.ndarray, y_hat: np.ndarray):
    """The orthogonal R minimising || X R - Y_hat ||_F, and M = X^T Y_hat."""
    m = cross(x, y_hat)
    u, _, vt = np.linalg.svd(m)
    return u @ vt, m


def distortion(x: np.ndarray, r: np.ndarray, codes: np.ndarray, codebook: np.ndarray) -> float:
    """E = sum_n || x_n R - y_hat_n ||^2 in float64 (R float64, codebook as given)."""
    y = np.asarray(x, np.float64) @ np.asarray(r, np.float64)
    diff = y - pq.decode(codes, np.asarray(codebook, np.float64))
    return float(np.einsum("nd,nd->", diff, diff))


def opq_fit(x: np.ndarray, init_rows: np.ndarray, m: int, outer_iters: int, pq_iters: int):
    """Alternating optimisation from R = I and the codebook seeded from the
    rows ``init_rows`` of x (the rotation by I leaves x unchanged).

    Each outer iteration: y = rotate(x, R); ``pq_iters`` Lloyd rounds on y
    from the current codebook (decisions by the float32 exact rule); codes of
    y against the new codebook; R = Procrustes(x, decode(codes)).  The
    codebook used by the decode and carried on is the float32 one.

    Returns dict(R float64 [d, d], codebook float64 (float32 values) [m, ks, d/m],
    objective [outer_iters] = E after each Procrustes step, rotations list).
    """
    d = x.shape[1]
    r = np.eye(d)
    cb = pq.init_codebook(x, init_rows, m).astype(np.float32).astype(np.float64)
    objective, rotations = [], []
    for _ in range(outer_iters):
        y = rotate(x, r)
        fit = pq.lloyd(y, None, m, pq_iters, decide="fp32", init_codebook_value=cb)
        cb = fit["codebook"].astype(np.float32).astype(np.float64)
        codes, _ = pq.encode(y, cb, decide="fp32")
        r, _ = procrustes(x, pq.decode(codes, cb))
        rotations.append(r)
        objective.append(distortion(x, r, codes, cb))
    return dict(R=r, codebook=cb, objective=np.array(objective), rotations=rotations)
