"""Reconstruction loss and its gradient with the codes held fixed.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With codes a fixed, x_hat_n = concat_j C_j[a_nj] and
    L = sum_n ||x_n - x_hat_n||^2                       (float64)
    dL/dx_n     = 2 (x_n - x_hat_n)
    dL/dC_j[k]  = 2 (cnt_jk C_j[k] - S_jk),  S_jk = sum of the subspace-j blocks
                  of the rows coded k, cnt_jk their number.
Setting dL/dC = 0 gives the k-means mean update of Section 2.1's fit, so right
after an update the codebook gradient for the codes used in it is zero.
An upstream scalar ``g`` multiplies both gradients.
"""

from __future__ import annotations

import numpy as np

from . import pq


def loss(x: np.ndarray, codes: np.ndarray, codebook: np.ndarray) -> float:
    diff = x.astype(np.float64) - pq.decode(codes, codebook)
    return float(np.einsum("nd,nd->", diff, diff))


def grads(x: np.ndarray, codes: np.ndarray, codebook: np.ndarray, g: float = 1.0):
    """(L, dL/dx [N, D], dL/dC [M, Ks, ds]) in float64."""
    cb = np.asarray(codebook, dtype=np.float64)
    m, ks, ds = cb.shape
    diff = x.astype(np.float64) - pq.decode(codes, cb)
    lval = float(np.einsum("nd,nd->", diff, diff))
    gx = 2.0 * g * diff
    gc = np.empty_like(cb)
    for j in range(m):
        lab = codes[:, j]
        cnt = np.bincount(lab, minlength=ks).astype(np.float64)
        xs = pq.block(x, j, ds).astype(np.float64)
        s = np.stack([np.bincount(lab, weights=xs[:, t], minlength=ks) for t in range(ds)], axis=1)
        gc[j] = 2.0 * g * (cnt[:, None] * cb[j] - s)
    return lval, gx, gc
