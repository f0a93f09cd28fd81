"""The float32 facts behind the ADC scan's exact skips, checked with IEEE
float32 arithmetic on the host (no GPU):

  * a row's score is a float32 sum of non-negative table entries taken in a
    fixed order, so its running sum never decreases (rounding is monotone);
  * the running sum over the first P subspaces is at least the sum, in the
    same order, of the smallest entry of each of those P table rows.

So a row whose running sum already exceeds the bound's score, and a list
whose sum of minima exceeds it, cannot reach the top k, and skipping them
leaves the results unchanged."""

import numpy as np
import pytest


def _seq_sum(terms):
    """float32 running sums of terms[..., 0..M-1], left to right."""
    s = terms[..., 0].astype(np.float32)
    out = [s]
    for u in range(1, terms.shape[-1]):
        s = (s + terms[..., u]).astype(np.float32)
        out.append(s)
    return np.stack(out, axis=-1)


@pytest.mark.parametrize("seed,scale", [(0, 1.0), (1, 1e-3), (2, 1e6), (3, 0.0)])
def test_running_sums_do_not_decrease_and_bound_by_table_minima(seed, scale):
    rng = np.random.default_rng(seed)
    m, ks, n = 16, 256, 20000
    # non-negative entries over many magnitudes, with exact zeros and ties
    lut = (rng.random((m, ks)) ** 4 * scale).astype(np.float32)
    lut[:, :3] = 0.0
    lut[:, 3:8] = lut[:, 8:13]
    codes = rng.integers(0, ks, size=(n, m))
    terms = lut[np.arange(m)[None, :], codes]
    run = _seq_sum(terms)
    assert np.all(np.diff(run, axis=1) >= 0)
    lb = _seq_sum(lut.min(axis=1)[None, :])[0]
    for p in range(1, m + 1):
        assert np.all(run[:, p - 1] >= lb[p - 1])
    # the skip rules: with the bound at the k-th smallest score, every row
    # that belongs to the top k passes the row test at every depth
    score = run[:, -1]
    kth = np.sort(score)[99]
    top = score <= kth
    for p in range(1, m + 1):
        assert np.all(run[top, p - 1] <= kth)
    assert lb[m - 1] <= kth
