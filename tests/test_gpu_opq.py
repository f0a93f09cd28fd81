"""GPU parity of optimized PQ (rotation, Procrustes step, alternating fit)
against the oracle: the rotation bit for bit, the cross matrix and the
rotation to float64 tolerances, the fit in lockstep (every outer iteration
restarted from the GPU's own rotation and codebook)."""

import numpy as np
import pytest
import torch

import paper_2604_21645_amd as mipq
from oracle import opq, pq
from synth import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _orthogonal(seed, d):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((d, d)))
    return q * np.sign(np.diag(r))[None, :]


def _correlated(seed, n, d, n_comp=30, sigma=0.1):
    x = wl.gaussian_mixture(seed, n, d, n_comp, sigma=sigma)
    return (x.astype(np.float64) @ _orthogonal(seed + 1, d)).astype(np.float32)


@pytest.mark.parametrize("n,d", [(1000, 128), (777, 48), (130, 256), (65, 3), (1, 1), (0, 16), (3001, 72)])
@pytest.mark.parametrize("kind", ["orthogonal", "general"])
def test_rotate_matches_oracle_bit_for_bit(n, d, kind):
    print("rotate", n, d, kind, flush=True)
    x = wl.gaussian_mixture(n + d, max(n, 1), d, 20, sigma=0.3)[:n]
    r = _orthogonal(d, d) if kind == "orthogonal" else np.random.default_rng(d).standard_normal((d, d))
    y = mipq.rotate(_t(x), _t(r)).cpu().numpy()
    np.testing.assert_array_equal(y, opq.rotate(x, r))


@pytest.mark.parametrize("n,d", [(5000, 48), (4000, 128), (3000, 256), (500, 7), (2, 2)])
def test_procrustes_matches_oracle(n, d):
    print("procrustes", n, d, flush=True)
    rng = np.random.default_rng(n + d)
    x = rng.standard_normal((n, d)).astype(np.float32)
    yh = (x + 0.5 * rng.standard_normal((n, d))).astype(np.float32)
    r, m, sw = mipq.procrustes(_t(x), _t(yh))
    rr, mref = opq.procrustes(x, yh)
    m = m.cpu().numpy()
    r = r.cpu().numpy()
    assert np.abs(m - mref).max() <= 1e-12 * np.abs(mref).max()
    np.testing.assert_allclose(r.T @ r, np.eye(d), atol=1e-12)
    np.testing.assert_allclose(r, rr, atol=1e-9)
    assert 0 < int(sw.item()) <= 64
    # results repeat bit for bit
    r2, m2, _, v = mipq.procrustes(_t(x), _t(yh), return_v=True)
    assert np.array_equal(r2.cpu().numpy(), r) and np.array_equal(m2.cpu().numpy(), m)
    # V is orthogonal and R = U V^T with U = M V S^-1 (full-rank M)
    vv = v.cpu().numpy()
    np.testing.assert_allclose(vv.T @ vv, np.eye(d), atol=1e-12)
    # a warm start (V of this M, or any orthogonal matrix) gives the same R
    r3, _, sw3 = mipq.procrustes(_t(x), _t(yh), v_init=v)
    np.testing.assert_allclose(r3.cpu().numpy(), rr, atol=1e-9)
    assert int(sw3.item()) <= 2 < int(sw.item()) or d <= 2
    r4, _, _ = mipq.procrustes(_t(x), _t(yh), v_init=_t(_orthogonal(d + 7, d)))
    np.testing.assert_allclose(r4.cpu().numpy(), rr, atol=1e-9)


def test_procrustes_recovers_a_known_rotation():
    x = _correlated(40, 6000, 64)
    q = _orthogonal(41, 64)
    yh = opq.rotate(x, q)
    r, _, _ = mipq.procrustes(_t(x), _t(yh))
    np.testing.assert_allclose(r.cpu().numpy(), q, atol=1e-5)


def test_procrustes_rank_deficient_and_empty():
    rng = np.random.default_rng(42)
    x = rng.standard_normal((2000, 32)).astype(np.float32)
    x[:, 5:10] = 0.0                        # M has five zero rows
    yh = rng.standard_normal((2000, 32)).astype(np.float32)
    r, _, sw = mipq.procrustes(_t(x), _t(yh))
    r = r.cpu().numpy()
    np.testing.assert_allclose(r.T @ r, np.eye(32), atol=1e-12)
    rr, _ = opq.procrustes(x, yh)
    x64, y64 = x.astype(np.float64), yh.astype(np.float64)
    best = np.linalg.norm(x64 @ rr - y64)
    assert np.linalg.norm(x64 @ r - y64) == pytest.approx(best, rel=1e-12)
    # no rows: M = 0 and R = I
    e = torch.empty((0, 12), dtype=torch.float32, device=DEV)
    r0, m0, _ = mipq.procrustes(e, e)
    np.testing.assert_array_equal(r0.cpu().numpy(), np.eye(12))
    assert not m0.cpu().numpy().any()
    # all-zero rows: the same
    z = torch.zeros((100, 12), dtype=torch.float32, device=DEV)
    rz, _, _ = mipq.procrustes(z, z)
    np.testing.assert_array_equal(rz.cpu().numpy(), np.eye(12))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_opq_fit_lockstep_with_oracle(prec):
    x = _correlated(43, 3000, 32)
    m, ks, outer, inner = 4, 16, 4, 2
    init = wl.init_rows_per_subspace(43, x.shape[0], m, ks)
    print("opq fit", prec, flush=True)
    out = mipq.opq_fit(_t(x), m, ks, outer, inner, _t(init), precision=prec, history=True)
    obj = out["objective"].cpu().numpy()
    r_prev = np.eye(32)
    cb_prev = pq.init_codebook(x, init, m).astype(np.float32).astype(np.float64)
    for it in range(outer):
        y = opq.rotate(x, r_prev)
        fit = pq.lloyd(y, None, m, inner, decide="fp32", init_codebook_value=cb_prev)
        cb = out["codebooks"][it].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(cb, fit["codebook"], rtol=1e-6, atol=1e-7)
        codes, _ = pq.encode(y, cb, decide="fp32")
        rr, _ = opq.procrustes(x, pq.decode(codes, cb).astype(np.float32))
        r = out["rotations"][it].cpu().numpy()
        np.testing.assert_allclose(r, rr, atol=1e-9)
        sse, _ = pq.sse_rmse(opq.rotate(x, r), codes, cb)
        assert obj[it] == pytest.approx(sse, rel=1e-12)
        r_prev, cb_prev = r, cb
    # the alternation lowers the distortion below plain PQ's
    codes0, _ = pq.encode(x, out["codebooks"][0].cpu().numpy().astype(np.float64), decide="fp32")
    e_pq, _ = pq.sse_rmse(x, codes0, out["codebooks"][0].cpu().numpy().astype(np.float64))
    assert obj[0] <= e_pq * (1 + 1e-6) and obj[-1] < e_pq
    assert np.all(np.diff(obj) <= 1e-5 * obj[:-1])
    codes = mipq.opq_encode(_t(x), out["R"], out["codebook"], prec).cpu().numpy().astype(np.int64)
    ref, _ = pq.encode(opq.rotate(x, out["R"].cpu().numpy()), out["codebook"].cpu().numpy().astype(np.float64),
                       decide="fp32")
    np.testing.assert_array_equal(codes, ref)


def test_full_size_rotation_sampled():
    """1M x 128 rows (the integer-valued headline shape) rotated by a random
    orthogonal R: sampled rows bit for bit against the oracle."""
    x = wl.integer_pq().x
    r = _orthogonal(44, x.shape[1])
    y = mipq.rotate(_t(x), _t(r))
    rows = np.random.default_rng(45).choice(x.shape[0], 2000, replace=False)
    np.testing.assert_array_equal(y.cpu().numpy()[rows], opq.rotate(x[rows], r))
