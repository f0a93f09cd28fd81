"""The encode that allocates nothing (mipq_pq_encode_noalloc) against the
workspace encode (mipq_pq_encode): two calls in a row on one GPU, the second
with fewer rows, outputs passed in by the caller, in every precision."""

import numpy as np
import pytest
import torch

import paper_2604_21645_amd as mipq
from oracle import pq
from synth import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_noalloc_encode_equals_the_workspace_encode(prec):
    x = wl.gaussian_mixture(11, 5003, 128, 40, mean_hi=255.0, sigma=20.0, integer_clip=(0, 255))
    rng = np.random.default_rng(12)
    rows = np.stack([rng.choice(x.shape[0], 256, replace=False) for _ in range(16)])
    cb = pq.init_codebook(x, rows, 16).astype(np.float32)
    cbt = _t(cb)
    for n in (5003, 1777):   # the second call uses fewer rows of the same scratch
        print("noalloc", prec, n, flush=True)
        xt = _t(x[:n])
        ref = mipq.pq_encode_ex(xt, cbt, prec, min_dist=True, sse_rmse=True, rescored=True)
        codes = torch.empty((n, 16), dtype=torch.uint8, device=DEV)
        md = torch.empty((n, 16), dtype=torch.float32, device=DEV)
        sr = torch.empty(2, dtype=torch.float64, device=DEV)
        rs = torch.empty(1, dtype=torch.int64, device=DEV)
        mipq.pq_encode_noalloc(xt, cbt, prec, codes=codes, min_dist=md, sse_rmse=sr, rescored=rs)
        torch.cuda.synchronize()
        assert torch.equal(codes, ref["codes"])
        assert torch.equal(md, ref["min_dist"])
        assert torch.equal(sr, ref["sse_rmse"])   # same kernels, same partial layout
        assert torch.equal(rs, ref["rescored"])
        ref32, _, _ = pq.assign(x[:n], cb.astype(np.float64), "fp32")
        np.testing.assert_array_equal(codes.cpu().numpy().astype(np.int64), ref32)
