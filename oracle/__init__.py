"""Plain, slow, CPU oracle for the PQ / inverted-index hot path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this package:
only the test suite, the smoke check in ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` may call it.  It shares no code, header,
table or helper with the HIP library; both sides only read the seeded inputs
produced by the ``synth`` package.

Precision.  Floating-point inputs are float32 and are promoted exactly to
float64.  Every quantity the paper defines (distances, centroid means,
reconstruction error, loss and gradient) is computed in float64.  Where a
floating-point comparison decides an integer (a code, a list label, a top-k
membership) the oracle can take the decision in float64 (the exact reference)
or in the arithmetic the GPU library uses for its final decision (the
``decide="fp32"`` mode), so that the two can be compared bit for bit; codes
from the two modes differ only where the two best float64 distances are
within 1e-5 relative, which the oracle counts and reports as near-ties.

Modules
  pq     -- subspace split, k-means codebook fit, encode, decode, RMSE (Section 2.1)
  ivf    -- coarse quantiser, residual PQ, posting lists, ADC top-k search (Section 2.2)
  grad   -- reconstruction loss and its gradient with codes held fixed
  chunked -- the paper's chunk-then-pool two-level fit (Section 3)
  opq    -- optimized PQ: an orthogonal rotation learnt before PQ (Section 3.1.1)
"""

from . import pq, ivf, grad, chunked, opq  # noqa: F401
