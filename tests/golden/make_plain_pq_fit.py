"""Write tests/golden/plain_pq_fit.npz: the oracle's results on the 10,000-row
plain PQ workload (D=128, 64-component mixture, M=8, Ks=256, 20 Lloyd rounds
from 256 seeded rows per subspace).  It calls only oracle/ and synth/ (about a
minute of CPU), so the GPU test that reads it does not rerun the oracle.

    python tests/golden/make_plain_pq_fit.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pq  # noqa: E402
from synth import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "plain_pq_fit.npz")


def main():
    w = wl.plain_pq()
    f32 = pq.lloyd(w.x, w.init_rows, w.m, w.iters, decide="fp32")
    codes, _, tie = pq.assign(w.x, f32["codebook"], "fp32")
    codes_f64, _, _ = pq.assign(w.x, f32["codebook"], "fp64")
    # the error of the codes against the float32 codebook the library works with
    sse, rmse = pq.sse_rmse(w.x, codes, f32["codebook"].astype(np.float32).astype(np.float64))
    f64 = pq.lloyd(w.x, w.init_rows, w.m, w.iters, decide="fp64")
    codes64, _, _ = pq.assign(w.x, f64["codebook"], "fp64")
    _, rmse64 = pq.sse_rmse(w.x, codes64, f64["codebook"].astype(np.float32).astype(np.float64))
    np.savez_compressed(OUT, codebook=f32["codebook"], labels=f32["codes"].astype(np.uint8),
                        objective=f32["objective"], near_ties=f32["near_ties"], codes=codes.astype(np.uint8),
                        codes_fp64_decision=codes_f64.astype(np.uint8),
                        codes_near_tie=np.packbits(tie), sse_rmse=np.array([sse, rmse]),
                        rmse_fp64_fit=np.array([rmse64]), objective_fp64_fit=f64["objective"])
    print("wrote", OUT, "rmse", rmse, "fp64-decision fit rmse", rmse64)


if __name__ == "__main__":
    main()
