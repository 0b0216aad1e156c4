"""Writes advdiff512_oracle_trajectory.json: the oracle's free-running trajectory of the
512 x 512 advection-diffusion sequence (GMRES(30), M = 20, SRHT s = 80, tol 1e-8, FP64),
steps 0..139: per-step iterations, kept ranks and initial relative residuals.

Calls only the input generators and the oracle.  About half an hour on 8 cores:
python tests/golden/make_advdiff512_trajectory.py
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from gen import config  # noqa: E402
from oracle.sequence import make_sequence  # noqa: E402


def main(steps=140):
    p, m = config(1)
    seq = make_sequence(p, m)
    out = []
    t0 = time.time()
    for i in range(steps):
        A = p.matrix(i).to_scipy()
        _, _, info = seq.step(A, p.rhs(i))
        out.append(dict(i=i, iters=int(info["iters"]), k=int(info["k"]), k2=int(info["k2"]),
                        relres0=float(info["relres0"]), relres=float(info["relres"])))
        print(i, info["iters"], f"{time.time() - t0:.0f}s", flush=True)
    meta = dict(workload="advdiff2d 512x512, M=20, SRHT s=80, Galerkin, GMRES(30), tol 1e-8, FP64",
                writer="tests/golden/make_advdiff512_trajectory.py (oracle only)")
    with open(os.path.join(HERE, "advdiff512_oracle_trajectory.json"), "w") as f:
        json.dump(dict(meta=meta, steps=out), f, indent=0)


if __name__ == "__main__":
    main()
