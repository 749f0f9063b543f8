"""Write the oracle's posterior mean for the 32x32 mesh, nt = 40 workload.

Calls only the oracle (and the seeded input module).  Output:
tests/golden/tiny_mean_oracle.npz with
  y_obs   observations F u_true + sigma * noise (seeds 0 and 1), shape (289, 40)
  mean    the MAP point by the data-space route, shape (961, 40)
  resid   its normal-equation residual with the time-stepping maps

Run:  python tests/golden/make_tiny_mean.py   (about a minute, ~8 GB RAM)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mean  # noqa: E402
from oracle.spacetime import Problem  # noqa: E402
import synthetic  # noqa: E402


def main():
    d = synthetic.TINY_FP64
    p = Problem.from_desc(d)
    t0 = time.time()
    y = mean.observe_data(p, synthetic.u_true(d), synthetic.yobs_noise(p.nobs, p.nt))
    u = mean.mean_dataspace(p, y)
    res = mean.normal_equation_residual(p, u, y)
    print("mean %.1f s, normal-equation residual %.3e" % (time.time() - t0, res), flush=True)
    np.savez_compressed(os.path.join(HERE, "tiny_mean_oracle.npz"), y_obs=y, mean=u, resid=res)


if __name__ == "__main__":
    main()
