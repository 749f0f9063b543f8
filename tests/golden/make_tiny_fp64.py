"""Write the oracle's expected values for the 32x32 mesh, nt = 40 workload.

Calls only the oracle (and the seeded input module).  Output:
tests/golden/tiny_fp64_oracle.npz with
  lam        top 40 pencil eigenvalues (data-space route)
  diag_k20   diag(Gamma_post,20), shape (961, 40)
  diag_exact diag((H_mis + P)^{-1}) by Woodbury in data space, shape (961, 40)
  dprior     diag(P^{-1}) over one step, shape (961,)
  vecs4      the first 4 P-orthonormal eigenvectors, shape (961*40, 4)

Run:  python tests/golden/make_tiny_fp64.py   (about 2-3 minutes, ~15 GB RAM)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import posterior  # noqa: E402
from oracle.spacetime import Problem  # noqa: E402
import synthetic  # noqa: E402


def main():
    d = synthetic.TINY_FP64
    p = Problem.from_desc(d)
    t0 = time.time()
    F = p.impulse_F()
    lam, V = posterior.eig_dataspace(p, 40, F=F)
    print("eig", time.time() - t0, lam[:4], flush=True)
    dprior = posterior.prior_diag_closed(p.N, p.alpha, p.tau)
    diag_k20 = posterior.post_diag_lowrank(p, lam[:20], V[:, :20], dprior)
    diag_exact = posterior.post_diag_exact_dataspace(p, F=F)
    print("exact", time.time() - t0, flush=True)
    np.savez_compressed(os.path.join(HERE, "tiny_fp64_oracle.npz"), lam=lam, diag_k20=diag_k20,
                        diag_exact=diag_exact, dprior=dprior, vecs4=V[:, :4])


if __name__ == "__main__":
    main()
