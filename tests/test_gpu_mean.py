"""GPU parity of the posterior mean (MAP point, Sec. 2 eq. map1): the
block-Lanczos solve of (G + I) u = P^{-1} sigma^{-2} F^T y against the
oracle's data-space solution of the normal equations, for the workload's
seeded u_true / y_obs."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import synthetic  # noqa: E402
from oracle import mean  # noqa: E402
from oracle.spacetime import Problem as OP  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_05638_amd import lrpost
    lrpost.load()
    return lrpost


def _rel_err(W1, W2, ref):
    got = W1.cpu().numpy().T @ W2
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


def test_posterior_mean_small_mesh_matches_oracle(lp):
    """16 x 16 mesh, nt = 10, tol 1e-12: the GPU mean against the oracle's
    data-space MAP point; the oracle's normal-equation residual of the GPU
    result is small too."""
    print("case posterior mean N=16 nt=10", flush=True)
    d = synthetic.ProblemDesc(N=16, nt=10, trunc_tol=1e-12, rank_cap=10)
    ora = OP.from_desc(d)
    y = mean.observe_data(ora, synthetic.u_true(d), synthetic.yobs_noise(ora.nobs, ora.nt))
    ref = mean.mean_dataspace(ora, y)
    prob = lp.Problem(d)
    assert prob.obs_count() == ora.nobs
    W1, W2, res = prob.posterior_mean(y, rtol=1e-10)
    err = _rel_err(W1, W2, ref)
    ne = mean.normal_equation_residual(ora, W1.cpu().numpy().T @ W2, y)
    print("mean rel err %.3e, residual estimate %.3e, oracle normal-equation residual %.3e, steps %d" %
          (err, res, ne, prob.stats()["lanczos_steps"]), flush=True)
    assert err < 1e-6
    assert ne < 1e-6


def test_posterior_mean_tiny_workload_matches_golden(lp):
    """32 x 32 mesh, nt = 40 (the tiny workload's problem and data, with the
    truncation tightened to 1e-12): the GPU mean against the oracle's stored
    data-space solution for u_true / y_obs.  The truncated applies bound what
    the residual can reach (their error scales with the largest eigenvalue,
    about 3.5e6, against the shift 1), and the error of the mean follows the
    residual times the ratio of the right-hand side to the solution."""
    print("case posterior mean tiny workload", flush=True)
    import dataclasses
    g = np.load(os.path.join(ROOT, "tests", "golden", "tiny_mean_oracle.npz"))
    d = dataclasses.replace(synthetic.TINY_FP64, trunc_tol=1e-12)
    prob = lp.Problem(d)
    W1, W2, res = prob.posterior_mean(g["y_obs"], max_vectors=1600, rtol=1e-9, allow_unconverged=True)
    err = _rel_err(W1, W2, g["mean"])
    print("tiny mean rel err %.3e, residual estimate %.3e, rank %d, steps %d" %
          (err, res, W1.shape[0], prob.stats()["lanczos_steps"]), flush=True)
    # conjugate gradients on G + I, whose spectrum spans 3.5e6 down to 0, gain
    # accuracy slowly: 800 Krylov vectors leave 1.4e-4, the bound below is for 1600
    assert err < 1e-4


def test_posterior_mean_vector_limit_returns_enoconv(lp):
    import torch  # noqa: F401
    print("case posterior mean enoconv", flush=True)
    d = synthetic.ProblemDesc(N=16, nt=10, trunc_tol=1e-12, rank_cap=10)
    ora = OP.from_desc(d)
    y = mean.observe_data(ora, synthetic.u_true(d), synthetic.yobs_noise(ora.nobs, ora.nt))
    prob = lp.Problem(d)
    with pytest.raises(lp.LrpostError) as ex:
        prob.posterior_mean(y, max_vectors=8, rtol=1e-12)
    assert ex.value.code == -3
    W1, W2, res = prob.posterior_mean(y, max_vectors=8, rtol=1e-12, allow_unconverged=True)
    assert res > 1e-12 and W1.shape[0] > 0
