"""The initial-condition problem of the paper's experiments on the GPU (Sec. 6,
eqs. misfit and postvar; Sec. 6.2) against the oracle: the Hessian apply, the
eigenpairs, the posterior variance, the full-observation closed form and the
paper's nine-sensor setting at 64 x 64, nt = 30."""
import dataclasses
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import synthetic  # noqa: E402
from oracle.initial import ICProblem, full_obs_ic_eigs  # noqa: E402
from synthetic import sensor_mask  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_05638_amd import lrpost
    lrpost.load()
    return lrpost


def _problem(lp, N, nt, sigma, precision="fp64", tol=1e-10, rank_cap=16, mask=None):
    d = synthetic.ProblemDesc(N=N, nt=nt, sigma=sigma, trunc_tol=tol, rank_cap=rank_cap, k=8, precision=precision)
    prob = lp.Problem(d)
    prob.set_obs_mask(sensor_mask(N) if mask is None else mask)
    return prob


def _gap_cut(lam, kmax):
    """The largest k <= kmax whose eigenvalue is separated from the next one
    (the sensor layout's symmetry makes some eigenvalues double, and a cut
    inside such a pair leaves the eigenvectors undetermined)."""
    for k in range(kmax, 1, -1):
        if lam[k - 1] - lam[k] > 1e-4 * lam[0]:
            return k
    return 1


def test_ic_apply_matches_oracle(lp):
    import torch
    print("case ic apply N=16 nt=10", flush=True)
    N, nt, sigma, c = 16, 10, 0.03, 10.0
    prob = _problem(lp, N, nt, sigma)
    ora = ICProblem(N, nt, sigma=sigma, prior_var=c)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((3, ora.nx))
    Y = prob.ic_apply(torch.tensor(U, device="cuda"), c).cpu().numpy()
    for j in range(3):
        ref = ora.G(U[j])
        err = np.abs(Y[j] - ref).max() / np.abs(ref).max()
        print("ic apply rel err %.3e" % err, flush=True)
        assert err < 1e-8


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 2e-5)])
def test_ic_eigenpairs_and_variance_match_oracle(lp, precision, tol):
    print("case ic eigen N=16 nt=10", precision, flush=True)
    N, nt, sigma, c = 16, 10, 0.03, 10.0
    prob = _problem(lp, N, nt, sigma, precision=precision)
    ora = ICProblem(N, nt, sigma=sigma, prior_var=c)
    k = _gap_cut(ora.eig(12)[0], 8)
    lam, V = ora.eig(k)
    vals, vecs, used = prob.ic_eigensolve(k, c)
    err = np.abs(vals - lam).max() / lam[0]
    print("ic eigenvalues rel err %.3e, basis %d" % (err, used), flush=True)
    assert err < tol
    Vg = vecs.cpu().numpy().T
    # orthonormal, and each eigenvector spans the oracle's (the sensor layout's
    # symmetry makes some eigenvalues double: compare the spanned subspaces)
    assert np.abs(Vg.T @ Vg - np.eye(k)).max() < 1e-8
    s = np.linalg.svd(V.T @ Vg, compute_uv=False)
    assert s.min() > 1 - 10 * tol
    D = prob.ic_post_variance(vals, vecs, c, on_device=False)
    Dref = ora.post_var_lowrank(lam, V)
    derr = np.abs(D - Dref).max() / Dref.max()
    print("ic variance rel err %.3e" % derr, flush=True)
    assert derr < tol


def test_ic_full_observation_closed_form_at_paper_size(lp):
    """64 x 64, nt = 30, every node observed: the 20 leading eigenvalues equal
    c sigma^-2 sum_k rho_p^2k."""
    print("case ic closed form N=64 nt=30", flush=True)
    N, nt, sigma, c = 64, 30, 0.1, 10.0
    prob = _problem(lp, N, nt, sigma, tol=1e-8, rank_cap=32, mask=np.ones((N - 1) ** 2, dtype=bool))
    vals, _, used = prob.ic_eigensolve(20, c, rtol=1e-7)
    ref = full_obs_ic_eigs(N, nt, 1.0, sigma, c)[:20]
    err = np.abs(vals - ref).max() / ref[0]
    print("ic closed form rel err %.3e, basis %d" % (err, used), flush=True)
    assert err < 1e-7


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-7), ("mixed", 1e-5)])
def test_ic_paper_setting(lp, precision, tol):
    """The paper's Sec. 6.2 setting: 64 x 64, nt = 30, nine sensors of area
    1/256, Gamma_prior = 10 I, noise weight 1e4 times the prior's (sigma^2 =
    1e-3): the 20 leading eigenvalues against the oracle (ARPACK on its
    matrix-free G), and the posterior variance from them."""
    print("case ic paper setting", precision, flush=True)
    N, nt, c = 64, 30, 10.0
    sigma = (1.0 / (1e4 / c)) ** 0.5
    prob = _problem(lp, N, nt, sigma, precision=precision, tol=1e-8, rank_cap=32)
    ora = ICProblem(N, nt, sigma=sigma, prior_var=c)
    lam, V = ora.eig_arpack(24)
    k = _gap_cut(lam, 20)
    lam, V = lam[:k], V[:, :k]
    vals, vecs, used = prob.ic_eigensolve(k, c, rtol=1e-7 if precision == "fp64" else 1e-5)
    err = np.abs(vals - lam).max() / lam[0]
    print("ic paper eigenvalues rel err %.3e, basis %d, lambda_1 %.6e" % (err, used, vals[0]), flush=True)
    assert err < tol
    D = prob.ic_post_variance(vals, vecs, c, on_device=False)
    Dref = ora.post_var_lowrank(lam, V)
    derr = np.abs(D - Dref).max() / c
    print("ic paper variance rel err %.3e, k %d, min variance %.4f" % (derr, k, D.min()), flush=True)
    assert derr < 10 * tol
    # never above the prior's, and lowest at a sensor node
    assert D.max() <= c * (1 + 1e-12)
    assert sensor_mask(N)[int(np.argmin(D))]


def test_ic_eigensolve_reports_no_convergence(lp):
    print("case ic enoconv", flush=True)
    prob = _problem(lp, 16, 10, 0.03)
    with pytest.raises(lp.LrpostError) as ex:
        prob.ic_eigensolve(8, 10.0, max_vectors=8, rtol=1e-14)
    assert ex.value.code == -3
    vals, _, used = prob.ic_eigensolve(8, 10.0, max_vectors=8, rtol=1e-14, allow_unconverged=True)
    assert used <= 8 and vals[0] > 0
