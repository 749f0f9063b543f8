"""Pins for the oracle's eigenpairs, posterior covariance, prior variance and samples."""
import numpy as np
import pytest

from oracle import closed_forms, posterior
from oracle.lowrank import lr_arnoldi
from oracle.spacetime import Problem

FULL = (0.0, 1.0, 0.0, 1.0)


def test_full_observation_spectrum_closed_form():
    """Every node observed: eigenvalues tau/(sigma^2 alpha (kappa+mu) s_q(B_p)^2), rank-1 eigenvectors."""
    N, nt, alpha, sigma = 6, 5, 2e-2, 3e-2
    p = Problem(N, nt, alpha=alpha, sigma=sigma, box=FULL)
    w, V = posterior.eig_dense(p)
    cf, tags = closed_forms.full_obs_eigs(N, nt, 1.0, alpha, sigma)
    assert np.allclose(w, cf, rtol=1e-10)
    # leading eigenvector is the separable mode phi_(1,1) (x) w_0 (rank one)
    i, j, q = tags[0]
    v = closed_forms.full_obs_eigvec(N, nt, 1.0, i, j, q).reshape(-1, order="F")
    v0 = V[:, 0]
    cos = abs(v @ (p.P_apply(v0.reshape((p.nx, nt), order="F")).reshape(-1, order="F")))
    cos /= np.sqrt(p.P_inner(v.reshape((p.nx, nt), order="F"), v.reshape((p.nx, nt), order="F")))
    assert cos == pytest.approx(1.0, abs=1e-10)
    assert np.linalg.matrix_rank(V[:, 0].reshape((p.nx, nt), order="F"), tol=1e-10 * np.abs(V[:, 0]).max()) == 1


def test_steady_case_lemma():
    """nt = 1: sine-mode eigenvectors with eigenvalues tau/(sigma^2 alpha (kappa+mu)(1+tau lambda)^2)."""
    N, alpha, sigma = 7, 1e-2, 1e-2
    p = Problem(N, 1, alpha=alpha, sigma=sigma, box=FULL)
    w, _ = posterior.eig_dense(p)
    assert np.allclose(w, closed_forms.steady_eigs(N, 1.0, alpha, sigma), rtol=1e-10)


def test_parameter_scaling():
    p1 = Problem(6, 4, alpha=1.0, sigma=1.0, box=(0.2, 0.6, 0.3, 0.9))
    p2 = Problem(6, 4, alpha=3e-2, sigma=7e-3, box=(0.2, 0.6, 0.3, 0.9))
    w1, _ = posterior.eig_dense(p1, 10)
    w2, _ = posterior.eig_dense(p2, 10)
    assert np.allclose(w2, w1 / (7e-3 ** 2 * 3e-2), rtol=1e-10)


def test_eigen_routes_agree():
    p = Problem(8, 6, alpha=1e-2, sigma=1e-2, box=(0.25, 0.75, 0.1, 0.5))
    k = 12
    w_d, V_d = posterior.eig_dense(p, k)
    w_s = posterior.eig_sym_root(p, k)
    w_ds, V_ds = posterior.eig_dataspace(p, k)
    w_a, _ = posterior.eig_arpack(p, k)
    for w in (w_s, w_ds, w_a):
        assert np.allclose(w, w_d, rtol=1e-9)
    # P-orthonormality and the pencil relation for the data-space vectors
    _, _, _, Pst = p.spacetime_matrices()
    assert np.allclose(V_ds.T @ (Pst @ V_ds), np.eye(k), atol=1e-9)
    for i in range(3):
        X = V_ds[:, i].reshape((p.nx, p.nt), order="F")
        assert np.allclose(p.G(X), w_ds[i] * X, rtol=1e-8, atol=1e-8 * np.abs(X).max() * w_ds[i])


def test_symmetric_box_gives_exact_pairs():
    """The centered box keeps the square's symmetry group: some eigenvalues come in exact pairs."""
    p = Problem(8, 4, box=(0.25, 0.75, 0.25, 0.75))
    w, _ = posterior.eig_dense(p, 30)
    rel = np.abs(np.diff(w)) / w[1:]
    assert np.min(rel) < 1e-10
    # an off-center box breaks the symmetry
    p2 = Problem(8, 4, box=(0.125, 0.625, 0.25, 0.875))
    w2, _ = posterior.eig_dense(p2, 30)
    assert np.min(np.abs(np.diff(w2)) / w2[1:]) > 1e-8


def test_posterior_identities():
    p = Problem(6, 4, alpha=1e-2, sigma=1e-2, box=(0.2, 0.8, 0.2, 0.6))
    w, V = posterior.eig_dense(p)
    exact = posterior.post_cov_exact(p)
    # full-rank Woodbury equals the inverse
    assert np.allclose(posterior.post_cov_lowrank(p, w, V), exact, rtol=1e-10, atol=1e-10 * np.abs(exact).max())
    dprior = posterior.prior_diag_closed(p.N, p.alpha, p.tau)
    dex = np.diag(exact).reshape((p.nx, p.nt), order="F")
    prev = None
    for k in (1, 3, 8, 20):
        dk = posterior.post_diag_lowrank(p, w[:k], V[:, :k], dprior)
        gap = dk - dex
        assert gap.min() >= -1e-12 * dex.max()
        bound = w[k] / (1 + w[k]) * dprior[:, None]
        assert np.all(gap <= bound + 1e-12 * dex.max())
        assert np.all(dk <= dprior[:, None] * (1 + 1e-12))
        if prev is not None:
            assert np.all(dk <= prev + 1e-12 * dex.max())
        prev = dk


def test_dataspace_exact_diagonal():
    p = Problem(6, 4, alpha=1e-2, sigma=1e-2, box=(0.2, 0.8, 0.2, 0.6))
    exact = np.diag(posterior.post_cov_exact(p)).reshape((p.nx, p.nt), order="F")
    assert np.allclose(posterior.post_diag_exact_dataspace(p), exact, rtol=1e-9)


@pytest.mark.parametrize("N", [5, 9])
def test_prior_variance_closed_form(N):
    a, tau = 2e-2, 0.1
    p = Problem(N, 10, alpha=a)
    assert np.allclose(posterior.prior_diag_closed(N, a, tau), posterior.prior_diag_dense(p), rtol=1e-12)


def test_samples_have_posterior_covariance():
    """The sample map (I - V diag(p) V^T P) L has covariance Gamma_post,k exactly."""
    p = Problem(5, 3, alpha=1e-2, sigma=1e-2, box=(0.2, 0.8, 0.2, 0.8))
    w, V = posterior.eig_dense(p, 6)
    n = p.nx * p.nt
    # column c of the sample map is the sample drawn from the unit vector e_c
    Xi = np.stack([np.eye(n)[c].reshape((p.nx, p.nt), order="F") for c in range(n)])
    Smap = np.stack([s.reshape(-1, order="F") for s in posterior.samples(p, w, V, Xi)], axis=1)
    cov = Smap @ Smap.T
    ref = posterior.post_cov_lowrank(p, w, V)
    assert np.allclose(cov, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_prior_root_squares_to_prior_covariance():
    p = Problem(6, 2, alpha=1e-2)
    n = p.nx
    L = np.stack([posterior.prior_sqrt_apply(p, np.eye(n * 2)[c].reshape((n, 2), order="F"))[:, 0]
                  for c in range(n)], axis=1)
    ref = np.linalg.inv((p.K + p.M).toarray()) / (p.alpha * p.tau)
    assert np.allclose(L @ L.T, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    assert np.allclose(L, L.T, atol=1e-11 * np.abs(L).max())


def test_low_rank_arnoldi_recovers_eigenvalues():
    """Sec. 6.2: low-rank Arnoldi with full re-orthogonalization recovers the leading eigenvalues."""
    p = Problem(8, 6, alpha=1e-2, sigma=1e-2, box=(0.25, 0.75, 0.1, 0.5))
    w, _ = posterior.eig_dense(p, 6)
    rng = np.random.default_rng(2)
    v1 = np.outer(rng.standard_normal(p.nx), rng.standard_normal(p.nt))
    H, basis = lr_arnoldi(p.G, p.P_inner, v1, steps=40, tol=1e-12)
    m = H.shape[1]
    Hm = H[:m, :m]
    theta = np.sort(np.linalg.eigvals(Hm).real)[::-1]
    assert np.allclose(theta[:6], w, rtol=1e-8)
    # with truncation the Hessenberg matrix is numerically symmetric (Lanczos case)
    assert np.abs(Hm - Hm.T).max() <= 1e-6 * np.abs(Hm).max()


def test_ritz_residual_bound():
    """|lambda - theta| <= ||G v - theta v||_P for P-unit v (symmetric pencil)."""
    p = Problem(6, 4, box=(0.2, 0.8, 0.2, 0.6))
    w, V = posterior.eig_dense(p, 4)
    rng = np.random.default_rng(9)
    for i in range(4):
        X = V[:, i].reshape((p.nx, p.nt), order="F") + 1e-3 * rng.standard_normal((p.nx, p.nt)) * np.abs(V[:, i]).max()
        X /= np.sqrt(p.P_inner(X, X))
        theta = p.P_inner(X, p.G(X))
        R = p.G(X) - theta * X
        res = np.sqrt(p.P_inner(R, R))
        assert np.min(np.abs(w - theta)) <= res * (1 + 1e-10)
