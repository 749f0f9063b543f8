"""Eigenpairs of the prior-preconditioned misfit Hessian and the posterior.

Test infrastructure (see the package docstring).

With A = F, Gamma_noise = sigma^2 I and Gamma_prior^{-1} = P, Sec. 2 eq.
postcov1 gives Gamma_post = (H_mis + P)^{-1}.  The prior-preconditioned
Hessian of Sec. 2 eq. prior_pre has the eigenvalues of the pencil
(H_mis, P); with P-orthonormal pencil eigenvectors v_i (v_i^T P v_j = delta_ij)
the Sherman-Morrison-Woodbury step of Sec. 2 gives

    Gamma_post,k = P^{-1} - sum_{i<=k} d_i v_i v_i^T,   d_i = lambda_i / (1 + lambda_i),

which is Gamma_prior^{1/2} (I - V Lambda~ V^T) Gamma_prior^{1/2} written with
v_i = Gamma_prior^{1/2} (eigenvector of the symmetric form).  The result does
not depend on which square root of Gamma_prior is used.

Three independent eigen routes:
  eig_dense      generalized dense eigh of (H_mis, P) from the explicit matrix
                 (micro grids)
  eig_sym_root   dense eigh of P^{-1/2} H_mis P^{-1/2} with the symmetric root
                 (micro grids)
  eig_dataspace  eigh of sigma^{-2} F P^{-1} F^T in data space, mapped back by
                 v = P^{-1} F^T q / (sigma sqrt(lambda))
  eig_arpack     ARPACK on the matrix-free pencil (any size the time stepping
                 reaches)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import fem
from .spacetime import Problem


def _vec(X):
    """vec() with space fastest: (nx, nt) -> nx*nt."""
    return np.asarray(X).reshape(-1, order="F")


def _unvec(x, nx, nt):
    return np.asarray(x).reshape((nx, nt), order="F")


def dense_hessian(prob: Problem):
    """Explicit H_mis = sigma^{-2} F^T F and P (dense), vec ordering space fastest."""
    F = prob.dense_F()
    H = F.T @ F / prob.sigma ** 2
    _, _, _, Pst = prob.spacetime_matrices()
    return H, Pst.toarray()


def eig_dense(prob: Problem, k=None):
    """Largest k eigenpairs of the pencil (H_mis, P) by dense generalized eigh.

    Returns lambda (descending) and V (nx*nt x k) with V^T P V = I.
    """
    H, P = dense_hessian(prob)
    w, V = sla.eigh(H, P)
    order = np.argsort(w)[::-1]
    w, V = w[order], V[:, order]
    if k is not None:
        w, V = w[:k], V[:, :k]
    return w, V


def eig_sym_root(prob: Problem, k=None):
    """Eigenvalues of Gamma_prior^{1/2} H_mis Gamma_prior^{1/2} with the symmetric root (dense)."""
    H, P = dense_hessian(prob)
    wp, Up = np.linalg.eigh(P)
    R = (Up / np.sqrt(wp)) @ Up.T  # P^{-1/2}
    Ht = R @ H @ R
    w = np.linalg.eigvalsh((Ht + Ht.T) / 2)[::-1]
    return w if k is None else w[:k]


def _prior_chol(prob: Problem):
    return np.linalg.cholesky((prob.K + prob.M).toarray())


def eig_dataspace(prob: Problem, k: int, F=None):
    """Top-k pencil eigenpairs through the data-space matrix sigma^{-2} F P^{-1} F^T.

    Returns lambda (descending, k), V (nx*nt x k, P-orthonormal).
    """
    if F is None:
        F = prob.impulse_F()
    nx, nt, nobs = prob.nx, prob.nt, prob.nobs
    L = _prior_chol(prob)  # K + M = L L^T
    # B = F (I kron L^{-T}) / sqrt(alpha tau); then sigma^{-2} F P^{-1} F^T = sigma^{-2} B B^T
    B = np.empty_like(F)
    for l in range(nt):
        blk = F[:, l * nx:(l + 1) * nx]
        B[:, l * nx:(l + 1) * nx] = sla.solve_triangular(L, blk.T, lower=True).T
    B /= np.sqrt(prob.alpha * prob.tau)
    A = (B @ B.T) / prob.sigma ** 2
    m = A.shape[0]
    w, Q = sla.eigh(A, subset_by_index=[m - k, m - 1])
    w, Q = w[::-1], Q[:, ::-1]
    # v = P^{-1} F^T q / (sigma sqrt(lambda))
    FtQ = F.T @ Q
    V = np.empty((nx * nt, k))
    for i in range(k):
        V[:, i] = _vec(prob.P_solve(_unvec(FtQ[:, i], nx, nt))) / (prob.sigma * np.sqrt(w[i]))
    return w, V


def eig_arpack(prob: Problem, k: int, tol=1e-13, ncv=None, v0=None):
    """Top-k pencil eigenpairs by ARPACK on the matrix-free H_mis with mass P."""
    nx, nt = prob.nx, prob.nt
    n = nx * nt
    Hop = spla.LinearOperator((n, n), matvec=lambda x: _vec(prob.H_mis(_unvec(x, nx, nt))), dtype=np.float64)
    Pop = spla.LinearOperator((n, n), matvec=lambda x: _vec(prob.P_apply(_unvec(x, nx, nt))), dtype=np.float64)
    Pinv = spla.LinearOperator((n, n), matvec=lambda x: _vec(prob.P_solve(_unvec(x, nx, nt))), dtype=np.float64)
    w, V = spla.eigsh(Hop, k=k, M=Pop, Minv=Pinv, which="LA", tol=tol, ncv=ncv, v0=v0)
    order = np.argsort(w)[::-1]
    w, V = w[order], V[:, order]
    # P-normalize
    for i in range(k):
        vi = V[:, i]
        V[:, i] = vi / np.sqrt(vi @ Pop.matvec(vi))
    return w, V


def prior_diag_dense(prob: Problem):
    """diag(P^{-1}) over one time step (nx,): (alpha tau)^{-1} diag((K+M)^{-1}), dense inverse."""
    Ainv = np.linalg.inv((prob.K + prob.M).toarray())
    return np.diag(Ainv) / (prob.alpha * prob.tau)


def prior_diag_closed(N: int, alpha: float, tau: float):
    """diag(P^{-1}) over one time step from the sine-transform eigenpairs (any N).

    (K+M)^{-1} = sum_p phi_p phi_p^T / (kappa_p + mu_p) with phi_p = s_i (x) s_j,
    so the diagonal at node (ii, jj) is sum_{i,j} s_i(ii)^2 s_j(jj)^2 / (kappa_ij + mu_ij):
    two n x n matrix products with the squared sine matrix.
    """
    S, kappa, mu = fem.modes_2d(N)
    Sq = S * S
    W = 1.0 / (kappa + mu)
    D = Sq @ W @ Sq.T  # D[ii, jj], ii along x1
    return D.T.reshape(-1) / (alpha * tau)


def post_diag_lowrank(prob: Problem, lam, V, dprior=None):
    """diag(Gamma_post,k) as an (nx, nt) array: diag(P^{-1}) - sum_i d_i v_i^2."""
    if dprior is None:
        dprior = prior_diag_closed(prob.N, prob.alpha, prob.tau)
    d = lam / (1.0 + lam)
    acc = (V * V) @ d
    return np.repeat(dprior[:, None], prob.nt, axis=1) - _unvec(acc, prob.nx, prob.nt)


def post_cov_exact(prob: Problem):
    """Gamma_post = (H_mis + P)^{-1} by dense inversion (micro grids)."""
    H, P = dense_hessian(prob)
    return np.linalg.inv(H + P)


def post_cov_lowrank(prob: Problem, lam, V):
    """Gamma_post,k = P^{-1} - V diag(d) V^T, dense (micro grids)."""
    _, _, _, Pst = prob.spacetime_matrices()
    Pinv = np.linalg.inv(Pst.toarray())
    d = lam / (1.0 + lam)
    return Pinv - (V * d) @ V.T


def post_diag_exact_dataspace(prob: Problem, F=None):
    """diag((H_mis + P)^{-1}) as (nx, nt) by Woodbury in data space.

    Gamma_post = P^{-1} - P^{-1} F^T (sigma^2 I + F P^{-1} F^T)^{-1} F P^{-1}.
    """
    if F is None:
        F = prob.impulse_F()
    nx, nt = prob.nx, prob.nt
    # X = P^{-1} F^T, column by column in blocks of time
    X = np.empty((nx * nt, F.shape[0]))
    Ft = F.T
    for l in range(nt):
        X[l * nx:(l + 1) * nx, :] = prob.prior_space_solve(Ft[l * nx:(l + 1) * nx, :]) / (prob.alpha * prob.tau)
    S = F @ X
    S[np.diag_indices_from(S)] += prob.sigma ** 2
    Lc = np.linalg.cholesky((S + S.T) / 2)
    Y = sla.solve_triangular(Lc, X.T, lower=True)  # (m, nx*nt)
    corr = np.sum(Y * Y, axis=0)
    dprior = prior_diag_closed(prob.N, prob.alpha, prob.tau)
    return np.repeat(dprior[:, None], nt, axis=1) - _unvec(corr, nx, nt)


def prior_sqrt_apply(prob: Problem, Xi):
    """L xi with L = (alpha tau)^{-1/2} (I kron (K+M)^{-1/2}), symmetric root via the sine basis.

    Xi has shape (nx, nt).  (K+M)^{-1/2} = Phi diag((kappa+mu)^{-1/2}) Phi^T with the
    Euclidean-orthonormal tensor sine basis Phi.
    """
    S, kappa, mu = fem.modes_2d(prob.N)
    n = prob.n
    W = 1.0 / np.sqrt(kappa + mu)  # [i, j]
    out = np.empty_like(np.asarray(Xi, dtype=np.float64))
    for k in range(prob.nt):
        G = Xi[:, k].reshape((n, n))  # G[jj, ii]  (row = x2 node, col = x1 node)
        C = S.T @ G @ S               # C[j, i] = sum s_j(jj) G s_i(ii)
        C = C * W.T
        out[:, k] = (S @ C @ S.T).reshape(-1)
    return out / np.sqrt(prob.alpha * prob.tau)


def samples(prob: Problem, lam, V, Xi):
    """Zero-mean posterior samples s = (I - V diag(p) V^T P) L xi, p_i = 1 - (1+lambda_i)^{-1/2}.

    The covariance of s is Gamma_post,k (derived from the Woodbury step of
    Sec. 2).  Xi: (ns, nx, nt); returns (ns, nx, nt).
    """
    pcoef = 1.0 - 1.0 / np.sqrt(1.0 + lam)
    out = np.empty_like(Xi, dtype=np.float64)
    for s in range(Xi.shape[0]):
        Lxi = prior_sqrt_apply(prob, Xi[s])
        PLxi = _vec(prob.P_apply(Lxi))
        c = V.T @ PLxi
        out[s] = Lxi - _unvec(V @ (pcoef * c), prob.nx, prob.nt)
    return out
