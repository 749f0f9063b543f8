"""Posterior mean (the maximum a posteriori point) of the linear-Gaussian problem.

Test infrastructure (see the package docstring).

With A = F, zero prior mean, zero noise mean, Gamma_noise = sigma^2 I and
Gamma_prior^{-1} = P, the MAP point of Sec. 2 (eq. map1 and the
minimization written after it) minimizes

    1/2 ||u||_P^2 + 1/2 sigma^{-2} ||y - F u||^2,

so it solves the normal equations (H_mis + P) u = sigma^{-2} F^T y, and for
this linear-Gaussian problem it is also the posterior mean.  Two routes:

  mean_dense      the normal equations with the explicit dense matrices
                  (micro grids)
  mean_dataspace  u = P^{-1} F^T (sigma^2 I + F P^{-1} F^T)^{-1} y, the same
                  point written in data space (Woodbury), of size nobs * nt

and the closed form of the fully observed case (every interior node in the
box), where the tensor sine basis diagonalizes K and M and the problem
separates into one nt x nt problem per spatial mode:

  mean_full_obs_closed

The workload's data: u_true and y_obs = F u_true + sigma * noise with the
seeded draws of the synthetic module (draws only; F is applied here).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import closed_forms, fem
from .posterior import dense_hessian
from .spacetime import Problem


def _vec(X):
    return np.asarray(X).reshape(-1, order="F")


def _unvec(x, nx, nt):
    return np.asarray(x).reshape((nx, nt), order="F")


def observe_data(prob: Problem, u_true, noise):
    """y_obs = F u_true + sigma * noise, shape (nobs, nt) (observation rows in mask order)."""
    return prob.F(u_true) + prob.sigma * np.asarray(noise, dtype=np.float64)


def mean_dense(prob: Problem, y):
    """Solve (H_mis + P) u = sigma^{-2} F^T y with the explicit matrices; returns (nx, nt)."""
    H, P = dense_hessian(prob)
    rhs = _vec(prob.FT(y)) / prob.sigma ** 2
    u = np.linalg.solve(H + P, rhs)
    return _unvec(u, prob.nx, prob.nt)


def mean_dataspace(prob: Problem, y, F=None):
    """u = P^{-1} F^T (sigma^2 I + F P^{-1} F^T)^{-1} vec(y); returns (nx, nt).

    F is the dense (nobs*nt) x (nx*nt) parameter-to-observable matrix (built by
    impulse responses when not given); vec(y) stacks the observations of one
    time step after another.
    """
    if F is None:
        F = prob.impulse_F()
    nx, nt = prob.nx, prob.nt
    X = np.empty((nx * nt, F.shape[0]))
    Ft = F.T
    for l in range(nt):
        X[l * nx:(l + 1) * nx, :] = prob.prior_space_solve(Ft[l * nx:(l + 1) * nx, :]) / (prob.alpha * prob.tau)
    S = F @ X
    S[np.diag_indices_from(S)] += prob.sigma ** 2
    w = sla.solve((S + S.T) / 2, _vec(y), assume_a="pos")
    return _unvec(X @ w, nx, nt)


def normal_equation_residual(prob: Problem, u, y):
    """||(H_mis + P) u - sigma^{-2} F^T y|| / ||sigma^{-2} F^T y|| with the matrix-free maps."""
    rhs = prob.FT(y) / prob.sigma ** 2
    lhs = prob.H_mis(u) + prob.P_apply(u)
    return np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs)


def mean_full_obs_closed(N: int, nt: int, T: float, alpha: float, sigma: float, y):
    """The MAP point when every interior node is observed, mode by mode.

    With the Euclidean-orthonormal tensor sine basis Phi (K = Phi diag(kappa)
    Phi^T, M = Phi diag(mu) Phi^T), mode p of the state obeys
    B_p yhat = tau uhat with B_p = (1 + tau lambda_p) I - S, lambda_p =
    kappa_p / mu_p; the prior precision of the mode is alpha tau
    (kappa_p + mu_p) I_nt and the noise stays sigma^2 I.  So
    uhat_p = (sigma^{-2} G^T G + alpha tau (kappa_p + mu_p) I)^{-1} sigma^{-2} G^T yhat_p
    with G = tau B_p^{-1}.  y: (nx, nt) observations at every node.
    """
    S, kappa, mu = fem.modes_2d(N)
    n = N - 1
    tau = T / nt
    Y = np.asarray(y, dtype=np.float64)
    # yhat[p, k] for p = (i, j): coefficient on s_i (x1) s_j (x2)
    out_hat = np.empty((n, n, nt))
    yk = Y.reshape((n, n, nt), order="C")  # [jj, ii, k]
    yhat = np.einsum("ai,bj,bak->ijk", S, S, yk)  # [i, j, k]
    for i in range(n):
        for j in range(n):
            lam = kappa[i, j] / mu[i, j]
            G = tau * np.linalg.inv(closed_forms.bidiag(nt, tau * lam))
            A = G.T @ G / sigma ** 2 + alpha * tau * (kappa[i, j] + mu[i, j]) * np.eye(nt)
            out_hat[i, j] = np.linalg.solve(A, G.T @ yhat[i, j] / sigma ** 2)
    U = np.einsum("ai,bj,ijk->bak", S, S, out_hat)  # [jj, ii, k]
    return U.reshape((n * n, nt), order="C")
