"""Spectra known in closed form, used to pin the oracle.

Test infrastructure (see the package docstring).

Sec. 5 shows that for the Poisson operator on a rectangle the eigenfunctions
of the misfit Hessian are products of sines (separation rank one; the Lemma of
Sec. 5), with continuum eigenvalues pi^2 ((m/a)^2 + (n/b)^2).  For the
space-time operator Sec. 5 diagonalizes the Kronecker sum through the SVD of
its factors and the pencil (L, M), so that eigenvectors are rank one in space
and time.  On the uniform Q1 mesh both K and M are diagonalized by the tensor
sine basis, which makes that argument exact when every node is observed:

  * per spatial mode p the state equation becomes the nt x nt bidiagonal
    system B_p z = tau g with B_p = (1 + tau lambda_p) I - S,
    lambda_p = kappa_p / mu_p;
  * the pencil (H_mis, P) then has eigenvalues
        tau / (sigma^2 alpha (kappa_p + mu_p) s_q(B_p)^2)
    over all modes p and singular values s_q of B_p, with eigenvectors
    phi_p (x) (right singular vector of B_p): rank one.
"""
from __future__ import annotations

import numpy as np

from . import fem


def continuum_laplace_eigs(m, n, a=1.0, b=1.0):
    """Dirichlet Laplacian eigenvalues pi^2 ((m/a)^2 + (n/b)^2) on [0,a] x [0,b] (Sec. 5)."""
    return np.pi ** 2 * ((np.asarray(m) / a) ** 2 + (np.asarray(n) / b) ** 2)


def bidiag(nt: int, lam_tau: float):
    """B = (1 + tau lambda) I - S, the per-mode implicit-Euler matrix."""
    return (1.0 + lam_tau) * np.eye(nt) - np.eye(nt, k=-1)


def full_obs_eigs(N: int, nt: int, T: float, alpha: float, sigma: float, modes=None):
    """Pencil eigenvalues when the box covers every node.

    modes: iterable of (i, j) 1-based sine modes; default all.  Returns
    (eigenvalues, list of (i, j, q)) sorted descending.
    """
    _, kappa, mu = fem.modes_2d(N)
    tau = T / nt
    n = N - 1
    if modes is None:
        modes = [(i, j) for j in range(1, n + 1) for i in range(1, n + 1)]
    vals, tags = [], []
    for (i, j) in modes:
        kp, mp = kappa[i - 1, j - 1], mu[i - 1, j - 1]
        s = np.linalg.svd(bidiag(nt, tau * kp / mp), compute_uv=False)
        ev = tau / (sigma ** 2 * alpha * (kp + mp) * s ** 2)
        for q, e in enumerate(ev):
            vals.append(e)
            tags.append((i, j, q))
    vals = np.asarray(vals)
    order = np.argsort(vals)[::-1]
    return vals[order], [tags[o] for o in order]


def full_obs_eigvec(N: int, nt: int, T: float, i: int, j: int, q: int):
    """Eigenvector phi_(i,j) (x) w_q for the full-observation pencil, as (nx, nt)
    (unnormalized; w_q the left singular vector of B_p for its q-th largest
    singular value, q 0-based as tagged by full_obs_eigs)."""
    _, kappa, mu = fem.modes_2d(N)
    tau = T / nt
    lam = kappa[i - 1, j - 1] / mu[i - 1, j - 1]
    U, _, _ = np.linalg.svd(bidiag(nt, tau * lam))
    return np.outer(fem.mode_vector(N, i, j), U[:, q])


def steady_eigs(N: int, T: float, alpha: float, sigma: float):
    """nt = 1: eigenvalues tau / (sigma^2 alpha (kappa_p + mu_p) (1 + tau lambda_p)^2), sorted descending.

    The one-step case is a steady problem; its eigenvectors are the sine modes,
    separation rank one as the Lemma of Sec. 5 states.
    """
    _, kappa, mu = fem.modes_2d(N)
    tau = T
    lam = kappa / mu
    ev = tau / (sigma ** 2 * alpha * (kappa + mu) * (1.0 + tau * lam) ** 2)
    return np.sort(ev.ravel())[::-1]


def single_mode_state(N: int, nt: int, T: float, i: int, j: int, g):
    """State for source u = phi_(i,j) (x) g: y = phi (x) tau (tau lambda_p I + C)^{-1} g."""
    _, kappa, mu = fem.modes_2d(N)
    tau = T / nt
    lam = kappa[i - 1, j - 1] / mu[i - 1, j - 1]
    C = np.eye(nt) - np.eye(nt, k=-1)
    z = tau * np.linalg.solve(tau * lam * np.eye(nt) + C, np.asarray(g, dtype=np.float64))
    return np.outer(fem.mode_vector(N, i, j), z)
