"""The initial-condition inverse problem of the paper's experiments (Sec. 6,
eqs. pde, obj, dis_obj, postvar, misfit; Sec. 6.2 heat equation).

Test infrastructure (see the package docstring).

The unknown is the initial state u = y(0) (one value per interior node); the
state follows the heat equation without source, y_t = Laplace(y), y = 0 on
the boundary, Q1 in space and implicit Euler in time:

    (M + tau K) y_1 = M u,   (M + tau K) y_k = M y_{k-1}   (k = 2..nt),

which is the all-at-once system K_st vec(Y) = C u with K_st = I kron tau K +
C_t kron M (C_t = I - S, S the sub-diagonal shift) and C = e_1 kron M.

Another spatial operator L may take the place of K (the convection-diffusion
operator of Sec. 6.3, which is not symmetric): the forward steps then solve
(M + tau L) y_k = M y_{k-1} and the adjoint steps the transposed system.

Readings of points the paper leaves open (they are listed with the design):
  * observations are nodal values at the nodes inside the sensor regions, at
    every step t_1..t_nt, with noise covariance sigma^2 I (the paper's noise
    weight beta_noise becomes sigma^-2);
  * the prior covariance is Gamma_prior = c I (the paper's experiments take
    c = 10, with beta_noise = 1e4 beta_prior = 1e4 / c);
  * the nine sensors of area 1/256 "uniformly distributed" are the closed
    squares of side 1/16 centred at (i/4, j/4), i, j = 1, 2, 3 (the input
    module's default sensor layout).

The misfit Hessian is H = sigma^-2 C^T K_st^-T B^T B K_st^-1 C (eq. postvar
without its prior term), the prior-preconditioned operator of eq. misfit is
G = Gamma_prior^1/2 H Gamma_prior^1/2 = c H, and the posterior covariance is
(H + Gamma_prior^-1)^-1 = c (I + G)^-1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synthetic import sensor_mask  # the sensor layout: an input shared with the library's tests

from . import fem


class ICProblem:
    """Operators of one initial-condition problem.  States are (nx, nt) arrays,
    column k at time t_{k+1}; parameters are nodal vectors (nx,)."""

    def __init__(self, N, nt, T=1.0, sigma=1e-2, prior_var=10.0, mask=None, L=None):
        self.N, self.nt, self.T = int(N), int(nt), float(T)
        self.sigma, self.c = float(sigma), float(prior_var)
        self.n = self.N - 1
        self.nx = self.n * self.n
        self.tau = self.T / self.nt
        self.K, self.M = fem.assemble_kronecker(self.N)
        # the spatial operator: the Laplacian's stiffness K, or another one
        # (the convection-diffusion operator of Sec. 6.3, not symmetric)
        self.L = self.K if L is None else sp.csr_matrix(L)
        self.mask = sensor_mask(self.N) if mask is None else np.asarray(mask, dtype=bool)
        self.obs_idx = np.nonzero(self.mask)[0]
        self._lu = spla.splu((self.M + self.tau * self.L).tocsc())

    def step_solve(self, b):
        """(M + tau L)^{-1} b."""
        return self._lu.solve(np.asarray(b, dtype=np.float64))

    def step_solve_t(self, b):
        """(M + tau L)^{-T} b (the adjoint step)."""
        return self._lu.solve(np.asarray(b, dtype=np.float64), trans="T")

    def forward(self, u):
        """Y = K_st^{-1} C u by implicit-Euler time stepping from y_0 = u: (M + tau L) y_k = M y_{k-1}."""
        Y = np.zeros((self.nx, self.nt))
        y = np.asarray(u, dtype=np.float64)
        for k in range(self.nt):
            y = self.step_solve(self.M @ y)
            Y[:, k] = y
        return Y

    def forward_source(self, F):
        """Y = K_st^{-1} vec(F) for a space-time source F (nx, nt): forward in
        time, (M + tau L) y_k = M y_{k-1} + f_k, y_0 = 0 (eq. st_pde with a
        general right-hand side)."""
        F = np.asarray(F, dtype=np.float64)
        Y = np.zeros((self.nx, self.nt))
        y = np.zeros(self.nx)
        for k in range(self.nt):
            y = self.step_solve(self.M @ y + F[:, k])
            Y[:, k] = y
        return Y

    def adjoint(self, Z):
        """P = K_st^{-T} vec(Z): backward in time, (M + tau L)^T p_k = M p_{k+1} + z_k, p_{nt+1} = 0."""
        Z = np.asarray(Z, dtype=np.float64)
        P = np.zeros((self.nx, self.nt))
        p = np.zeros(self.nx)
        for k in range(self.nt - 1, -1, -1):
            p = self.step_solve_t(self.M @ p + Z[:, k])
            P[:, k] = p
        return P

    def F(self, u):
        """Parameter-to-observable map B K_st^{-1} C: observed nodal values, (nobs, nt)."""
        return self.forward(u)[self.obs_idx, :]

    def FT(self, D):
        """Adjoint C^T K_st^{-T} B^T: scatter to the observed nodes, solve backward,
        and C^T vec(P) = M p_1."""
        Z = np.zeros((self.nx, self.nt))
        Z[self.obs_idx, :] = D
        return self.M @ self.adjoint(Z)[:, 0]

    def H(self, u):
        """Misfit Hessian sigma^{-2} F^T F u."""
        return self.FT(self.F(u)) / self.sigma ** 2

    def G(self, u):
        """Prior-preconditioned misfit Hessian c H u (eq. misfit with Gamma_prior = c I)."""
        return self.c * self.H(u)

    # ---- explicit matrices (small problems only) -------------------------
    def dense_G(self):
        """G column by column through the matrix-free apply."""
        return np.column_stack([self.G(e) for e in np.eye(self.nx)])

    def dense_G_allatonce(self):
        """G from the sparse all-at-once system: c sigma^-2 (B K_st^-1 C)^T (B K_st^-1 C)
        (a route independent of the time stepping above)."""
        nt, nx = self.nt, self.nx
        Ct = sp.eye(nt) - sp.eye(nt, k=-1)
        Kst = (sp.kron(sp.eye(nt), self.tau * self.L) + sp.kron(Ct, self.M)).tocsc()
        e1 = np.zeros((nt, 1))
        e1[0, 0] = 1.0
        Cm = sp.kron(sp.csr_matrix(e1), self.M).tocsc()
        X = spla.spsolve(Kst, Cm.toarray())
        obs = (np.arange(nt)[:, None] * nx + self.obs_idx[None, :]).ravel()
        F = X[obs, :]
        return self.c * (F.T @ F) / self.sigma ** 2

    def eig(self, k=None):
        """Leading eigenpairs of G (dense symmetric eigensolve), descending."""
        w, V = np.linalg.eigh(self.dense_G())
        order = np.argsort(w)[::-1]
        w, V = w[order], V[:, order]
        if k is not None:
            w, V = w[:k], V[:, :k]
        return w, V

    def eig_arpack(self, k, tol=1e-12):
        """k leading eigenpairs of G by ARPACK (scipy's eigsh) on the matrix-free apply, descending."""
        op = spla.LinearOperator((self.nx, self.nx), matvec=self.G, dtype=np.float64)
        w, V = spla.eigsh(op, k=k, which="LA", tol=tol, v0=np.ones(self.nx))
        order = np.argsort(w)[::-1]
        return w[order], V[:, order]

    def post_var_lowrank(self, lam, V):
        """diag of c (I + G)^{-1} from k eigenpairs of G (Sherman-Morrison-Woodbury):
        c - c sum_i lam_i / (1 + lam_i) v_i^2."""
        lam = np.asarray(lam, dtype=np.float64)
        return self.c - self.c * (np.asarray(V) ** 2) @ (lam / (1.0 + lam))

    def post_var_exact(self):
        """diag of the posterior covariance (H + Gamma_prior^-1)^-1 = c (I + G)^-1 (eq. postvar)."""
        return np.diag(self.c * np.linalg.inv(np.eye(self.nx) + self.dense_G()))


def full_obs_ic_eigs(N: int, nt: int, T: float, sigma: float, prior_var: float):
    """Eigenvalues of G when every interior node is observed.

    K and M are diagonalized by the orthonormal tensor sine basis, so the step
    map (M + tau K)^{-1} M is symmetric with eigenvalues rho_p = mu_p / (mu_p +
    tau kappa_p) on mode p, y_k = rho_p^k u_p, and G has eigenvalues
    c sigma^-2 sum_{k=1}^{nt} rho_p^{2k} on the sine modes.  Descending."""
    _, kappa, mu = fem.modes_2d(N)
    tau = T / nt
    rho = (mu / (mu + tau * kappa)).ravel()
    r2 = rho ** 2
    s = r2 * (1.0 - r2 ** nt) / (1.0 - r2)
    return np.sort(prior_var * s / sigma ** 2)[::-1]
