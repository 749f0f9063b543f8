"""Space-time forward and adjoint maps of the heat-equation inverse problem.

Test infrastructure (see the package docstring).

State equation y_t = Laplace(y) + u on the unit square, y = 0 on the boundary,
y(0) = 0, Q1 in space, implicit Euler with tau = T/nt.  In the all-at-once form
of Sec. 3 eq. KKT2 (state block) and Sec. 6.1 eq. st_pde the discrete state
Y = [y_1 .. y_nt] solves

    (I_nt kron tau K + C kron M) vec(Y) = (I_nt kron tau M) vec(U),

with C = I - S (S the sub-diagonal shift): step by step
(M + tau K) y_k = M y_{k-1} + tau M u_k.  The source block tau N with N = M
is the control block of KKT2 (D3 kron tau N).

Readings of points the paper leaves open (they are listed with the design):
  * y_0 = 0; the parameter is the space-time source u (the paper's Sec. 6
    experiments use the initial condition instead);
  * the source enters at the right end point t_k through tau M u_k;
  * observations are nodal values inside the closed box at t_1..t_nt, with
    noise covariance sigma^2 I;
  * the prior precision is alpha tau (I_nt kron (K + M)).

The parameter-to-observable map is F = B K^{-1} S with B = I_nt kron B_x,
the misfit Hessian H_mis = sigma^{-2} F^T F (Sec. 2 eq. postcov1 with
A = F and Gamma_noise = sigma^2 I), the prior precision
P = alpha tau (I kron (K+M)), and the prior-preconditioned operator
G = P^{-1} H_mis, which is similar to Gamma_prior^{1/2} H_mis Gamma_prior^{1/2}
(Sec. 2 eq. prior_pre) and has the same eigenvalues.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


class Problem:
    """Operators of one problem instance.  Arrays are (nx, nt): column k is time t_{k+1}."""

    def __init__(self, N, nt, T=1.0, alpha=1e-2, sigma=1e-2, box=(0.25, 0.75, 0.25, 0.75)):
        self.N, self.nt, self.T = int(N), int(nt), float(T)
        self.alpha, self.sigma = float(alpha), float(sigma)
        self.box = tuple(float(b) for b in box)
        self.n = self.N - 1
        self.h = 1.0 / self.N
        self.nx = self.n * self.n
        self.tau = self.T / self.nt
        self.K, self.M = fem.assemble_kronecker(self.N)
        h = self.h
        g = np.arange(1, self.N) * h
        x1 = np.tile(g, self.n)
        x2 = np.repeat(g, self.n)
        lo1, hi1, lo2, hi2 = self.box
        eps = 1e-12
        self.mask = (x1 >= lo1 - eps) & (x1 <= hi1 + eps) & (x2 >= lo2 - eps) & (x2 <= hi2 + eps)
        self.obs_idx = np.nonzero(self.mask)[0]
        self.nobs = int(self.obs_idx.size)
        self._lu_step = spla.splu((self.M + self.tau * self.K).tocsc())
        self._lu_prior = spla.splu((self.K + self.M).tocsc())

    @classmethod
    def from_desc(cls, d):
        return cls(d.N, d.nt, d.T, d.alpha, d.sigma, d.box)

    # ---- spatial pieces -------------------------------------------------
    def step_solve(self, b):
        """(M + tau K)^{-1} b."""
        return self._lu_step.solve(np.asarray(b, dtype=np.float64))

    def prior_space_solve(self, b):
        """(K + M)^{-1} b."""
        return self._lu_prior.solve(np.asarray(b, dtype=np.float64))

    # ---- space-time maps (full arrays) ----------------------------------
    def forward(self, U):
        """Y = K^{-1} S vec(U) by implicit-Euler time stepping, y_0 = 0."""
        U = np.asarray(U, dtype=np.float64)
        Y = np.zeros((self.nx, self.nt))
        y = np.zeros(self.nx)
        for k in range(self.nt):
            y = self.step_solve(self.M @ y + self.tau * (self.M @ U[:, k]))
            Y[:, k] = y
        return Y

    def forward_source(self, Fsrc):
        """Y with (I kron tau K + C kron M) vec(Y) = vec(Fsrc): a general right-hand side."""
        Fsrc = np.asarray(Fsrc, dtype=np.float64)
        Y = np.zeros((self.nx, self.nt))
        y = np.zeros(self.nx)
        for k in range(self.nt):
            y = self.step_solve(self.M @ y + Fsrc[:, k])
            Y[:, k] = y
        return Y

    def adjoint_source(self, Z):
        """P with (I kron tau K + C^T kron M) vec(P) = vec(Z): backward in time, p_{nt+1} = 0."""
        Z = np.asarray(Z, dtype=np.float64)
        P = np.zeros((self.nx, self.nt))
        p = np.zeros(self.nx)
        for k in range(self.nt - 1, -1, -1):
            p = self.step_solve(self.M @ p + Z[:, k])
            P[:, k] = p
        return P

    def observe(self, Y):
        """B vec(Y): nodal values in the box, shape (nobs, nt)."""
        return np.asarray(Y)[self.obs_idx, :]

    def observe_T(self, D):
        """B^T vec(D): scatter (nobs, nt) back to (nx, nt)."""
        Z = np.zeros((self.nx, self.nt))
        Z[self.obs_idx, :] = D
        return Z

    def F(self, U):
        """Parameter-to-observable map F = B K^{-1} S."""
        return self.observe(self.forward(U))

    def FT(self, D):
        """Adjoint F^T = S^T K^{-T} B^T, with S^T = tau (I kron M)."""
        P = self.adjoint_source(self.observe_T(D))
        return self.tau * (self.M @ P)

    def H_mis(self, U):
        """Data-misfit Hessian sigma^{-2} F^T F applied to U."""
        return self.FT(self.F(U)) / self.sigma ** 2

    def P_apply(self, U):
        """Prior precision alpha tau (I kron (K + M)) applied to U."""
        return self.alpha * self.tau * ((self.K + self.M) @ np.asarray(U, dtype=np.float64))

    def P_solve(self, U):
        """Prior covariance (alpha tau)^{-1} (I kron (K + M))^{-1} applied to U."""
        return self.prior_space_solve(np.asarray(U, dtype=np.float64)) / (self.alpha * self.tau)

    def G(self, U):
        """Prior-preconditioned misfit Hessian G = P^{-1} H_mis applied to U."""
        return self.P_solve(self.H_mis(U))

    def P_inner(self, U, V):
        """<U, V>_P = vec(U)^T P vec(V)."""
        return float(np.sum(np.asarray(U) * self.P_apply(V)))

    # ---- explicit matrices (small problems only) -------------------------
    def spacetime_matrices(self):
        """Sparse all-at-once matrices: Kst = I kron tau K + C kron M, Sst = I kron tau M,
        Bst = I kron B_x, Pst = alpha tau I kron (K+M).  vec ordering: space fastest."""
        nt = self.nt
        C = sp.eye(nt) - sp.eye(nt, k=-1)
        It = sp.eye(nt)
        Kst = (sp.kron(It, self.tau * self.K) + sp.kron(C, self.M)).tocsc()
        Sst = sp.kron(It, self.tau * self.M).tocsc()
        Bx = sp.csr_matrix((np.ones(self.nobs), (np.arange(self.nobs), self.obs_idx)),
                           shape=(self.nobs, self.nx))
        Bst = sp.kron(It, Bx).tocsc()
        Pst = (self.alpha * self.tau * sp.kron(It, self.K + self.M)).tocsc()
        return Kst, Sst, Bst, Pst

    def dense_F(self):
        """F as a dense (nobs*nt) x (nx*nt) matrix from the all-at-once system."""
        Kst, Sst, Bst, _ = self.spacetime_matrices()
        X = spla.spsolve(Kst, Sst.toarray())
        return Bst @ X

    def impulse_F(self):
        """F as a dense matrix built from impulse responses (a route independent of dense_F).

        Time invariance makes F block lower-triangular Toeplitz in time: the block
        (k, l), k >= l, is the observed response at step k to a unit source in
        step l, which depends on k - l only.
        """
        nt, nx, nobs = self.nt, self.nx, self.nobs
        # response to source tau M e_x at step 1: y_1 = (M+tau K)^{-1} tau M e_x, y_k = A y_{k-1}
        Yk = self.step_solve(self.tau * self.M.toarray())  # nx x nx: column x = y_1 for source e_x
        blocks = []
        for _ in range(nt):
            blocks.append(Yk[self.obs_idx, :].copy())
            Yk = self.step_solve(self.M @ Yk)
        F = np.zeros((nobs * nt, nx * nt))
        for k in range(nt):
            for l in range(k + 1):
                F[k * nobs:(k + 1) * nobs, l * nx:(l + 1) * nx] = blocks[k - l]
        return F
