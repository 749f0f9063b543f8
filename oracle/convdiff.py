"""The convection-diffusion operator of the paper's second experiment (Sec. 6.3,
and Sec. 6 eq. pde with L = -nu Laplace + w . grad), discretized by
streamline-upwind Petrov-Galerkin (SUPG) bilinear elements on the uniform
N x N mesh of the unit square, homogeneous Dirichlet conditions.

Test infrastructure (see the package docstring).

Readings of points the paper leaves open (they are listed with the design):
  * the stabilization is the streamline-diffusion form of SUPG used for Q1
    elements: the test function v + delta w . grad v multiplies the steady
    operator only.  For bilinear functions on rectangles the Laplacian of the
    trial function vanishes inside every element, so the stabilized stiffness
    matrix is nu K + N + delta S with the convection matrix
    N_ij = (w . grad phi_j, phi_i) and the streamline matrix
    S_ij = (w . grad phi_j, w . grad phi_i).  The time derivative keeps the
    plain mass matrix M, as in the space-time system of eq. st_pde
    (I kron L + C kron M);
  * delta per element follows the element Peclet number
    Pe = |w| h_w / (2 nu): delta = h_w / (2 |w|) (1 - 1 / Pe) when Pe > 1,
    else 0, with h_w the length of the element along the wind through its
    centre;
  * the boundary data of the paper's textbook example only shift the state
    by a fixed field: the Hessian, its eigenpairs and the posterior
    covariance depend on the homogeneous problem alone, which is what is
    built here (zero Dirichlet values on the whole boundary).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# two-point Gauss rule on [0, 1]: exact for polynomials of degree 3 per
# variable, which covers every product of two bilinear functions or their
# derivatives
_GP = np.array([0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)])
_GW = np.array([0.5, 0.5])

# local nodes counter-clockwise from the lower-left corner: reference
# coordinates of each corner
_CORNERS = [(0, 0), (1, 0), (1, 1), (0, 1)]


def _shape(xi: float, eta: float):
    """Bilinear shape functions on [0,1]^2 and their reference derivatives."""
    phi = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta])
    dxi = np.array([-(1 - eta), (1 - eta), eta, -eta])
    deta = np.array([-(1 - xi), -xi, xi, (1 - xi)])
    return phi, dxi, deta


def supg_delta(N: int, nu: float, wind) -> float:
    """Stabilization parameter of a square element of side h = 1/N: element
    Peclet number Pe = |w| h_w / (2 nu) with h_w = h / max(|w1|, |w2|) * |w|
    (the element's length along the wind through its centre); delta =
    h_w / (2 |w|) (1 - 1/Pe) for Pe > 1, else 0."""
    w1, w2 = float(wind[0]), float(wind[1])
    wn = math.hypot(w1, w2)
    if wn == 0.0:
        return 0.0
    h = 1.0 / N
    hw = h * wn / max(abs(w1), abs(w2))
    pe = wn * hw / (2.0 * nu)
    if pe <= 1.0:
        return 0.0
    return hw / (2.0 * wn) * (1.0 - 1.0 / pe)


def element_matrices(h: float, nu: float, wind, delta: float):
    """Local diffusion, convection, streamline-diffusion and mass matrices of a
    square element of side h (rows: test function, columns: trial function),
    by 2 x 2 Gauss quadrature."""
    w1, w2 = float(wind[0]), float(wind[1])
    D = np.zeros((4, 4))
    C = np.zeros((4, 4))
    S = np.zeros((4, 4))
    Mloc = np.zeros((4, 4))
    for gx, wx in zip(_GP, _GW):
        for gy, wy in zip(_GP, _GW):
            phi, dxi, deta = _shape(gx, gy)
            gxv, gyv = dxi / h, deta / h  # physical gradients
            wgt = wx * wy * h * h
            conv = w1 * gxv + w2 * gyv  # w . grad phi_b for each local b
            for a in range(4):
                for b in range(4):
                    D[a, b] += wgt * nu * (gxv[b] * gxv[a] + gyv[b] * gyv[a])
                    C[a, b] += wgt * conv[b] * phi[a]
                    S[a, b] += wgt * delta * conv[b] * conv[a]
                    Mloc[a, b] += wgt * phi[b] * phi[a]
    return D, C, S, Mloc


def assemble_supg(N: int, nu: float, wind, delta: float | None = None):
    """L = nu K + N + delta S and M on the interior nodes (index (j-1) n +
    (i-1), x1 fastest), by a loop over the N^2 elements.  delta None: the
    element Peclet rule of supg_delta.  Returns CSR matrices (L, M)."""
    n = N - 1
    h = 1.0 / N
    nx = n * n
    if delta is None:
        delta = supg_delta(N, nu, wind)
    D, C, S, Mloc = element_matrices(h, nu, wind, delta)
    Lloc = D + C + S
    rows, cols, lv, mv = [], [], [], []
    for ey in range(N):
        for ex in range(N):
            gidx = []
            for (ci, cj) in _CORNERS:
                gi, gj = ex + ci, ey + cj
                gidx.append((gj - 1) * n + (gi - 1) if (1 <= gi <= n and 1 <= gj <= n) else -1)
            for a in range(4):
                if gidx[a] < 0:
                    continue
                for b in range(4):
                    if gidx[b] < 0:
                        continue
                    rows.append(gidx[a])
                    cols.append(gidx[b])
                    lv.append(Lloc[a, b])
                    mv.append(Mloc[a, b])
    L = sp.csr_matrix((lv, (rows, cols)), shape=(nx, nx))
    M = sp.csr_matrix((mv, (rows, cols)), shape=(nx, nx))
    L.sum_duplicates()
    M.sum_duplicates()
    return L, M


def cd_ic_problem(N: int, nt: int, nu: float, wind=(0.0, 1.0), delta: float | None = None, T: float = 1.0,
                  sigma: float = math.sqrt(1e-3), prior_var: float = 10.0, mask=None):
    """The initial-condition problem of the paper's experiments with the SUPG
    convection-diffusion operator in place of the Laplacian: the forward steps
    solve (M + tau L) y_k = M y_{k-1}, the adjoint steps the transposed
    system (M + tau L)^T p_k = M p_{k+1} + z_k (eq. postvar's K^-T)."""
    from .initial import ICProblem

    L, _ = assemble_supg(N, nu, wind, delta)
    return ICProblem(N, nt, T=T, sigma=sigma, prior_var=prior_var, mask=mask, L=L)

