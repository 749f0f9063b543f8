"""Q1 finite elements on the uniform N x N mesh of the unit square.

Test infrastructure (see the package docstring).

Interior nodes (i h, j h), i, j = 1..n with h = 1/N, n = N-1, are numbered
(j-1) n + (i-1): x1 runs fastest.  Homogeneous Dirichlet conditions remove the
boundary nodes.  The paper discretizes the heat equation with Q1 elements on
the unit square (Sec. 6, first paragraph, and Sec. 6.2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Bilinear element matrices on a square of side h, local nodes counter-clockwise
# from the lower-left corner.  Stiffness is h-independent in 2D; mass scales h^2.
KE = np.array([[4, -1, -2, -1],
               [-1, 4, -1, -2],
               [-2, -1, 4, -1],
               [-1, -2, -1, 4]], dtype=np.float64) / 6.0
ME_UNIT = np.array([[4, 2, 1, 2],
                    [2, 4, 2, 1],
                    [1, 2, 4, 2],
                    [2, 1, 2, 4]], dtype=np.float64) / 36.0


def node_index(i: int, j: int, n: int) -> int:
    """Global index of interior node (i, j), 1-based grid coordinates."""
    return (j - 1) * n + (i - 1)


def assemble_elementwise(N: int):
    """K and M by a loop over the N^2 elements (route (i)); returns CSR matrices."""
    n = N - 1
    h = 1.0 / N
    nx = n * n
    rows, cols, kv, mv = [], [], [], []
    for ey in range(N):
        for ex in range(N):
            # element corners in grid coordinates, counter-clockwise
            corners = [(ex, ey), (ex + 1, ey), (ex + 1, ey + 1), (ex, ey + 1)]
            gidx = []
            for (ci, cj) in corners:
                if 1 <= ci <= n and 1 <= cj <= n:
                    gidx.append(node_index(ci, cj, n))
                else:
                    gidx.append(-1)
            for a in range(4):
                if gidx[a] < 0:
                    continue
                for b in range(4):
                    if gidx[b] < 0:
                        continue
                    rows.append(gidx[a])
                    cols.append(gidx[b])
                    kv.append(KE[a, b])
                    mv.append(ME_UNIT[a, b] * h * h)
    K = sp.csr_matrix((kv, (rows, cols)), shape=(nx, nx))
    M = sp.csr_matrix((mv, (rows, cols)), shape=(nx, nx))
    K.sum_duplicates()
    M.sum_duplicates()
    return K, M


def matrices_1d(N: int):
    """1D P1 stiffness h^{-1} tridiag(-1,2,-1) and mass (h/6) tridiag(1,4,1) on n interior nodes."""
    n = N - 1
    h = 1.0 / N
    e = np.ones(n)
    K1 = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1]) / h
    M1 = sp.diags([e[:-1], 4 * e, e[:-1]], [-1, 0, 1]) * (h / 6.0)
    return K1.tocsr(), M1.tocsr()


def assemble_kronecker(N: int):
    """K = K1 kron M1 + M1 kron K1 and M = M1 kron M1 (route (ii)); CSC matrices."""
    K1, M1 = matrices_1d(N)
    K = (sp.kron(K1, M1) + sp.kron(M1, K1)).tocsc()
    M = sp.kron(M1, M1).tocsc()
    return K, M


def dst_1d(N: int):
    """Sine-transform eigenpairs shared by K1 and M1.

    Returns S (n x n, columns s_j with entries sqrt(2h) sin(i j pi h)), the
    stiffness eigenvalues k_j = (4/h) sin^2(j pi h / 2) and the mass
    eigenvalues m_j = (h/3)(2 + cos(j pi h)), j = 1..n.
    """
    n = N - 1
    h = 1.0 / N
    idx = np.arange(1, n + 1)
    S = np.sqrt(2.0 * h) * np.sin(np.outer(idx, idx) * np.pi * h)
    k = (4.0 / h) * np.sin(idx * np.pi * h / 2.0) ** 2
    m = (h / 3.0) * (2.0 + np.cos(idx * np.pi * h))
    return S, k, m


def modes_2d(N: int):
    """2D eigenvalues of K and M on the tensor sine basis s_i (x) s_j.

    Mode (i, j) (i for x1, j for x2) has eigenvector with node value
    s_i(x1 node) s_j(x2 node); kappa = k_i m_j + m_i k_j, mu = m_i m_j.
    Returns S, kappa (n x n, [i, j]), mu (n x n).
    """
    S, k, m = dst_1d(N)
    kappa = np.outer(k, m) + np.outer(m, k)
    mu = np.outer(m, m)
    return S, kappa, mu


def mode_vector(N: int, i: int, j: int) -> np.ndarray:
    """Euclidean-normalized nodal vector of 2D sine mode (i, j), 1-based."""
    S, _, _ = dst_1d(N)
    # node index (jj-1) n + (ii-1) holds s_i(ii) s_j(jj): x1 fastest
    return np.kron(S[:, j - 1], S[:, i - 1])
