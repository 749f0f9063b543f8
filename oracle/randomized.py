"""Two-pass randomized eigensolver for the pencil (H_mis, P).

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may use the oracle.

The method is the two-pass randomized range finder followed by Rayleigh-Ritz
(Halko, Martinsson and Tropp, SIAM Review 2011: Algorithm 4.1 for the range,
Algorithm 5.3 for the eigenvalue decomposition of a self-adjoint operator),
carried out in the P inner product so that G = P^{-1} H_mis is self-adjoint:

1. Y_j = G Omega_j for the given probes Omega_j (space-time arrays).
2. A P-orthonormal basis Q of range(Y): with the Gram matrix
   Gy = [<Y_i, Y_j>_P] = U diag(mu) U^T, Q_c = sum_j Y_j U_jc / sqrt(mu_c),
   keeping the directions with mu_c > 1e-14 max(mu).
3. T = [<Q_a, G Q_b>_P] (second pass of applies), symmetrized.
4. T = V diag(theta) V^T; Ritz pairs (theta_i, sum_c Q_c V_ci), largest first.

Every apply is the oracle's exact FP64 G (time stepping with a sparse LU).
The eigenvalue problem of the pencil is the one of Sec. 2 (prior-preconditioned
Hessian, eq. prior_pre); the randomized solver itself is not in the paper.
"""
import numpy as np

from .spacetime import Problem


def randomized_eig(prob: Problem, probes, k: int):
    """Top-k Ritz pairs from the probes (list of (nx, nt) arrays).

    Returns (theta (k,), X list of (nx, nt) arrays with <X_i, X_j>_P = delta_ij,
    residual norms ||G X_i - theta_i X_i||_P).
    """
    Y = [prob.G(np.asarray(w, dtype=np.float64)) for w in probes]
    l = len(Y)
    Gy = np.array([[prob.P_inner(Y[i], Y[j]) for j in range(l)] for i in range(l)])
    mu, U = np.linalg.eigh(0.5 * (Gy + Gy.T))
    keep = np.where(mu > 1e-14 * mu.max())[0][::-1]
    Q = [sum(Y[j] * (U[j, c] / np.sqrt(mu[c])) for j in range(l)) for c in keep]
    W = [prob.G(q) for q in Q]
    m = len(Q)
    T = np.array([[prob.P_inner(Q[a], W[b]) for b in range(m)] for a in range(m)])
    theta, V = np.linalg.eigh(0.5 * (T + T.T))
    order = np.argsort(theta)[::-1][:k]
    X = [sum(Q[c] * V[c, i] for c in range(m)) for i in order]
    GX = [sum(W[c] * V[c, i] for c in range(m)) for i in order]
    res = np.array([np.sqrt(max(prob.P_inner(g - t * x, g - t * x), 0.0))
                    for g, t, x in zip(GX, theta[order], X)])
    return theta[order], X, res


def probes_from_factors(G1, G2):
    """Probe arrays Omega_j = G1[j] G2[j]^T / sqrt(rank) from (count, nx, r) and (count, nt, r) factors."""
    r = G1.shape[2]
    return [G1[j] @ G2[j].T / np.sqrt(r) for j in range(G1.shape[0])]
