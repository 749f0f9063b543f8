"""Low-rank space-time vectors and the low-rank Arnoldi process (Sec. 4).

Test infrastructure (see the package docstring).

A space-time vector v = vec(V), V in R^{nx x nt}, is kept as factors
V = W1 W2^T (Sec. 4 eq. lr_vec).  Sums concatenate factors (Sec. 4 eq.
lanczos2) and truncation keeps the smallest rank r with
sqrt(sum_{i>r} s_i^2) <= tol * ||s||_2 (relative Frobenius), computed here from
a dense SVD of the represented matrix, the plainest form of the truncated SVD
the paper names.
"""
from __future__ import annotations

import numpy as np


def truncate_dense(X, tol, rank_cap=None):
    """Factors (W1, W2) of the relative-Frobenius truncation of dense X."""
    U, s, Vt = np.linalg.svd(np.asarray(X, dtype=np.float64), full_matrices=False)
    r = truncation_rank(s, tol)
    if rank_cap is not None:
        r = min(r, rank_cap)
    return U[:, :r] * s[:r], Vt[:r].T


def truncation_rank(s, tol):
    """Smallest r with sqrt(sum_{i>r} s_i^2) <= tol * ||s||_2 (0 for a zero vector)."""
    s = np.asarray(s, dtype=np.float64)
    total = np.sqrt(np.sum(s * s))
    if total == 0.0:
        return 0
    tail = np.sqrt(np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]]))
    for r in range(len(s) + 1):
        if tail[r] <= tol * total:
            return r
    return len(s)


def lr_arnoldi(apply, inner, v1, steps, tol, rank_cap=None):
    """Low-rank Arnoldi with modified Gram-Schmidt (Sec. 4 Algorithm 1).

    apply(X) -> dense image of the operator on dense X; inner(X, Y) -> scalar.
    The operator image and every update are truncated back to low rank at
    tolerance tol.  Returns the Hessenberg matrix H ((steps+1) x steps) and the
    list of basis vectors as (W1, W2) factor pairs.
    """
    W1, W2 = truncate_dense(v1, tol, rank_cap)
    nrm = np.sqrt(inner(W1 @ W2.T, W1 @ W2.T))
    basis = [(W1 / nrm, W2)]
    H = np.zeros((steps + 1, steps))
    for j in range(steps):
        Vj = basis[j][0] @ basis[j][1].T
        w = apply(Vj)
        w1, w2 = truncate_dense(w, tol, rank_cap)
        w = w1 @ w2.T
        for i in range(j + 1):
            Vi = basis[i][0] @ basis[i][1].T
            H[i, j] = inner(w, Vi)
            w1, w2 = truncate_dense(w - H[i, j] * Vi, tol, rank_cap)
            w = w1 @ w2.T
        H[j + 1, j] = np.sqrt(max(inner(w, w), 0.0))
        if j + 1 < steps + 1 and H[j + 1, j] > 0:
            basis.append((w1 / H[j + 1, j], w2))
        else:
            break
    return H, basis
