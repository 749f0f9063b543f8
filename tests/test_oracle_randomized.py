"""Pins of the oracle's randomized eigensolver (two-pass range finder plus
Rayleigh-Ritz in the P inner product) against facts fixed by the mathematics."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import posterior  # noqa: E402
from oracle.randomized import probes_from_factors, randomized_eig  # noqa: E402
from oracle.spacetime import Problem  # noqa: E402

BOX = (0.2, 0.8, 0.2, 0.8)


def test_probes_spanning_the_space_give_the_exact_spectrum():
    """Rank-one probes that span all of R^{nx x nt}: the Ritz values are the
    pencil's nonzero eigenvalues (the null space of H_mis drops out of range(Y))."""
    p = Problem(4, 2, alpha=1e-2, sigma=1e-2, box=BOX)
    n = p.nx * p.nt
    rng = np.random.default_rng(11)
    probes = [np.outer(rng.standard_normal(p.nx), rng.standard_normal(p.nt)) for _ in range(n)]
    lam, _ = posterior.eig_dense(p)
    k = int(np.sum(lam > 1e-10 * lam[0]))
    theta, _, res = randomized_eig(p, probes, k)
    assert np.allclose(theta, lam[:k], rtol=1e-9)
    assert np.all(res <= 1e-8 * theta)


def test_ritz_values_interlace_below_the_eigenvalues():
    """Rayleigh-Ritz on any subspace: theta_i <= lambda_i (Cauchy interlacing)."""
    p = Problem(8, 4, alpha=1e-2, sigma=1e-2, box=BOX)
    G1 = np.random.default_rng(3).standard_normal((6, p.nx, 2))
    G2 = np.random.default_rng(4).standard_normal((6, p.nt, 2))
    theta, X, _ = randomized_eig(p, probes_from_factors(G1, G2), 6)
    lam, _ = posterior.eig_dense(p, 6)
    assert np.all(theta <= lam * (1 + 1e-10))
    # the Ritz vectors are P-orthonormal
    Gx = np.array([[p.P_inner(a, b) for b in X] for a in X])
    assert np.allclose(Gx, np.eye(len(X)), atol=1e-10)


def test_invariant_subspace_probes_give_exact_pairs():
    """Probes spanning the top-5 eigenvectors: exact eigenvalues, zero residuals."""
    p = Problem(8, 4, alpha=1e-2, sigma=1e-2, box=BOX)
    lam, V = posterior.eig_dense(p, 5)
    rng = np.random.default_rng(5)
    mix = rng.standard_normal((5, 5))
    probes = [(V @ mix[:, j]).reshape((p.nx, p.nt), order="F") for j in range(5)]
    theta, _, res = randomized_eig(p, probes, 5)
    assert np.allclose(theta, lam, rtol=1e-10)
    assert np.all(res <= 1e-8 * lam)
