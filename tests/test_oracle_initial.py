"""Pins of the oracle's initial-condition problem (Sec. 6, eqs. pde, dis_obj,
postvar, misfit; Sec. 6.2): closed forms, an independent all-at-once route,
symmetry, the Woodbury identity and the sensor layout."""
import os
import sys

import numpy as np
import scipy.sparse.linalg as spla

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import fem  # noqa: E402
from oracle.initial import ICProblem, full_obs_ic_eigs  # noqa: E402
from synthetic import sensor_mask  # noqa: E402


def test_full_observation_spectrum_closed_form():
    """Every node observed: the spectrum of G is c sigma^-2 sum_k rho_p^2k over the sine modes."""
    N, nt = 8, 6
    p = ICProblem(N, nt, sigma=0.05, prior_var=10.0, mask=np.ones((N - 1) ** 2, dtype=bool))
    w, _ = p.eig()
    ref = full_obs_ic_eigs(N, nt, 1.0, 0.05, 10.0)
    assert np.allclose(w, ref, rtol=1e-10, atol=1e-12 * ref[0])


def test_time_stepping_equals_all_at_once_system():
    """G by forward/adjoint time stepping equals G from the sparse space-time system."""
    p = ICProblem(8, 5, sigma=0.03, prior_var=10.0)
    A = p.dense_G()
    B = p.dense_G_allatonce()
    assert np.abs(A - B).max() <= 1e-10 * np.abs(B).max()


def test_single_step_is_the_step_map():
    """nt = 1: G = c sigma^-2 T^T B^T B T with T = (M + tau K)^{-1} M."""
    p = ICProblem(8, 1, sigma=0.1, prior_var=2.0)
    Tm = spla.spsolve((p.M + p.tau * p.K).tocsc(), p.M.toarray())
    Bm = np.eye(p.nx)[p.obs_idx]
    ref = 2.0 * (Bm @ Tm).T @ (Bm @ Tm) / 0.1 ** 2
    assert np.abs(p.dense_G() - ref).max() <= 1e-11 * np.abs(ref).max()


def test_G_is_symmetric():
    rng = np.random.default_rng(0)
    p = ICProblem(16, 7, sigma=0.02, prior_var=10.0)
    u, v = rng.standard_normal(p.nx), rng.standard_normal(p.nx)
    a, b = np.dot(p.G(u), v), np.dot(u, p.G(v))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_woodbury_posterior_variance():
    """All eigenpairs: c - c sum lam/(1+lam) v^2 equals diag(c (I + G)^{-1})."""
    p = ICProblem(8, 4, sigma=0.02, prior_var=10.0)
    lam, V = p.eig()
    assert np.allclose(p.post_var_lowrank(lam, V), p.post_var_exact(), rtol=1e-10, atol=1e-12)
    # fewer pairs never go below the exact variance
    assert np.all(p.post_var_lowrank(lam[:5], V[:, :5]) >= p.post_var_exact() - 1e-12)


def test_nine_sensors_of_area_one_256th():
    """At 64 x 64 each sensor square (side 1/16 = 4h, centred on a node) holds 5 x 5 nodes."""
    m = sensor_mask(64)
    assert m.sum() == 9 * 25
    n = 63
    ij = np.argwhere(m.reshape(n, n))  # (x2 index, x1 index)
    centres = {(a * 16 - 1, b * 16 - 1) for a in (1, 2, 3) for b in (1, 2, 3)}
    for a, b in centres:
        assert m.reshape(n, n)[a, b]
    assert ij.min() == 16 - 1 - 2 and ij.max() == 48 - 1 + 2


def test_closed_form_uses_the_sine_basis():
    """The step map's eigenvectors are the sine modes (the closed form's premise)."""
    N, nt = 8, 3
    p = ICProblem(N, nt, mask=np.ones((N - 1) ** 2, dtype=bool))
    v = fem.mode_vector(N, 2, 3)
    _, kappa, mu = fem.modes_2d(N)
    rho = mu[1, 2] / (mu[1, 2] + p.tau * kappa[1, 2])
    y1 = p.forward(v)[:, 0]
    assert np.allclose(y1, rho * v, atol=1e-13)


def test_arpack_route_equals_dense_eigensolve():
    p = ICProblem(16, 6, sigma=0.03, prior_var=10.0)
    w, _ = p.eig(8)
    wa, _ = p.eig_arpack(8)
    assert np.allclose(wa, w, rtol=1e-9)
