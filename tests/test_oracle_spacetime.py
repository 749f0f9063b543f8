"""Pins for the oracle's forward/adjoint maps and Hessian."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import closed_forms, fem
from oracle.spacetime import Problem


def _rng(seed=11):
    return np.random.default_rng(seed)


def test_time_stepping_equals_all_at_once_system():
    p = Problem(6, 5, alpha=1e-2, sigma=1e-2, box=(0.3, 0.7, 0.2, 0.9))
    Kst, Sst, _, _ = p.spacetime_matrices()
    U = _rng().standard_normal((p.nx, p.nt))
    y_all = spla.spsolve(Kst, Sst @ U.reshape(-1, order="F"))
    assert np.allclose(p.forward(U).reshape(-1, order="F"), y_all, rtol=1e-13, atol=1e-15)


def test_two_routes_to_dense_F_agree():
    p = Problem(5, 4, box=(0.2, 0.8, 0.4, 1.0))
    assert np.allclose(p.dense_F(), p.impulse_F(), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("ij", [(1, 1), (2, 3), (4, 1)])
def test_single_mode_solution(ij):
    """A sine mode in space stays a sine mode; time follows the per-mode bidiagonal system."""
    N, nt = 8, 7
    p = Problem(N, nt)
    g = _rng(3).standard_normal(nt)
    U = np.outer(fem.mode_vector(N, *ij), g)
    assert np.allclose(p.forward(U), closed_forms.single_mode_state(N, nt, 1.0, *ij, g), rtol=1e-12, atol=1e-15)


def test_adjoint_identity_and_hessian_symmetry():
    p = Problem(12, 9, alpha=3e-2, sigma=2e-2, box=(0.25, 0.75, 0.1, 0.6))
    rng = _rng(5)
    X = rng.standard_normal((p.nx, p.nt))
    Z = rng.standard_normal((p.nobs, p.nt))
    lhs = np.sum(p.F(X) * Z)
    rhs = np.sum(X * p.FT(Z))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    Y = rng.standard_normal((p.nx, p.nt))
    a, b = np.sum(p.H_mis(X) * Y), np.sum(X * p.H_mis(Y))
    assert abs(a - b) <= 1e-12 * abs(a)
    assert np.sum(p.H_mis(X) * X) >= 0
    # G is self-adjoint in the prior-precision inner product
    a, b = p.P_inner(p.G(X), Y), p.P_inner(X, p.G(Y))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_mask_is_closed_box():
    p = Problem(32, 2)  # nodes at multiples of 1/32; 0.25 and 0.75 are nodes
    assert p.nobs == 17 * 17
    p2 = Problem(32, 2, box=(0.0, 1.0, 0.0, 1.0))
    assert p2.nobs == p2.nx
