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


def test_forward_source_solves_the_all_at_once_system():
    """forward_source is the solve of Sec. 6.1 eq. st_pde with L = tau K and
    C = I - S, for any right-hand side: checked against a sparse direct solve
    of the Kronecker-form matrix (no time stepping), and against the
    parameter-to-state map when the right-hand side is the source tau M U."""
    p = Problem(7, 6, box=(0.2, 0.9, 0.1, 0.6))
    Kst, Sst, _, _ = p.spacetime_matrices()
    rng = _rng(23)
    F = rng.standard_normal((p.nx, p.nt))
    ref = spla.spsolve(Kst, F.reshape(-1, order="F")).reshape((p.nx, p.nt), order="F")
    assert np.allclose(p.forward_source(F), ref, rtol=1e-13, atol=1e-14 * np.abs(ref).max())
    U = rng.standard_normal((p.nx, p.nt))
    assert np.allclose(p.forward_source(p.tau * (p.M @ U)), p.forward(U), rtol=1e-13, atol=1e-15)


def test_adjoint_source_solves_the_transposed_system():
    """adjoint_source solves (I kron tau K + C^T kron M) vec(P) = vec(Z): the
    transpose of the all-at-once matrix (K and M are symmetric), checked by a
    sparse direct solve with Kst^T."""
    p = Problem(7, 5, box=(0.2, 0.9, 0.1, 0.6))
    Kst, _, _, _ = p.spacetime_matrices()
    Z = _rng(29).standard_normal((p.nx, p.nt))
    ref = spla.spsolve(Kst.T.tocsc(), Z.reshape(-1, order="F")).reshape((p.nx, p.nt), order="F")
    assert np.allclose(p.adjoint_source(Z), ref, rtol=1e-13, atol=1e-14 * np.abs(ref).max())
