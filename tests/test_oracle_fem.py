"""Pins for the oracle's Q1 operators (assembly, stencils, sine-transform spectra)."""
import numpy as np
import pytest

from oracle import closed_forms, fem


@pytest.mark.parametrize("N", [3, 4, 8, 13])
def test_two_assemblies_agree(N):
    Ke, Me = fem.assemble_elementwise(N)
    Kk, Mk = fem.assemble_kronecker(N)
    assert np.allclose(Ke.toarray(), Kk.toarray(), rtol=0, atol=1e-14)
    assert np.allclose(Me.toarray(), Mk.toarray(), rtol=0, atol=1e-18)


def test_stencil_values_and_row_sums():
    N = 10
    n, h = N - 1, 1.0 / N
    K, M = fem.assemble_elementwise(N)
    K, M = K.toarray(), M.toarray()
    c = fem.node_index(5, 5, n)
    nb = {(di, dj): fem.node_index(5 + di, 5 + dj, n) for di in (-1, 0, 1) for dj in (-1, 0, 1)}
    assert K[c, c] == pytest.approx(8.0 / 3.0)
    for (di, dj), j in nb.items():
        if (di, dj) != (0, 0):
            assert K[c, j] == pytest.approx(-1.0 / 3.0)
    assert M[c, c] == pytest.approx(4 * h * h / 9)
    assert M[c, nb[(1, 0)]] == pytest.approx(h * h / 9)
    assert M[c, nb[(0, 1)]] == pytest.approx(h * h / 9)
    assert M[c, nb[(1, 1)]] == pytest.approx(h * h / 36)
    # rows of nodes not adjacent to the boundary: mass sums to h^2, stiffness to 0
    for i in range(2, n):
        for j in range(2, n):
            r = fem.node_index(i, j, n)
            assert M[r].sum() == pytest.approx(h * h, rel=1e-13)
            assert abs(K[r].sum()) < 1e-13
    # the stiffness matrix of a Dirichlet problem is positive definite
    assert np.linalg.eigvalsh(K).min() > 0


@pytest.mark.parametrize("N", [5, 16])
def test_sine_basis_diagonalizes_1d_and_2d(N):
    K1, M1 = fem.matrices_1d(N)
    S, k, m = fem.dst_1d(N)
    assert np.allclose(S.T @ S, np.eye(N - 1), atol=1e-13)
    assert np.allclose(K1 @ S, S * k, atol=1e-12)
    assert np.allclose(M1 @ S, S * m, atol=1e-14)
    K, M = fem.assemble_elementwise(N)
    _, kappa, mu = fem.modes_2d(N)
    for (i, j) in [(1, 1), (2, 1), (1, 3), (N - 1, N - 2)]:
        phi = fem.mode_vector(N, i, j)
        assert np.allclose(K @ phi, kappa[i - 1, j - 1] * phi, atol=1e-12)
        assert np.allclose(M @ phi, mu[i - 1, j - 1] * phi, atol=1e-16)


def test_discrete_spectrum_converges_to_continuum():
    """Sec. 5: Dirichlet Laplacian eigenvalues pi^2 (m^2 + n^2) on the unit square.
    Q1 generalized eigenvalues kappa/mu converge at O(h^2)."""
    errs = []
    for N in (16, 32, 64):
        _, kappa, mu = fem.modes_2d(N)
        lam = kappa / mu
        for (m_, n_) in [(1, 1), (1, 2), (2, 3)]:
            exact = closed_forms.continuum_laplace_eigs(m_, n_)
            assert lam[m_ - 1, n_ - 1] > exact  # conforming FEM overestimates
        errs.append(lam[0, 0] - closed_forms.continuum_laplace_eigs(1, 1))
    # halving h divides the error by about 4
    assert 3.5 < errs[0] / errs[1] < 4.5
    assert 3.5 < errs[1] / errs[2] < 4.5
