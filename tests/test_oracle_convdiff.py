"""Pins of the oracle's SUPG convection-diffusion operator and of the
initial-condition problem built on it (Sec. 6 eqs. pde, dis_obj, postvar;
Sec. 6.3): reductions to the Q1 heat matrices, the Kronecker form of a wind
along x2 from 1D integrals, skew symmetry of the convection part, exactness
on linear fields, the Peclet rule, and the all-at-once route that pins the
transposed adjoint."""
import math
import os
import sys

import numpy as np
import scipy.sparse as sp

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import fem  # noqa: E402
from oracle.convdiff import assemble_supg, cd_ic_problem, supg_delta  # noqa: E402
from oracle.initial import ICProblem  # noqa: E402


def _dense(A):
    return A.toarray() if sp.issparse(A) else np.asarray(A)


def test_no_wind_unit_viscosity_is_the_heat_stiffness():
    """nu = 1, w = 0: the quadrature loop reproduces the Q1 stiffness and mass."""
    N = 9
    L, M = assemble_supg(N, 1.0, (0.0, 0.0))
    K, Mk = fem.assemble_kronecker(N)
    assert np.abs(_dense(L) - _dense(K)).max() <= 1e-13
    assert np.abs(_dense(M) - _dense(Mk)).max() <= 1e-16


def test_wind_along_x2_has_the_kronecker_form():
    """w = (0, w2), constant delta: L = (nu + delta w2^2) K1 (x) M1 + nu M1 (x) K1
    + w2 C1 (x) M1 (first factor acting along x2, the slow index), with the 1D
    convection matrix C1_ij = int phi_j' phi_i = +-1/2 off the diagonal."""
    N, nu, w2 = 12, 3e-3, 0.7
    delta = supg_delta(N, nu, (0.0, w2))
    assert delta > 0
    L, _ = assemble_supg(N, nu, (0.0, w2))
    K1, M1 = fem.matrices_1d(N)
    e = np.ones(N - 2)
    C1 = sp.diags([-0.5 * e, 0.5 * e], [-1, 1])
    ref = (nu + delta * w2 * w2) * sp.kron(K1, M1) + nu * sp.kron(M1, K1) + w2 * sp.kron(C1, M1)
    assert np.abs(_dense(L) - _dense(ref)).max() <= 1e-14 * np.abs(_dense(ref)).max()


def test_convection_part_is_skew():
    """Galerkin convection with a constant wind and zero boundary values:
    N + N^T = 0 (any wind direction)."""
    N = 10
    Lc, _ = assemble_supg(N, 1.0, (0.3, -0.8), delta=0.0)
    L0, _ = assemble_supg(N, 1.0, (0.0, 0.0), delta=0.0)
    Nc = _dense(Lc) - _dense(L0)
    assert np.abs(Nc).max() > 0.2 / N  # entries of order h
    assert np.abs(Nc + Nc.T).max() <= 1e-13 * np.abs(Nc).max()


def test_exact_on_linear_fields():
    """u = a x1 + b x2 (Laplacian zero, w . grad u = w1 a + w2 b constant): at
    rows whose neighbours are all interior, (L u)_i = h^2 (w1 a + w2 b); the
    streamline term integrates a derivative of phi_i and gives zero."""
    N, nu, w = 16, 1e-3, (0.4, 0.9)
    L, _ = assemble_supg(N, nu, w)
    n, h = N - 1, 1.0 / N
    x1 = np.tile(np.arange(1, n + 1) * h, n)
    x2 = np.repeat(np.arange(1, n + 1) * h, n)
    a, b = 0.37, -1.3
    r = L @ (a * x1 + b * x2)
    i = np.tile(np.arange(1, n + 1), n)
    j = np.repeat(np.arange(1, n + 1), n)
    inner = (i > 1) & (i < n) & (j > 1) & (j < n)
    assert np.abs(r[inner] - h * h * (w[0] * a + w[1] * b)).max() <= 1e-14


def test_peclet_rule():
    """Pe <= 1: no stabilization; wind along a grid line with Pe > 1:
    nu + delta |w| = h / 2 (the streamwise stencil becomes the upwind
    difference); diagonal wind: h_w = h sqrt(2)."""
    N = 32
    h = 1.0 / N
    assert supg_delta(N, 1.0, (0.0, 1.0)) == 0.0
    assert supg_delta(N, h / 2, (0.0, 1.0)) == 0.0  # Pe = 1 exactly
    for nu in (1e-2, 1e-3):
        d = supg_delta(N, nu, (0.0, 1.0))
        assert abs(nu + d - h / 2) <= 1e-17
    d = supg_delta(N, 1e-3, (1.0, 1.0))
    hw = h * math.sqrt(2.0)
    pe = math.sqrt(2.0) * hw / 2e-3
    assert abs(d - hw / (2 * math.sqrt(2.0)) * (1 - 1 / pe)) <= 1e-17
    # the x2 stencil of (nu + delta) K1 + C1 at Pe > 1 has no downstream entry
    K1, _ = fem.matrices_1d(N)
    e = np.ones(N - 2)
    C1 = sp.diags([-0.5 * e, 0.5 * e], [-1, 1])
    A = _dense((1e-3 + supg_delta(N, 1e-3, (0.0, 1.0))) * K1 + C1)
    assert np.abs(np.diag(A, 1)).max() <= 1e-15
    assert np.allclose(np.diag(A, -1), -1.0) and np.allclose(np.diag(A), 1.0)


def test_time_stepping_equals_all_at_once_with_convection():
    """G by forward steps and transposed adjoint steps equals G from the
    sparse space-time system (which never forms an adjoint step): a plain
    adjoint (untransposed L) fails this."""
    p = cd_ic_problem(8, 5, 1e-2, sigma=0.03)
    A = p.dense_G()
    B = p.dense_G_allatonce()
    assert np.abs(A - B).max() <= 1e-10 * np.abs(B).max()
    assert np.abs(A - A.T).max() <= 1e-10 * np.abs(A).max()


def test_adjoint_identity_with_convection():
    rng = np.random.default_rng(3)
    p = cd_ic_problem(12, 7, 1e-3)
    u = rng.standard_normal(p.nx)
    D = rng.standard_normal((len(p.obs_idx), p.nt))
    lhs = np.sum(p.F(u) * D)
    rhs = np.dot(u, p.FT(D))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_no_wind_reduces_to_the_heat_problem():
    """w = 0, nu = 1: the convection-diffusion problem is the heat problem."""
    p = cd_ic_problem(8, 4, 1.0, wind=(0.0, 0.0), sigma=0.02)
    q = ICProblem(8, 4, sigma=0.02, prior_var=10.0)
    A, B = p.dense_G(), q.dense_G()
    assert np.abs(A - B).max() <= 1e-11 * np.abs(B).max()


def test_woodbury_variance_with_convection():
    p = cd_ic_problem(8, 6, 1e-3)
    lam, V = p.eig()
    assert np.allclose(p.post_var_lowrank(lam, V), p.post_var_exact(), rtol=1e-10, atol=1e-12)


def test_source_solves_equal_the_all_at_once_system():
    """Forward steps with a general source, and the transposed adjoint steps,
    equal sparse solves with K_st = I kron tau L + C_t kron M and its
    transpose (eq. st_pde)."""
    import scipy.sparse.linalg as spla
    p = cd_ic_problem(10, 6, 1e-3)
    rng = np.random.default_rng(11)
    F = rng.standard_normal((p.nx, p.nt))
    Ct = sp.eye(p.nt) - sp.eye(p.nt, k=-1)
    Kst = (sp.kron(sp.eye(p.nt), p.tau * p.L) + sp.kron(Ct, p.M)).tocsc()
    fwd = spla.spsolve(Kst, F.T.reshape(-1)).reshape(p.nt, p.nx).T
    adj = spla.spsolve(Kst.T.tocsc(), F.T.reshape(-1)).reshape(p.nt, p.nx).T
    assert np.abs(p.forward_source(F) - fwd).max() <= 1e-12 * np.abs(fwd).max()
    assert np.abs(p.adjoint(F) - adj).max() <= 1e-12 * np.abs(adj).max()
