"""Pins for the oracle's posterior mean (MAP point, Sec. 2 eq. map1)."""
import numpy as np

import synthetic
from oracle import mean
from oracle.spacetime import Problem

FULL = (0.0, 1.0, 0.0, 1.0)


def _data(p, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((p.nx, p.nt))
    return mean.observe_data(p, u, rng.standard_normal((p.nobs, p.nt)))


def test_two_routes_agree():
    """Normal equations with the dense matrices == the data-space (Woodbury) form."""
    p = Problem(6, 5, alpha=2e-2, sigma=3e-2, box=(0.2, 0.7, 0.3, 0.8))
    y = _data(p, 1)
    a = mean.mean_dense(p, y)
    b = mean.mean_dataspace(p, y)
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(a)


def test_normal_equations_hold_with_the_time_stepping_maps():
    """The data-space point satisfies (H_mis + P) u = sigma^{-2} F^T y evaluated
    with the matrix-free time-stepping maps (a route independent of the dense F)."""
    p = Problem(8, 6, alpha=1e-2, sigma=1e-2)
    y = _data(p, 2)
    u = mean.mean_dataspace(p, y)
    assert mean.normal_equation_residual(p, u, y) < 1e-10


def test_full_observation_closed_form():
    """Every node observed: the per-mode nt x nt solves of the sine basis give the same point."""
    N, nt, alpha, sigma = 6, 5, 2e-2, 3e-2
    p = Problem(N, nt, alpha=alpha, sigma=sigma, box=FULL)
    y = _data(p, 3)
    a = mean.mean_dataspace(p, y)
    b = mean.mean_full_obs_closed(N, nt, 1.0, alpha, sigma, y)
    assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(a)


def test_map_point_minimizes_the_objective():
    """J(u) = 1/2 ||u||_P^2 + 1/2 sigma^-2 ||y - F u||^2 grows in every direction
    away from the point (by exactly 1/2 ||d||^2_{H_mis + P})."""
    p = Problem(6, 4, alpha=1e-2, sigma=5e-2, box=(0.1, 0.5, 0.2, 0.9))
    y = _data(p, 4)
    u = mean.mean_dataspace(p, y)

    def J(v):
        r = y - p.F(v)
        return 0.5 * p.P_inner(v, v) + 0.5 * np.sum(r * r) / p.sigma ** 2

    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.standard_normal(u.shape) * 1e-2
        growth = J(u + d) - J(u)
        quad = 0.5 * (np.sum(d * p.H_mis(d)) + p.P_inner(d, d))
        assert growth > 0
        assert abs(growth - quad) <= 1e-8 * quad


def test_workload_data_shapes():
    """u_true and y_obs of the workload recipe (seeds 0 and 1)."""
    d = synthetic.ProblemDesc(N=8, nt=5)
    p = Problem.from_desc(d)
    u = synthetic.u_true(d)
    y = mean.observe_data(p, u, synthetic.yobs_noise(p.nobs, p.nt))
    assert u.shape == (p.nx, p.nt) and y.shape == (p.nobs, p.nt)
    assert np.all(np.isfinite(y))
