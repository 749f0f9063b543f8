"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds workload descriptions and random draws only: problem sizes,
parameters, observation boxes, seeded Gaussian factors, request streams.  It
contains none of the method's arithmetic (no operators, no solves), so that
both sides of a parity test can take their inputs from here without sharing
any computation.

Random numbers come from NumPy's PCG64 generator with fixed seeds:
  0  noise added to the true source u_true
  1  observation noise for y_obs
  2  Lanczos start block
  3  randomized-eigensolver probe factors
  4  serving request stream
  5  standard-normal draws for posterior samples
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

SEED_UTRUE, SEED_YOBS, SEED_LANCZOS, SEED_PROBES, SEED_SERVING, SEED_SAMPLES = 0, 1, 2, 3, 4, 5


@dataclasses.dataclass(frozen=True)
class ProblemDesc:
    """A heat-equation inverse problem on the unit square.

    N      mesh cells per side (n = N-1 interior nodes per side, nx = n*n)
    nt     implicit-Euler steps over [0, T] (tau = T/nt)
    alpha  prior precision scale: Gamma_prior^{-1} = alpha*tau*(I_nt kron (K+M))
    sigma  noise standard deviation: Gamma_noise = sigma^2 I
    box    closed observation box (x1lo, x1hi, x2lo, x2hi)
    """
    N: int
    nt: int
    T: float = 1.0
    alpha: float = 1e-2
    sigma: float = 1e-2
    box: Tuple[float, float, float, float] = (0.25, 0.75, 0.25, 0.75)
    trunc_tol: float = 1e-6
    rank_cap: int = 64
    k: int = 20
    precision: str = "fp64"  # "fp64" | "mixed"

    @property
    def n(self) -> int:
        return self.N - 1

    @property
    def nx(self) -> int:
        return (self.N - 1) ** 2

    @property
    def tau(self) -> float:
        return self.T / self.nt


# The five workloads.  Names say what they are.
TINY_FP64 = ProblemDesc(N=32, nt=40, alpha=1e-2, sigma=1e-2, trunc_tol=1e-10, rank_cap=40, k=20)
MESH256_NT200 = ProblemDesc(N=256, nt=200, alpha=1e-2, sigma=1e-2, trunc_tol=1e-6, rank_cap=64, k=50)
MESH512_NT500_PROBES = ProblemDesc(N=512, nt=500, alpha=1e-3, sigma=5e-3, trunc_tol=1e-6, rank_cap=32, k=64,
                                   precision="mixed")
MESH1024_NT1000 = ProblemDesc(N=1024, nt=1000, alpha=1e-2, sigma=1e-2, trunc_tol=1e-6, rank_cap=128, k=100,
                              precision="mixed")
PROBE_COUNT, PROBE_OVERSAMPLE, PROBE_RANK = 64, 10, 32


def node_coords(N: int) -> Tuple[np.ndarray, np.ndarray]:
    """Coordinates of interior nodes, lexicographic with x1 fastest."""
    h = 1.0 / N
    x = np.arange(1, N) * h
    x1 = np.tile(x, N - 1)
    x2 = np.repeat(x, N - 1)
    return x1, x2


def sensor_mask(N: int, centers=None, side: float = 1.0 / 16.0) -> np.ndarray:
    """Observed interior nodes of a sensor layout: the nodes inside closed
    axis-aligned squares of the given side centred at `centers` (default: the
    paper's nine sensors of area 1/256 spread uniformly, side 1/16 at the
    points (i/4, j/4), i, j = 1..3).  Node index j n + i holds ((i+1) h,
    (j+1) h), x1 fastest.  Layout only; no arithmetic of the method."""
    if centers is None:
        centers = [(a / 4.0, b / 4.0) for b in (1, 2, 3) for a in (1, 2, 3)]
    x1, x2 = node_coords(N)
    eps = 1e-12
    mask = np.zeros(x1.size, dtype=bool)
    for c1, c2 in centers:
        mask |= (np.abs(x1 - c1) <= side / 2 + eps) & (np.abs(x2 - c2) <= side / 2 + eps)
    return mask


def u_true(desc: ProblemDesc) -> np.ndarray:
    """sin(pi x1) sin(pi x2) exp(-t_k) plus seeded N(0, 0.1^2) noise, shape (nx, nt)."""
    x1, x2 = node_coords(desc.N)
    t = desc.tau * np.arange(1, desc.nt + 1)
    base = np.outer(np.sin(np.pi * x1) * np.sin(np.pi * x2), np.exp(-t))
    rng = np.random.Generator(np.random.PCG64(SEED_UTRUE))
    return base + 0.1 * rng.standard_normal((desc.nx, desc.nt))


def yobs_noise(nobs: int, nt: int) -> np.ndarray:
    """Standard-normal observation noise, shape (nobs, nt); y_obs = F u_true + sigma * this."""
    rng = np.random.Generator(np.random.PCG64(SEED_YOBS))
    return rng.standard_normal((nobs, nt))


def lanczos_start(nx: int, nt: int, b: int = 4) -> Tuple[np.ndarray, np.ndarray]:
    """Start block of b rank-1 space-time vectors a_j (x) b_j: returns (A nx x b, B nt x b)."""
    rng = np.random.Generator(np.random.PCG64(SEED_LANCZOS))
    A = rng.standard_normal((nx, b))
    B = rng.standard_normal((nt, b))
    return A, B


def probe_factors(nx: int, nt: int, count: int = PROBE_COUNT + PROBE_OVERSAMPLE,
                  rank: int = PROBE_RANK, seed: int = SEED_PROBES) -> Tuple[np.ndarray, np.ndarray]:
    """Gaussian probe factors: probe j is G1[:, j] G2[:, j]^T / sqrt(rank).

    Returns G1 of shape (count, nx, rank) and G2 of shape (count, nt, rank),
    drawn probe by probe in that order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    G1 = np.empty((count, nx, rank))
    G2 = np.empty((count, nt, rank))
    for j in range(count):
        G1[j] = rng.standard_normal((nx, rank))
        G2[j] = rng.standard_normal((nt, rank))
    return G1, G2


def sample_normals(ns: int, nx: int, nt: int) -> np.ndarray:
    """Standard-normal draws for posterior samples, shape (ns, nx, nt)."""
    rng = np.random.Generator(np.random.PCG64(SEED_SAMPLES))
    return rng.standard_normal((ns, nx, nt))


@dataclasses.dataclass(frozen=True)
class Request:
    arrival_s: float
    desc: ProblemDesc


def serving_stream(count: int = 256, rate_per_s: float = 20.0, k: int = 30,
                   seed: int = SEED_SERVING) -> List[Request]:
    """Poisson arrivals of posterior requests with uneven mesh and time sizes.

    Mesh side from {64,128,256}, nt from {50,100,200}, sigma and alpha from
    {1e-3,1e-2}; the observation box covers a fraction a ~ U[0.10,0.40] of the
    domain with aspect rho ~ logU[1/2,2], its lower corner uniform, and its
    edges snapped outward to mesh nodes so that it holds at least one node.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out: List[Request] = []
    t = 0.0
    for _ in range(count):
        t += rng.exponential(1.0 / rate_per_s)
        N = int(rng.choice([64, 128, 256]))
        nt = int(rng.choice([50, 100, 200]))
        sigma = float(rng.choice([1e-3, 1e-2]))
        alpha = float(rng.choice([1e-3, 1e-2]))
        a = rng.uniform(0.10, 0.40)
        rho = math.exp(rng.uniform(math.log(0.5), math.log(2.0)))
        w = min(math.sqrt(a * rho), 1.0)
        hh = min(math.sqrt(a / rho), 1.0)
        lo1 = rng.uniform(0.0, 1.0 - w)
        lo2 = rng.uniform(0.0, 1.0 - hh)
        h = 1.0 / N
        # snap outward to nodes, clamp to interior nodes
        b = (math.floor(lo1 / h) * h, math.ceil((lo1 + w) / h) * h,
             math.floor(lo2 / h) * h, math.ceil((lo2 + hh) / h) * h)
        b = (max(b[0], h), min(b[1], 1 - h), max(b[2], h), min(b[3], 1 - h))
        out.append(Request(arrival_s=t, desc=ProblemDesc(N=N, nt=nt, alpha=alpha, sigma=sigma, box=b,
                                                          trunc_tol=1e-6, rank_cap=64, k=k)))
    return out
