"""Pins for the oracle's truncation rule."""
import numpy as np

from oracle.lowrank import truncate_dense, truncation_rank


def test_truncation_rank_rule():
    s = np.array([1.0, 1e-3, 1e-7, 1e-9])
    # tail after r=2 is sqrt(1e-14 + 1e-18) ~ 1e-7 > 1e-8; after r=3 it is 1e-9 <= 1e-8
    assert truncation_rank(s, 1e-8) == 3
    assert truncation_rank(s, 1e-6) == 2
    assert truncation_rank(s, 0.0) == 4
    assert truncation_rank(np.zeros(3), 1e-8) == 0


def test_truncate_exact_low_rank():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((50, 4)) @ rng.standard_normal((4, 30))
    W1, W2 = truncate_dense(A, 1e-12)
    assert W1.shape[1] == 4
    assert np.allclose(W1 @ W2.T, A, atol=1e-12 * np.abs(A).max())
    W1, W2 = truncate_dense(A, 1e-12, rank_cap=2)
    assert W1.shape[1] == 2
