"""The allocation-free Gram entry point (lrpost_gram_noalloc) against the
allocating one (lrpost_gram): same kernels and chunking, so equal bits; two
calls in a row, the second smaller, share the static scratch."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import synthetic  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_05638_amd import lrpost
    lrpost.load()
    return lrpost


def test_noalloc_gram_equals_allocating_gram(lp):
    import torch
    print("case gram noalloc", flush=True)
    prob = lp.Problem(synthetic.ProblemDesc(N=256, nt=4, trunc_tol=1e-6, rank_cap=8))
    rng = np.random.default_rng(99)
    for m, q in ((180, 70), (37, 12)):  # the second call smaller than the first
        A = torch.tensor(rng.standard_normal((m, prob.nx)), device="cuda")
        B = torch.tensor(rng.standard_normal((q, prob.nx)), device="cuda")
        C = torch.full((q, m), float("nan"), dtype=torch.float64, device="cuda")
        prob.gram_noalloc(A, B, C)
        torch.cuda.synchronize()
        got = C.cpu().numpy().T
        ref = prob.gram(A, B)
        print("m=%d q=%d noalloc vs gram max abs diff %.3e" % (m, q, np.abs(got - ref).max()), flush=True)
        assert np.array_equal(got, ref)
        ref64 = A.cpu().numpy() @ B.cpu().numpy().T
        assert np.abs(got - ref64).max() <= 1e-13 * np.abs(ref64).max()


def test_noalloc_gram_rejects_sizes_beyond_the_scratch(lp):
    import torch
    print("case gram noalloc too large", flush=True)
    prob = lp.Problem(synthetic.ProblemDesc(N=32, nt=4, trunc_tol=1e-6, rank_cap=8))
    A = torch.zeros((4096, prob.nx), dtype=torch.float64, device="cuda")
    C = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda")
    with pytest.raises(lp.LrpostError) as ex:
        prob.gram_noalloc(A, A, C)
    assert ex.value.code == -1 and "scratch" in str(ex.value)
