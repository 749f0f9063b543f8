"""HIP-graph replay of the multigrid V-cycles and the autotuned stencil
strips: both must give exactly the bits of the plain kernel-by-kernel path.

Graph replays are interleaved with eager work of the same problem (stencil
applies, Gram products, synchronizations) and every replay is compared with
the eager result, so that a replay that reads stale buffers or parameters
would show."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import synthetic  # noqa: E402
from oracle.spacetime import Problem as OP  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_05638_amd import lrpost
    lrpost.load()
    return lrpost


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("N", [16, 64, 256])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replayed_vcycles_equal_eager(lp, N, precision):
    import torch
    print("case graphs mg N=%d %s" % (N, precision), flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        prob = lp.Problem(synthetic.ProblemDesc(N=N, nt=4, trunc_tol=1e-6, rank_cap=8, precision=precision),
                          stream=stream)
        rng = np.random.default_rng(N)
        coef = np.array([[1.0, 1.0], [1.0 / 200, 1.0], [1e-3, 50.0]])
        B = _dev(rng.standard_normal((3, prob.nx)))
        prob.set_graphs(False)
        ref = prob.mg_solve(B, coef, 3).cpu().numpy()
        prob.set_graphs(True)
        c0, l0 = prob.graph_info()
        outs = []
        for rep in range(4):
            outs.append(prob.mg_solve(B, coef, 3).cpu().numpy())
            # eager work of the same problem between the replays
            prob.stencil_apply(B, np.tile([1.0, 1.0, 0.0], (3, 1)))
            prob.gram(B, B)
            torch.cuda.synchronize()
        c1, l1 = prob.graph_info()
        print("graphs captured %d, graph launches %d" % (c1 - c0, l1 - l0), flush=True)
        assert c1 - c0 >= 1 and l1 - l0 >= 4 * 3
        for o in outs:
            assert np.array_equal(o, ref)
        prob.close()


def test_graph_replayed_hessian_apply_equals_eager(lp):
    """A whole Hessian apply (pole solves, prior solve) with graphs on and off:
    the same bits; and against the oracle's G to its tolerance."""
    import torch
    print("case graphs hessian apply", flush=True)
    d = synthetic.ProblemDesc(N=32, nt=20, trunc_tol=1e-10, rank_cap=20)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        prob = lp.Problem(d, stream=stream)
        ora = OP.from_desc(d)
        rng = np.random.default_rng(8)
        A = rng.standard_normal((prob.nx, 2))
        B = np.cumsum(rng.standard_normal((d.nt, 2)), axis=0)
        prob.set_graphs(False)
        E1, E2 = prob.hess_apply(_dev(A.T), B.T)
        eager = E1.cpu().numpy().T @ E2
        prob.set_graphs(True)
        for rep in range(3):
            G1, G2 = prob.hess_apply(_dev(A.T), B.T)
            got = G1.cpu().numpy().T @ G2
            assert np.array_equal(got, eager)
        assert prob.graph_info()[1] > 0
        ref = ora.G(A @ B.T)
        assert np.linalg.norm(eager - ref) / np.linalg.norm(ref) < 1e-8
        prob.close()


@pytest.mark.parametrize("N,ncols", [(64, 6), (256, 9), (512, 40)])
def test_autotuned_stencil_strips_give_the_same_bits(lp, N, ncols):
    """The strip-height autotuner changes timing only: a shape class launched
    first under the fixed rule, then timed (all three heights, the result
    coming from the 32-row variant), then with the chosen height, gives the
    same bits each time, equal to the assembled operators to rounding."""
    from oracle import fem
    print("case autotune stencil N=%d ncols=%d" % (N, ncols), flush=True)
    prob = lp.Problem(synthetic.ProblemDesc(N=N, nt=4, trunc_tol=1e-6, rank_cap=8))
    rng = np.random.default_rng(N + ncols)
    # an unusual coefficient set so that this class is new to the process
    X = _dev(rng.standard_normal((ncols, prob.nx)))
    coef = np.tile([0.7, 1.3, 0.0], (ncols, 1))
    lp.set_autotune(False)
    r1 = prob.stencil_apply(X, coef).cpu().numpy()
    lp.set_autotune(True)
    r2 = prob.stencil_apply(X, coef).cpu().numpy()
    r3 = prob.stencil_apply(X, coef).cpu().numpy()
    report = lp.autotune_report()
    print(report, flush=True)
    assert "n=%d " % (N - 1) in report
    assert np.array_equal(r1, r2) and np.array_equal(r2, r3)
    K, M = fem.assemble_kronecker(N)
    Xh = X.cpu().numpy()
    ref = 0.7 * (K @ Xh.T) + 1.3 * (M @ Xh.T)
    assert np.abs(r3.T - ref).max() <= 1e-13 * np.abs(ref).max()
