"""PCG iterations replayed from a captured HIP graph (MI355X only).

With options.graph every iteration after the first is one launch of a graph
captured from the second.  The replays run between the solver's own eager
work (convergence checkpoints that drain the stream, float64 residual
replacements in mixed precision, the derivative build after the solve),
and every result must be bitwise that of the eager launches: likelihood,
gradient, the Lanczos record of every column, predictive variances."""
import sys

import numpy as np
import pytest

from workloads import generators as G

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    from paper_2405_14492_amd import fsa
    fsa.lib()
    return fsa


def run(F, graph, precision, clustered=False, **kw):
    n, m = 6000, 200
    locs = G.clustered_locations(n, 31) if clustered else G.uniform_locations(n, 31)
    ind = G.random_subset_inducing(locs, m, 32)
    th = (G.MATERN32, 1.0, 0.08, 0.05)
    y = G.rff_response(locs, th[0], th[1], th[2], th[3], 128, 33)
    gamma = G.taper_range_by_count(locs, 40, sample=2000) if clustered else G.taper_range_for_uniform(n, 40)
    pred = G.uniform_locations(700, 34)
    import torch
    s = torch.cuda.Stream()  # a graph is captured on the context's own stream (never the null stream)
    with F.FSA(locs, y, th, ind, gamma, num_probes=9, seed=5, precision=precision, graph=graph,
               stream=s.cuda_stream, **kw) as f:
        nll, grad, st = f.nll_grad()
        lz = f.export_lanczos()
        nll2, grad2, _ = f.nll_grad(theta=(th[0], 1.1, 0.07, 0.06))
        var, _, stp = f.predict_var(pred, 6)
    s.synchronize()
    return nll, grad, st, lz, nll2, grad2, var, stp


@pytest.mark.parametrize("prec,clustered", [("fp64", False), ("mixed", False), ("mixed", True), ("bf16a", False)])
def test_graph_replay_is_bitwise_eager(F, prec, clustered):
    precision = {"fp64": F.FP64, "mixed": F.MIXED_FP32, "bf16a": F.MIXED_BF16A}[prec]
    tol = 1e-8 if prec == "fp64" else 1e-6
    say(f"case: graph vs eager {prec} clustered={clustered}")
    eager = run(F, False, precision, clustered, tol=tol, rr_period=5)
    graph = run(F, True, precision, clustered, tol=tol, rr_period=5)
    again = run(F, True, precision, clustered, tol=tol, rr_period=5)
    say("iters", eager[2]["iters_max"], graph[2]["iters_max"], "nll", eager[0], graph[0])
    assert eager[2]["iters_max"] > 3  # the graph was replayed
    for res in (graph, again):
        assert res[0] == eager[0] and np.array_equal(res[1], eager[1])
        assert res[2]["iters_min"] == eager[2]["iters_min"] and res[2]["iters_max"] == eager[2]["iters_max"]
        for k in ("iters", "alpha", "beta", "weight", "slq"):
            a, b = np.asarray(eager[3][k]), np.asarray(res[3][k])
            if k in ("alpha", "beta"):  # entries past a column's count are undefined
                its = np.asarray(eager[3]["iters"])
                mask = np.arange(a.shape[0])[:, None] < its[None, :]
                a, b = a[mask], b[mask]
            assert np.array_equal(a, b), k
        assert res[4] == eager[4] and np.array_equal(res[5], eager[5])
        assert np.array_equal(res[6], eager[6])


def test_graph_option_on_the_null_stream_runs_eager(F):
    """The null stream cannot be captured: graph is ignored there."""
    n, m = 3000, 100
    locs = G.uniform_locations(n, 41)
    ind = G.random_subset_inducing(locs, m, 42)
    th = (G.EXPONENTIAL, 1.0, 0.1, 0.1)
    y = G.rff_response(locs, th[0], th[1], th[2], th[3], 64, 43)
    gamma = G.taper_range_for_uniform(n, 30)
    out = []
    for graph in (False, True):
        with F.FSA(locs, y, th, ind, gamma, num_probes=4, seed=6, graph=graph) as f:
            out.append(f.nll_grad())
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])


def test_graph_replay_fixed_iterations(F):
    say("case: graph vs eager fp64 fixed_iter=14")
    eager = run(F, False, F.FP64, fixed_iter=14)
    graph = run(F, True, F.FP64, fixed_iter=14)
    assert graph[0] == eager[0] and np.array_equal(graph[1], eager[1]) and np.array_equal(graph[6], eager[6])
    assert graph[2]["iters_max"] == 14
