"""Differentiated likelihood on the GPU: the autograd Function, finite
differences with fixed probes, and L-BFGS on the clustered ill-conditioned
workload (n = 200,000, half in 10 blobs of sd 0.02, exponential, rho = 0.2,
sigma1^2 = 2, sigma^2 = 0.01, m = 300, ~50 nonzeros per row, t = 50)."""
import sys

import numpy as np
import pytest

from oracle import fsa_oracle as O
from workloads import configs
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


def small():
    locs = G.clustered_locations(3000, 41)
    ind = G.random_subset_inducing(locs, 60, 42)
    gamma = G.taper_range_by_count(locs, 30, sample=3000)
    y = G.rff_response(locs, O.EXPONENTIAL, 2.0, 0.2, 0.05, 500, 43)
    return locs, y, (O.EXPONENTIAL, 2.0, 0.2, 0.05), ind, gamma


def test_autograd_equals_direct_gradient(F):
    import torch
    from paper_2405_14492_amd.autograd import fsa_nll
    locs, y, theta, ind, gamma = small()
    with F.FSA(locs, y, theta, ind, gamma, num_probes=8, seed=3, tol=1e-10, max_iter=2000) as f:
        nll, grad, _ = f.nll_grad()
        th = torch.tensor(theta[1:], dtype=torch.float64, requires_grad=True)
        val = fsa_nll(th, f, theta[0])
        val.backward()
    assert float(val.detach()) == nll
    np.testing.assert_array_equal(th.grad.numpy(), grad)


@pytest.mark.parametrize("which", [0, 1, 2])
def test_quadratic_term_matches_central_difference(F, which):
    """d/dtheta (y^T Sigma~^{-1} y) = -u^T dSigma~ u: deterministic, so the
    central difference (h = 1e-5 relative) must agree closely."""
    locs, y, theta, ind, gamma = small()
    with F.FSA(locs, y, theta, ind, gamma, num_probes=2, seed=3, tol=1e-12, max_iter=3000) as f:
        _, _, st = f.nll_grad()
        qd = st["grad_quad"][which]
        h = 1e-5 * theta[which + 1]
        tp = list(theta); tp[which + 1] += h
        tm = list(theta); tm[which + 1] -= h
        _, _, sp = f.nll_grad(theta=tuple(tp), with_grad=False)
        _, _, sm = f.nll_grad(theta=tuple(tm), with_grad=False)
    fd = (sp["quad"] - sm["quad"]) / (2 * h)
    say("quad fd", fd, "analytic", -qd)
    assert abs(fd + qd) <= 1e-5 * abs(qd) + 1e-8


def test_gradient_matches_dense_exact_within_monte_carlo(F):
    """Stochastic gradient with many probes vs the exact dense FSA gradient."""
    locs, y, theta, ind, gamma = small()
    locs, y = locs[:800], y[:800]
    ind = ind[:30]
    from tests import dense_fsa as DF
    S = DF.dense_fsa(locs, ind, theta, gamma)
    Si = np.linalg.inv(S)
    u = Si @ y
    exact = []
    for k in range(3):
        dS = DF.fd_operator(locs, ind, theta, gamma, k)
        exact.append(0.5 * np.trace(Si @ dS) - 0.5 * u @ dS @ u)
    exact = np.array(exact)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=1000, seed=9, tol=1e-10, max_iter=3000) as f:
        _, grad, st = f.nll_grad()
    scale = np.abs(np.array(st["grad_trace"]))
    say("grad", grad, "exact", exact, "trace scale", scale)
    assert np.all(np.abs(grad - exact) <= 0.05 * 0.5 * scale + 1e-6 * np.abs(exact))


@pytest.mark.slow
def test_clustered_workload_fd_and_lbfgs(F):
    """Full-size clustered workload: quadratic-term central differences and
    20 L-BFGS steps from a perturbed start (NLL must decrease)."""
    from paper_2405_14492_amd.autograd import fit_lbfgs
    w = configs.clustered_grad()
    say("clustered workload", w.name, "gamma", w.gamma)
    th0 = (w.sigma1_sq * 1.5, w.rho * 0.6, w.sigma_sq * 2.0)
    with F.FSA(w.locs, w.y, w.theta, w.inducing, w.gamma, num_probes=w.num_probes, seed=w.seed, tol=1e-8,
               max_iter=3000) as f:
        nll0, grad0, st0 = f.nll_grad()
        say("nll", nll0, "grad", grad0, "iters", st0["iters_max"], "ms", st0["ms_total"])
        h = 1e-5 * w.rho
        tp = list(w.theta); tp[2] += h
        tm = list(w.theta); tm[2] -= h
        _, _, sp = f.nll_grad(theta=tuple(tp), with_grad=False)
        _, _, sm = f.nll_grad(theta=tuple(tm), with_grad=False)
        fd = (sp["quad"] - sm["quad"]) / (2 * h)
        say("rho quad fd", fd, "analytic", -st0["grad_quad"][1])
        assert abs(fd + st0["grad_quad"][1]) <= 1e-3 * abs(st0["grad_quad"][1])
        theta, trace = fit_lbfgs(f, th0, w.kind, steps=20)
    for row in trace:
        say("lbfgs eval", row)
    finite = [r for r in trace if np.isfinite(r[0])]
    assert finite[-1][0] < trace[0][0]
    assert min(r[0] for r in finite) < trace[0][0]
