"""The boundary's memory and output variants on the MI355X: device memory
from the caller's allocator (torch's caching allocator through the C ABI's
callbacks), and the likelihood with device outputs.

The problem statement (Section 2) fixes the inputs and outputs; the caller's
framework owns device memory.  Results must not depend on where the memory
comes from (same kernels, same order: bit for bit), and every block the
library takes must go back to the caller's allocator."""
import sys

import numpy as np
import pytest

from oracle import fsa_oracle as O
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


def small_case(n=5000, m=120, seed=0):
    locs = G.uniform_locations(n, 1500 + seed)
    ind = G.random_subset_inducing(locs, m, 1600 + seed)
    gamma = G.taper_range_for_uniform(n, 40)
    y = G.rff_response(locs, O.MATERN32, 1.0, 0.05, 0.1, 300, 1700 + seed)
    return locs, y, (O.MATERN32, 1.0, 0.05, 0.1), ind, gamma


def run_all(F, prec, locs, y, theta, ind, gamma, pred):
    with F.FSA(locs, y, theta, ind, gamma, num_probes=6, seed=4, tol=1e-7, precision=prec) as f:
        nll, grad, _ = f.nll_grad()
        th2 = (theta[0], 1.2, 0.06, 0.12)
        nll2, grad2, _ = f.nll_grad(theta=th2)
        var, mean, _ = f.predict_var(pred, 8, with_mean=True)
    return nll, grad, nll2, grad2, var, mean


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_caller_allocator_receives_every_block(F, prec):
    """Build, likelihood + gradient, revaluation at a new theta (the
    derivative rebuilt), prediction and destroy with torch's caching
    allocator registered: every block handed out comes back, torch's
    allocated bytes return to where they were, and every result is
    bitwise that of the library's own pool."""
    import torch
    precision = F.FP64 if prec == "fp64" else F.MIXED_FP32
    locs, y, theta, ind, gamma = small_case()
    pred = G.uniform_locations(300, 1800)
    ref = run_all(F, precision, locs, y, theta, ind, gamma, pred)
    alloc = F.TorchAllocator()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    F.fsa_set_allocator(alloc)
    try:
        got = run_all(F, precision, locs, y, theta, ind, gamma, pred)
        torch.cuda.synchronize()
    finally:
        F.fsa_set_allocator(None)
    say("blocks", alloc.allocs, "returned", alloc.releases, "live", len(alloc.live),
        "torch bytes before", base, "after", torch.cuda.memory_allocated())
    assert alloc.allocs > 20
    assert alloc.releases == alloc.allocs and not alloc.live
    assert torch.cuda.memory_allocated() == base
    for a, b in zip(ref, got):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_nll_grad_dev_writes_device_outputs(F):
    """fsa_nll_grad_dev leaves the NLL and the gradient in device tensors,
    equal to the host-output call's values bit for bit."""
    import torch
    locs, y, theta, ind, gamma = small_case(seed=1)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=6, seed=9, fixed_iter=15) as f:
        nll, grad, _ = f.nll_grad()
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        g = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        st = f.nll_grad_dev(out, g)
        out2 = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        f.nll_grad_dev(out2, None, theta=(theta[0], 1.1, 0.05, 0.1))
        nll3, _, _ = f.nll_grad(theta=(theta[0], 1.1, 0.05, 0.1), with_grad=False)
    say("nll", nll, float(out), "grad", grad, g.cpu().numpy())
    assert float(out.item()) == nll
    assert np.array_equal(g.cpu().numpy(), grad)
    assert float(out2.item()) == nll3
    assert st["iters_max"] == 15
