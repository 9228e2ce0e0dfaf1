"""GPU parity of the Vecchia-Laplace approximation (Section 5.1) for
Bernoulli responses against the oracle (MI355X only).

Both sides take the same Newton steps from b = 0, each solve by the
FITC-preconditioned CG, and the same SLQ probes at the mode.  With a fixed
number of Newton steps and CG iterations the mode and the NLL must agree to
1e-9 relative (float64 on both sides, differing by summation order and the
factorization of the conditioning systems); run to convergence, to the
method's tolerance.  The mode must also satisfy its stationarity equation
Sigma_V^{-1} b = y - pi(b) on the device's own operator."""
import numpy as np
import pytest

from oracle import fsa_oracle as F
from oracle import vecchia_oracle as VO
from workloads import generators as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _case(n, mv, m, seed, rho=0.1, kind=F.MATERN32, s1=1.5, clustered=False):
    locs = G.clustered_locations(n, seed) if clustered else G.uniform_locations(n, seed)
    ind = G.random_subset_inducing(locs, m, seed + 1)
    y = G.bernoulli_responses(locs, kind, s1, rho, 200, seed + 2)
    return locs, ind, y, (kind, s1, rho)


def _both(locs, ind, y, th, mv, t, seed, **kw):
    from paper_2405_14492_amd import fsa
    print(f"case: laplace n={locs.shape[0]} mv={mv} m={ind.shape[0]} t={t} {kw}", flush=True)
    with fsa.Vecchia(_dev(locs), _dev(ind), th[0], th[1], th[2], mv, _dev(np.full(locs.shape[0], 0.25))) as v:
        mode, nll, st = v.laplace(_dev(y), t, seed, **kw)
        # stationarity on the device's operator: Sigma_V^{-1} b - (y - pi)
        qb = v.apply(fsa.V_PRECISION, mode).cpu().numpy()
    mode = mode.cpu().numpy()
    M = VO.Vecchia(locs, ind, th, mv, np.full(locs.shape[0], 0.25))
    ref = VO.laplace(M, y, t, seed, **kw)
    return mode, nll, st, qb, ref


@pytest.mark.parametrize("n,mv,m,clustered", [(1500, 10, 40, False), (1200, 20, 30, True), (300, 4, 12, False)])
def test_fixed_steps_match_oracle(n, mv, m, clustered):
    locs, ind, y, th = _case(n, mv, m, seed=11 + n, clustered=clustered)
    mode, nll, st, _, ref = _both(locs, ind, y, th, mv, 6, 5, fixed_iter=25, fixed_newton=4)
    assert st["newton_steps"] == 4 == ref["newton_steps"]
    assert np.linalg.norm(mode - ref["mode"]) <= 1e-9 * np.linalg.norm(ref["mode"])
    assert abs(st["loglik"] - ref["loglik"]) <= 1e-9 * abs(ref["loglik"])
    assert abs(st["quad"] - ref["quad"]) <= 1e-9 * abs(ref["quad"])
    assert abs(st["sum_log_d"] - ref["sum_log_d"]) <= 1e-9 * abs(ref["sum_log_d"]) + 1e-9
    assert abs(st["logdet"] - ref["logdet"]) <= 1e-9 * abs(ref["logdet"])
    assert abs(nll - ref["nll"]) <= 1e-9 * abs(ref["nll"])


def test_converged_mode_matches_oracle_and_is_stationary():
    locs, ind, y, th = _case(2000, 16, 50, seed=23, rho=0.05, kind=F.EXPONENTIAL, s1=2.0)
    mode, nll, st, qb, ref = _both(locs, ind, y, th, 16, 8, 7, tol=1e-11, max_iter=600, newton_tol=1e-10)
    assert st["converged"] == 1 and ref["converged"]
    assert st["newton_steps"] == ref["newton_steps"]
    assert np.linalg.norm(mode - ref["mode"]) <= 1e-8 * np.linalg.norm(ref["mode"])
    assert abs(nll - ref["nll"]) <= 1e-8 * abs(ref["nll"])
    g = y - 1.0 / (1.0 + np.exp(-mode))
    assert np.linalg.norm(qb - g) <= 1e-7 * np.linalg.norm(g)


def test_rejects_responses_that_are_not_binary():
    from paper_2405_14492_amd import fsa
    locs, ind, y, th = _case(200, 4, 10, seed=3)
    y = y.copy()
    y[7] = 0.5
    with fsa.Vecchia(_dev(locs), _dev(ind), th[0], th[1], th[2], 4, _dev(np.full(200, 0.25))) as v:
        with pytest.raises(fsa.FsaError, match="not 0 or 1"):
            v.laplace(_dev(y), 4, 1)
        with pytest.raises(fsa.FsaError):
            v.laplace(_dev(np.zeros(200)), 0, 1)
