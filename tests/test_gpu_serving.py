"""The serving loop (MI355X only): likelihood + gradient and prediction
requests of uneven size admitted by footprint, run concurrently on several
streams.

Checked through the C ABI:
  - every request's NLL, gradient and predictive variances are the same run
    alone (one worker, one request at a time) and in a mix of overlapping
    requests on four workers: float64 within 1e-9 relative, mixed precision
    within 1e-4 (the method's bars; the kernels and their reductions are the
    same, so the results agree bit for bit);
  - admission never reserves more than the budget, no request holds more
    device memory than its footprint, and with a budget below the trace's
    total some requests wait for memory;
  - a request larger than the whole budget is refused with OOM while the
    others complete;
  - a served request matches the oracle (fixed iterations, float64, 1e-9)."""
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


def small_trace(n_req=14, seed=11):
    tr = configs.serving_trace(n_requests=n_req, rate=200.0, n_lo=1500, n_hi=12000, m_choices=(50, 100, 200),
                               num_samples=8, seed=seed)
    return [(r, r.materialize(n_features=64)) for r in tr]


def submit(F, srv, r, arrays, arrival_ms):
    locs, y, ind, pred = arrays
    kind = F.REQ_NLL_GRAD if r.kind == "nll_grad" else F.REQ_PREDICT_VAR
    return srv.submit(kind, locs, y, r.theta, ind, r.gamma, pred, r.num_samples, arrival_ms=arrival_ms)


def run_alone(F, trace, **opts):
    out = []
    with F.Server(slots=1, hbm_budget=8 << 30, **opts) as srv:
        for r, a in trace:
            say(f"case: alone request {r.index} kind={r.kind} n={r.n} m={r.m}")
            out.append(srv.wait(submit(F, srv, r, a, 0.0)))
    return out


def run_mix(F, trace, slots=4, budget=8 << 30, spacing_ms=3.0, **opts):
    with F.Server(slots=slots, hbm_budget=budget, **opts) as srv:
        t0 = srv.clock_ms() + 20.0
        say(f"case: mix of {len(trace)} requests on {slots} workers, budget {budget}")
        ids = [submit(F, srv, r, a, t0 + spacing_ms * k) for k, (r, a) in enumerate(trace)]
        res = [srv.wait(i) for i in ids]
        return res, srv.stats()


def compare(trace, alone, mix, rtol):
    for (r, _), (ra, va), (rm, vm) in zip(trace, alone, mix):
        assert ra["status"] == 0 and rm["status"] == 0, (r.index, ra["message"], rm["message"])
        if r.kind == "nll_grad":
            assert abs(rm["nll"] - ra["nll"]) <= rtol * abs(ra["nll"]), (r.index, rm["nll"], ra["nll"])
            scale = np.abs(ra["grad"]).max()
            np.testing.assert_allclose(rm["grad"], ra["grad"], rtol=rtol, atol=rtol * scale)
        else:
            np.testing.assert_allclose(vm, va, rtol=rtol, atol=rtol * np.abs(va).max())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_alone_and_in_the_mix_agree(F, prec):
    precision = F.FP64 if prec == "fp64" else F.MIXED_FP32
    tol = 1e-8 if prec == "fp64" else 1e-6
    trace = small_trace()
    alone = run_alone(F, trace, num_probes=8, seed=3, tol=tol, precision=precision, rr_period=10)
    mix, st = run_mix(F, trace, num_probes=8, seed=3, tol=tol, precision=precision, rr_period=10)
    say("stats", st)
    compare(trace, alone, mix, 1e-9 if prec == "fp64" else 1e-4)
    bitwise = all(a[0]["nll"] == m[0]["nll"] and np.array_equal(a[0]["grad"], m[0]["grad"]) and
                  (a[1] is None or np.array_equal(a[1], m[1])) for a, m in zip(alone, mix))
    say("bitwise equal:", bitwise)
    assert bitwise
    assert st["completed"] == len(trace) and st["failed"] == 0
    assert st["peak_active"] >= 2  # requests did overlap on the device
    for (res, _) in mix:
        assert res["peak_bytes"] <= res["footprint"]
        assert res["admit_ms"] >= res["arrival_ms"]


def test_admission_respects_the_budget(F):
    trace = small_trace(n_req=12, seed=12)
    fps = [F.request_footprint(F.REQ_NLL_GRAD if r.kind == "nll_grad" else F.REQ_PREDICT_VAR, a[0], a[1], r.theta,
                               a[2], r.gamma, a[3], r.num_samples, num_probes=8, precision=F.MIXED_FP32)
           for r, a in trace]
    budget = int(max(fps) * 1.6)
    assert budget < sum(fps)
    mix, st = run_mix(F, trace, slots=6, budget=budget, spacing_ms=0.0, num_probes=8, seed=5, tol=1e-6,
                      precision=F.MIXED_FP32)
    say("stats", st, "footprints", fps)
    assert st["peak_reserved"] <= st["hbm_budget"] <= budget
    assert st["failed"] == 0
    for (res, _), fp in zip(mix, fps):
        assert res["status"] == 0, res["message"]
        assert res["footprint"] >= fp and res["peak_bytes"] <= res["footprint"]
    # with room for at most one large request, some had to wait for memory
    waited = sum(res["admit_ms"] - res["arrival_ms"] > 1.0 for res, _ in mix)
    assert waited >= 1


def test_oversized_request_is_refused(F):
    trace = small_trace(n_req=4, seed=13)
    big_locs = G.uniform_locations(60_000, 77)
    big_y = G.rff_response(big_locs, G.EXPONENTIAL, 1.0, 0.1, 0.1, 32, 78)
    big_ind = G.random_subset_inducing(big_locs, 500, 79)
    with F.Server(slots=2, hbm_budget=96 << 20, num_probes=4, tol=1e-6, precision=F.MIXED_FP32) as srv:
        say("case: oversized request beside small ones, budget 96 MiB")
        small = [r for r in trace if F.request_footprint(
            F.REQ_NLL_GRAD if r[0].kind == "nll_grad" else F.REQ_PREDICT_VAR, r[1][0], r[1][1], r[0].theta, r[1][2],
            r[0].gamma, r[1][3], r[0].num_samples, num_probes=4, precision=F.MIXED_FP32) < (96 << 20)]
        ids = [submit(F, srv, r, a, 0.0) for r, a in small]
        bid = srv.submit(F.REQ_NLL_GRAD, big_locs, big_y, (0, 1.0, 0.1, 0.1), big_ind,
                         G.taper_range_for_uniform(60_000, 60))
        rb, _ = srv.wait(bid)
        assert rb["status"] == 2 and "budget" in rb["message"], rb
        for i in ids:
            assert srv.wait(i)[0]["status"] == 0
    with pytest.raises(F.FsaError):
        with F.Server(slots=1, hbm_budget=64 << 20) as srv:
            srv.submit(F.REQ_NLL_GRAD, big_locs[:10], big_y[:10], (0, 1.0, 0.1, 0.1), big_ind[:20], 0.1)


def test_served_requests_match_the_oracle(F):
    trace = small_trace(n_req=6, seed=14)
    r1, (locs, y, ind, _) = next(x for x in trace if x[0].kind == "nll_grad")
    with F.Server(slots=2, hbm_budget=4 << 30, num_probes=5, seed=21, fixed_iter=12, precision=F.FP64) as srv:
        say(f"case: oracle check of likelihood request {r1.index} n={r1.n} m={r1.m}")
        rr, _ = srv.wait(submit(F, srv, r1, (locs, y, ind, None), 0.0))
    assert rr["status"] == 0, rr["message"]
    ref = O.nll_grad(O.FSA(locs, ind, r1.theta, r1.gamma), y, 5, 21, fixed_iter=12)
    assert abs(rr["nll"] - ref["nll"]) <= 1e-9 * abs(ref["nll"])
    np.testing.assert_allclose(rr["grad"], ref["grad"], rtol=1e-9, atol=1e-9 * np.abs(ref["grad"]).max())
    r2, (locs, y, ind, pred) = next(x for x in trace if x[0].kind == "predict_var")
    with F.Server(slots=2, hbm_budget=4 << 30, num_probes=2, seed=22, tol=1e-12, max_iter=3000,
                  precision=F.FP64) as srv:
        say(f"case: oracle check of prediction request {r2.index} n={r2.n} m={r2.m} n_p={r2.n_p}")
        rp, var = srv.wait(submit(F, srv, r2, (locs, y, ind, pred), 0.0))
    assert rp["status"] == 0, rp["message"]
    ref_var, _ = O.predict_var(O.FSA(locs, ind, r2.theta, r2.gamma), pred, r2.num_samples, 22, tol=1e-12,
                               max_iter=3000)
    assert np.abs(var - ref_var).max() / np.abs(ref_var).max() < 1e-9
