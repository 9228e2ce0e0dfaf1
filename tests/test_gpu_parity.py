"""GPU path vs the CPU oracle on identical seeded inputs (MI355X only).

Bars: the taper pattern is bit-exact; float64 operators and values agree to
1e-11 relative; float64 NLL / gradient to 1e-9 relative (identical probes,
fixed iteration count, or both converged to a tight tolerance)."""
import sys

import numpy as np
import pytest

from oracle import fsa_oracle as O
from tests import dense_fsa as DF
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


def case(n=700, m=40, kind=O.EXPONENTIAL, rho=0.1, s1=1.0, s2=0.05, n_gamma=25, seed=0, clustered=False):
    locs = G.clustered_locations(n, 100 + seed) if clustered else G.uniform_locations(n, 100 + seed)
    ind = G.random_subset_inducing(locs, m, 200 + seed)
    gamma = G.taper_range_by_count(locs, n_gamma, sample=min(n, 5000)) if clustered else \
        G.taper_range_for_uniform(n, n_gamma)
    y = G.rff_response(locs, kind, s1, rho, s2, 300, 300 + seed)
    return locs, y, (kind, s1, rho, s2), ind, gamma


CASES = {
    "exp_n700_m40": dict(),
    "m32_n1500_m100": dict(n=1500, m=100, kind=O.MATERN32, rho=0.05, s2=0.1, n_gamma=40, seed=1),
    "exp_clustered_n2000_m70": dict(n=2000, m=70, rho=0.2, s1=2.0, s2=0.01, n_gamma=30, seed=2, clustered=True),
    "ragged_n333_m7": dict(n=333, m=7, kind=O.MATERN32, rho=0.15, n_gamma=12, seed=3),
}


@pytest.mark.parametrize("name", list(CASES))
def test_pattern_bit_exact(F, name):
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    with F.FSA(locs, y, theta, ind, gamma, num_probes=2) as f:
        rp, col, vals = f.export_csr(with_values=True)
    orp, ocol = O.taper_pattern(locs, locs, gamma)
    assert np.array_equal(rp, orp)
    assert np.array_equal(col, ocol)


def test_pattern_ties_bit_exact(F):
    g = np.arange(40) / 64.0
    locs = np.array([(a, b) for a in g for b in g])
    gamma = 2.0 / 64.0
    y = np.ones(locs.shape[0])
    ind = locs[::97].copy()
    with F.FSA(locs, y, (O.EXPONENTIAL, 1.0, 0.1, 0.1), ind, gamma, num_probes=2) as f:
        rp, col, _ = f.export_csr()
    orp, ocol = O.taper_pattern(locs, locs, gamma)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)


@pytest.mark.parametrize("name", list(CASES))
def test_values_and_fitc_match_oracle(F, name):
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    mdl = O.FSA(locs, ind, theta, gamma)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=2) as f:
        _, _, vals = f.export_csr(with_values=True)
        D, logdet_P = f.export_diag()
    scale = np.abs(mdl.vals).max()
    np.testing.assert_allclose(vals, mdl.vals, rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(D, mdl.D, rtol=1e-11)
    assert abs(logdet_P - mdl.logdet_P) <= 1e-11 * abs(mdl.logdet_P) + 1e-9


@pytest.mark.parametrize("name", list(CASES))
def test_operators_match_oracle(F, name):
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    mdl = O.FSA(locs, ind, theta, gamma)
    X = np.random.default_rng(5).standard_normal((locs.shape[0], 5))
    with F.FSA(locs, y, theta, ind, gamma, num_probes=3, seed=11) as f:
        got = {
            "sigma": f.apply(F.OP_SIGMA_DAGGER, X),
            "sparse": f.apply(F.OP_SIGMA_S, X),
            "pinv": f.apply(F.OP_P_INV, X),
            "dsigma1": f.apply(F.OP_D_SIGMA1, X),
            "drho": f.apply(F.OP_D_RHO, X),
            "probes": f.apply(F.OP_PROBES, None, ncols=3),
        }
    ref = {
        "sigma": mdl.matvec(X),
        "sparse": mdl.sparse_matvec(X),
        "pinv": mdl.precond_solve(X),
        "dsigma1": mdl.dmatvec(0, X),
        "drho": mdl.dmatvec(1, X),
        "probes": O.probes(mdl, 3, 11),
    }
    for k in ref:
        err = np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max()
        say(k, err)
        assert err < 1e-10, (k, err)


@pytest.mark.parametrize("name", list(CASES))
def test_nll_grad_fixed_iterations_match_oracle(F, name):
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    mdl = O.FSA(locs, ind, theta, gamma)
    t, k = 6, 15
    ref = O.nll_grad(mdl, y, t, 77, fixed_iter=k)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=t, seed=77, fixed_iter=k) as f:
        nll, grad, st = f.nll_grad()
    say("nll", nll, ref["nll"], "grad", grad, ref["grad"])
    assert abs(nll - ref["nll"]) <= 1e-9 * abs(ref["nll"])
    gscale = np.maximum(np.abs(ref["grad"]), 0.5 * np.abs(ref["trace_terms"]).mean(1))
    assert np.all(np.abs(grad - ref["grad"]) <= 1e-9 * gscale + 1e-12), (grad, ref["grad"])
    assert st["iters_min"] == k and st["iters_max"] == k


def lanczos_tridiagonal(alpha, beta, k):
    """T of Algorithm 2 from a column's CG coefficients (same entries as the
    oracle's pcg_lanczos records)."""
    d = np.array([1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0) for j in range(k)])
    e = np.array([np.sqrt(beta[j]) / alpha[j] for j in range(k - 1)])
    return d, e


@pytest.mark.parametrize("name,kw", [("m32_n1500_m100", dict(tol=1e-11, max_iter=2000)),
                                     ("exp_n700_m40", dict(tol=1e-11, max_iter=2000)),
                                     ("exp_clustered_n2000_m70", dict(tol=1e-6, max_iter=3000)),
                                     ("ragged_n333_m7", dict(fixed_iter=40))])
def test_quadrature_matches_oracle_on_device_coefficients(F, name, kw):
    """The device's e_1^T log(T) e_1 (implicit QL) against the oracle's
    eigendecomposition of the same T, built from the device's own CG
    coefficients, 1e-12 relative per probe; the converged runs hold
    near-multiple Ritz values (gaps below 1e-14)."""
    say("case", name, kw)
    locs, y, theta, ind, gamma = case(**CASES[name])
    with F.FSA(locs, y, theta, ind, gamma, num_probes=8, seed=5, **kw) as f:
        f.nll_grad(with_grad=False)
        rec = f.export_lanczos()
    worst = 0.0
    for c in range(1, 9):
        k = int(rec["iters"][c])
        d, e = lanczos_tridiagonal(rec["alpha"][:, c], rec["beta"][:, c], k)
        ref = rec["weight"][c] * O.e1_log_e1(d, e)
        err = abs(rec["slq"][c] - ref) / abs(ref)
        worst = max(worst, err)
        if err > 1e-12:
            say("column", c, "k", k, "device", rec["slq"][c], "oracle", ref)
    say("worst", worst)
    assert worst < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3])
def test_quadrature_of_short_krylov_spaces_matches_oracle(F, k):
    """1-3 iterations: T of order 1 (a single node of weight 1), 2 and 3."""
    locs, y, theta, ind, gamma = case(**CASES["ragged_n333_m7"])
    ref = O.nll_grad(O.FSA(locs, ind, theta, gamma), y, 5, 31, fixed_iter=k, with_grad=False)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=5, seed=31, fixed_iter=k) as f:
        nll, _, st = f.nll_grad(with_grad=False)
    say("k", k, "nll", nll, ref["nll"])
    assert abs(nll - ref["nll"]) <= 1e-9 * abs(ref["nll"])


@pytest.mark.parametrize("name", ["exp_n700_m40", "m32_n1500_m100"])
def test_nll_converged_matches_oracle(F, name):
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    mdl = O.FSA(locs, ind, theta, gamma)
    ref = O.nll_grad(mdl, y, 8, 5, tol=1e-11, max_iter=2000)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=8, seed=5, tol=1e-11, max_iter=2000) as f:
        nll, grad, st = f.nll_grad()
    say("iters", st["iters_min"], st["iters_max"], ref["iters"].min(), ref["iters"].max())
    assert abs(nll - ref["nll"]) <= 1e-9 * abs(ref["nll"])
    assert abs(st["iters_max"] - ref["iters"].max()) <= 1


def test_revalue_same_pattern(F):
    locs, y, theta, ind, gamma = case(**CASES["exp_n700_m40"])
    th2 = (theta[0], 1.3, 0.07, 0.2)
    ref = O.nll_grad(O.FSA(locs, ind, th2, gamma), y, 4, 3, fixed_iter=10)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=4, seed=3, fixed_iter=10) as f:
        f.nll_grad()
        nll, grad, _ = f.nll_grad(theta=th2)
    assert abs(nll - ref["nll"]) <= 1e-9 * abs(ref["nll"])
    np.testing.assert_allclose(grad, ref["grad"], rtol=1e-8)


@pytest.mark.parametrize("name", ["exp_n700_m40", "m32_n1500_m100", "exp_clustered_n2000_m70"])
def test_mixed_precision_matches_oracle(F, name):
    """float32 blocks + float64 dots and residual replacement, converged to
    1e-6: NLL within 1e-4 relative of the float64 oracle converged to 1e-10
    with the same probes; each gradient component within 1e-4 of its scale."""
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    mdl = O.FSA(locs, ind, theta, gamma)
    ref = O.nll_grad(mdl, y, 8, 5, tol=1e-10, max_iter=3000)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=8, seed=5, tol=1e-6, max_iter=3000,
               precision=F.MIXED_FP32, rr_period=10) as f:
        nll, grad, st = f.nll_grad()
    say("mixed nll", nll, ref["nll"], "grad", grad, ref["grad"], "iters", st["iters_max"], ref["iters"].max())
    assert abs(nll - ref["nll"]) <= 1e-4 * abs(ref["nll"])
    gscale = np.maximum(np.abs(ref["grad"]), 0.5 * np.abs(ref["trace_terms"]).mean(1))
    assert np.all(np.abs(grad - ref["grad"]) <= 1e-4 * gscale), (grad, ref["grad"])


@pytest.mark.parametrize("name", ["exp_n700_m40", "m32_n1500_m100", "exp_clustered_n2000_m70", "ragged_n333_m7"])
def test_predictive_variances_match_oracle(F, name):
    """Algorithm 1 (float64, tight tolerance, identical Rademacher draws) and
    the predictive mean; includes prediction points outside the training
    region and far from every training point."""
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    pred = np.vstack([G.uniform_locations(257, 900), [[1.3, 0.5], [-0.2, -0.2], [0.5, 0.5], [5.0, 5.0]]])
    mdl = O.FSA(locs, ind, theta, gamma)
    u = O.pcg_lanczos(mdl.matvec, mdl.precond_solve, y[:, None], 1e-13, 3000).U[:, 0]
    ref_var, det = O.predict_var(mdl, pred, 16, 21, tol=1e-12, max_iter=3000, u=u)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=2, seed=21, tol=1e-12, max_iter=3000) as f:
        f.nll_grad(with_grad=False)
        var, mean, st = f.predict_var(pred, 16, with_mean=True)
    err = np.abs(var - ref_var).max() / np.abs(ref_var).max()
    merr = np.abs(mean - det["mean"]).max() / np.abs(det["mean"]).max()
    say("var err", err, "mean err", merr, "iters", st["iters_max"])
    assert err < 1e-9
    assert merr < 1e-9


def test_predictive_variances_mixed_precision(F):
    locs, y, theta, ind, gamma = case(**CASES["m32_n1500_m100"])
    pred = G.uniform_locations(300, 901)
    mdl = O.FSA(locs, ind, theta, gamma)
    ref_var, _ = O.predict_var(mdl, pred, 16, 22, tol=1e-12, max_iter=3000)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=2, seed=22, tol=1e-7, max_iter=3000,
               precision=F.MIXED_FP32) as f:
        var, _, _ = f.predict_var(pred, 16)
    err = np.abs(var - ref_var) / np.abs(ref_var)
    say("mixed var rel err max", err.max())
    assert err.max() < 1e-4


@pytest.mark.parametrize("name", ["exp_n700_m40", "m32_n1500_m100", "ragged_n333_m7"])
def test_bf16a_matches_oracle_of_rounded_model(F, name):
    """MIXED_BF16A is MIXED_FP32 on the model whose whitened factor is
    rounded to bfloat16: against the float64 oracle of that model (converged
    to 1e-10, same probes) the bar is the mixed-precision one, NLL within
    1e-4 relative and each gradient component within 1e-4 of its scale.  The
    deviation from the unrounded model is printed beside it.  The sigma1^2
    derivative is that of the rounded model scaled with sigma1^2."""
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    mdl = DF.RoundedFSA(locs, ind, theta, gamma, smn_T=DF.bf16_cross_covariance(locs, ind, theta))
    ref = O.nll_grad(mdl, y, 8, 5, tol=1e-10, max_iter=3000)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=8, seed=5, tol=1e-6, max_iter=3000,
               precision=F.MIXED_BF16A, rr_period=10) as f:
        nll, grad, st = f.nll_grad()
    exact = O.nll_grad(O.FSA(locs, ind, theta, gamma), y, 8, 5, tol=1e-10, max_iter=3000)
    gscale = np.maximum(np.abs(ref["grad"]), 0.5 * np.abs(ref["trace_terms"]).mean(1))
    say("bf16a nll", nll, "rounded-model oracle", ref["nll"], "rel", abs(nll - ref["nll"]) / abs(ref["nll"]),
        "grad err / scale", np.abs(grad - ref["grad"]) / gscale, "iters", st["iters_max"])
    say("rounding of A moves the nll by", abs(ref["nll"] - exact["nll"]) / abs(exact["nll"]),
        "and the gradient by", np.abs(ref["grad"] - exact["grad"]) / gscale, "of its scale")
    assert abs(nll - ref["nll"]) <= 1e-4 * abs(ref["nll"])
    assert np.all(np.abs(grad - ref["grad"]) <= 1e-4 * gscale), (grad, ref["grad"])
    assert 0.0 < st["rel_res_max"] < 1e-6


def test_bf16a_wide_block_matches_oracle_of_rounded_model(F):
    """60 probes: 61 columns exceed the 52 the bfloat16-MFMA expansion holds
    in LDS, so that pass widens A to float32 while the residual pass stays
    on the bfloat16 MFMA; both against the rounded model's oracle with
    fixed iterations."""
    locs, y, theta, ind, gamma = case(**CASES["ragged_n333_m7"])
    mdl = DF.RoundedFSA(locs, ind, theta, gamma, smn_T=DF.bf16_cross_covariance(locs, ind, theta))
    ref = O.nll_grad(mdl, y, 60, 9, fixed_iter=12)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=60, seed=9, fixed_iter=12, precision=F.MIXED_BF16A,
               rr_period=5) as f:
        nll, grad, st = f.nll_grad()
    gscale = np.maximum(np.abs(ref["grad"]), 0.5 * np.abs(ref["trace_terms"]).mean(1))
    say("bf16a t=60 nll rel", abs(nll - ref["nll"]) / abs(ref["nll"]), "grad/scale", np.abs(grad - ref["grad"]) / gscale)
    assert abs(nll - ref["nll"]) <= 1e-4 * abs(ref["nll"])
    assert np.all(np.abs(grad - ref["grad"]) <= 1e-4 * gscale)


def test_bf16a_predictive_variances_match_oracle_of_rounded_model(F):
    locs, y, theta, ind, gamma = case(**CASES["m32_n1500_m100"])
    pred = G.uniform_locations(300, 901)
    mdl = O.FSA(locs, ind, theta, gamma, smn_T=DF.bf16_cross_covariance(locs, ind, theta))
    ref_var, _ = O.predict_var(mdl, pred, 16, 22, tol=1e-12, max_iter=3000,
                               smp_T=DF.bf16_cross_covariance(locs, ind, theta, pred=pred))
    with F.FSA(locs, y, theta, ind, gamma, num_probes=2, seed=22, tol=1e-7, max_iter=3000,
               precision=F.MIXED_BF16A) as f:
        var, _, _ = f.predict_var(pred, 16)
    err = np.abs(var - ref_var) / np.abs(ref_var)
    say("bf16a var rel err max", err.max())
    assert err.max() < 1e-4


def test_bf16a_rejects_rounded_model_with_negative_residual_diagonal(F):
    """Clustered points with inducing points among them and a small nugget
    (sigma^2 = 0.01, sigma1^2 = 2): at an inducing point the unrounded
    residual diagonal is the nugget alone, and the bfloat16 rounding of A
    moves ||A_i||^2 by more than that, so the rounded model is not positive
    definite.  The build must refuse it rather than run PCG on it."""
    locs, y, theta, ind, gamma = case(**CASES["exp_clustered_n2000_m70"])
    mdl_T = DF.bf16_cross_covariance(locs, ind, theta)
    kind, s1, rho, s2 = theta
    import scipy.linalg as sla
    from scipy.spatial.distance import cdist
    Sm = O.covariance(cdist(ind, ind), s1, rho, kind)
    Ar = sla.solve_triangular(np.linalg.cholesky(Sm), mdl_T.T, lower=True)  # = A~
    dmin = (s1 + s2 - (Ar * Ar).sum(0)).min()
    say("rounded residual diagonal min", dmin)
    assert dmin < -1e-4
    with pytest.raises(F.FsaError, match="NOT_SPD"):
        with F.FSA(locs, y, theta, ind, gamma, num_probes=4, seed=5, precision=F.MIXED_BF16A) as f:
            f.nll_grad()
    # float32 mixed precision keeps the unrounded model and runs
    with F.FSA(locs, y, theta, ind, gamma, num_probes=4, seed=5, tol=1e-6, precision=F.MIXED_FP32) as f:
        f.nll_grad()


def test_contexts_return_device_memory(F):
    """Every context's device buffers and every temporary go back to the
    library's pool: after build / solve / gradient / destroy cycles and a
    pool trim, the device has the free memory it had before."""
    import torch
    from paper_2405_14492_amd import fsa as Fm
    locs, y, theta, ind, gamma = case(n=30000, m=200, kind=O.MATERN32, rho=0.05, s2=0.1, n_gamma=30, seed=4)
    Fm.lib().fsa_pool_trim()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for prec in (F.FP64, F.MIXED_FP32, F.MIXED_BF16A, F.FP64):
        with F.FSA(locs, y, theta, ind, gamma, num_probes=4, seed=1, tol=1e-6, precision=prec) as f:
            f.nll_grad()
            f.predict_var(locs[:500], 4)
    Fm.lib().fsa_pool_trim()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    say("device free before", free0 >> 20, "MiB, after", free1 >> 20, "MiB")
    assert free0 - free1 < (64 << 20)


@pytest.mark.gpu
def test_kernel_timer_class_mask(F):
    """options.profile times exactly the kernel classes in its bit mask; the
    result does not depend on which classes are timed."""
    locs, y, theta, ind, gamma = case(n=20000, m=150, kind=O.MATERN32, rho=0.05, s2=0.1, n_gamma=30, seed=6)
    out = {}
    for prof in (0, 1, 1 << 2, True):
        with F.FSA(locs, y, theta, ind, gamma, num_probes=4, seed=1, tol=1e-6, precision=F.MIXED_FP32,
                   profile=prof) as f:
            out[prof] = f.nll_grad()
    mask = {0: 0, 1: 1, 4: 4, True: 0x1f}
    for prof, (nll, grad, st) in out.items():
        timed = [k for k in range(5) if st["kernel_launches"][k] > 0]
        assert timed == [k for k in range(5) if (mask[prof] >> k) & 1], (prof, st["kernel_launches"])
        assert all(st["kernel_ms"][k] > 0 for k in timed)
        assert abs(nll - out[0][0]) <= 1e-12 * abs(out[0][0])
        np.testing.assert_allclose(grad, out[0][1], rtol=1e-12, atol=0)


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["dense_cells_n3000_m60", "exp_clustered_n2000_m70"])
def test_float32_operator_tracks_float64(F, name):
    """The float32 iteration's operator (the sparse product on pre-scattered
    MFMA-order tiles, here with cells of more than one 32-row group) against
    the float64 one: with no residual replacement, the first Lanczos
    coefficients of the float32 solve match the float64 solve's to float32
    accuracy.  A misplaced tile entry moves them by orders of magnitude more."""
    cases = dict(CASES, dense_cells_n3000_m60=dict(n=3000, m=60, kind=O.MATERN32, rho=0.1, s2=0.1, n_gamma=150,
                                                   seed=7))
    say("case", name)
    locs, y, theta, ind, gamma = case(**cases[name])
    h = gamma * (1.0 + 2.0 ** -20)
    cell = np.floor((locs - locs.min(0)) / h).astype(np.int64)
    counts = np.unique(cell[:, 0] * 100003 + cell[:, 1], return_counts=True)[1]
    say("largest cell", counts.max(), "points")
    assert counts.max() > 32  # some cells hold two or more row groups
    rec = {}
    for prec in (F.FP64, F.MIXED_FP32):
        with F.FSA(locs, y, theta, ind, gamma, num_probes=4, seed=3, fixed_iter=6, precision=prec,
                   rr_period=0) as f:
            f.nll_grad(with_grad=False)
            rec[prec] = f.export_lanczos()
    for key in ("alpha", "beta"):
        a64, a32 = rec[F.FP64][key][:6], rec[F.MIXED_FP32][key][:6]
        err = np.abs(a32 - a64).max() / np.abs(a64).max()
        say(key, "max rel diff", err)
        assert err < 1e-4, key


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["exp_n700_m40", "m32_n1500_m100", "ragged_n333_m7"])
@pytest.mark.parametrize("mode", ["one", "opt", "opt_printed"])
def test_gradient_control_variate_matches_oracle(F, name, mode):
    """The FITC preconditioner as control variate (App. E): the float64
    gradient with c = 1, the centred c_opt or the printed c_opt against the
    oracle with the same probes and fixed iterations, together with the
    coefficients and the exact traces Tr(P^{-1} dP/dtheta)."""
    say("case", name, mode)
    cvm = {"one": F.CV_ONE, "opt": F.CV_OPT, "opt_printed": F.CV_OPT_PRINTED}[mode]
    locs, y, theta, ind, gamma = case(**CASES[name])
    mdl = O.FSA(locs, ind, theta, gamma)
    t, k = 8, 20
    ref = O.nll_grad(mdl, y, t, 41, fixed_iter=k, control_variate=mode)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=t, seed=41, fixed_iter=k, control_variate=cvm) as f:
        nll, grad, st = f.nll_grad()
    gscale = np.maximum(np.abs(ref["grad"]), 0.5 * np.abs(ref["trace_terms"]).mean(1))
    say("grad", grad, ref["grad"], "c", st["cv_c"], ref["cv_c"], "trace_P", st["trace_P"], ref["trace_P"])
    np.testing.assert_allclose(st["trace_P"], ref["trace_P"], rtol=1e-9)
    np.testing.assert_allclose(st["cv_c"], ref["cv_c"], rtol=1e-7, atol=1e-12)
    assert np.all(np.abs(grad - ref["grad"]) <= 1e-9 * gscale + 1e-12), (grad, ref["grad"])


@pytest.mark.gpu
def test_gradient_control_variate_mixed_and_bf16a(F):
    """The control variate on the float32 solves: MIXED_FP32 against the
    float64 oracle, MIXED_BF16A against the oracle of its rounded model
    (whose sigma1^2 derivative, of Sigma~ and of P, scales with sigma1^2), at
    the mixed-precision bar.  The exact Tr(P^{-1} dP/dtheta) is float64 work
    on the derivative factor F, which MIXED_FP32 forms as a float32 product
    (float32 accuracy, 1e-6) and MIXED_BF16A in float64 (1e-9)."""
    locs, y, theta, ind, gamma = case(**CASES["m32_n1500_m100"])
    for prec, mdl in ((F.MIXED_FP32, O.FSA(locs, ind, theta, gamma)),
                      (F.MIXED_BF16A, DF.RoundedFSA(locs, ind, theta, gamma,
                                                    smn_T=DF.bf16_cross_covariance(locs, ind, theta)))):
        ref = O.nll_grad(mdl, y, 8, 5, tol=1e-10, max_iter=3000, control_variate="opt")
        with F.FSA(locs, y, theta, ind, gamma, num_probes=8, seed=5, tol=1e-6, max_iter=3000, precision=prec,
                   rr_period=10, control_variate=F.CV_OPT) as f:
            nll, grad, st = f.nll_grad()
        gscale = np.maximum(np.abs(ref["grad"]), 0.5 * np.abs(ref["trace_terms"]).mean(1))
        say(prec, "grad err / scale", np.abs(grad - ref["grad"]) / gscale, "trace_P", st["trace_P"], ref["trace_P"])
        np.testing.assert_allclose(st["trace_P"], ref["trace_P"], rtol=1e-6 if prec == F.MIXED_FP32 else 1e-9)
        assert np.all(np.abs(grad - ref["grad"]) <= 1e-4 * gscale), (prec, grad, ref["grad"])


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["m32_n1500_m100", "exp_clustered_n2000_m70", "ragged_n333_m7"])
@pytest.mark.parametrize("mode", ["one", "opt", "opt_printed"])
def test_predictive_variance_control_variate_matches_oracle(F, name, mode):
    """Algorithm 1 with D_s as control variate for its stochastic diagonal
    (App. E), float64 at a tight tolerance, identical Rademacher draws."""
    say("case", name, mode)
    cvm = {"one": F.CV_ONE, "opt": F.CV_OPT, "opt_printed": F.CV_OPT_PRINTED}[mode]
    locs, y, theta, ind, gamma = case(**CASES[name])
    pred = np.vstack([G.uniform_locations(257, 902), [[1.3, 0.5], [5.0, 5.0]]])
    mdl = O.FSA(locs, ind, theta, gamma)
    ref, det = O.predict_var(mdl, pred, 16, 23, tol=1e-12, max_iter=3000, control_variate=mode)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=2, seed=23, tol=1e-12, max_iter=3000,
               control_variate=cvm) as f:
        var, _, st = f.predict_var(pred, 16)
    err = np.abs(var - ref).max() / np.abs(ref).max()
    say("var err", err, "c range", det["cv_c"].min(), det["cv_c"].max())
    assert err < 1e-9


@pytest.mark.gpu
def test_scores_match_oracle(F):
    """Log-score, CRPS and RMSE of the predictive distribution at held-out
    points (Section 4) against the oracle's, from the same means and
    variances; and the refusal of a non-positive variance."""
    locs, y, theta, ind, gamma = case(**CASES["m32_n1500_m100"])
    pred = G.uniform_locations(400, 903)
    ytest = G.rff_response(pred, O.MATERN32, 1.0, 0.05, 0.1, 300, 301)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=2, seed=3, tol=1e-10, max_iter=3000) as f:
        f.nll_grad(with_grad=False)
        # enough samples that the stochastic diagonal leaves every variance
        # positive (with a few dozen, one of these 400 went below zero)
        var, mean, _ = f.predict_var(pred, 512, with_mean=True)
    say("smallest predictive variance", var.min())
    assert var.min() > 0
    got = F.fsa_scores(ytest, mean, var)
    ref = O.scores(ytest, mean, var)
    say("scores", got, ref)
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    bad = var.copy()
    bad[7] = 0.0
    with pytest.raises(F.FsaError):
        F.fsa_scores(ytest, mean, bad)


@pytest.mark.gpu
def test_control_variate_with_one_probe(F):
    """One probe: the centred and printed coefficients have nothing to
    regress on (c = 0, the plain estimate); c = 1 still applies.  Against the
    oracle with fixed iterations; no NaN anywhere."""
    locs, y, theta, ind, gamma = case(**CASES["ragged_n333_m7"])
    mdl = O.FSA(locs, ind, theta, gamma)
    for mode, cvm in (("one", F.CV_ONE), ("opt", F.CV_OPT), ("opt_printed", F.CV_OPT_PRINTED)):
        ref = O.nll_grad(mdl, y, 1, 13, fixed_iter=10, control_variate=mode)
        with F.FSA(locs, y, theta, ind, gamma, num_probes=1, seed=13, fixed_iter=10, control_variate=cvm) as f:
            nll, grad, st = f.nll_grad()
        assert np.all(np.isfinite(grad)) and np.all(np.isfinite(st["cv_c"]))
        np.testing.assert_allclose(st["cv_c"], ref["cv_c"], atol=1e-12)
        gscale = np.maximum(np.abs(ref["grad"]), 0.5 * np.abs(ref["trace_terms"]).mean(1))
        assert np.all(np.abs(grad - ref["grad"]) <= 1e-9 * gscale + 1e-12), (mode, grad, ref["grad"])
