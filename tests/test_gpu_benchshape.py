"""Oracle parity at the shapes of the timed configuration's kernel variants,
and the two small configurations run as written (MI355X only).

The timed likelihood has m = 500 inducing points (padded to 512: the float64
Woodbury expansion runs as two 256-k passes with the partial sum held in
the output block, the float32 one keeps a 128 KiB G tile in LDS) and t = 50
probes (51 right-hand-side columns: one 64-column block, and the
bfloat16-MFMA expansion at its 52-column limit).  The cases below keep those
shapes at n = 4,000 so that the oracle finishes in seconds; m = 300 (padded
to 320: one 256-k and one 64-k pass) covers a ragged k split, and one case is
clustered.

Bars (the method's): float64 with identical probes and a fixed iteration
count within 1e-9 relative (NLL) and 1e-9 of each gradient component's
scale; mixed precision within 1e-4; the true float64 residual
||b - Sigma~ u|| / ||b|| of every column of a mixed solve at or below the
tolerance.

Configurations as written:
  - n = 2,000 uniform, exponential (sigma1^2 = 1, rho = 0.1, sigma^2 = 0.05),
    m = 50 random subset, ~30 nonzeros per row, t = 10, tolerance 1e-8:
    against the oracle (fixed iterations) and against dense Cholesky
    (within the Monte-Carlo error of the probes);
  - Algorithm 1 on a 2,000-point training set (exponential, rho = 0.1,
    sigma^2 = 0.1, m = 500, ~60 nonzeros per row, s = 100) against the
    dense float64 FSA predictive variances (eq. MuPredFSA), within the
    standard error of the simulated term."""
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


def case(n=4000, m=500, kind=O.MATERN32, rho=0.05, s1=1.0, s2=0.1, n_gamma=80, seed=0, clustered=False):
    locs = G.clustered_locations(n, 600 + seed) if clustered else G.uniform_locations(n, 600 + seed)
    ind = G.kmeanspp_inducing(locs, m, 700 + seed)
    gamma = G.taper_range_by_count(locs, n_gamma, sample=n) if clustered else G.taper_range_for_uniform(n, n_gamma)
    y = G.rff_response(locs, kind, s1, rho, s2, 500, 800 + seed)
    return locs, y, (kind, s1, rho, s2), ind, gamma


CASES = {
    "m500_uniform": dict(),
    "m300_uniform": dict(m=300, seed=1),
    "m500_clustered": dict(kind=O.EXPONENTIAL, rho=0.2, s1=2.0, s2=0.05, n_gamma=50, seed=2, clustered=True),
}
T = 50


def gscale(ref):
    return np.maximum(np.abs(ref["grad"]), 0.5 * np.abs(ref["trace_terms"]).mean(1))


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_fixed_iterations_at_bench_shape(F, name):
    """The float64 kernel variants of the timed shape (two-pass expansion at
    mp = 512, 320 = 256 + 64 at m = 300) against the oracle, 1e-9."""
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    k = 10
    ref = O.nll_grad(O.FSA(locs, ind, theta, gamma), y, T, 91, fixed_iter=k)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=T, seed=91, fixed_iter=k) as f:
        nll, grad, st = f.nll_grad()
    err = np.abs(grad - ref["grad"]) / gscale(ref)
    say("nll", nll, ref["nll"], "rel", abs(nll - ref["nll"]) / abs(ref["nll"]), "grad err / scale", err)
    assert abs(nll - ref["nll"]) <= 1e-9 * abs(ref["nll"])
    assert np.all(err <= 1e-9)
    assert st["iters_min"] == k and st["iters_max"] == k


@pytest.mark.parametrize("products", ["split", "mfma"])
@pytest.mark.parametrize("name", list(CASES))
def test_mixed_fixed_iterations_at_bench_shape(F, name, products):
    """The float32 kernels of the timed shape (tiled sparse product, the
    residual pass and the expansion, their float32 products either split into
    bfloat16 parts or on the float32 matrix cores with the 128 KiB G tile)
    with the float64 residual replacement every 5 iterations, against the
    oracle with the same probes and iteration count: 1e-4."""
    say("case", name, products)
    locs, y, theta, ind, gamma = case(**CASES[name])
    k = 12
    ref = O.nll_grad(O.FSA(locs, ind, theta, gamma), y, T, 92, fixed_iter=k)
    fp = {"split": F.F32P_SPLIT, "mfma": F.F32P_MFMA}[products]
    with F.FSA(locs, y, theta, ind, gamma, num_probes=T, seed=92, fixed_iter=k, precision=F.MIXED_FP32,
               rr_period=5, fp32_products=fp) as f:
        nll, grad, st = f.nll_grad()
    err = np.abs(grad - ref["grad"]) / gscale(ref)
    say("nll rel", abs(nll - ref["nll"]) / abs(ref["nll"]), "grad err / scale", err)
    assert abs(nll - ref["nll"]) <= 1e-4 * abs(ref["nll"])
    assert np.all(err <= 1e-4)


@pytest.mark.parametrize("t", [12, 20])
@pytest.mark.parametrize("name", ["m500_uniform", "m500_clustered"])
def test_mixed_narrow_blocks_against_oracle(F, name, t):
    """Blocks of at most 16 and 32 columns (t' = 13 and 21, the serving
    stream's width): the split residual pass and expansion multiply one or
    two of their four 16-column tiles and the tiled sparse product leaves its
    empty column tiles out.  Against the oracle with the same probes and
    iteration count: 1e-4."""
    say("case", name, "t", t)
    locs, y, theta, ind, gamma = case(**CASES[name])
    k = 12
    ref = O.nll_grad(O.FSA(locs, ind, theta, gamma), y, t, 96, fixed_iter=k)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=t, seed=96, fixed_iter=k, precision=F.MIXED_FP32,
               rr_period=5) as f:
        nll, grad, st = f.nll_grad()
    err = np.abs(grad - ref["grad"]) / gscale(ref)
    say("nll rel", abs(nll - ref["nll"]) / abs(ref["nll"]), "grad err / scale", err)
    assert abs(nll - ref["nll"]) <= 1e-4 * abs(ref["nll"])
    assert np.all(err <= 1e-4)
    assert st["iters_min"] == k and st["iters_max"] == k


@pytest.mark.parametrize("name", ["m500_uniform", "m500_clustered"])
def test_split_products_agree_with_fp32_mfma(F, name):
    """The two ways of taking MIXED_FP32's low-rank products (bfloat16 parts,
    float32 matrix cores) are both float32 products: with the same probes and
    a fixed iteration count the likelihood, gradient and every column's
    Lanczos coefficients agree to float32 rounding propagated through the
    iterations (gradient components against the gradient's scale: the
    larger of the component and a hundredth of the largest one, since the
    sigma1^2 component can be a small difference of large terms)."""
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    out = {}
    for fp in (F.F32P_SPLIT, F.F32P_MFMA):
        with F.FSA(locs, y, theta, ind, gamma, num_probes=T, seed=95, fixed_iter=15, precision=F.MIXED_FP32,
                   rr_period=5, fp32_products=fp) as f:
            nll, grad, st = f.nll_grad()
            out[fp] = (nll, grad, f.export_lanczos())
    (n1, g1, l1), (n2, g2, l2) = out[F.F32P_SPLIT], out[F.F32P_MFMA]
    a1, a2 = np.asarray(l1["alpha"]), np.asarray(l2["alpha"])
    say("nll rel", abs(n1 - n2) / abs(n2), "grad rel", np.abs(g1 - g2) / np.abs(g2),
        "alpha rel max", (np.abs(a1 - a2) / np.abs(a2)).max())
    assert abs(n1 - n2) <= 1e-6 * abs(n2)
    assert np.all(np.abs(g1 - g2) <= 1e-5 * np.maximum(np.abs(g2), 0.01 * np.abs(g2).max()))
    assert (np.abs(a1 - a2) / np.abs(a2)).max() <= 1e-4


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_converged_at_bench_shape_with_true_residual(F, name):
    """MIXED_FP32 at tolerance 1e-6 with residual replacement every 20
    iterations (the timed settings) against the oracle converged to 1e-10:
    NLL and gradient within 1e-4; and the true residual b - Sigma~ u of every
    column, formed from the exported solution with the float64 operator, at
    or below the tolerance (the library's reported figure agrees)."""
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    tol = 1e-6
    ref = O.nll_grad(O.FSA(locs, ind, theta, gamma), y, T, 93, tol=1e-10, max_iter=3000)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=T, seed=93, tol=tol, max_iter=3000, precision=F.MIXED_FP32,
               rr_period=20) as f:
        nll, grad, st = f.nll_grad()
        U = f.export_solution()
        Z = f.apply(F.OP_PROBES, None, ncols=T)
        SU = f.apply(F.OP_SIGMA_DAGGER, U)
    B = np.column_stack([y, Z])
    rel = np.linalg.norm(B - SU, axis=0) / np.linalg.norm(B, axis=0)
    err = np.abs(grad - ref["grad"]) / gscale(ref)
    say("nll rel", abs(nll - ref["nll"]) / abs(ref["nll"]), "grad err / scale", err, "iters", st["iters_max"],
        ref["iters"].max(), "true residual max", rel.max(), "reported", st["rel_res_max"])
    assert abs(nll - ref["nll"]) <= 1e-4 * abs(ref["nll"])
    assert np.all(err <= 1e-4)
    assert rel.max() <= tol
    assert 0.0 < st["rel_res_max"] <= tol
    assert abs(st["rel_res_max"] - rel.max()) <= 1e-3 * rel.max()


@pytest.mark.parametrize("name", ["m500_uniform", "m300_uniform"])
def test_bf16a_at_bench_shape_matches_oracle_of_rounded_model(F, name):
    """MIXED_BF16A at 51 columns (the bfloat16-MFMA expansion at its LDS
    limit) against the oracle of the model with A rounded to bfloat16."""
    say("case", name)
    locs, y, theta, ind, gamma = case(**CASES[name])
    mdl = DF.RoundedFSA(locs, ind, theta, gamma, smn_T=DF.bf16_cross_covariance(locs, ind, theta))
    ref = O.nll_grad(mdl, y, T, 94, tol=1e-10, max_iter=3000)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=T, seed=94, tol=1e-6, max_iter=3000,
               precision=F.MIXED_BF16A, rr_period=20) as f:
        nll, grad, st = f.nll_grad()
    err = np.abs(grad - ref["grad"]) / gscale(ref)
    say("bf16a nll rel", abs(nll - ref["nll"]) / abs(ref["nll"]), "grad err / scale", err)
    assert abs(nll - ref["nll"]) <= 1e-4 * abs(ref["nll"])
    assert np.all(err <= 1e-4)
    assert 0.0 < st["rel_res_max"] <= 1e-6


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_predictive_variances_at_m500(F, prec):
    """Algorithm 1 with m = 500 (the sparse solves then carry 512 + s
    columns) against the oracle with the same draws: 1e-9 in float64, 1e-4
    per variance in mixed precision."""
    locs, y, theta, ind, gamma = case(**CASES["m500_uniform"])
    pred = G.uniform_locations(300, 905)
    ref, _ = O.predict_var(O.FSA(locs, ind, theta, gamma), pred, 16, 24, tol=1e-12, max_iter=3000)
    precision, tol = (F.FP64, 1e-12) if prec == "fp64" else (F.MIXED_FP32, 1e-7)
    with F.FSA(locs, y, theta, ind, gamma, num_probes=2, seed=24, tol=tol, max_iter=3000, precision=precision) as f:
        var, _, st = f.predict_var(pred, 16)
    if prec == "fp64":
        err = np.abs(var - ref).max() / np.abs(ref).max()
        say("fp64 var err", err, "iters", st["iters_max"])
        assert err < 1e-9
    else:
        err = (np.abs(var - ref) / np.abs(ref)).max()
        say("mixed var rel err", err, "iters", st["iters_max"])
        assert err < 1e-4


# ---------------------------------------------------------------- configurations as written
def test_small_configuration_against_oracle_and_dense_cholesky(F):
    """n = 2,000, m = 50, t = 10, tolerance 1e-8.  Fixed iterations (the
    converged run's count): NLL and gradient within 1e-9 of the oracle.
    Converged: the NLL within four Monte-Carlo standard errors of the dense
    Cholesky NLL (the SLQ estimate's error is the probes' sample spread over
    sqrt(t)), and each gradient component within four standard errors of the
    dense exact gradient."""
    w = configs.small_fp64()
    mdl = O.FSA(w.locs, w.inducing, w.theta, w.gamma)
    with F.FSA(w.locs, w.y, w.theta, w.inducing, w.gamma, num_probes=w.num_probes, seed=w.seed, tol=w.tol) as f:
        nll, grad, st = f.nll_grad()
        rec = f.export_lanczos()
    k = int(st["iters_max"])
    ref = O.nll_grad(mdl, w.y, w.num_probes, w.seed, fixed_iter=k)
    with F.FSA(w.locs, w.y, w.theta, w.inducing, w.gamma, num_probes=w.num_probes, seed=w.seed,
               fixed_iter=k) as f:
        nll_k, grad_k, _ = f.nll_grad()
    say("fixed", k, "nll", nll_k, ref["nll"], "grad", grad_k, ref["grad"])
    assert abs(nll_k - ref["nll"]) <= 1e-9 * abs(ref["nll"])
    assert np.all(np.abs(grad_k - ref["grad"]) <= 1e-9 * gscale(ref) + 1e-12)
    # dense Cholesky
    S = DF.dense_fsa(w.locs, w.inducing, w.theta, w.gamma)
    L = np.linalg.cholesky(S)
    dense_nll = 0.5 * w.n * np.log(2 * np.pi) + np.log(np.diag(L)).sum() + 0.5 * w.y @ np.linalg.solve(S, w.y)
    terms = rec["slq"][1:]
    se_nll = 0.5 * terms.std(ddof=1) / np.sqrt(w.num_probes)
    Si = np.linalg.inv(S)
    u = Si @ w.y
    conv = O.nll_grad(mdl, w.y, w.num_probes, w.seed, tol=w.tol)
    exact = np.empty(3)
    se_g = np.empty(3)
    for j in range(3):
        dS = DF.fd_operator(w.locs, w.inducing, w.theta, w.gamma, j)
        exact[j] = 0.5 * np.trace(Si @ dS) - 0.5 * u @ dS @ u
        se_g[j] = 0.5 * conv["trace_terms"][j].std(ddof=1) / np.sqrt(w.num_probes)
    say("nll", nll, "dense", dense_nll, "se", se_nll, "grad", grad, "exact", exact, "se", se_g, "iters", k,
        "rel_res", st["rel_res_max"])
    assert st["rel_res_max"] < w.tol
    assert abs(nll - dense_nll) <= 4 * se_nll
    assert np.all(np.abs(grad - exact) <= 4 * se_g)


def test_predictive_variances_against_dense_subproblem(F):
    """Algorithm 1 (s = 100) on a 2,000-point training set of the prediction
    workload's recipe against the dense float64 FSA predictive variances.
    Only the simulated diagonal D_l is random; with Rademacher draws its
    per-point variance is sum_{k != j} M_jk^2 / s, M = Sigma^s_{n n_p}^T
    Sigma~_s^{-1} Sigma^s_{n n_p}, which gives each point's standard error.
    Every point within 5 standard errors, the mean error within 4 standard
    errors of the mean, and the mean squared standardized error near 1."""
    w = configs.predictive(n=2000, n_p=400, m=500, s=100)
    with F.FSA(w.locs, w.y, w.theta, w.inducing, w.gamma, num_probes=2, seed=w.seed, tol=1e-10,
               max_iter=3000) as f:
        var, _, st = f.predict_var(w.pred_locs, w.num_samples)
    exact, _, _ = DF.dense_pred_var(w.locs, w.inducing, w.pred_locs, w.theta, w.gamma)
    p = DF.dense_parts(w.locs, w.inducing, w.theta, w.gamma)
    from scipy.spatial.distance import cdist
    kind, s1, rho, s2 = w.theta
    Sm = O.covariance(cdist(w.inducing, w.inducing), s1, rho, kind)
    Smp = O.covariance(cdist(w.inducing, w.pred_locs), s1, rho, kind)
    Snp = O.covariance(cdist(w.locs, w.pred_locs), s1, rho, kind)
    Sl_np = p["Smn"].T @ np.linalg.solve(Sm, Smp)
    Scross = (Snp - Sl_np) * O.wendland_taper(cdist(w.locs, w.pred_locs), w.gamma)
    M = Scross.T @ np.linalg.solve(p["Ss"], Scross)
    se = np.sqrt((np.sum(M * M, axis=1) - np.diag(M) ** 2) / w.num_samples)
    se = np.sqrt(se * se + 1e-16)  # the solves' own error (tolerance 1e-10) where a point has no spread
    z = (var - exact) / se
    say("n_p", len(var), "max |z|", np.abs(z).max(), "mean z^2", np.mean(z * z), "mean err", np.mean(var - exact),
        "se of mean", np.sqrt(np.sum(se * se)) / len(var), "iters", st["iters_max"])
    assert np.abs(z).max() < 5.0
    assert abs(np.mean(var - exact)) <= 4 * np.sqrt(np.sum(se * se)) / len(var)
    assert 0.7 < np.mean(z * z) < 1.3


def test_mixed_falls_back_to_fp64_where_float32_cannot_resolve(F):
    """A strongly low-rank problem (n = 6,313, m = 500, Matern-3/2 with rho =
    0.153: |A A^T| exceeds the nugget by ~10^4): the float32 Woodbury
    application loses most of its digits, the float32 iteration stalls, and
    MIXED_FP32 repeats the solve in float64 (the likelihood is then the
    float64 one bit for bit, and the stats say so; the gradient's derivative
    factor stays the float32 one of the mixed mode, so the gradient agrees to
    the mixed-precision bar).  A well-conditioned request of the same stream
    stays in float32."""
    trace = configs.serving_trace()
    hard = next(r for r in trace if r.index == 5)
    locs, y, ind, _ = hard.materialize()
    with F.FSA(locs, y, hard.theta, ind, hard.gamma, num_probes=20, seed=4005, tol=1e-6, max_iter=2000) as f:
        nll64, grad64, st64 = f.nll_grad()
    with F.FSA(locs, y, hard.theta, ind, hard.gamma, num_probes=20, seed=4005, tol=1e-6, max_iter=2000,
               precision=F.MIXED_FP32, rr_period=20) as f:
        nll, grad, st = f.nll_grad()
    say("hard: fallback", st["fp64_fallback"], "abandoned probe-iterations", st["fallback_probe_iters"],
        "iters", st["iters_max"], st64["iters_max"])
    assert st["fp64_fallback"] == 1 and st["fallback_probe_iters"] > 0
    assert nll == nll64
    scale = np.maximum(np.abs(grad64), 0.01 * np.abs(grad64).max())
    assert np.all(np.abs(grad - grad64) <= 1e-4 * scale)
    easy = next(r for r in trace if r.index == 0)
    locs, y, ind, _ = easy.materialize()
    with F.FSA(locs, y, easy.theta, ind, easy.gamma, num_probes=20, seed=4005, tol=1e-6, max_iter=2000,
               precision=F.MIXED_FP32, rr_period=20) as f:
        nll, grad, st = f.nll_grad()
    assert st["fp64_fallback"] == 0 and st["fallback_probe_iters"] == 0
