"""Pins of the CPU oracle against the paper's definitions, closed forms,
special cases, brute force and published values (no GPU needed)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.special import gamma as Gamma
from scipy.special import kv

from oracle import fsa_oracle as O
from tests import dense_fsa as DF
from workloads import generators as G

EXP, M32 = O.EXPONENTIAL, O.MATERN32


def small_case(n=300, m=30, kind=EXP, rho=0.1, s1=1.0, s2=0.1, n_gamma=20, seed=0):
    locs = G.uniform_locations(n, 10 + seed)
    ind = G.random_subset_inducing(locs, m, 20 + seed)
    gamma = G.taper_range_for_uniform(n, n_gamma)
    theta = (kind, s1, rho, s2)
    return locs, ind, theta, gamma


# ---------------------------------------------------------------- covariance

@pytest.mark.parametrize("kind,nu", [(EXP, 0.5), (M32, 1.5)])
def test_covariance_is_matern_bessel_form(kind, nu):
    """Matérn in its Bessel form with argument sqrt(2 nu) d / rho."""
    d = np.linspace(1e-4, 0.6, 97)
    rho, s1 = 0.07, 1.7
    x = math.sqrt(2 * nu) * d / rho
    ref = s1 * 2 ** (1 - nu) / Gamma(nu) * x ** nu * kv(nu, x)
    np.testing.assert_allclose(O.covariance(d, s1, rho, kind), ref, rtol=1e-12)
    assert O.covariance(0.0, s1, rho, kind) == s1


def test_matern32_effective_range_matches_section4(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "effective_range.json")))
    for re_, rho_printed in zip(g["effective_ranges"], g["rho_printed"]):
        corr = O.covariance(re_, 1.0, rho_printed, M32)
        assert abs(corr - g["correlation_at_effective_range"]) < 0.005
        assert abs(rho_printed - re_ / 2.7) < 1e-4


@pytest.mark.parametrize("kind", [EXP, M32])
def test_covariance_drho_central_difference(kind):
    d = np.linspace(0.0, 0.5, 51)
    rho, s1, h = 0.05, 1.3, 1e-6
    fd = (O.covariance(d, s1, rho + h, kind) - O.covariance(d, s1, rho - h, kind)) / (2 * h)
    np.testing.assert_allclose(O.covariance_drho(d, s1, rho, kind), fd, rtol=1e-7, atol=1e-9)


def test_wendland_taper_properties():
    gamma = 0.3
    assert O.wendland_taper(0.0, gamma) == 1.0
    assert O.wendland_taper(gamma, gamma) == 0.0
    assert O.wendland_taper(2 * gamma, gamma) == 0.0
    # C^2 at the support boundary: first and second derivatives vanish at r = 1.
    r = 1 - 1e-4
    assert O.wendland_taper(r * gamma, gamma) < 1e-14
    # positive definite in 2-D: taper matrix of random points has no negative eigenvalue
    pts = G.uniform_locations(400, 5)
    from scipy.spatial.distance import cdist
    T = O.wendland_taper(cdist(pts, pts), 0.2)
    assert np.linalg.eigvalsh(T).min() > -1e-10


def test_wendland_taper_is_wendlands_phi31():
    """The taper is Wendland's phi_{3,1}: his integral operator
    (I f)(r) = int_r^1 t f(t) dt applied once to the truncated power
    (1 - r)^3_+, normalised to 1 at r = 0, evaluated here by numerical
    quadrature (independent of the closed form); and one interior value by
    hand, W(1/2) = (1/2)^4 (1 + 2) = 3/16."""
    from scipy.integrate import quad
    gamma = 0.7
    f0 = quad(lambda t: t * (1 - t) ** 3, 0.0, 1.0, epsabs=1e-15, epsrel=1e-14)[0]
    for r in (0.0, 0.1, 0.25, 0.5, 0.8, 0.95):
        ref = quad(lambda t: t * (1 - t) ** 3, r, 1.0, epsabs=1e-15, epsrel=1e-14)[0] / f0
        assert abs(float(O.wendland_taper(r * gamma, gamma)) - ref) < 1e-12, r
    assert abs(float(O.wendland_taper(0.5 * gamma, gamma)) - 3.0 / 16.0) < 1e-15


# ---------------------------------------------------------------- pattern

def test_pattern_equals_bruteforce_random():
    locs = G.uniform_locations(1500, 3)
    gamma = 0.04
    rp, cl = O.taper_pattern(locs, locs, gamma)
    rb, cb = O.taper_pattern_bruteforce(locs, locs, gamma)
    assert np.array_equal(rp, rb) and np.array_equal(cl, cb)


def test_pattern_excludes_exact_ties():
    """Lattice points at exactly distance gamma are excluded (taper is zero
    at d >= gamma); values are exact binary fractions so d^2 == gamma^2."""
    g = np.arange(24) / 64.0
    locs = np.array([(a, b) for a in g for b in g])
    gamma = 2.0 / 64.0
    rp, cl = O.taper_pattern(locs, locs, gamma)
    rb, cb = O.taper_pattern_bruteforce(locs, locs, gamma)
    assert np.array_equal(rp, rb) and np.array_equal(cl, cb)
    # interior lattice point: itself, 4 axis neighbours at 1/64 and 4 diagonals at sqrt2/64
    i = 10 * 24 + 10
    assert rp[i + 1] - rp[i] == 9


def test_cross_pattern_equals_bruteforce():
    a = G.uniform_locations(700, 4)
    b = G.uniform_locations(300, 5)
    rp, cl = O.taper_pattern(a, b, 0.05)
    rb, cb = O.taper_pattern_bruteforce(a, b, 0.05)
    assert np.array_equal(rp, rb) and np.array_equal(cl, cb)


def test_pattern_density_matches_appendix_h(golden_dir):
    """gamma = 0.016 gives about 80 nonzeros per row at n = 100000."""
    g = json.load(open(os.path.join(golden_dir, "taper_density.json")))
    assert abs(G.mean_neighbours_uniform(g["n"], g["gamma"]) - g["n_gamma"]) / g["n_gamma"] < 0.01
    locs = G.uniform_locations(g["n"], 7)
    rp, _ = O.taper_pattern(locs, locs, g["gamma"])
    assert abs(rp[-1] / g["n"] - g["n_gamma"]) / g["n_gamma"] < 0.02


# ---------------------------------------------------------------- operator

def test_operator_equals_dense_definition():
    locs, ind, theta, gamma = small_case(kind=M32, rho=0.08)
    mdl = O.FSA(locs, ind, theta, gamma)
    X = np.random.default_rng(0).standard_normal((locs.shape[0], 3))
    ref = DF.dense_fsa(locs, ind, theta, gamma) @ X
    np.testing.assert_allclose(mdl.matvec(X), ref, rtol=1e-10, atol=1e-10)


def test_supplied_cross_covariance_equals_dense_definition():
    """FSA with a rounded low-rank part (whitened factor in bfloat16): the
    operator, FITC solve and log det P follow the dense definitions built on
    the same Sigma_mn; the diagonal stays sigma1^2 + sigma^2 because the
    residual absorbs the low-rank part on it; the rho-derivative keeps the
    exact dSigma_mn (dense: dSmn^T K + K^T dSmn - K^T dSm K with K = Sm^{-1} Smn,
    then tapered); bf16_round is exact on bfloat16 values and moves others by
    at most half a bfloat16 unit."""
    from scipy.spatial.distance import cdist
    locs, ind, theta, gamma = small_case(kind=M32, rho=0.08)
    kind, s1, rho, s2 = theta
    n = locs.shape[0]
    smn_T = DF.bf16_cross_covariance(locs, ind, theta)
    exact_T = O.covariance(cdist(locs, ind), s1, rho, kind)
    assert 0 < np.abs(smn_T - exact_T).max() < 1e-2
    mdl = O.FSA(locs, ind, theta, gamma, smn_T=smn_T)
    p = DF.dense_parts(locs, ind, theta, gamma, Smn=smn_T.T)
    X = np.random.default_rng(0).standard_normal((n, 3))
    np.testing.assert_allclose(mdl.matvec(X), p["full"] @ X, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(np.diag(p["full"]), s1 + s2, rtol=1e-12)
    P = np.diag(np.diag(p["Ss"])) + p["Sl"]
    np.testing.assert_allclose(mdl.precond_solve(X), np.linalg.solve(P, X), rtol=1e-9, atol=1e-9)
    assert abs(mdl.logdet_P - np.linalg.slogdet(P)[1]) < 1e-9 * abs(np.linalg.slogdet(P)[1])
    K = np.linalg.solve(p["Sm"], smn_T.T)
    dSm = O.covariance_drho(cdist(ind, ind), s1, rho, kind)
    dSmn = O.covariance_drho(cdist(ind, locs), s1, rho, kind)
    dSl = dSmn.T @ K + K.T @ dSmn - K.T @ dSm @ K
    dS = (O.covariance_drho(cdist(locs, locs), s1, rho, kind) - dSl) * p["T"] + dSl
    np.testing.assert_allclose(mdl.dmatvec(1, X), dS @ X, rtol=1e-9, atol=1e-9 * np.abs(dS @ X).max())
    # the sigma1^2 derivative of the rounded model by proportionality is the
    # oracle's exact one on the unrounded model
    plain = O.FSA(locs, ind, theta, gamma)
    np.testing.assert_allclose(plain.dmatvec(0, X), (plain.matvec(X) - s2 * X) / s1, rtol=1e-9,
                               atol=1e-9 * np.abs(X).max())
    rnd = DF.RoundedFSA(locs, ind, theta, gamma, smn_T=smn_T)
    np.testing.assert_allclose(rnd.dmatvec(0, X), (p["full"] @ X - s2 * X) / s1, rtol=1e-9, atol=1e-9)
    v = np.array([1.0, -2.5, 3.0e-3, 0.1, 1.0078125])
    r = DF.bf16_round(v)
    np.testing.assert_array_equal(r[[0, 1, 4]], v[[0, 1, 4]])
    assert np.all(np.abs(r - v) <= np.abs(v) * 2.0 ** -8)
    # a tie rounds to the even neighbour: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert DF.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert DF.bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_inducing_equal_to_locations_gives_exact_gp():
    """S* = S makes Sigma_l = Sigma, so Sigma~_dagger = Sigma + sigma^2 I and
    the FITC preconditioner is exact too."""
    locs = G.uniform_locations(150, 11)
    theta = (EXP, 1.2, 0.2, 0.3)
    mdl = O.FSA(locs, locs, theta, 0.05)
    from scipy.spatial.distance import cdist
    exact = O.covariance(cdist(locs, locs), 1.2, 0.2, EXP) + 0.3 * np.eye(150)
    X = np.random.default_rng(1).standard_normal((150, 2))
    np.testing.assert_allclose(mdl.matvec(X), exact @ X, rtol=1e-8, atol=1e-8)
    assert abs(mdl.logdet_P - np.linalg.slogdet(exact)[1]) < 1e-7 * abs(np.linalg.slogdet(exact)[1])


def test_residual_is_psd():
    locs, ind, theta, gamma = small_case(n=400, m=40, kind=M32, rho=0.1, n_gamma=40)
    mdl = O.FSA(locs, ind, theta, gamma)
    S = mdl.S.toarray()
    assert np.allclose(S, S.T)
    assert np.linalg.eigvalsh(S - theta[3] * np.eye(400)).min() > -1e-10


def test_woodbury_and_sylvester_match_dense_fitc():
    locs, ind, theta, gamma = small_case(kind=M32, rho=0.06)
    mdl = O.FSA(locs, ind, theta, gamma)
    P = DF.dense_fitc(locs, ind, theta, gamma)
    R = np.random.default_rng(2).standard_normal((locs.shape[0], 4))
    np.testing.assert_allclose(mdl.precond_solve(R), np.linalg.solve(P, R), rtol=1e-9, atol=1e-9)
    assert abs(mdl.logdet_P - np.linalg.slogdet(P)[1]) < 1e-9 * abs(np.linalg.slogdet(P)[1])


def test_tiny_taper_reduces_to_fitc_one_iteration():
    """gamma below the minimum distance: Sigma~_dagger equals P, so PCG needs
    one iteration and SLQ returns log det P exactly."""
    locs, ind, theta, _ = small_case(n=200, m=20)
    mdl = O.FSA(locs, ind, theta, 1e-7)
    assert mdl.col.size == 200
    y = np.random.default_rng(3).standard_normal(200)
    out = O.nll_grad(mdl, y, 5, 9, tol=1e-12, with_grad=False)
    assert np.all(out["iters"] == 1)
    assert abs(out["logdet"] - mdl.logdet_P) < 1e-10 * abs(mdl.logdet_P)
    P = DF.dense_fitc(locs, ind, theta, 1e-7)
    np.testing.assert_allclose(out["pcg"].U[:, 0], np.linalg.solve(P, y), rtol=1e-10)


# ---------------------------------------------------------------- RNG and probes

def test_splitmix64_known_answers(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64_seed0.json")))
    got = O.splitmix64(g["seed"], np.arange(3))
    assert [int(v) for v in got] == [int(h, 16) for h in g["outputs_hex"]]


def test_rademacher_is_balanced_and_keyed():
    Z = O.rademacher(4242, O.STREAM_RHO, 20000, 4)
    assert set(np.unique(Z)) == {-1.0, 1.0}
    assert np.all(np.abs(Z.mean(0)) < 4 / math.sqrt(20000))
    assert not np.array_equal(Z, O.rademacher(4243, O.STREAM_RHO, 20000, 4))
    assert not np.array_equal(Z, O.rademacher(4242, O.STREAM_E, 20000, 4))
    # column c of a wider draw equals column c of a narrower one (counter-based)
    np.testing.assert_array_equal(Z[:, :2], O.rademacher(4242, O.STREAM_RHO, 20000, 2))


def test_probe_covariance_is_preconditioner():
    """Cov z = D_s + Sigma_mn^T Sigma_m^{-1} Sigma_mn (App. F)."""
    locs, ind, theta, gamma = small_case(n=40, m=8, n_gamma=6)
    mdl = O.FSA(locs, ind, theta, gamma)
    Z = O.probes(mdl, 40000, 77)
    emp = Z @ Z.T / Z.shape[1]
    P = DF.dense_fitc(locs, ind, theta, gamma)
    se = np.sqrt((np.outer(np.diag(P), np.diag(P)) + P ** 2) / Z.shape[1])
    assert np.max(np.abs(emp - P) / se) < 5.5


# ---------------------------------------------------------------- PCG / Lanczos / SLQ

def test_pcg_solves_match_dense():
    locs, ind, theta, gamma = small_case(kind=M32, rho=0.08)
    mdl = O.FSA(locs, ind, theta, gamma)
    B = np.random.default_rng(4).standard_normal((locs.shape[0], 5))
    res = O.pcg_lanczos(mdl.matvec, mdl.precond_solve, B, 1e-12, 500)
    ref = np.linalg.solve(DF.dense_fsa(locs, ind, theta, gamma), B)
    np.testing.assert_allclose(res.U, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
    assert np.all(res.rel_res < 1e-12)


def _explicit_lanczos(A, v, k):
    """Lanczos with full reorthogonalisation; returns the k x k tridiagonal."""
    n = A.shape[0]
    Q = np.zeros((n, k + 1))
    Q[:, 0] = v / np.linalg.norm(v)
    a, b = np.zeros(k), np.zeros(k)
    for j in range(k):
        w = A @ Q[:, j]
        a[j] = Q[:, j] @ w
        w -= Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        w -= Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        b[j] = np.linalg.norm(w)
        Q[:, j + 1] = w / b[j]
    return a, b[:k - 1]


def test_cg_coefficients_give_lanczos_tridiagonal():
    """T built from the CG alphas/betas (Algorithm 2) equals the Lanczos
    matrix of P^{-1/2} Sigma~ P^{-1/2} started at P^{-1/2} z."""
    locs, ind, theta, gamma = small_case(n=250, m=20, kind=EXP, rho=0.15)
    mdl = O.FSA(locs, ind, theta, gamma)
    z = O.probes(mdl, 1, 5)
    k = 8
    res = O.pcg_lanczos(mdl.matvec, mdl.precond_solve, z, 0.0, k, fixed_iter=k)
    P = DF.dense_fitc(locs, ind, theta, gamma)
    L = np.linalg.cholesky(P)
    A = sla.solve_triangular(L, sla.solve_triangular(L, DF.dense_fsa(locs, ind, theta, gamma), lower=True).T,
                             lower=True)
    a, b = _explicit_lanczos(A, sla.solve_triangular(L, z[:, 0], lower=True), k)
    np.testing.assert_allclose(res.diags[0], a, rtol=1e-8)
    np.testing.assert_allclose(res.offs[0], b, rtol=1e-7)


def test_quadrature_equals_dense_quadratic_form_at_convergence():
    locs, ind, theta, gamma = small_case(n=250, m=25, kind=M32, rho=0.08)
    mdl = O.FSA(locs, ind, theta, gamma)
    z = O.probes(mdl, 1, 6)
    res = O.pcg_lanczos(mdl.matvec, mdl.precond_solve, z, 1e-13, 400)
    w = float(z[:, 0] @ res.Q0[:, 0])
    est = w * O.e1_log_e1(res.diags[0], res.offs[0])
    P = DF.dense_fitc(locs, ind, theta, gamma)
    L = np.linalg.cholesky(P)
    A = sla.solve_triangular(L, sla.solve_triangular(L, DF.dense_fsa(locs, ind, theta, gamma), lower=True).T,
                             lower=True)
    lam, V = np.linalg.eigh(A)
    v = V.T @ sla.solve_triangular(L, z[:, 0], lower=True)
    exact = float(np.sum(v ** 2 * np.log(lam)))
    assert abs(est - exact) < 1e-8 * abs(exact)


def test_e1_log_e1_special_cases():
    assert abs(O.e1_log_e1([2.0], []) - math.log(2.0)) < 1e-15
    d, e = np.array([2.0, 3.0, 4.0]), np.array([0.5, 0.25])
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    lam, V = np.linalg.eigh(T)
    assert abs(O.e1_log_e1(d, e) - (V[0] ** 2 @ np.log(lam))) < 1e-14


def test_slq_converges_to_exact_logdet():
    locs, ind, theta, gamma = small_case(n=200, m=20, kind=EXP, rho=0.1)
    mdl = O.FSA(locs, ind, theta, gamma)
    y = np.zeros(200)
    out = O.nll_grad(mdl, y, 600, 31, tol=1e-11, with_grad=False)
    exact = np.linalg.slogdet(DF.dense_fsa(locs, ind, theta, gamma))[1]
    terms = out["slq_terms"]
    se = terms.std(ddof=1) / math.sqrt(terms.size)
    assert abs(out["logdet"] - exact) < 4 * se + 1e-9
    # fewer probes -> larger spread of the estimate
    assert se < terms.std(ddof=1)


def test_fitc_preconditioner_reduces_iterations(golden_dir):
    """Trend of Table 1: FITC needs far fewer CG iterations than none."""
    g = json.load(open(os.path.join(golden_dir, "table1_iterations.json")))
    assert all(f < nn for f, nn in zip(g["fitc"], g["none"]))
    locs = G.uniform_locations(3000, 12)
    ind = G.kmeanspp_inducing(locs, 100, 13, subsample=3000, lloyd_iters=5)
    theta = (M32, 1.0, 0.2 / 2.7, 1.0)
    mdl = O.FSA(locs, ind, theta, G.taper_range_for_uniform(3000, 30))
    y = G.rff_response(locs, M32, 1.0, 0.2 / 2.7, 1.0, 500, 14)[:, None]
    fitc = O.pcg_lanczos(mdl.matvec, mdl.precond_solve, y, 1e-3 / np.linalg.norm(y), 2000).iters[0]
    none = O.pcg_lanczos(mdl.matvec, lambda r: r.copy(), y, 1e-3 / np.linalg.norm(y), 2000).iters[0]
    assert fitc * 3 < none


# ---------------------------------------------------------------- NLL and gradient

def test_quadratic_term_and_nll_match_dense():
    locs, ind, theta, gamma = small_case(n=300, m=30, kind=EXP, rho=0.1, s2=0.05)
    mdl = O.FSA(locs, ind, theta, gamma)
    y = G.rff_response(locs, EXP, 1.0, 0.1, 0.05, 300, 8)
    out = O.nll_grad(mdl, y, 400, 19, tol=1e-11, with_grad=False)
    S = DF.dense_fsa(locs, ind, theta, gamma)
    assert abs(out["quad"] - y @ np.linalg.solve(S, y)) < 1e-9 * abs(out["quad"])
    se = out["slq_terms"].std(ddof=1) / math.sqrt(400)
    assert abs(out["nll"] - DF.dense_nll(S, y)) < 0.5 * 4 * se + 1e-8


@pytest.mark.parametrize("which", [0, 1, 2])
@pytest.mark.parametrize("kind", [EXP, M32])
def test_derivative_operator_equals_finite_difference(which, kind):
    locs, ind, theta, gamma = small_case(n=200, m=20, kind=kind, rho=0.09, s1=1.4, s2=0.2)
    mdl = O.FSA(locs, ind, theta, gamma)
    X = np.random.default_rng(9).standard_normal((200, 2))
    got = mdl.dmatvec(which, X)
    ref = DF.fd_operator(locs, ind, theta, gamma, which) @ X
    np.testing.assert_allclose(got, ref, rtol=2e-6, atol=2e-6 * np.abs(ref).max())


def test_dense_gradient_is_fd_of_dense_nll():
    """eq. DNEGLL on the dense FSA matrix vs a central difference of eq. NEGLL."""
    locs, ind, theta, gamma = small_case(n=150, m=15, kind=M32, rho=0.1, s2=0.1)
    y = G.rff_response(locs, M32, 1.0, 0.1, 0.1, 200, 21)
    S = DF.dense_fsa(locs, ind, theta, gamma)
    Si = np.linalg.inv(S)
    u = Si @ y
    for k in range(3):
        dS = DF.fd_operator(locs, ind, theta, gamma, k)
        g = 0.5 * np.trace(Si @ dS) - 0.5 * u @ dS @ u
        th = list(theta)
        h = 1e-5 * th[k + 1]
        th[k + 1] += h
        fp = DF.dense_nll(DF.dense_fsa(locs, ind, tuple(th), gamma), y)
        th[k + 1] -= 2 * h
        fm = DF.dense_nll(DF.dense_fsa(locs, ind, tuple(th), gamma), y)
        assert abs(g - (fp - fm) / (2 * h)) < 1e-5 * max(1.0, abs(g))


def test_stochastic_gradient_matches_exact_trace():
    locs, ind, theta, gamma = small_case(n=250, m=25, kind=EXP, rho=0.12, s1=1.0, s2=0.1)
    mdl = O.FSA(locs, ind, theta, gamma)
    y = G.rff_response(locs, EXP, 1.0, 0.12, 0.1, 300, 22)
    t = 500
    out = O.nll_grad(mdl, y, t, 23, tol=1e-11)
    S = DF.dense_fsa(locs, ind, theta, gamma)
    Si = np.linalg.inv(S)
    u = Si @ y
    for k in range(3):
        dS = DF.fd_operator(locs, ind, theta, gamma, k)
        exact = 0.5 * np.trace(Si @ dS) - 0.5 * u @ dS @ u
        terms = out["trace_terms"][k]
        se = 0.5 * terms.std(ddof=1) / math.sqrt(t)
        assert abs(out["grad"][k] - exact) < 4 * se + 1e-5 * abs(exact), (k, out["grad"][k], exact, se)


# ---------------------------------------------------------------- control variate (App. E)

@pytest.mark.parametrize("which", [0, 1, 2])
def test_preconditioner_derivative_equals_finite_difference(which):
    """dP/dtheta X against a central difference of the dense FITC matrix
    D_s + Sigma_l (eq. eqfitcp) built from the definitions."""
    locs, ind, theta, gamma = small_case(n=200, m=20, kind=M32, rho=0.09, s1=1.3, s2=0.15)
    mdl = O.FSA(locs, ind, theta, gamma)
    X = np.random.default_rng(11).standard_normal((200, 3))
    th = list(theta)
    h = 1e-5 * th[which + 1]
    th[which + 1] += h
    Pp = DF.dense_fitc(locs, ind, tuple(th), gamma)
    th[which + 1] -= 2 * h
    Pm = DF.dense_fitc(locs, ind, tuple(th), gamma)
    ref = (Pp - Pm) / (2 * h) @ X
    got = mdl.precond_dmatvec(which, X)
    np.testing.assert_allclose(got, ref, rtol=2e-6, atol=2e-6 * np.abs(ref).max())


@pytest.mark.parametrize("kind", [EXP, M32])
def test_preconditioner_trace_is_derivative_of_its_logdet(kind):
    """Jacobi's formula: Tr(P^{-1} dP/dtheta) = d log det P / dtheta, the
    right side by central differences of slogdet of the dense FITC matrix."""
    locs, ind, theta, gamma = small_case(n=180, m=18, kind=kind, rho=0.1, s1=0.8, s2=0.2)
    got = O.FSA(locs, ind, theta, gamma).precond_trace_deriv()
    for k in range(3):
        th = list(theta)
        h = 1e-5 * th[k + 1]
        th[k + 1] += h
        lp = np.linalg.slogdet(DF.dense_fitc(locs, ind, tuple(th), gamma))[1]
        th[k + 1] -= 2 * h
        lm = np.linalg.slogdet(DF.dense_fitc(locs, ind, tuple(th), gamma))[1]
        fd = (lp - lm) / (2 * h)
        assert abs(got[k] - fd) < 1e-6 * max(1.0, abs(fd)), (k, got[k], fd)


def test_c_opt_is_least_squares_slope():
    """The control-variate coefficients as regression slopes of the samples
    a_i on b_i: c_opt (centred reading) is the ordinary least-squares slope
    with intercept, so a_i - c b_i has the smallest sample variance; the
    printed form minimises sum_i (a_i - mean a - c b_i)^2, the slope through
    the origin of the centred samples."""
    locs, ind, theta, gamma = small_case(n=250, m=25, kind=EXP, rho=0.12, s1=1.0, s2=0.1)
    mdl = O.FSA(locs, ind, theta, gamma)
    y = G.rff_response(locs, EXP, 1.0, 0.12, 0.1, 300, 31)
    out = O.nll_grad(mdl, y, 12, 32, tol=1e-11, control_variate="opt")
    outp = O.nll_grad(mdl, y, 12, 32, tol=1e-11, control_variate="opt_printed")
    for k in range(3):
        a, b = out["trace_terms"][k], out["cv_terms"][k]
        slope = np.polyfit(b, a, 1)[0]
        assert abs(out["cv_c"][k] - slope) <= 1e-9 * max(1.0, abs(slope))
        v = lambda c: np.var(a - c * b)
        assert v(out["cv_c"][k]) <= min(v(out["cv_c"][k] * 1.01), v(out["cv_c"][k] * 0.99), v(1.0), v(0.0))
        slope0 = np.linalg.lstsq(b[:, None], a - a.mean(), rcond=None)[0][0]
        assert abs(outp["cv_c"][k] - slope0) <= 1e-12 * max(1.0, abs(slope0))
        # b_i with exact solves: (P^{-1} z_i)^T dP (P^{-1} z_i)
    P = DF.dense_fitc(locs, ind, theta, gamma)
    Z = O.probes(mdl, 12, 32)
    X = np.linalg.solve(P, Z)
    th = list(theta)
    h = 1e-5 * th[2]
    th[2] += h
    Pp = DF.dense_fitc(locs, ind, tuple(th), gamma)
    th[2] -= 2 * h
    dP = (Pp - DF.dense_fitc(locs, ind, tuple(th), gamma)) / (2 * h)
    np.testing.assert_allclose(out["cv_terms"][1], np.einsum("ij,ij->j", X, dP @ X), rtol=1e-5)


def test_control_variate_is_unbiased_and_reduces_variance():
    """Over independent probe sets the plain and control-variate gradient
    estimates all centre on the dense gradient (within four standard
    errors), and c_opt lowers the spread of the sigma1^2 and rho components
    (App. E, Fig. GradNEGLL)."""
    locs, ind, theta, gamma = small_case(n=200, m=20, kind=M32, rho=0.1, s1=1.0, s2=0.1)
    mdl = O.FSA(locs, ind, theta, gamma)
    y = G.rff_response(locs, M32, 1.0, 0.1, 0.1, 300, 33)
    S = DF.dense_fsa(locs, ind, theta, gamma)
    Si = np.linalg.inv(S)
    u = Si @ y
    exact = []
    for k in range(3):
        dS = DF.fd_operator(locs, ind, theta, gamma, k)
        exact.append(0.5 * np.trace(Si @ dS) - 0.5 * u @ dS @ u)
    est = {cv: [] for cv in (None, "one", "opt", "opt_printed")}
    for seed in range(40):
        for cv in est:
            est[cv].append(O.nll_grad(mdl, y, 8, 100 + seed, tol=1e-11, control_variate=cv)["grad"])
    sd = {cv: np.std(np.array(v), axis=0, ddof=1) for cv, v in est.items()}
    for cv, v in est.items():
        m = np.mean(np.array(v), axis=0)
        assert np.all(np.abs(m - exact) < 4 * sd[cv] / math.sqrt(40) + 1e-6 * np.abs(exact)), (cv, m, exact)
    # sigma1^2 and rho: b_i tracks a_i and the spread falls (by about 2.3x
    # for rho here); sigma^2 (b_i = |P^{-1} z_i|^2) gains little, and c
    # estimated from eight samples may cost a few percent there
    assert np.all(sd["opt"][:2] < 0.8 * sd[None][:2]), (sd["opt"], sd[None])
    assert sd["opt"][2] < 1.1 * sd[None][2], (sd["opt"], sd[None])
    assert np.all(sd["opt"][:2] < 1.05 * sd["one"][:2]), (sd["opt"], sd["one"])


def dense_residual_cross(locs, ind, pred, theta, gamma):
    """Sigma^s_{n n_p} = (Sigma_{n n_p} - Sigma^l_{n n_p}) o T_{n n_p}, dense."""
    from scipy.spatial.distance import cdist
    kind, s1, rho, s2 = theta
    Sm = O.covariance(cdist(ind, ind), s1, rho, kind)
    Smn = O.covariance(cdist(ind, locs), s1, rho, kind)
    Smp = O.covariance(cdist(ind, pred), s1, rho, kind)
    Snp = O.covariance(cdist(locs, pred), s1, rho, kind)
    low = Smn.T @ np.linalg.solve(Sm, Smp)
    return (Snp - low) * O.wendland_taper(cdist(locs, pred), gamma)


def test_diagonal_control_variate_is_unbiased_and_reduces_variance():
    """Algorithm 1's stochastic diagonal with D_s as control variate (App.
    E): the exact term diag(S^T D_s^{-1} S) against the dense definition; the
    c slopes as regressions; over independent draws every estimate centres
    on the exact diagonal (dense solve) and c_opt spreads far less than the
    plain estimate.  c = 1 spreads more here: S^T D_s^{-1} S is a loose
    stand-in for S^T Sigma~_s^{-1} S and c = 1 over-corrects."""
    locs, ind, theta, gamma = small_case(n=300, m=30, kind=M32, rho=0.1, s1=1.0, s2=0.1, n_gamma=25)
    mdl = O.FSA(locs, ind, theta, gamma)
    pred = G.uniform_locations(60, 901)
    _, det0 = O.predict_var(mdl, pred, 8, 0, tol=1e-12, exact_Dl=True)
    S = dense_residual_cross(locs, ind, pred, theta, gamma)
    _, d1 = O.predict_var(mdl, pred, 8, 5, tol=1e-12, control_variate="opt")
    np.testing.assert_allclose(d1["cv_E"], np.einsum("ij,ij->j", S, S / mdl.D[:, None]), rtol=1e-10)
    _, dp = O.predict_var(mdl, pred, 8, 5, tol=1e-12, control_variate="opt_printed")
    for j in (0, 7, 31):
        a, b = d1["cv_a"][j], d1["cv_b"][j]
        if np.ptp(b) > 0:
            assert abs(d1["cv_c"][j] - np.polyfit(b, a, 1)[0]) <= 1e-8 * max(1.0, abs(d1["cv_c"][j]))
        slope0 = np.linalg.lstsq(b[:, None], a - a.mean(), rcond=None)[0][0]
        assert abs(dp["cv_c"][j] - slope0) <= 1e-10 * max(1.0, abs(slope0))
    est = {cv: [] for cv in (None, "one", "opt", "opt_printed")}
    for seed in range(30):
        for cv in est:
            est[cv].append(O.predict_var(mdl, pred, 8, 200 + seed, tol=1e-12, control_variate=cv)[1]["Dl"])
    exact = det0["Dl"]
    sd = {cv: np.std(np.array(v), axis=0, ddof=1) for cv, v in est.items()}
    for cv, v in est.items():
        m = np.mean(np.array(v), axis=0)
        assert np.all(np.abs(m - exact) < 4.5 * sd[cv] / math.sqrt(30) + 1e-9), cv
    ratio_opt = np.median(sd["opt"] / sd[None])
    assert ratio_opt < 0.5, ratio_opt


# ---------------------------------------------------------------- predictive variances

def test_algorithm1_with_exact_diagonal_equals_dense():
    locs, ind, theta, gamma = small_case(n=300, m=25, kind=EXP, rho=0.1, s2=0.1, n_gamma=25)
    pred = G.uniform_locations(80, 99)
    mdl = O.FSA(locs, ind, theta, gamma)
    var, det = O.predict_var(mdl, pred, 0, 0, tol=1e-13, exact_Dl=True)
    ref, cross, S = DF.dense_pred_var(locs, ind, pred, theta, gamma)
    np.testing.assert_allclose(var, ref, rtol=1e-9, atol=1e-10)
    # the predictive mean from the same pieces
    y = G.rff_response(locs, EXP, 1.0, 0.1, 0.1, 200, 98)
    u = np.linalg.solve(S, y)
    _, det2 = O.predict_var(mdl, pred, 0, 0, tol=1e-13, exact_Dl=True, u=u)
    np.testing.assert_allclose(det2["mean"], cross.T @ u, rtol=1e-9, atol=1e-10)


def test_algorithm1_stochastic_term_is_unbiased():
    """Proposition 1: the simulated diagonal is unbiased; mean over seeds is
    within 4 standard errors of the exact value."""
    locs, ind, theta, gamma = small_case(n=250, m=20, kind=M32, rho=0.1, s2=0.1, n_gamma=25)
    pred = G.uniform_locations(60, 97)
    mdl = O.FSA(locs, ind, theta, gamma)
    exact, _ = O.predict_var(mdl, pred, 0, 0, tol=1e-12, exact_Dl=True)
    draws = np.array([O.predict_var(mdl, pred, 50, s, tol=1e-12)[0] for s in range(40)])
    se = draws.std(0, ddof=1) / math.sqrt(draws.shape[0])
    assert np.all(np.abs(draws.mean(0) - exact) < 4.5 * se + 1e-12)


def test_row_sampled_oracle_equals_assembled_oracle():
    """FSARows (rows on demand, low-rank sums streamed in chunks) gives the
    same pattern rows, values, D_s, operator rows and probe rows as the
    assembled FSA on a problem small enough to assemble."""
    locs = G.uniform_locations(900, 61)
    ind = G.random_subset_inducing(locs, 40, 62)
    theta = (M32, 1.3, 0.08, 0.07)
    gamma = G.taper_range_for_uniform(900, 25)
    full = O.FSA(locs, ind, theta, gamma)
    rows = O.FSARows(locs, ind, theta, gamma, chunk=128)
    idx = np.array([0, 5, 17, 450, 899, 233])
    rp, col, vals, D = rows.value_rows(idx)
    for k, i in enumerate(idx):
        a, b = full.row_ptr[i], full.row_ptr[i + 1]
        assert np.array_equal(col[rp[k]:rp[k + 1]], full.col[a:b])
        np.testing.assert_allclose(vals[rp[k]:rp[k + 1]], full.vals[a:b], rtol=0, atol=1e-13)
    np.testing.assert_allclose(D, full.D[idx], rtol=1e-13)
    X = np.random.default_rng(63).standard_normal((900, 3))
    np.testing.assert_allclose(rows.matvec_rows(idx, X), full.matvec(X)[idx], rtol=0, atol=1e-12)
    np.testing.assert_allclose(rows.probe_rows(idx, 4, 64), O.probes(full, 4, 64)[idx], rtol=0, atol=1e-12)


# ---------------------------------------------------------------- scores (Section 4)

def test_scores_match_definitions():
    """Log-score against scipy's normal log density; the closed-form CRPS
    against its definition, the integral of (F(x) - 1{x >= y})^2 over x,
    by quadrature; RMSE of the means."""
    from scipy import integrate, stats
    rng = np.random.default_rng(3)
    n = 40
    mu = rng.normal(size=n)
    var = rng.uniform(0.05, 2.0, size=n)
    y = mu + rng.normal(size=n) * np.sqrt(var) * 1.5
    ls, crps, rmse = O.scores(y, mu, var)
    assert abs(ls + np.mean(stats.norm.logpdf(y, mu, np.sqrt(var)))) < 1e-12
    c = []
    for i in range(n):
        F = lambda x: stats.norm.cdf(x, mu[i], math.sqrt(var[i]))
        lo, hi = mu[i] - 12 * math.sqrt(var[i]), mu[i] + 12 * math.sqrt(var[i])
        c.append(integrate.quad(lambda x: F(x) ** 2, lo, y[i], epsabs=1e-13, limit=200)[0]
                 + integrate.quad(lambda x: (1.0 - F(x)) ** 2, y[i], hi, epsabs=1e-13, limit=200)[0])
    assert abs(crps - np.mean(c)) < 1e-9
    assert abs(rmse - math.sqrt(np.mean((y - mu) ** 2))) < 1e-15
