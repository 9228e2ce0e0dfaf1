"""Pins of the Vecchia oracle (Section 5) against what the definitions fix.

A Vecchia approximation that conditions every point on all earlier points is
exact; the k nearest earlier points are a brute-force fact; the triangular
solves, the preconditioner and the linear solve are checked against dense
inverses; the log-determinant assembly against a dense slogdet; and the
preconditioned quadrature, run to the full Krylov dimension, against the
dense quadratic form of the matrix logarithm.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.spatial.distance import cdist

from oracle import fsa_oracle as F
from oracle import vecchia_oracle as V
from workloads import generators as G

TH = (F.MATERN32, 1.0, 0.1)


def dense_sigma(locs, theta=TH):
    kind, s1, rho = theta
    return F.covariance(cdist(locs, locs), s1, rho, kind)


def model(n, mv, m=20, seed=0, theta=TH):
    locs = G.uniform_locations(n, seed)
    ind = G.random_subset_inducing(locs, m, seed + 1)
    w = G.laplace_weights(n, seed + 2)
    return V.Vecchia(locs, ind, theta, mv, w)


def sigma_v_dense(M):
    B = M.B.toarray()
    return np.linalg.inv(B.T @ np.diag(1.0 / M.Dv) @ B)


@pytest.mark.parametrize("theta", [TH, (F.EXPONENTIAL, 2.0, 0.3)])
def test_full_conditioning_is_exact(theta):
    """m_v = n - 1: every point conditions on all earlier ones, so
    B^T D^{-1} B is the exact precision Sigma^{-1}."""
    M = model(40, 39, theta=theta)
    S = dense_sigma(M.locs, theta)
    np.testing.assert_allclose(sigma_v_dense(M), S, rtol=1e-8, atol=1e-8)


def test_exact_factor_is_ldl_of_precision():
    """With full conditioning, D_i is the conditional variance of b_i given
    b_0..b_{i-1}: the squared diagonal of the Cholesky factor of Sigma."""
    M = model(30, 29)
    L = np.linalg.cholesky(dense_sigma(M.locs))
    np.testing.assert_allclose(M.Dv, np.diag(L) ** 2, rtol=1e-9)


def test_neighbours_are_the_nearest_earlier_points():
    locs = G.uniform_locations(300, 5)
    mv = 7
    nbr = V.neighbors(locs, mv)
    for i in range(300):
        k = min(mv, i)
        assert np.all(nbr[i, k:] == -1)
        if i == 0:
            continue
        d = cdist(locs[i:i + 1], locs[:i])[0]
        want = np.argsort(d, kind="stable")[:k]
        assert set(nbr[i, :k]) == set(want)
        assert np.all(nbr[i, :k] < i)
        # nearest first
        assert np.all(np.diff(d[nbr[i, :k]]) >= 0)
        # nothing outside the set is nearer than its farthest member
        rest = np.setdiff1d(np.arange(i), nbr[i, :k])
        if rest.size:
            assert d[rest].min() >= d[nbr[i, :k]].max()


def test_neighbour_ties_go_to_the_lower_index():
    locs = np.array([[0.5, 0.5], [0.6, 0.5], [0.4, 0.5], [0.5, 0.6], [0.5, 0.5 + 1e-3]])
    nbr = V.neighbors(locs, 2)
    # point 3 is 0.1 from 0 and about 0.1414 from 1 and 2 (equal): takes 0, then 1
    assert list(nbr[3]) == [0, 1]
    # point 4 is nearest to 0 (1e-3); then 3 is at 0.099 (< 0.1)
    assert list(nbr[4]) == [0, 3]


def test_sigma_v_product_matches_dense_inverse():
    M = model(120, 6)
    X = np.random.default_rng(1).standard_normal((120, 3))
    SV = sigma_v_dense(M)
    np.testing.assert_allclose(M.cov_matvec(X), SV @ X, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(M.prec_matvec(X), np.linalg.solve(SV, X), rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(M.prec_matvec(M.cov_matvec(X)), X, rtol=1e-9, atol=1e-9)


def test_preconditioner_matches_dense_inverse():
    M = model(150, 5, m=25)
    S = dense_sigma(M.locs)
    Sl = M.Smn_T @ np.linalg.solve(M.Sigma_m, M.Smn_T.T)
    P = Sl + np.diag(np.diag(S - Sl) + 1.0 / M.w)
    R = np.random.default_rng(2).standard_normal((150, 4))
    np.testing.assert_allclose(M.precond_solve(R), np.linalg.solve(P, R), rtol=1e-8, atol=1e-9)
    assert abs(M.logdet_P - np.linalg.slogdet(P)[1]) < 1e-8 * abs(M.logdet_P)


def test_printed_equivalent_system_is_not_the_inverse():
    """1 x 1: (1/s + w)^{-1} = s / (1 + s w); the printed form
    w (s + 1/w)^{-1} / s differs, the form used, (s + 1/w)^{-1} s / w, does not."""
    s, w = 0.7, 0.2
    target = 1.0 / (1.0 / s + w)
    printed = w / (s + 1.0 / w) / s
    used = (1.0 / (s + 1.0 / w)) * s / w
    assert abs(printed - target) > 0.1 * target
    assert abs(used - target) < 1e-15


def test_solve_matches_dense():
    M = model(200, 8)
    v = np.random.default_rng(3).standard_normal(200)
    out = V.solve_logdet(M, v, 4, seed=11, tol=1e-12, max_iter=400)
    A = np.linalg.inv(sigma_v_dense(M)) + np.diag(M.w)
    np.testing.assert_allclose(out["x"], np.linalg.solve(A, v), rtol=1e-8, atol=1e-9)


def test_logdet_assembly_matches_dense():
    M = model(160, 6)
    SV = sigma_v_dense(M)
    lhs = np.linalg.slogdet(np.linalg.inv(SV) + np.diag(M.w))[1]
    rhs = M.logdet_offset() + np.linalg.slogdet(SV + np.diag(1.0 / M.w))[1]
    assert abs(lhs - rhs) < 1e-9 * abs(lhs)


def test_quadrature_exact_at_full_dimension():
    """With the Lanczos run to the full dimension, w_i e_1^T log(T_i) e_1
    = u_i^T log(P^{-1/2} K P^{-1/2}) u_i, u_i = P^{-1/2} z_i."""
    n = 50
    M = model(n, 4, m=8)
    K = sigma_v_dense(M) + np.diag(1.0 / M.w)
    S = dense_sigma(M.locs)
    Sl = M.Smn_T @ np.linalg.solve(M.Sigma_m, M.Smn_T.T)
    P = Sl + np.diag(np.diag(S - Sl) + 1.0 / M.w)
    lamP, QP = np.linalg.eigh(P)
    Pmh = QP @ np.diag(lamP ** -0.5) @ QP.T
    lam, Q = np.linalg.eigh(Pmh @ K @ Pmh)
    logM = Q @ np.diag(np.log(lam)) @ Q.T
    out = V.solve_logdet(M, np.ones(n), 3, seed=4, tol=1e-14, max_iter=n)
    Z = out["B"][:, 1:]
    for i in range(3):
        u = Pmh @ Z[:, i]
        assert abs(out["slq_terms"][i] - u @ logM @ u) < 1e-7 * abs(u @ logM @ u) + 1e-9


def test_slq_estimate_near_dense_logdet():
    """Many probes: the estimate lands within a few standard errors."""
    M = model(300, 8, m=30)
    SV = sigma_v_dense(M)
    exact = np.linalg.slogdet(np.linalg.inv(SV) + np.diag(M.w))[1]
    out = V.solve_logdet(M, np.ones(300), 200, seed=9, tol=1e-10, max_iter=300)
    se = np.std(out["slq_terms"]) / np.sqrt(200)
    assert abs(out["logdet"] - exact) < 4 * se + 1e-8


# ---------------------------------------------------------------- Vecchia-Laplace (Bernoulli-logit)
def bernoulli_case(n=180, mv=8, m=20, seed=3, theta=TH):
    locs = G.uniform_locations(n, seed)
    ind = G.random_subset_inducing(locs, m, seed + 1)
    M = V.Vecchia(locs, ind, theta, mv, np.full(n, 0.25))
    rng = np.random.default_rng(seed + 2)
    # responses from a smooth latent field, so the mode is not trivial
    field = np.sin(6 * locs[:, 0]) + np.cos(5 * locs[:, 1])
    y = (rng.uniform(size=n) < 1.0 / (1.0 + np.exp(-2.0 * field))).astype(np.float64)
    return M, y


def test_laplace_mode_matches_a_general_optimizer():
    """The Newton/CG mode equals the minimiser of -log p(y|b) + b^T Q b / 2
    (Q = B^T D^{-1} B) found by scipy's trust-region method on the dense
    objective."""
    from scipy.optimize import minimize
    M, y = bernoulli_case()
    Q = (M.B.T @ sp_diag(1.0 / M.Dv) @ M.B).toarray()

    def f(b):
        return -V.bernoulli_loglik(y, b) + 0.5 * b @ Q @ b

    def g(b):
        return -(y - V.logistic(b)) + Q @ b

    def h(b):
        p = V.logistic(b)
        return Q + np.diag(p * (1 - p))

    opt = minimize(f, np.zeros(M.n), jac=g, hess=h, method="trust-exact", options={"gtol": 1e-12})
    out = V.laplace(M, y, 4, seed=1, tol=1e-13, max_iter=500, newton_tol=1e-12)
    assert out["converged"]
    assert np.linalg.norm(out["mode"] - opt.x) <= 1e-8 * np.linalg.norm(opt.x)


def sp_diag(v):
    import scipy.sparse as sp
    return sp.diags(v)


def test_laplace_mode_is_stationary():
    """At the mode, Sigma_V^{-1} b = y - pi(b) (checked with the sparse
    factor, no solve)."""
    M, y = bernoulli_case(seed=5, theta=(F.EXPONENTIAL, 1.5, 0.2))
    out = V.laplace(M, y, 4, seed=2, tol=1e-13, max_iter=500, newton_tol=1e-12)
    b = out["mode"]
    r = M.prec_matvec(b) - (y - V.logistic(b))
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(y - V.logistic(b))


def test_laplace_nll_matches_dense_laplace():
    """NLL = -log p(y|b) + b^T Sigma_V^{-1} b / 2 + log det(I + Sigma_V W) / 2:
    its deterministic part equals the dense evaluation, and the SLQ term lands
    within a few standard errors of the dense log-determinant."""
    M, y = bernoulli_case(n=240, seed=7)
    t = 400
    out = V.laplace(M, y, t, seed=3, tol=1e-12, max_iter=500, newton_tol=1e-12)
    b = out["mode"]
    B = M.B.toarray()
    SV = np.linalg.inv(B.T @ np.diag(1.0 / M.Dv) @ B)
    p = V.logistic(b)
    W = p * (1 - p)
    exact_ld = np.linalg.slogdet(np.eye(M.n) + SV * W[None, :])[1]
    quad = b @ np.linalg.solve(SV, b)
    det_part = -V.bernoulli_loglik(y, b) + 0.5 * quad
    assert abs(out["quad"] - quad) <= 1e-8 * abs(quad)
    assert abs(-out["loglik"] + 0.5 * out["quad"] - det_part) <= 1e-10 * abs(det_part)
    # log det(I + Sigma_V W) = sum log D + log det(Sigma_V^{-1} + W)
    se = np.std(out["slq_terms"]) / np.sqrt(t)
    assert abs(out["sum_log_d"] + out["logdet"] - exact_ld) < 4 * se + 1e-8
    exact_nll = det_part + 0.5 * exact_ld
    assert abs(out["nll"] - exact_nll) < 2 * se + 1e-8


def test_laplace_one_point_is_the_textbook_formula():
    """n = 1: the Laplace approximation of int p(y|b) N(b; 0, s) db is
    p(y|b*) N(b*; 0, s) sqrt(2 pi / H), H = 1/s + pi (1 - pi) at the mode b*,
    which solves b/s = y - pi(b) (found here by bisection)."""
    s = 1.7
    locs = np.array([[0.3, 0.6]])
    M = V.Vecchia(locs, locs, (F.EXPONENTIAL, s, 0.2), 0, np.array([0.25]))
    for yv in (0.0, 1.0):
        y = np.array([yv])
        lo, hi = -20.0, 20.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid / s - (yv - V.logistic(mid)) > 0:
                hi = mid
            else:
                lo = mid
        bs = 0.5 * (lo + hi)
        p = V.logistic(bs)
        H = 1.0 / s + p * (1 - p)
        log_lp = yv * bs - np.logaddexp(0.0, bs) - 0.5 * np.log(2 * np.pi * s) - bs * bs / (2 * s)
        textbook = -(log_lp + 0.5 * np.log(2 * np.pi / H))
        out = V.laplace(M, y, 1, seed=0, tol=1e-14, max_iter=5, newton_tol=1e-14)
        assert abs(out["mode"][0] - bs) < 1e-10
        assert abs(out["nll"] - textbook) < 1e-10 * abs(textbook)
