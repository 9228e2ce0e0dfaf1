"""GPU parity of the Vecchia path (Section 5) against the oracle.

The neighbour lists are integer results decided by float64 squared
distances evaluated the same way on both sides: they must agree exactly,
order included.  The coefficients A_i solve Sigma_{N(i)} a = Sigma_{N(i),i}
by different factorizations on the two sides (Cholesky here, LU in the
oracle): each is allowed 64 eps cond(Sigma_{N(i)}) |a|, the first-order
bound of the rounding of a backward-stable solve.  Products and solves are
compared relative to the size of the result; the PCG runs compare iteration
counts and the SLQ log-determinant on the same probes.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import fsa_oracle as F
from oracle import vecchia_oracle as VO
from workloads import generators as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = np.finfo(np.float64).eps


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _case(n, mv, m, seed, rho=0.05, clustered=False):
    locs = G.clustered_locations(n, seed) if clustered else G.uniform_locations(n, seed)
    ind = G.random_subset_inducing(locs, m, seed + 1)
    w = G.laplace_weights(n, seed + 2)
    return locs, ind, w, (F.MATERN32, 1.0, rho)


def _gpu(locs, ind, w, th, mv):
    from paper_2405_14492_amd import fsa
    return fsa.Vecchia(_dev(locs), _dev(ind), th[0], th[1], th[2], mv, _dev(w))


def _coef_tol(locs, nbr, coef, theta):
    kind, s1, rho = theta
    tol = np.zeros_like(coef)
    for i in range(nbr.shape[0]):
        N = nbr[i][nbr[i] >= 0]
        if N.size == 0:
            continue
        SN = F.covariance(cdist(locs[N], locs[N]), s1, rho, kind)
        tol[i, :N.size] = 64 * EPS * np.linalg.cond(SN) * np.abs(coef[i, :N.size]).max()
    return tol


@pytest.mark.parametrize("n,mv,m,clustered", [(3000, 30, 64, False), (2500, 10, 40, True), (700, 32, 20, False)])
def test_factor_matches_oracle(n, mv, m, clustered):
    locs, ind, w, th = _case(n, mv, m, seed=7, clustered=clustered)
    nbr_o = VO.neighbors(locs, mv)
    coef_o, D_o = VO.factor(locs, nbr_o, th)
    with _gpu(locs, ind, w, th, mv) as v:
        nbr, coef, D = (t.cpu().numpy() for t in v.factor())
    assert np.array_equal(nbr.astype(np.int64), nbr_o)
    tol = _coef_tol(locs, nbr_o, coef_o, th)
    assert np.all(np.abs(coef - coef_o) <= tol + 1e-300)
    # D_i = sigma1^2 - a . s: the same bound scaled by |s| ~ sigma1^2
    np.testing.assert_allclose(D, D_o, rtol=0, atol=float(tol.max()) * mv + 64 * EPS)


@pytest.mark.parametrize("which", [0, 1, 2, 3])
def test_products_match_oracle(which):
    from paper_2405_14492_amd import fsa
    n, mv, m = 2000, 12, 48
    locs, ind, w, th = _case(n, mv, m, seed=3)
    M = VO.Vecchia(locs, ind, th, mv, w)
    X = np.random.default_rng(5).standard_normal((n, 7))
    ref = {fsa.V_SIGMA: M.cov_matvec, fsa.V_PRECISION: M.prec_matvec, fsa.V_OPERATOR: M.matvec,
           fsa.V_P_INV: M.precond_solve}[which](X)
    with _gpu(locs, ind, w, th, mv) as v:
        Y = v.apply(which, _dev(X)).cpu().numpy()
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err < 1e-9, err


@pytest.mark.parametrize("ncols", [64, 65, 130])
def test_sigma_product_over_64_columns(ncols):
    """Blocks wider than one 64-lane pass of the triangular solves: each pass
    reads its own slice of the point's row and reuses the list, on the
    one-point levels (one workgroup, point after point) and on the others."""
    from paper_2405_14492_amd import fsa
    n, mv, m = 1200, 30, 32
    locs, ind, w, th = _case(n, mv, m, seed=17, clustered=True)
    M = VO.Vecchia(locs, ind, th, mv, w)
    X = np.random.default_rng(8).standard_normal((n, ncols))
    ref = M.cov_matvec(X)
    with _gpu(locs, ind, w, th, mv) as v:
        Y = v.apply(fsa.V_SIGMA, _dev(X)).cpu().numpy()
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err < 1e-9, err


def test_chain_of_one_point_levels():
    """Points in order along a line: each point's nearest earlier points are
    the ones just before it, so every level holds one point (n levels) and
    each pass of the triangular solves is one stretch, one workgroup walking
    all n points."""
    from paper_2405_14492_amd import fsa
    n, mv = 400, 5
    x = np.linspace(0.0, 1.0, n)
    locs = np.column_stack([x, np.full(n, 0.5)])
    ind = locs[::25][:16].copy()
    w = G.laplace_weights(n, 4)
    th = (F.MATERN32, 1.0, 0.01)
    M = VO.Vecchia(locs, ind, th, mv, w)
    X = np.random.default_rng(6).standard_normal((n, 3))
    ref = M.cov_matvec(X)
    with _gpu(locs, ind, w, th, mv) as v:
        Y = v.apply(fsa.V_SIGMA, _dev(X)).cpu().numpy()
        _, _, st = v.solve_logdet(_dev(X[:, 0]), 2, seed=1, fixed_iter=3)
    assert st["nlevels"] == n
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err < 1e-9, err


def test_products_are_inverse_of_each_other():
    from paper_2405_14492_amd import fsa
    n, mv, m = 1500, 20, 30
    locs, ind, w, th = _case(n, mv, m, seed=9, clustered=True)
    X = _dev(np.random.default_rng(1).standard_normal((n, 3)))
    with _gpu(locs, ind, w, th, mv) as v:
        Y = v.apply(fsa.V_PRECISION, v.apply(fsa.V_SIGMA, X))
    assert float((Y - X).abs().max() / X.abs().max()) < 1e-8


@pytest.mark.parametrize("n,mv,m,t,clustered", [(3000, 10, 64, 8, False), (1800, 30, 40, 5, True),
                                                 (257, 4, 16, 3, False)])
def test_solve_logdet_matches_oracle(n, mv, m, t, clustered):
    locs, ind, w, th = _case(n, mv, m, seed=11, clustered=clustered)
    vv = np.random.default_rng(2).standard_normal(n)
    M = VO.Vecchia(locs, ind, th, mv, w)
    o = VO.solve_logdet(M, vv, t, seed=21, tol=1e-8, max_iter=2000)
    with _gpu(locs, ind, w, th, mv) as v:
        x, logdet, st = v.solve_logdet(_dev(vv), t, 21, tol=1e-8, max_iter=2000)
    x = x.cpu().numpy()
    assert st["converged"] == 1
    assert abs(st["iters_rhs"] - int(o["iters"][0])) <= 1
    assert abs(st["iters_max"] - int(o["iters"].max())) <= 1
    assert abs(st["logdet_P"] - o["logdet_P"]) < 1e-10 * abs(o["logdet_P"])
    assert abs(st["logdet_offset"] - M.logdet_offset()) < 1e-10 * abs(M.logdet_offset())
    # both sides stop at ||r|| < 1e-8 ||b||: the solutions differ by about
    # that times the conditioning of the system
    np.testing.assert_allclose(x, o["x"], rtol=0, atol=1e-6 * np.abs(o["x"]).max())
    assert abs(logdet - o["logdet"]) < 1e-6 * abs(o["logdet"])


@pytest.mark.parametrize("n,mv,m,t,k,clustered", [(3000, 10, 64, 8, 12, False), (1800, 30, 40, 5, 20, True),
                                                   (257, 4, 16, 3, 7, False)])
def test_solve_logdet_fixed_iterations_match_oracle(n, mv, m, t, k, clustered):
    """With a fixed iteration count both sides run the same Krylov
    sequence on the same probes, so the float64 results agree to the
    method's 1e-9: the solution, the SLQ estimate of log det(Sigma_V +
    W^{-1}) and the log det of Sigma_V^{-1} + W."""
    locs, ind, w, th = _case(n, mv, m, seed=13, clustered=clustered)
    vv = np.random.default_rng(4).standard_normal(n)
    M = VO.Vecchia(locs, ind, th, mv, w)
    o = VO.solve_logdet(M, vv, t, seed=23, fixed_iter=k)
    with _gpu(locs, ind, w, th, mv) as v:
        x, logdet, st = v.solve_logdet(_dev(vv), t, 23, fixed_iter=k)
    x = x.cpu().numpy()
    assert st["iters_rhs"] == k and st["iters_max"] == k and st["probe_iters"] == k * (t + 1)
    xerr = np.abs(x - o["x"]).max() / np.abs(o["x"]).max()
    swerr = abs(st["logdet_sw"] - o["logdet_sw"]) / abs(o["logdet_sw"])
    lerr = abs(logdet - o["logdet"]) / abs(o["logdet"])
    print("x", xerr, "logdet_sw", swerr, "logdet", lerr, flush=True)
    assert xerr < 1e-9
    assert swerr < 1e-9
    assert lerr < 1e-9


def _transformed_residual(v, fsa, x, w, vv):
    """The CG runs on (Sigma_V + W^{-1}) u = Sigma_V v with u = W x and
    stops on that residual; (Sigma_V^{-1} + W) x - v is Sigma_V^{-1} times
    it, amplified by |Sigma_V^{-1}| ~ 1 / min D_i."""
    b = v.apply(fsa.V_SIGMA, vv)
    r = v.apply(fsa.V_OPERATOR, _dev(w) * x) - b
    return float(r.norm() / b.norm())


def test_solve_residual_small():
    from paper_2405_14492_amd import fsa
    n, mv, m = 2000, 15, 40
    locs, ind, w, th = _case(n, mv, m, seed=4)
    vv = _dev(np.random.default_rng(8).standard_normal(n))
    with _gpu(locs, ind, w, th, mv) as v:
        x, _, _ = v.solve_logdet(vv, 2, 3, tol=1e-10, max_iter=3000)
        rel = _transformed_residual(v, fsa, x, w, vv)
        r = v.apply(fsa.V_PRECISION, x) + _dev(w) * x - vv
        D = v.factor()[2]
    # the recurrence residual is below 1e-10; the true one drifts a little
    assert rel < 1e-9, rel
    assert float(r.norm() / vv.norm()) < 1e-9 / float(D.min()), float(r.norm() / vv.norm())


@pytest.mark.parametrize("n,mv", [(1, 30), (2, 30), (40, 0), (33, 32)])
def test_degenerate_sizes(n, mv):
    from paper_2405_14492_amd import fsa
    m = min(n, 8)
    locs, ind, w, th = _case(n, mv, m, seed=13)
    nbr_o = VO.neighbors(locs, mv)
    coef_o, D_o = VO.factor(locs, nbr_o, th)
    M = VO.Vecchia(locs, ind, th, mv, w)
    X = np.random.default_rng(3).standard_normal((n, 2))
    with _gpu(locs, ind, w, th, mv) as v:
        nbr, coef, D = (t.cpu().numpy() for t in v.factor())
        Y = v.apply(fsa.V_SIGMA, _dev(X)).cpu().numpy()
    assert np.array_equal(nbr.astype(np.int64).reshape(n, mv), nbr_o)
    np.testing.assert_allclose(D, D_o, rtol=1e-9)
    np.testing.assert_allclose(Y, M.cov_matvec(X), rtol=1e-9, atol=1e-12)
    if mv == 0:  # no conditioning: Sigma_V = sigma1^2 I
        np.testing.assert_allclose(Y, X * th[1], rtol=1e-15)


def test_invalid_arguments():
    from paper_2405_14492_amd import fsa
    locs, ind, w, th = _case(50, 5, 8, seed=1)
    with pytest.raises(fsa.FsaError):
        fsa.Vecchia(_dev(locs), _dev(ind), th[0], th[1], th[2], 33, _dev(w))
    w_bad = w.copy()
    w_bad[7] = 0.0
    with pytest.raises(fsa.FsaError):
        fsa.Vecchia(_dev(locs), _dev(ind), th[0], th[1], th[2], 5, _dev(w_bad))
    with pytest.raises(fsa.FsaError):
        fsa.Vecchia(_dev(locs), _dev(ind[:0]), th[0], th[1], th[2], 5, _dev(w))
    with _gpu(locs, ind, w, th, 5) as v:
        with pytest.raises(fsa.FsaError):
            v.solve_logdet(_dev(np.ones(50)), 0, 1)
        with pytest.raises(fsa.FsaError):
            v.apply(9, _dev(np.ones((50, 2))))


def test_fullsize_sampled_rows_and_identities():
    """n = 100,000, m_v = 30, m = 200, 50 probes (the Section 5 setting):
    sampled neighbour rows and coefficients against the oracle computed row
    by row, the precision/covariance products as inverses, and the solve's
    residual."""
    from paper_2405_14492_amd import fsa
    n, mv, m, t = 100_000, 30, 200, 50
    locs, ind, w, th = _case(n, mv, m, seed=17, rho=0.05)
    rows = np.random.default_rng(0).choice(n, 40, replace=False)
    rows = np.concatenate([[0, 1, 29, 30, 31, n - 1], rows])
    nbr_o = VO.neighbors(locs, mv, rows)
    coef_o, D_o = VO.factor(locs, nbr_o, th, rows)
    vv = _dev(np.random.default_rng(8).standard_normal(n))
    with _gpu(locs, ind, w, th, mv) as v:
        nbr, coef, D = (t_.cpu().numpy() for t_ in v.factor())
        assert np.array_equal(nbr[rows].astype(np.int64), nbr_o)
        tol = _coef_tol(locs, nbr_o, coef_o, th)
        assert np.all(np.abs(coef[rows] - coef_o) <= tol + 1e-300)
        X = _dev(np.random.default_rng(2).standard_normal((n, 4)))
        Y = v.apply(fsa.V_PRECISION, v.apply(fsa.V_SIGMA, X))
        # the round trip (two triangular solves, two products) loses digits in
        # proportion to the conditioning of B: at this density the A_i of the
        # Matern-3/2 covariance reach O(10) with cancelling signs (1e-6
        # measured); a wrong coefficient, order or schedule gives O(1)
        assert float((Y - X).abs().max() / X.abs().max()) < 1e-5
        x, logdet, st = v.solve_logdet(vv, t, 5, tol=1e-6, max_iter=3000)
        rel = _transformed_residual(v, fsa, x, w, vv)
    assert st["converged"] == 1
    assert rel < 1e-5, rel
    assert np.isfinite(logdet)


def test_exponential_covariance_matches_oracle():
    n, mv, m, t = 1500, 12, 32, 4
    locs = G.uniform_locations(n, 31)
    ind = G.random_subset_inducing(locs, m, 32)
    w = G.laplace_weights(n, 33)
    th = (F.EXPONENTIAL, 1.5, 0.1)
    nbr_o = VO.neighbors(locs, mv)
    coef_o, D_o = VO.factor(locs, nbr_o, th)
    M = VO.Vecchia(locs, ind, th, mv, w)
    vv = np.random.default_rng(4).standard_normal(n)
    o = VO.solve_logdet(M, vv, t, seed=7, tol=1e-8, max_iter=2000)
    with _gpu(locs, ind, w, th, mv) as v:
        nbr, coef, D = (t_.cpu().numpy() for t_ in v.factor())
        x, logdet, st = v.solve_logdet(_dev(vv), t, 7, tol=1e-8, max_iter=2000)
    assert np.array_equal(nbr.astype(np.int64), nbr_o)
    assert np.all(np.abs(coef - coef_o) <= _coef_tol(locs, nbr_o, coef_o, th) + 1e-300)
    np.testing.assert_allclose(D, D_o, rtol=1e-9)
    assert abs(st["iters_rhs"] - int(o["iters"][0])) <= 1
    np.testing.assert_allclose(x.cpu().numpy(), o["x"], rtol=0, atol=1e-6 * np.abs(o["x"]).max())
    assert abs(logdet - o["logdet"]) < 1e-6 * abs(o["logdet"])


def test_solution_does_not_depend_on_the_probes():
    """Every column runs CG on its own scalars, so the right-hand side's
    column comes out the same whatever probes share the block."""
    n, mv, m = 1200, 10, 24
    locs, ind, w, th = _case(n, mv, m, seed=41)
    vv = _dev(np.random.default_rng(5).standard_normal(n))
    with _gpu(locs, ind, w, th, mv) as v:
        x1, l1, s1 = v.solve_logdet(vv, 3, 1, tol=1e-9, max_iter=2000)
        x2, l2, s2 = v.solve_logdet(vv, 9, 2, tol=1e-9, max_iter=2000)
    assert s1["iters_rhs"] == s2["iters_rhs"]
    assert torch.equal(x1, x2)
    assert l1 != l2


def test_side_stream():
    """Built and run on a caller's non-default stream: bitwise the same
    results (every sum has a fixed order, and the points of a level take their
    positions in index order on every build)."""
    from paper_2405_14492_amd import fsa
    n, mv, m = 900, 8, 16
    locs, ind, w, th = _case(n, mv, m, seed=43)
    X = _dev(np.random.default_rng(6).standard_normal((n, 3)))
    vv = _dev(np.random.default_rng(7).standard_normal(n))
    with _gpu(locs, ind, w, th, mv) as v:
        Y0 = v.apply(fsa.V_SIGMA, X)
        x0, l0, _ = v.solve_logdet(vv, 4, 3, tol=1e-9)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dl, di, dw = _dev(locs), _dev(ind), _dev(w)
        s.synchronize()
        with fsa.Vecchia(dl, di, th[0], th[1], th[2], mv, dw, stream=s) as v:
            Y1 = v.apply(fsa.V_SIGMA, X)
            x1, l1, _ = v.solve_logdet(vv, 4, 3, tol=1e-9)
        s.synchronize()
    assert torch.equal(Y0, Y1)
    assert torch.equal(x0, x1)
    assert l0 == l1
