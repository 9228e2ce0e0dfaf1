"""CPU FP64 oracle for the full-scale-approximation (FSA) iterative path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this module; the product path
never calls it.  It shares no code with the HIP path: it builds the
covariance, the taper pattern, the FITC preconditioner, the preconditioned
CG with Lanczos coefficients, the SLQ log-determinant, the stochastic
gradient and the simulation-based predictive variances from the paper's
definitions, in plain numpy/scipy, in float64.

Paper: Gyger, Furrer & Sigrist, "Iterative Methods for Full-Scale Gaussian
Process Approximations for Large Spatial Data" (arXiv 2405.14492).

Readings where the paper is silent (each also listed in the design notes):
  * covariance: Matérn 1/2 is sigma1^2 exp(-d/rho); Matérn 3/2 is
    sigma1^2 (1 + sqrt3 d/rho) exp(-sqrt3 d/rho), whose 0.05-correlation
    distance is 2.74 rho, matching the "rho ~ effective range / 2.7" of
    Section 4;
  * taper: Wendland (1-r)^4_+ (1+4r), r = d/gamma, zero for d >= gamma as
    Section 2.1 requires; a pair is kept iff dx*dx + dy*dy < gamma*gamma in
    float64 with no fused multiply-add;
  * probes: z = Sigma_mn^T L_m^{-T} e + D_s^{1/2} rho (the sampling recipe
    of Appendix F) with Rademacher e and rho, so Cov z = P exactly;
  * Rademacher signs: top bit of the c-th output of SplitMix64 (Steele, Lea
    & Flood 2014) keyed by the seed, c = stream<<60 | column<<40 | index;
  * SLQ weight: z^T P^{-1} z by default (the exact quadrature weight), the
    paper's n on request;
  * CG stopping: per column ||r|| / ||b|| < tol, converged columns frozen;
  * Algorithm 1: Sigma~_dagger^{-1} Sigma_mn^T is taken as V M^{-1} Sigma_m
    with V = Sigma~_s^{-1} Sigma_mn^T (an identity of eq. SWMFSA).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist

EXPONENTIAL = 0
MATERN32 = 1

SQRT3 = math.sqrt(3.0)

# ---------------------------------------------------------------------------
# Covariance function and taper (Section 2, Section 2.1)
# ---------------------------------------------------------------------------


# A control-variate coefficient is taken as 0 when its b_i hardly vary: the
# centred sum of squares at most this fraction of sum_i b_i^2 (then any c
# leaves the estimate unchanged up to rounding, and the ratio is noise).
CV_DEGENERATE = 1e-12


def covariance(d, sigma1_sq, rho, kind):
    """c(s_i, s_j) as a function of the Euclidean distance d (Section 2;
    Assumption 3 form sigma1^2 r(d) with r(0) = 1)."""
    d = np.asarray(d, dtype=np.float64)
    if kind == EXPONENTIAL:
        return sigma1_sq * np.exp(-d / rho)
    x = SQRT3 * d / rho
    return sigma1_sq * (1.0 + x) * np.exp(-x)


def covariance_dsigma1(d, sigma1_sq, rho, kind):
    """Partial derivative of c with respect to sigma1^2."""
    return covariance(d, 1.0, rho, kind)


def covariance_drho(d, sigma1_sq, rho, kind):
    """Partial derivative of c with respect to the range rho."""
    d = np.asarray(d, dtype=np.float64)
    if kind == EXPONENTIAL:
        return sigma1_sq * (d / (rho * rho)) * np.exp(-d / rho)
    x = SQRT3 * d / rho
    return sigma1_sq * (x * x / rho) * np.exp(-x)


def wendland_taper(d, gamma):
    """Compactly supported correlation c_taper(d; gamma), zero for d >= gamma
    (Section 2.1)."""
    r = np.asarray(d, dtype=np.float64) / gamma
    w = (1.0 - r) ** 4 * (1.0 + 4.0 * r)
    return np.where(r < 1.0, w, 0.0)


def taper_pattern(row_locs, col_locs, gamma):
    """Nonzero pattern of T(gamma) between two point sets (Section 2.1):
    pair (i, j) is kept iff (x_i-x_j)^2 + (y_i-y_j)^2 < gamma^2 in float64.

    Candidates come from a k-d tree with a slightly larger radius; the exact
    predicate decides.  Returns CSR (row_ptr int64, col int32) with columns
    ascending; the diagonal is included when both sets are the same."""
    row_locs = np.ascontiguousarray(row_locs, dtype=np.float64)
    col_locs = np.ascontiguousarray(col_locs, dtype=np.float64)
    nr = row_locs.shape[0]
    ta = cKDTree(row_locs)
    tb = cKDTree(col_locs)
    pairs = ta.sparse_distance_matrix(tb, gamma * (1.0 + 1e-6), output_type="ndarray")
    i = pairs["i"].astype(np.int64)
    j = pairs["j"].astype(np.int64)
    dx = row_locs[i, 0] - col_locs[j, 0]
    dy = row_locs[i, 1] - col_locs[j, 1]
    keep = (dx * dx + dy * dy) < gamma * gamma
    i, j = i[keep], j[keep]
    order = np.lexsort((j, i))
    i, j = i[order], j[order]
    row_ptr = np.zeros(nr + 1, dtype=np.int64)
    np.cumsum(np.bincount(i, minlength=nr), out=row_ptr[1:])
    return row_ptr, j.astype(np.int32)


def taper_pattern_bruteforce(row_locs, col_locs, gamma):
    """The same predicate over all pairs (for small inputs)."""
    dx = row_locs[:, 0][:, None] - col_locs[:, 0][None, :]
    dy = row_locs[:, 1][:, None] - col_locs[:, 1][None, :]
    keep = (dx * dx + dy * dy) < gamma * gamma
    i, j = np.nonzero(keep)
    row_ptr = np.zeros(row_locs.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(i, minlength=row_locs.shape[0]), out=row_ptr[1:])
    return row_ptr, j.astype(np.int32)


def _pair_dots(X, Y, rows, cols, chunk=1 << 16):
    """sum_k X[rows[p], k] * Y[cols[p], k] for each pair p (X, Y stored
    point-major, n x m)."""
    out = np.empty(rows.shape[0])
    for s in range(0, rows.shape[0], chunk):
        out[s:s + chunk] = np.einsum("ij,ij->i", X[rows[s:s + chunk]], Y[cols[s:s + chunk]])
    return out


def _pair_dist(A, B, rows, cols):
    dx = A[rows, 0] - B[cols, 0]
    dy = A[rows, 1] - B[cols, 1]
    return np.sqrt(dx * dx + dy * dy)


# ---------------------------------------------------------------------------
# Counter-based Rademacher signs (SplitMix64)
# ---------------------------------------------------------------------------

_SM_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_SM_M1 = np.uint64(0xBF58476D1CE4E5B9)
_SM_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, counter):
    """The (counter+1)-th output of SplitMix64 started from state `seed`
    (Steele, Lea & Flood 2014): state = seed + (counter+1) * 0x9E37...15,
    then the variant-13 finaliser."""
    with np.errstate(over="ignore"):
        c = np.asarray(counter, dtype=np.uint64)
        z = np.uint64(seed) + (c + np.uint64(1)) * _SM_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _SM_M1
        z = (z ^ (z >> np.uint64(27))) * _SM_M2
        return z ^ (z >> np.uint64(31))


STREAM_RHO, STREAM_E, STREAM_PRED = 0, 1, 2


def rademacher_rows(seed, stream, rows, n_cols):
    """Rows `rows` of the +-1 matrix: entry (i, c) is +1 iff the top bit of
    splitmix64(seed, stream<<60 | c<<40 | i) is 0."""
    i = np.asarray(rows, dtype=np.uint64)[:, None]
    c = np.arange(n_cols, dtype=np.uint64)[None, :]
    ctr = (np.uint64(stream) << np.uint64(60)) | (c << np.uint64(40)) | i
    top = splitmix64(seed, ctr) >> np.uint64(63)
    return 1.0 - 2.0 * top.astype(np.float64)


def rademacher(seed, stream, n_rows, n_cols):
    """(n_rows, n_cols) matrix of +-1 (rows 0 .. n_rows-1 of rademacher_rows)."""
    return rademacher_rows(seed, stream, np.arange(n_rows), n_cols)


# ---------------------------------------------------------------------------
# The FSA covariance and the FITC preconditioner (Sections 2.1, 3.3, App. F)
# ---------------------------------------------------------------------------


class FSA:
    """Sigma~_dagger = Sigma_mn^T Sigma_m^{-1} Sigma_mn + Sigma_s + sigma^2 I
    (Section 2.1) with its FITC preconditioner (eq. eqfitcp)."""

    def __init__(self, locs, inducing, theta, gamma, jitter=0.0, smn_T=None):
        """smn_T: the n x m matrix to take as Sigma_mn^T in place of the
        covariance between locations and inducing points (default).  The
        construction of Section 2.1 holds for any such matrix; tests use it
        for a model whose low-rank part was rounded.  The derivatives keep
        the exact dSigma_mn/dtheta."""
        kind, s1, rho, s2 = theta
        self.locs = np.ascontiguousarray(locs, dtype=np.float64)
        self.inducing = np.ascontiguousarray(inducing, dtype=np.float64)
        self.theta = (int(kind), float(s1), float(rho), float(s2))
        self.gamma = float(gamma)
        self.jitter = float(jitter)
        n, m = self.locs.shape[0], self.inducing.shape[0]
        self.n, self.m = n, m
        # Sigma_m (m x m) and Sigma_mn, stored point-major as Sigma_mn^T (n x m).
        self.Sigma_m = covariance(cdist(self.inducing, self.inducing), s1, rho, kind)
        self.Sigma_m[np.diag_indices(m)] += jitter * s1
        if smn_T is None:
            self.Smn_T = covariance(cdist(self.locs, self.inducing), s1, rho, kind)
        else:
            self.Smn_T = np.ascontiguousarray(smn_T, dtype=np.float64)
            if self.Smn_T.shape != (n, m):
                raise ValueError("smn_T must be n x m")
        self.chol_m = sla.cho_factor(self.Sigma_m, lower=True)
        # K = Sigma_m^{-1} Sigma_mn, stored point-major as K^T (n x m).
        self.K_T = np.ascontiguousarray(sla.cho_solve(self.chol_m, self.Smn_T.T).T)
        # Taper pattern and the residual values (Sigma - Sigma_l) o T + sigma^2 I.
        self.row_ptr, self.col = taper_pattern(self.locs, self.locs, self.gamma)
        self.rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(self.row_ptr))
        cols = self.col.astype(np.int64)
        self.pair_d = _pair_dist(self.locs, self.locs, self.rows, cols)
        self.pair_w = wendland_taper(self.pair_d, self.gamma)
        low = _pair_dots(self.Smn_T, self.K_T, self.rows, cols)
        vals = (covariance(self.pair_d, s1, rho, kind) - low) * self.pair_w
        self.is_diag = self.rows == cols
        vals[self.is_diag] += s2
        self.vals = vals
        self.S = sp.csr_matrix((vals, self.col, self.row_ptr), shape=(n, n))
        self.D = vals[self.is_diag].copy()
        if self.D.shape[0] != n:
            raise ValueError("diagonal missing from the taper pattern")
        # FITC: P = D_s + Sigma_mn^T Sigma_m^{-1} Sigma_mn (eq. eqfitcp); its
        # Woodbury matrix Sigma_m + Sigma_mn D_s^{-1} Sigma_mn^T (App. F).
        self.M_P = self.Sigma_m + self.Smn_T.T @ (self.Smn_T / self.D[:, None])
        self.chol_P = sla.cho_factor(self.M_P, lower=True)
        # log det P by Sylvester's theorem (App. F).
        self.logdet_P = (2.0 * np.sum(np.log(np.diag(self.chol_P[0])))
                         - 2.0 * np.sum(np.log(np.diag(self.chol_m[0])))
                         + np.sum(np.log(self.D)))
        self._dcache = {}

    # -- operators ---------------------------------------------------------
    def lowrank_matvec(self, X):
        """Sigma_mn^T Sigma_m^{-1} Sigma_mn X."""
        return self.Smn_T @ sla.cho_solve(self.chol_m, self.Smn_T.T @ X)

    def sparse_matvec(self, X):
        """Sigma~_s X."""
        return self.S @ X

    def matvec(self, X):
        """Sigma~_dagger X, O(n (m + n_gamma)) per column (Section 3.1)."""
        return self.sparse_matvec(X) + self.lowrank_matvec(X)

    def precond_solve(self, R):
        """P^{-1} R by the Sherman-Woodbury-Morrison formula (App. F)."""
        DR = R / self.D[:, None] if R.ndim == 2 else R / self.D
        t = sla.cho_solve(self.chol_P, self.Smn_T.T @ DR)
        corr = self.Smn_T @ t
        return DR - (corr / self.D[:, None] if R.ndim == 2 else corr / self.D)

    def diag_solve(self, R):
        """P_s^{-1} R with P_s = D_s (Section 3.3)."""
        return R / self.D[:, None] if R.ndim == 2 else R / self.D

    # -- derivatives (eq. NEGLLDNEGLLFSA and the two displays after it) -----
    def _deriv(self, which):
        """Matrices for dSigma~_dagger/dtheta, theta = sigma1^2 (0), rho (1)."""
        if which in self._dcache:
            return self._dcache[which]
        kind, s1, rho, s2 = self.theta
        dc = covariance_dsigma1 if which == 0 else covariance_drho
        dSm = dc(cdist(self.inducing, self.inducing), s1, rho, kind)
        dSmn_T = dc(cdist(self.locs, self.inducing), s1, rho, kind)
        if which == 0 and self.jitter:
            dSm[np.diag_indices(self.m)] += self.jitter
        # (dSigma_l)_ij = dSmn_i . K_j + K_i . dSmn_j - K_i . dSm K_j
        cols = self.col.astype(np.int64)
        dSmK_T = self.K_T @ dSm.T        # rows: (dSigma_m K)_{:, j}^T
        dl = (_pair_dots(dSmn_T, self.K_T, self.rows, cols)
              + _pair_dots(self.K_T, dSmn_T, self.rows, cols)
              - _pair_dots(self.K_T, dSmK_T, self.rows, cols))
        dvals = (dc(self.pair_d, s1, rho, kind) - dl) * self.pair_w
        dS = sp.csr_matrix((dvals, self.col, self.row_ptr), shape=(self.n, self.n))
        self._dcache[which] = (dSm, dSmn_T, dS)
        return self._dcache[which]

    def dmatvec(self, which, X):
        """(dSigma~_dagger / dtheta) X for theta = (sigma1^2, rho, sigma^2)[which]:
        dSigma~_s/dtheta + dSigma_l/dtheta with
        dSigma~_s/dtheta = (dSigma/dtheta - dSigma_l/dtheta) o T + dsigma^2/dtheta I and
        dSigma_l/dtheta = dSmn^T Sm^{-1} Smn + Smn^T Sm^{-1} dSmn - Smn^T Sm^{-1} dSm Sm^{-1} Smn."""
        if which == 2:
            return X.copy()
        dSm, dSmn_T, dS = self._deriv(which)
        KX = self.K_T.T @ X
        low = dSmn_T @ KX + self.K_T @ (dSmn_T.T @ X) - self.K_T @ (dSm @ KX)
        return dS @ X + low

    def precond_dmatvec(self, which, X):
        """(dP/dtheta) X for the FITC preconditioner P = D_s + Sigma_l (eq.
        eqfitcp): D_s = diag(Sigma~_s), so dP/dtheta = diag(dSigma~_s/dtheta)
        + dSigma_l/dtheta, and dP/dsigma^2 = I."""
        if which == 2:
            return X.copy()
        dSm, dSmn_T, dS = self._deriv(which)
        dD = dS.diagonal()
        KX = self.K_T.T @ X
        low = dSmn_T @ KX + self.K_T @ (dSmn_T.T @ X) - self.K_T @ (dSm @ KX)
        return (dD[:, None] * X if X.ndim == 2 else dD * X) + low

    def precond_dense(self):
        """P as a dense n x n matrix (small n only)."""
        return np.diag(self.D) + self.Smn_T @ sla.cho_solve(self.chol_m, self.Smn_T.T)

    def precond_trace_deriv(self):
        """Tr(P^{-1} dP/dtheta) for theta = (sigma1^2, rho, sigma^2), from the
        dense definition (small n only): the deterministic term of the
        control variate (App. E)."""
        P = self.precond_dense()
        eye = np.eye(self.n)
        return np.array([np.trace(np.linalg.solve(P, self.precond_dmatvec(k, eye))) for k in range(3)])


class FSARows:
    """The quantities of FSA for requested rows only, for inputs too large to
    assemble: Sigma_m and its Cholesky factor once; taper rows, residual
    values, D_s, rows of Sigma~_dagger X and rows of the probe block on
    demand.  The low-rank sum Sigma_m^{-1} Sigma_mn X over all points is
    streamed in chunks.  Same definitions as FSA (Section 2.1, App. F)."""

    def __init__(self, locs, inducing, theta, gamma, jitter=0.0, chunk=1 << 15):
        kind, s1, rho, s2 = theta
        self.locs = np.ascontiguousarray(locs, dtype=np.float64)
        self.inducing = np.ascontiguousarray(inducing, dtype=np.float64)
        self.theta = (int(kind), float(s1), float(rho), float(s2))
        self.gamma = float(gamma)
        self.n, self.m = self.locs.shape[0], self.inducing.shape[0]
        self.chunk = chunk
        self.Sigma_m = covariance(cdist(self.inducing, self.inducing), s1, rho, kind)
        self.Sigma_m[np.diag_indices(self.m)] += jitter * s1
        self.chol_m = sla.cho_factor(self.Sigma_m, lower=True)

    def smn_T(self, idx):
        """Sigma_mn^T rows idx (len(idx) x m)."""
        kind, s1, rho, _ = self.theta
        return covariance(cdist(self.locs[idx], self.inducing), s1, rho, kind)

    def k_T(self, idx):
        """(Sigma_m^{-1} Sigma_mn)^T rows idx."""
        return np.ascontiguousarray(sla.cho_solve(self.chol_m, self.smn_T(idx).T).T)

    def pattern_rows(self, idx):
        """Taper pattern of rows idx against all points (CSR over idx)."""
        return taper_pattern(self.locs[np.asarray(idx)], self.locs, self.gamma)

    def value_rows(self, idx):
        """Pattern, residual values and D_s of rows idx: (c(d) - Sigma_l)
        o T + sigma^2 on the diagonal."""
        kind, s1, rho, s2 = self.theta
        idx = np.asarray(idx, dtype=np.int64)
        rp, col = self.pattern_rows(idx)
        r_loc = np.repeat(np.arange(idx.shape[0], dtype=np.int64), np.diff(rp))
        cols = col.astype(np.int64)
        d = _pair_dist(self.locs[idx], self.locs, r_loc, cols)
        uc, inv = np.unique(cols, return_inverse=True)
        low = _pair_dots(self.smn_T(idx), self.k_T(uc), r_loc, inv)
        vals = (covariance(d, s1, rho, kind) - low) * wendland_taper(d, self.gamma)
        diag = idx[r_loc] == cols
        vals[diag] += s2
        D = np.zeros(idx.shape[0])
        D[r_loc[diag]] = vals[diag]
        return rp, col, vals, D

    def lowrank_sum(self, X):
        """Sigma_m^{-1} Sigma_mn X (m x k), streamed over the points."""
        X = np.asarray(X, dtype=np.float64)
        acc = np.zeros((self.m, X.shape[1]))
        for s in range(0, self.n, self.chunk):
            e = min(self.n, s + self.chunk)
            acc += self.smn_T(np.arange(s, e)).T @ X[s:e]
        return sla.cho_solve(self.chol_m, acc)

    def matvec_rows(self, idx, X):
        """Rows idx of Sigma~_dagger X."""
        idx = np.asarray(idx, dtype=np.int64)
        rp, col, vals, _ = self.value_rows(idx)
        S = sp.csr_matrix((vals, col, rp), shape=(idx.shape[0], self.n))
        return S @ X + self.smn_T(idx) @ self.lowrank_sum(X)

    def probe_rows(self, idx, t, seed):
        """Rows idx of the probe block z = Sigma_mn^T L_m^{-T} e + D_s^{1/2} rho."""
        idx = np.asarray(idx, dtype=np.int64)
        e = rademacher(seed, STREAM_E, self.m, t)
        r = rademacher_rows(seed, STREAM_RHO, idx, t)
        Lm = np.tril(self.chol_m[0])
        D = self.value_rows(idx)[3]
        return self.smn_T(idx) @ sla.solve_triangular(Lm, e, lower=True, trans="T") + np.sqrt(D)[:, None] * r


# ---------------------------------------------------------------------------
# Preconditioned CG with Lanczos coefficients (Appendix A, Algorithm 2)
# ---------------------------------------------------------------------------


class PCGResult:
    def __init__(self, U, Q0, diags, offs, iters, rel_res):
        self.U, self.Q0, self.diags, self.offs, self.iters, self.rel_res = U, Q0, diags, offs, iters, rel_res


def pcg_lanczos(matvec, precond, B, tol, max_iter, fixed_iter=0):
    """Algorithm 2 run independently on every column of B; the columns share
    each operator application (matrix-matrix products, Section 3.1).

    Column j stops once ||r||_2 / ||b||_2 < tol (its Lanczos matrix then stops
    growing) unless fixed_iter > 0, in which case every column runs exactly
    fixed_iter iterations.  Lanczos entries: T_{l+1,l+1} = 1/alpha_{l+1} +
    beta_l/alpha_l and T_{l,l+1} = sqrt(beta_l)/alpha_l, alpha_0 = 1, beta_0 = 0."""
    B = np.asarray(B, dtype=np.float64)
    n, k = B.shape
    U = np.zeros_like(B)
    R = B.copy()
    Z = precond(R)
    Q0 = Z.copy()
    H = Z.copy()
    rz = np.einsum("ij,ij->j", R, Z)
    alpha_prev = np.ones(k)
    beta_prev = np.zeros(k)
    bnorm = np.linalg.norm(B, axis=0)
    active = bnorm > 0
    diags = [[] for _ in range(k)]
    offs = [[] for _ in range(k)]
    iters = np.zeros(k, dtype=np.int64)
    L = fixed_iter if fixed_iter > 0 else max_iter
    for l in range(L):
        if not active.any():
            break
        V = matvec(H)
        hv = np.einsum("ij,ij->j", H, V)
        a = np.nonzero(active)[0]
        if np.any(hv[a] <= 0) or not np.all(np.isfinite(hv[a])):
            raise FloatingPointError("CG breakdown: h^T A h <= 0")
        alpha = np.ones(k)
        alpha[a] = rz[a] / hv[a]
        U[:, a] += alpha[a] * H[:, a]
        R[:, a] -= alpha[a] * V[:, a]
        Zn = precond(R)
        rz_new = np.einsum("ij,ij->j", R, Zn)
        beta = np.zeros(k)
        beta[a] = rz_new[a] / rz[a]
        for j in a:
            diags[j].append(1.0 / alpha[j] + beta_prev[j] / alpha_prev[j])
            if l > 0:
                offs[j].append(math.sqrt(beta_prev[j]) / alpha_prev[j])
        H[:, a] = Zn[:, a] + beta[a] * H[:, a]
        alpha_prev[a] = alpha[a]
        beta_prev[a] = beta[a]
        rz[a] = rz_new[a]
        iters[a] += 1
        if fixed_iter <= 0:
            rel = np.linalg.norm(R[:, a], axis=0) / bnorm[a]
            active[a[rel < tol]] = False
    with np.errstate(invalid="ignore", divide="ignore"):
        rel_res = np.where(bnorm > 0, np.linalg.norm(R, axis=0) / np.where(bnorm > 0, bnorm, 1), 0.0)
    return PCGResult(U, Q0, diags, offs, iters, rel_res)


def e1_log_e1(diag, off):
    """e_1^T log(T) e_1 for a symmetric tridiagonal T (diag, off), via its
    eigendecomposition: sum_k Q_{1k}^2 log(lambda_k)."""
    d = np.asarray(diag, dtype=np.float64)
    if d.size == 0:
        return 0.0
    if d.size == 1:
        return math.log(d[0])
    lam, Q = sla.eigh_tridiagonal(d, np.asarray(off, dtype=np.float64))
    return float(np.sum(Q[0] ** 2 * np.log(lam)))


# ---------------------------------------------------------------------------
# Likelihood and gradient (eq. NEGLLDNEGLLFSA, Sections 3.1 and 3.3)
# ---------------------------------------------------------------------------


def probes(model, t, seed):
    """t probe vectors z ~ (0, P): z = Sigma_mn^T L_m^{-T} e + D_s^{1/2} rho
    with Rademacher e (m) and rho (n) (App. F sampling recipe)."""
    e = rademacher(seed, STREAM_E, model.m, t)
    r = rademacher(seed, STREAM_RHO, model.n, t)
    Lm = np.tril(model.chol_m[0])
    return model.Smn_T @ sla.solve_triangular(Lm, e, lower=True, trans="T") + np.sqrt(model.D)[:, None] * r


def nll_grad(model, y, num_probes, seed, tol=1e-8, max_iter=1000, fixed_iter=0,
             slq_weight_n=False, with_grad=True, control_variate=None):
    """Negative log-likelihood and its gradient in (sigma1^2, rho, sigma^2).

    log det: preconditioned SLQ, (1/t) sum_i w_i e_1^T log(T_i) e_1 + log det P
    (Section 3.3); quadratic term y^T Sigma~^{-1} y from the same PCG run;
    gradient: (1/2) STE of Tr(Sigma~^{-1} dSigma~) with P^{-1} z_i (Section 3.3)
    minus (1/2) u^T dSigma~ u, u = Sigma~^{-1} y (eq. NEGLLDNEGLLFSA).

    control_variate (App. E, eq. Troptc): None for the plain estimate;
    otherwise subtract c * b_i, b_i = (P^{-1} z_i)^T dP/dtheta (P^{-1} z_i), from
    each sample a_i and add c Tr(P^{-1} dP/dtheta), per parameter, with
    "one": c = 1;
    "opt": c = sum_i (a_i - mean a)(b_i - mean b) / sum_i (b_i - mean b)^2, the
           coefficient that minimises the sample variance of a_i - c b_i
           (the printed c_opt with its denominator centred, the reading under
           which it is the optimal coefficient the text describes);
    "opt_printed": c = sum_i (a_i - mean a) b_i / sum_i b_i^2, as printed."""
    n = model.n
    y = np.asarray(y, dtype=np.float64)
    Z = probes(model, num_probes, seed)
    B = np.column_stack([y, Z])
    res = pcg_lanczos(model.matvec, model.precond_solve, B, tol, max_iter, fixed_iter)
    if slq_weight_n:
        w = np.full(num_probes, float(n))
    else:
        w = np.einsum("ij,ij->j", Z, res.Q0[:, 1:])
    q = np.array([e1_log_e1(res.diags[i + 1], res.offs[i + 1]) for i in range(num_probes)])
    logdet = float(np.mean(w * q)) + model.logdet_P
    u = res.U[:, 0]
    quad = float(y @ u)
    nll = 0.5 * n * math.log(2.0 * math.pi) + 0.5 * logdet + 0.5 * quad
    out = {"nll": nll, "logdet": logdet, "logdet_P": model.logdet_P, "quad": quad,
           "iters": res.iters, "rel_res": res.rel_res, "slq_terms": w * q, "pcg": res}
    if with_grad:
        X = np.column_stack([u, res.Q0[:, 1:]])
        grad = np.empty(3)
        trace_terms = np.empty((3, num_probes))
        quad_terms = np.empty(3)
        for k in range(3):
            dX = model.dmatvec(k, X)
            trace_terms[k] = np.einsum("ij,ij->j", res.U[:, 1:], dX[:, 1:])
            quad_terms[k] = float(u @ dX[:, 0])
            grad[k] = 0.5 * np.mean(trace_terms[k]) - 0.5 * quad_terms[k]
        out["trace_terms"] = trace_terms
        if control_variate is not None:
            Xp = res.Q0[:, 1:]  # P^{-1} z_i
            cv_terms = np.array([np.einsum("ij,ij->j", Xp, model.precond_dmatvec(k, Xp)) for k in range(3)])
            trace_P = model.precond_trace_deriv()
            c = np.ones(3)
            for k in range(3):
                a, b = trace_terms[k], cv_terms[k]
                if control_variate in ("opt", "opt_printed"):
                    bc = b - np.mean(b) if control_variate == "opt" else b
                    den = np.sum(bc * bc)
                    # b_i (nearly) constant: any c leaves the estimate as it is
                    c[k] = np.sum((a - np.mean(a)) * bc) / den if den > CV_DEGENERATE * np.sum(b * b) else 0.0
                elif control_variate != "one":
                    raise ValueError("control_variate must be None, 'one', 'opt' or 'opt_printed'")
                est = np.mean(a - c[k] * b) + c[k] * trace_P[k]
                grad[k] = 0.5 * est - 0.5 * quad_terms[k]
            out.update(cv_terms=cv_terms, trace_P=trace_P, cv_c=c)
        out["grad"] = grad
    return out


# ---------------------------------------------------------------------------
# Predictive variances by simulation (Section 3.2, Algorithm 1)
# ---------------------------------------------------------------------------


def predict_var(model, pred_locs, num_samples, seed, tol=1e-8, max_iter=1000, fixed_iter=0,
                exact_Dl=False, u=None, smp_T=None, control_variate=None):
    """Algorithm 1: D^p = sigma1^2 + sigma^2 - D1 - 2 D2 + D3 - D_l.

    Sigma~_s solves use CG preconditioned by D_s (Section 3.3).  With
    exact_Dl the stochastic diagonal is replaced by its exact value (dense,
    small inputs only).  Returns (variances, details); with u =
    Sigma~^{-1} y given, also the predictive mean (Section 2.3).  smp_T
    replaces Sigma_{m n_p}^T as smn_T does Sigma_mn^T in FSA.

    control_variate (App. E, second display): None for the plain D_l;
    otherwise, with P_s = D_s and per prediction point, the samples
    a_i = z_i o (S^T Sigma~_s^{-1} S z_i) get c o b_i subtracted, b_i =
    z_i o (S^T D_s^{-1} S z_i), and c o diag(S^T D_s^{-1} S) added (S =
    Sigma^s_{n n_p}); c as in nll_grad ("one", "opt" centred, "opt_printed")."""
    kind, s1, rho, s2 = model.theta
    P = np.ascontiguousarray(pred_locs, dtype=np.float64)
    n_p = P.shape[0]
    if smp_T is None:
        Smp_T = covariance(cdist(P, model.inducing), s1, rho, kind)   # Sigma_{m n_p}^T
    else:
        Smp_T = np.ascontiguousarray(smp_T, dtype=np.float64)
    G_T = np.ascontiguousarray(sla.cho_solve(model.chol_m, Smp_T.T).T)   # (Sigma_m^{-1} Sigma_{m n_p})^T
    # Sigma^s_{n n_p} = (Sigma_{n n_p} - Sigma^l_{n n_p}) o T_{n n_p}(gamma), stored n x n_p.
    rp, cl = taper_pattern(model.locs, P, model.gamma)
    rows = np.repeat(np.arange(model.n, dtype=np.int64), np.diff(rp))
    cols = cl.astype(np.int64)
    d = _pair_dist(model.locs, P, rows, cols)
    low = _pair_dots(model.Smn_T, G_T, rows, cols)
    vals = (covariance(d, s1, rho, kind) - low) * wendland_taper(d, model.gamma)
    Ss = sp.csr_matrix((vals, cl, rp), shape=(model.n, n_p))
    SsT = Ss.T.tocsr()
    # V = Sigma~_s^{-1} Sigma_mn^T and M = Sigma_m + Sigma_mn V (App. B).
    V = pcg_lanczos(model.sparse_matvec, model.diag_solve, model.Smn_T, tol, max_iter, fixed_iter).U
    M = model.Sigma_m + model.Smn_T.T @ V
    cM = sla.cho_factor(M, lower=True)
    # Sigma~_dagger^{-1} Sigma_mn^T = V M^{-1} Sigma_m (eq. SWMFSA).
    W = V @ sla.cho_solve(cM, model.Sigma_m)
    SmnW = model.Smn_T.T @ W                                             # Sigma_mn Sigma~^{-1} Sigma_mn^T
    D1 = np.einsum("ij,ij->j", G_T.T, SmnW @ G_T.T)
    SsTW = SsT @ W                                                       # n_p x m
    D2 = np.einsum("ij,ij->i", SsTW, G_T)
    Y = SsT @ V
    D3 = np.einsum("ij,ij->i", Y, sla.cho_solve(cM, Y.T).T)
    if exact_Dl:
        S_dense = model.S.toarray()
        Dl = np.einsum("ij,ij->j", Ss.toarray(), np.linalg.solve(S_dense, Ss.toarray()))
        Z1 = None
    else:
        Z1 = rademacher(seed, STREAM_PRED, n_p, num_samples)
        X = Ss @ Z1
        Wl = pcg_lanczos(model.sparse_matvec, model.diag_solve, X, tol, max_iter, fixed_iter).U
        Z2 = SsT @ Wl
        Dl = np.mean(Z1 * Z2, axis=1)
        if control_variate is not None:
            a = Z1 * Z2
            b = Z1 * (SsT @ (X / model.D[:, None]))
            E = np.asarray(Ss.multiply(Ss).T @ (1.0 / model.D)).ravel()   # diag(S^T D_s^{-1} S)
            if control_variate == "one":
                c = np.ones(n_p)
            elif control_variate in ("opt", "opt_printed"):
                bc = b - b.mean(axis=1, keepdims=True) if control_variate == "opt" else b
                num = np.sum((a - Dl[:, None]) * bc, axis=1)
                den = np.sum(bc * bc, axis=1)
                c = np.divide(num, den, out=np.zeros(n_p), where=den > CV_DEGENERATE * np.sum(b * b, axis=1))
            else:
                raise ValueError("control_variate must be None, 'one', 'opt' or 'opt_printed'")
            Dl = np.mean(a - c[:, None] * b, axis=1) + c * E
            det_cv = {"cv_c": c, "cv_E": E, "cv_a": a, "cv_b": b}
        else:
            det_cv = {}
    var = s1 + s2 - D1 - 2.0 * D2 + D3 - Dl
    det = {"D1": D1, "D2": D2, "D3": D3, "Dl": Dl, "cross_row_ptr": rp, "cross_col": cl}
    if not exact_Dl:
        det.update(det_cv)
    if u is not None:
        det["mean"] = G_T @ (model.Smn_T.T @ u) + SsT @ u
    return var, det


# ---------------------------------------------------------------------------
# Scores of a Gaussian predictive distribution (Section 4)
# ---------------------------------------------------------------------------


def scores(y, mean, var):
    """(log-score, CRPS, RMSE) of predictive means and variances against test
    responses y, averaged over the points: log-score -log phi(y; mu, sigma^2),
    CRPS in the closed form for a normal predictive distribution,
    sigma (-1/sqrt(pi) + 2 phi(z) + z (2 Phi(z) - 1)) with z = (y - mu)/sigma,
    and the root mean squared error of the means."""
    y, mu, v = (np.asarray(a, dtype=np.float64) for a in (y, mean, var))
    sd = np.sqrt(v)
    z = (y - mu) / sd
    ls = np.mean(0.5 * np.log(2.0 * math.pi * v) + 0.5 * z * z)
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    Phi = 0.5 * erfc(-z / math.sqrt(2.0))
    crps = np.mean(sd * (-1.0 / math.sqrt(math.pi) + 2.0 * phi + z * (2.0 * Phi - 1.0)))
    rmse = math.sqrt(np.mean((y - mu) ** 2))
    return float(ls), float(crps), float(rmse)

