"""CPU FP64 oracle for the FITC preconditioner in iterative methods for
Vecchia approximations (Section 5 of Gyger, Furrer & Sigrist, arXiv
2405.14492).

TEST INFRASTRUCTURE ONLY.  Only the test-suite and the benchmark's
CPU-baseline leg may import this module; the product path never calls it.
It shares no code with the HIP path.  It reuses the FSA oracle's covariance
function, probe recipe, preconditioned CG with Lanczos coefficients and
tridiagonal quadrature (all test infrastructure of the same kind).

What it computes (Section 5.1), with the readings taken where the paper is
silent or garbled (each also listed in the design notes):
  * Vecchia approximation of the latent process b ~ N(0, Sigma): the
    ordering is the input order; N(i) holds the min(m_v, i) nearest of
    s_0 .. s_{i-1}, nearest first, a tie in distance going to the lower
    index; squared distances are dx*dx + dy*dy in float64 with no fused
    multiply-add;
  * A_i = Sigma_{N(i),i}^T Sigma_{N(i)}^{-1}, D_i = Sigma_ii - A_i
    Sigma_{N(i),i}, B unit lower triangular with B_{i,N(i)} = -A_i, and
    Sigma_V^{-1} = B^T D^{-1} B; no jitter is added to Sigma_{N(i)};
  * linear solves (Sigma_V^{-1} + W)^{-1} v: the equivalent form printed as
    eq. VL_v2 does not equal this inverse (a 1 x 1 case gives
    w^2 / (s (1 + s w)) against s / (1 + s w)); the form taken is
    W^{-1} (Sigma_V + W^{-1})^{-1} Sigma_V v, which is the inverse, so CG
    runs on Sigma_V + W^{-1} with the FITC preconditioner
    P = Sigma_mn^T Sigma_m^{-1} Sigma_mn + D_s,
    D_s = diag(Sigma - Sigma_mn^T Sigma_m^{-1} Sigma_mn) + W^{-1};
  * Sigma_V X = B^{-1} (D (B^{-T} X)) by two sparse triangular solves;
  * log det(Sigma_V^{-1} + W) = sum log W - sum log D + log det(Sigma_V +
    W^{-1}), the last by preconditioned SLQ with probes z ~ (0, P) as for
    the FSA (Section 3.3), weight z^T P^{-1} z;
  * the Vecchia-Laplace approximation that Section 5.1 applies these solves
    and log-determinants to, for Bernoulli responses with the logistic link:
    Newton's method for the mode (each step one solve with the current W,
    the preconditioner rebuilt for it) and the Laplace negative log marginal
    likelihood at the mode (laplace()).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular
from scipy.spatial.distance import cdist

from oracle import fsa_oracle as F


def neighbors(locs, mv, rows=None):
    """N(i) for i in rows (default all): the min(mv, i) nearest earlier
    points, ordered by (squared distance, index); -1 pads to mv entries."""
    locs = np.asarray(locs, dtype=np.float64)
    n = locs.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    out = np.full((rows.shape[0], mv), -1, dtype=np.int64)
    for r, i in enumerate(rows):
        i = int(i)
        if i == 0 or mv == 0:
            continue
        dx = locs[:i, 0] - locs[i, 0]
        dy = locs[:i, 1] - locs[i, 1]
        d2 = dx * dx + dy * dy
        k = min(mv, i)
        order = np.lexsort((np.arange(i), d2))[:k]
        out[r, :k] = order
    return out


def factor(locs, nbr, theta, rows=None):
    """Coefficients A_i (padded with 0 to the width of nbr) and conditional
    variances D_i for i in rows (default all), Section 5.1."""
    kind, s1, rho = theta
    locs = np.asarray(locs, dtype=np.float64)
    rows = np.arange(locs.shape[0]) if rows is None else np.asarray(rows, dtype=np.int64)
    mv = nbr.shape[1]
    coef = np.zeros((rows.shape[0], mv))
    D = np.empty(rows.shape[0])
    for r, i in enumerate(rows):
        N = nbr[r][nbr[r] >= 0]
        if N.size == 0:
            D[r] = s1
            continue
        SN = F.covariance(cdist(locs[N], locs[N]), s1, rho, kind)
        sNi = F.covariance(cdist(locs[N], locs[int(i)][None, :])[:, 0], s1, rho, kind)
        a = np.linalg.solve(SN, sNi)
        coef[r, :N.size] = a
        D[r] = s1 - a @ sNi
    return coef, D


class Vecchia:
    """Sigma_V (Section 5.1) with W and the FITC preconditioner of
    Sigma + W^{-1} (Section 5.1, eq. eqfitcp with D_s + W^{-1})."""

    def __init__(self, locs, inducing, theta, mv, w, jitter=0.0):
        kind, s1, rho = theta
        self.locs = np.ascontiguousarray(locs, dtype=np.float64)
        self.inducing = np.ascontiguousarray(inducing, dtype=np.float64)
        self.theta = (int(kind), float(s1), float(rho))
        self.w = np.asarray(w, dtype=np.float64)
        n, m = self.locs.shape[0], self.inducing.shape[0]
        self.n, self.m, self.mv = n, m, int(mv)
        self.nbr = neighbors(self.locs, self.mv)
        self.coef, self.Dv = factor(self.locs, self.nbr, self.theta)
        rows = np.repeat(np.arange(n), self.mv)
        cols = self.nbr.ravel()
        keep = cols >= 0
        off = sp.csr_matrix((-self.coef.ravel()[keep], (rows[keep], cols[keep])), shape=(n, n))
        self.B = (sp.identity(n, format="csr") + off).tocsr()
        self.Bt = self.B.T.tocsr()
        # FITC preconditioner of Sigma + W^{-1}
        self.Sigma_m = F.covariance(cdist(self.inducing, self.inducing), s1, rho, kind)
        self.Sigma_m[np.diag_indices(m)] += jitter * s1
        self.Smn_T = F.covariance(cdist(self.locs, self.inducing), s1, rho, kind)
        self.chol_m = sla.cho_factor(self.Sigma_m, lower=True)
        K_T = sla.cho_solve(self.chol_m, self.Smn_T.T).T
        self.diag_s = s1 - np.einsum("ij,ij->i", self.Smn_T, K_T)  # diag(Sigma - Sigma_nm Sigma_m^-1 Sigma_mn)
        self.set_w(self.w)

    def set_w(self, w):
        """Take new weights W: the FITC preconditioner of Sigma + W^{-1}
        changes with them, the Vecchia factor does not."""
        self.w = np.asarray(w, dtype=np.float64)
        self.D = self.diag_s + 1.0 / self.w
        self.M_P = self.Sigma_m + self.Smn_T.T @ (self.Smn_T / self.D[:, None])
        self.chol_P = sla.cho_factor(self.M_P, lower=True)
        self.logdet_P = (2.0 * np.sum(np.log(np.diag(self.chol_P[0])))
                         - 2.0 * np.sum(np.log(np.diag(self.chol_m[0])))
                         + np.sum(np.log(self.D)))

    def _cols(self, X):
        X = np.asarray(X, dtype=np.float64)
        return X if X.ndim == 2 else X[:, None]

    def cov_matvec(self, X):
        """Sigma_V X = B^{-1} (D (B^{-T} X))."""
        X2 = self._cols(X)
        Z = spsolve_triangular(self.Bt, X2, lower=False, unit_diagonal=True)
        Y = spsolve_triangular(self.B, self.Dv[:, None] * Z, lower=True, unit_diagonal=True)
        return Y if np.ndim(X) == 2 else Y[:, 0]

    def prec_matvec(self, X):
        """Sigma_V^{-1} X = B^T D^{-1} B X."""
        X2 = self._cols(X)
        Y = self.Bt @ ((self.B @ X2) / self.Dv[:, None])
        return Y if np.ndim(X) == 2 else Y[:, 0]

    def matvec(self, X):
        """(Sigma_V + W^{-1}) X, the CG operator."""
        X2 = self._cols(X)
        Y = self.cov_matvec(X2) + X2 / self.w[:, None]
        return Y if np.ndim(X) == 2 else Y[:, 0]

    def precond_solve(self, R):
        """P^{-1} R by the Sherman-Woodbury-Morrison formula (App. F)."""
        R2 = self._cols(R)
        DR = R2 / self.D[:, None]
        t = sla.cho_solve(self.chol_P, self.Smn_T.T @ DR)
        Z = DR - (self.Smn_T @ t) / self.D[:, None]
        return Z if np.ndim(R) == 2 else Z[:, 0]

    def logdet_offset(self):
        """log det(Sigma_V^{-1} + W) - log det(Sigma_V + W^{-1})
        = sum log W - sum log D."""
        return float(np.sum(np.log(self.w)) - np.sum(np.log(self.Dv)))


def solve_logdet(model, v, num_probes, seed, tol=1e-8, max_iter=1000, fixed_iter=0):
    """x = (Sigma_V^{-1} + W)^{-1} v and the SLQ estimate of
    log det(Sigma_V^{-1} + W) from one block PCG run on Sigma_V + W^{-1}
    over [Sigma_V v, z_1 .. z_t]."""
    v = np.asarray(v, dtype=np.float64)
    y = model.cov_matvec(v)
    Z = F.probes(model, num_probes, seed)
    B = np.column_stack([y, Z])
    res = F.pcg_lanczos(model.matvec, model.precond_solve, B, tol, max_iter, fixed_iter)
    x = res.U[:, 0] / model.w
    wt = np.einsum("ij,ij->j", Z, res.Q0[:, 1:])
    q = np.array([F.e1_log_e1(res.diags[i + 1], res.offs[i + 1]) for i in range(num_probes)])
    logdet_sw = float(np.mean(wt * q)) + model.logdet_P
    return {"x": x, "logdet": model.logdet_offset() + logdet_sw, "logdet_sw": logdet_sw,
            "logdet_P": model.logdet_P, "slq_terms": wt * q, "iters": res.iters, "rel_res": res.rel_res,
            "pcg": res, "B": B}


# ---------------------------------------------------------------------------
# Vecchia-Laplace approximation for Bernoulli-logit responses (Section 5.1)
# ---------------------------------------------------------------------------


def bernoulli_loglik(y, b):
    """log p(y | b) = sum_i y_i b_i - log(1 + e^{b_i}) for y_i in {0, 1}
    (logistic link)."""
    y = np.asarray(y, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sum(y * b - np.logaddexp(0.0, b)))


def logistic(b):
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(b, dtype=np.float64)))


def laplace(model, y, num_probes, seed, tol=1e-8, max_iter=1000, fixed_iter=0, newton_tol=1e-8, max_newton=50,
            fixed_newton=0):
    """Vecchia-Laplace approximation of the negative log marginal likelihood
    of Bernoulli-logit responses y under the Vecchia prior b ~ N(0, Sigma_V).

    The mode of log p(y|b) - b^T Sigma_V^{-1} b / 2 by Newton's method from
    b = 0: with pi = 1/(1 + e^{-b}), W = diag(pi (1 - pi)) (the negative
    second derivatives of the log-likelihood),
        b <- (Sigma_V^{-1} + W)^{-1} (W b + y - pi),
    each solve by the FITC-preconditioned CG of solve_logdet (the
    preconditioner is rebuilt for every W).  The iteration stops when
    ||b_new - b|| <= newton_tol ||b_new|| (or after exactly fixed_newton
    steps).  At the mode, with W there,
        NLL = -log p(y|b) + b^T Sigma_V^{-1} b / 2 + log det(Sigma_V W + I) / 2,
        log det(Sigma_V W + I) = sum log D + log det(Sigma_V^{-1} + W),
    the last term by SLQ with num_probes probes (solve_logdet)."""
    y = np.asarray(y, dtype=np.float64)
    b = np.zeros(model.n)
    steps = 0
    converged = False
    limit = fixed_newton if fixed_newton > 0 else max_newton
    for _ in range(limit):
        pi = logistic(b)
        model.set_w(pi * (1.0 - pi))
        rhs = model.w * b + y - pi
        out = solve_logdet(model, rhs, 1, seed, tol, max_iter, fixed_iter)
        step = np.linalg.norm(out["x"] - b)
        b = out["x"]
        steps += 1
        if fixed_newton <= 0 and step <= newton_tol * max(np.linalg.norm(b), 1e-300):
            converged = True
            break
    pi = logistic(b)
    model.set_w(pi * (1.0 - pi))
    out = solve_logdet(model, y - pi, num_probes, seed, tol, max_iter, fixed_iter)
    ll = bernoulli_loglik(y, b)
    quad = float(b @ model.prec_matvec(b))
    sum_log_d = float(np.sum(np.log(model.Dv)))
    nll = -ll + 0.5 * quad + 0.5 * (sum_log_d + out["logdet"])
    return {"mode": b, "nll": nll, "loglik": ll, "quad": quad, "sum_log_d": sum_log_d, "logdet": out["logdet"],
            "slq_terms": out["slq_terms"], "newton_steps": steps, "converged": converged}
