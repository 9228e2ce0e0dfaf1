"""Dense (n <= ~2000) assembly of the FSA quantities straight from their
definitions, for pinning the oracle on small inputs.

Everything here is built as full matrices with numpy: the covariance of all
pairs, the taper of all pairs (zero beyond gamma), Hadamard products and
dense inverses/log-determinants.  No sparse pattern, no Woodbury, no
Sylvester, no CG.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial.distance import cdist

from oracle import fsa_oracle as O


def dense_parts(locs, inducing, theta, gamma, jitter=0.0, Smn=None):
    """Smn (m x n) replaces the cross covariance when given."""
    kind, s1, rho, s2 = theta
    n = locs.shape[0]
    Sig = O.covariance(cdist(locs, locs), s1, rho, kind)
    Sm = O.covariance(cdist(inducing, inducing), s1, rho, kind) + jitter * s1 * np.eye(inducing.shape[0])
    if Smn is None:
        Smn = O.covariance(cdist(inducing, locs), s1, rho, kind)
    Sl = Smn.T @ np.linalg.solve(Sm, Smn)
    T = O.wendland_taper(cdist(locs, locs), gamma)
    Ss = (Sig - Sl) * T + s2 * np.eye(n)
    return {"Sigma": Sig, "Sm": Sm, "Smn": Smn, "Sl": Sl, "T": T, "Ss": Ss, "full": Sl + Ss}


def dense_fsa(locs, inducing, theta, gamma, jitter=0.0):
    return dense_parts(locs, inducing, theta, gamma, jitter)["full"]


def dense_fitc(locs, inducing, theta, gamma):
    p = dense_parts(locs, inducing, theta, gamma)
    return np.diag(np.diag(p["Ss"])) + p["Sl"]


def dense_nll(S, y):
    sign, ld = np.linalg.slogdet(S)
    assert sign > 0
    return 0.5 * S.shape[0] * math.log(2 * math.pi) + 0.5 * ld + 0.5 * y @ np.linalg.solve(S, y)


def fd_operator(locs, inducing, theta, gamma, which, h_rel=1e-5):
    """Central finite difference of the dense FSA matrix in theta[which+1]."""
    th = list(theta)
    h = h_rel * th[which + 1]
    th[which + 1] += h
    Sp = dense_fsa(locs, inducing, tuple(th), gamma)
    th[which + 1] -= 2 * h
    Sm = dense_fsa(locs, inducing, tuple(th), gamma)
    return (Sp - Sm) / (2 * h)


def dense_pred_var(locs, inducing, pred, theta, gamma):
    """diag of the FSA predictive covariance (eq. MuPredFSA), dense."""
    kind, s1, rho, s2 = theta
    Sm = O.covariance(cdist(inducing, inducing), s1, rho, kind)
    Smn = O.covariance(cdist(inducing, locs), s1, rho, kind)
    Smp = O.covariance(cdist(inducing, pred), s1, rho, kind)
    Snp = O.covariance(cdist(locs, pred), s1, rho, kind)
    Sl_np = Smn.T @ np.linalg.solve(Sm, Smp)
    Tnp = O.wendland_taper(cdist(locs, pred), gamma)
    cross = Sl_np + (Snp - Sl_np) * Tnp
    S = dense_fsa(locs, inducing, theta, gamma)
    return s1 + s2 - np.einsum("ij,ij->j", cross, np.linalg.solve(S, cross)), cross, S


def bf16_round(x):
    """float64 -> float32 (nearest) -> bfloat16 (nearest, ties to even),
    returned as float64: the rounding of the MIXED_BF16A factor."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    h = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32)
    return (h << 16).view(np.float32).astype(np.float64)


def bf16_cross_covariance(locs, inducing, theta, pred=None):
    """Sigma_mn^T (n x m) of the model whose whitened factor
    A = L_m^{-1} Sigma_mn is rounded to bfloat16: L_m A~ with A~ rounded, so
    Sigma_mn^T Sigma_m^{-1} Sigma_mn = A~^T A~.  With pred, the same for the
    prediction locations."""
    import scipy.linalg as sla
    kind, s1, rho, s2 = theta
    Sm = O.covariance(cdist(inducing, inducing), s1, rho, kind)
    L = np.linalg.cholesky(Sm)
    pts = locs if pred is None else pred
    Smn = O.covariance(cdist(inducing, pts), s1, rho, kind)
    A = sla.solve_triangular(L, Smn, lower=True)
    return np.ascontiguousarray((L @ bf16_round(A)).T)


class RoundedFSA(O.FSA):
    """The oracle's FSA on a supplied cross covariance, differentiated in
    sigma1^2 as a model proportional to sigma1^2 (the unrounded FSA is, with
    no jitter): dSigma~/dsigma1^2 = (Sigma~ - sigma^2 I) / sigma1^2.  The
    rho-derivative is the oracle's (exact dSigma_mn, dSigma_m)."""

    def dmatvec(self, which, X):
        if which == 0:
            return (self.matvec(X) - self.theta[3] * X) / self.theta[1]
        return super().dmatvec(which, X)

    def precond_dmatvec(self, which, X):
        """The preconditioner under the same convention: dP/dsigma1^2 =
        (P - sigma^2 I) / sigma1^2."""
        if which == 0:
            DX = self.D[:, None] * X if X.ndim == 2 else self.D * X
            return (DX + self.lowrank_matvec(X) - self.theta[3] * X) / self.theta[1]
        return super().precond_dmatvec(which, X)
