"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds no arithmetic of the FSA method itself: it only draws
locations, inducing points, responses and taper ranges that both sides then
receive as identical inputs.  Shapes and distributions follow the paper's
simulation study (Section 4: uniform locations on the unit square, Matérn
covariance, m inducing points by kmeans++, a taper range giving a target mean
number of nonzeros per row).
"""
from __future__ import annotations

import math
import os

import numpy as np

EXPONENTIAL = 0   # Matérn smoothness 1/2
MATERN32 = 1      # Matérn smoothness 3/2


def uniform_locations(n: int, seed: int) -> np.ndarray:
    """n points uniform on [0,1]^2, row-major (n, 2) float64 (Section 4)."""
    return np.random.default_rng(seed).random((n, 2))


def clustered_locations(n: int, seed: int, n_blobs: int = 10, sd: float = 0.02) -> np.ndarray:
    """Half uniform on [0,1]^2, half in Gaussian blobs (sd `sd`) whose centres
    are uniform on [0.1,0.9]^2; blob draws falling outside the unit square are
    redrawn."""
    rng = np.random.default_rng(seed)
    n_u = n // 2
    n_c = n - n_u
    out = np.empty((n, 2))
    out[:n_u] = rng.random((n_u, 2))
    centres = 0.1 + 0.8 * rng.random((n_blobs, 2))
    which = rng.integers(0, n_blobs, n_c)
    pts = centres[which] + sd * rng.standard_normal((n_c, 2))
    bad = np.any((pts < 0) | (pts > 1), axis=1)
    while bad.any():
        pts[bad] = centres[which[bad]] + sd * rng.standard_normal((int(bad.sum()), 2))
        bad = np.any((pts < 0) | (pts > 1), axis=1)
    out[n_u:] = pts
    return out


def random_subset_inducing(locs: np.ndarray, m: int, seed: int) -> np.ndarray:
    """m inducing points sampled uniformly without replacement from the
    locations (the paper's Assumption 2)."""
    idx = np.random.default_rng(seed).choice(locs.shape[0], size=m, replace=False)
    return np.ascontiguousarray(locs[np.sort(idx)])


def kmeanspp_inducing(locs: np.ndarray, m: int, seed: int, subsample: int = 20000,
                      lloyd_iters: int = 50) -> np.ndarray:
    """kmeans++ seeding (Arthur & Vassilvitskii 2007) on a seeded subsample,
    followed by Lloyd iterations until the assignment is stable or
    `lloyd_iters` is reached.  Returns cluster centres (m, 2)."""
    rng = np.random.default_rng(seed)
    n = locs.shape[0]
    pts = locs[rng.choice(n, size=min(subsample, n), replace=False)] if n > subsample else locs.copy()
    k = pts.shape[0]
    m = min(m, k)
    centres = np.empty((m, 2))
    centres[0] = pts[rng.integers(k)]
    d2 = np.sum((pts - centres[0]) ** 2, axis=1)
    for c in range(1, m):
        p = d2 / d2.sum()
        centres[c] = pts[rng.choice(k, p=p)]
        d2 = np.minimum(d2, np.sum((pts - centres[c]) ** 2, axis=1))
    assign = None
    for _ in range(lloyd_iters):
        new = np.empty(k, dtype=np.int64)

        def nearest(s):
            blk = pts[s:s + 2048]
            d2 = (blk[:, 0:1] - centres[None, :, 0]) ** 2 + (blk[:, 1:2] - centres[None, :, 1]) ** 2
            new[s:s + 2048] = d2.argmin(1)

        _parallel(nearest, range(0, k, 2048))
        if assign is not None and np.array_equal(new, assign):
            break
        assign = new
        cnt = np.bincount(assign, minlength=m)
        sx = np.bincount(assign, weights=pts[:, 0], minlength=m)
        sy = np.bincount(assign, weights=pts[:, 1], minlength=m)
        nz = cnt > 0
        centres[nz, 0] = sx[nz] / cnt[nz]
        centres[nz, 1] = sy[nz] / cnt[nz]
    return np.ascontiguousarray(centres)


def rff_response(locs: np.ndarray, kind: int, sigma1_sq: float, rho: float, sigma_sq: float,
                 n_features: int, seed: int) -> np.ndarray:
    """y = sqrt(2 sigma1^2 / F) sum_f cos(w_f . s + b_f) + N(0, sigma^2).

    Frequencies are drawn from the spectral density of the Matérn kernel in
    the parameterisation c(d) = sigma1^2 e^{-d/rho} (smoothness 1/2) and
    sigma1^2 (1 + sqrt(3) d/rho) e^{-sqrt(3) d/rho} (smoothness 3/2): a 2-D
    Student-t with 2 nu degrees of freedom scaled by 1/rho, i.e.
    w = g sqrt(2 nu / u) / rho with g ~ N(0, I_2) and u ~ chi^2_{2 nu}."""
    rng = np.random.default_rng(seed)
    w, b = _rff_frequencies(rng, kind, rho, n_features)
    y = np.empty(locs.shape[0])
    amp = math.sqrt(2 * sigma1_sq / n_features)

    def chunk(s):
        blk = locs[s:s + 8192]
        y[s:s + 8192] = amp * np.cos(blk @ w.T + b).sum(1)

    _parallel(chunk, range(0, locs.shape[0], 8192))
    y += math.sqrt(sigma_sq) * rng.standard_normal(locs.shape[0])
    return y


def _rff_frequencies(rng, kind, rho, n_features):
    nu = 0.5 if kind == EXPONENTIAL else 1.5
    g = rng.standard_normal((n_features, 2))
    u = rng.chisquare(2 * nu, size=n_features)
    w = g * (np.sqrt(2 * nu / u) / rho)[:, None]
    b = rng.uniform(0, 2 * np.pi, n_features)
    return w, b


def rff_response_torch(torch):
    """rff_response with the feature sum on torch's current CUDA device (the
    same draws; equal up to rounding): for generating many large inputs fast."""
    def response(locs, kind, sigma1_sq, rho, sigma_sq, n_features, seed):
        rng = np.random.default_rng(seed)
        w, b = _rff_frequencies(rng, kind, rho, n_features)
        L = torch.from_numpy(np.ascontiguousarray(locs)).cuda()
        W = torch.from_numpy(w).cuda()
        B = torch.from_numpy(b).cuda()
        y = (math.sqrt(2 * sigma1_sq / n_features) * torch.cos(L @ W.T + B).sum(1)).cpu().numpy()
        return y + math.sqrt(sigma_sq) * rng.standard_normal(locs.shape[0])
    return response


def _parallel(fn, items):
    """Run fn over items on a thread pool (numpy releases the GIL); the
    result does not depend on the number of threads."""
    from concurrent.futures import ThreadPoolExecutor
    nt = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(fn, items))


def mean_neighbours_uniform(n: int, gamma: float) -> float:
    """Expected nonzeros per row (self included) for n uniform points on the
    unit square: 1 + (n-1) F(gamma), F the CDF of the distance between two
    uniform points, F(r) = pi r^2 - 8 r^3 / 3 + r^4 / 2 for r <= 1."""
    r = gamma
    return 1.0 + (n - 1) * (math.pi * r * r - 8.0 * r ** 3 / 3.0 + 0.5 * r ** 4)


def taper_range_for_uniform(n: int, n_gamma: float) -> float:
    """Taper range giving `n_gamma` expected nonzeros per row (self included)
    for uniform points on the unit square (bisection on the closed form)."""
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_neighbours_uniform(n, mid) < n_gamma:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def taper_range_by_count(locs: np.ndarray, n_gamma: float, sample: int = 20000, seed: int = 0) -> float:
    """Taper range whose counted mean nonzeros per row (self included) on a
    sample of rows equals `n_gamma` (bisection; used for clustered inputs)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    tree = cKDTree(locs)
    rows = locs[rng.choice(locs.shape[0], size=min(sample, locs.shape[0]), replace=False)]
    lo, hi = 0.0, 0.5
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        cnt = np.mean([len(x) for x in tree.query_ball_point(rows, mid)])
        if cnt < n_gamma:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def poisson_arrivals(n_requests: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process with `rate` requests per second."""
    return np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, n_requests))


def laplace_weights(n: int, seed: int, lo: float = 0.05, hi: float = 0.25) -> np.ndarray:
    """n diagonal weights uniform on [lo, hi]: the range that the negative
    second derivative of a Bernoulli-logit log-likelihood takes for latent
    values |b| <= 3 (its maximum is 1/4)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, n)


def bernoulli_responses(locs: np.ndarray, kind: int, sigma1_sq: float, rho: float, n_features: int,
                        seed: int) -> np.ndarray:
    """Binary responses y_i ~ Bernoulli(1 / (1 + e^{-b_i})) of a latent
    Gaussian process b drawn by random Fourier features (rff_response with a
    negligible nugget): the setting of the Vecchia-Laplace experiments
    (binary likelihood, Section 5)."""
    b = rff_response(locs, kind, sigma1_sq, rho, 1e-12, n_features, seed)
    u = np.random.default_rng(seed + 1).uniform(size=locs.shape[0])
    return (u < 1.0 / (1.0 + np.exp(-b))).astype(np.float64)
