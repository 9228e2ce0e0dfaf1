"""The five workload recipes: sizes, covariance parameters, seeds.

Seeds are 1000+c (locations), 2000+c (inducing points), 3000+c (response),
4000+c (probe key) for configuration c.  Every array is built by
`generators`; nothing here computes any part of the FSA method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import generators as g


@dataclass
class Workload:
    name: str
    locs: np.ndarray
    y: np.ndarray
    inducing: np.ndarray
    kind: int
    sigma1_sq: float
    rho: float
    sigma_sq: float
    gamma: float
    num_probes: int
    seed: int
    tol: float
    pred_locs: np.ndarray | None = None
    num_samples: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.locs.shape[0]

    @property
    def m(self) -> int:
        return self.inducing.shape[0]

    @property
    def theta(self) -> tuple:
        return (self.kind, self.sigma1_sq, self.rho, self.sigma_sq)


def small_fp64(n: int = 2000) -> Workload:
    """n=2000 uniform, exponential (sigma1^2=1, rho=0.1, sigma^2=0.05), m=50
    random subset, ~30 nonzeros/row, 1000 RFF features, t=10, tol 1e-8."""
    c = 1
    locs = g.uniform_locations(n, 1000 + c)
    ind = g.random_subset_inducing(locs, 50, 2000 + c)
    y = g.rff_response(locs, g.EXPONENTIAL, 1.0, 0.1, 0.05, 1000, 3000 + c)
    gamma = g.taper_range_for_uniform(n, 30)
    return Workload("n2000_m50_exp_t10", locs, y, ind, g.EXPONENTIAL, 1.0, 0.1, 0.05, gamma, 10,
                    4000 + c, 1e-8)


def large_matern(n: int = 500_000, m: int = 500, t: int = 50) -> Workload:
    """n=500k uniform, Matérn-3/2 (sigma1^2=1, rho=0.05, sigma^2=0.1), m=500
    kmeans++ on a 20k subsample, ~80 nonzeros/row, 2000 RFF features, t=50."""
    c = 2
    locs = g.uniform_locations(n, 1000 + c)
    ind = g.kmeanspp_inducing(locs, m, 2000 + c)
    y = g.rff_response(locs, g.MATERN32, 1.0, 0.05, 0.1, 2000, 3000 + c)
    gamma = g.taper_range_for_uniform(n, 80)
    return Workload(f"n{n}_m{m}_matern32_t{t}", locs, y, ind, g.MATERN32, 1.0, 0.05, 0.1, gamma, t,
                    4000 + c, 1e-8)


def clustered_grad(n: int = 200_000, m: int = 300, t: int = 50) -> Workload:
    """n=200k, half uniform and half in 10 blobs (sd 0.02), exponential
    (sigma1^2=2, rho=0.2, sigma^2=0.01), m=300 kmeans++, ~50 nonzeros/row."""
    c = 3
    locs = g.clustered_locations(n, 1000 + c)
    ind = g.kmeanspp_inducing(locs, m, 2000 + c)
    y = g.rff_response(locs, g.EXPONENTIAL, 2.0, 0.2, 0.01, 1000, 3000 + c)
    gamma = g.taper_range_by_count(locs, 50)
    return Workload(f"n{n}_m{m}_exp_clustered_t{t}", locs, y, ind, g.EXPONENTIAL, 2.0, 0.2, 0.01,
                    gamma, t, 4000 + c, 1e-8)


def predictive(n: int = 200_000, n_p: int = 200_000, m: int = 500, s: int = 100) -> Workload:
    """Training and prediction sets uniform, exponential (sigma1^2=1, rho=0.1,
    sigma^2=0.1), m=500 kmeans++, ~60 nonzeros/row, s=100 simulated samples."""
    c = 4
    locs = g.uniform_locations(n, 1000 + c)
    pred = g.uniform_locations(n_p, 5000 + c)
    ind = g.kmeanspp_inducing(locs, m, 2000 + c)
    y = g.rff_response(locs, g.EXPONENTIAL, 1.0, 0.1, 0.1, 1000, 3000 + c)
    gamma = g.taper_range_for_uniform(n, 60)
    return Workload(f"n{n}_np{n_p}_m{m}_exp_s{s}", locs, y, ind, g.EXPONENTIAL, 1.0, 0.1, 0.1, gamma,
                    10, 4000 + c, 1e-8, pred_locs=pred, num_samples=s)


# ---------------------------------------------------------------- serving stream
@dataclass
class ServingRequest:
    """One request of the serving stream: its arrival time and the recipe of
    its inputs (drawn by `materialize`)."""
    index: int
    arrival_s: float
    kind: str           # "nll_grad" or "predict_var"
    n: int
    m: int
    cov: int
    sigma1_sq: float
    rho: float
    sigma_sq: float
    n_gamma: float
    gamma: float
    n_p: int
    num_samples: int
    seed: int

    @property
    def theta(self) -> tuple:
        return (self.cov, self.sigma1_sq, self.rho, self.sigma_sq)

    def materialize(self, n_features: int = 256, response=None):
        """(locs, y, inducing, pred_locs or None).  `response` may replace
        g.rff_response (same arguments) with an equivalent generator."""
        locs = g.uniform_locations(self.n, self.seed)
        ind = g.random_subset_inducing(locs, self.m, self.seed + 1)
        rf = response or g.rff_response
        y = rf(locs, self.cov, self.sigma1_sq, self.rho, self.sigma_sq, n_features, self.seed + 2)
        pred = g.uniform_locations(self.n_p, self.seed + 3) if self.kind == "predict_var" else None
        return locs, y, ind, pred


def serving_trace(n_requests: int = 512, rate: float = 50.0, n_lo: int = 5000, n_hi: int = 300_000,
                  m_choices=(100, 200, 500), p_grad: float = 0.7, num_samples: int = 20,
                  seed: int = 5) -> list:
    """The serving stream: Poisson arrivals at `rate` per second; n
    log-uniform in [n_lo, n_hi]; m from `m_choices`; exponential or
    Matérn-3/2 with probability 1/2; rho ~ U[0.03, 0.2], sigma^2 ~ U[0.01,
    0.2], sigma1^2 = 1; ~U[40, 80] nonzeros per row; a fraction p_grad of
    likelihood + gradient requests, the rest predictive variances at n/4
    uniform locations with `num_samples` simulated samples; random-subset
    inducing points.  Seeded by `seed` (the trace) and per request."""
    rng = np.random.default_rng(5000 + seed)
    arr = g.poisson_arrivals(n_requests, rate, 6000 + seed)
    out = []
    for i in range(n_requests):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(rng.choice(np.asarray(m_choices)))
        cov = g.EXPONENTIAL if rng.uniform() < 0.5 else g.MATERN32
        rho = float(rng.uniform(0.03, 0.2))
        s2 = float(rng.uniform(0.01, 0.2))
        ng = float(rng.uniform(40.0, 80.0))
        kind = "nll_grad" if rng.uniform() < p_grad else "predict_var"
        out.append(ServingRequest(i, float(arr[i]), kind, n, min(m, n), cov, 1.0, rho, s2, ng,
                                  g.taper_range_for_uniform(n, ng), max(1, n // 4) if kind == "predict_var" else 0,
                                  num_samples if kind == "predict_var" else 0, (1000 + seed) * 100_000 + 10 * i))
    return out
