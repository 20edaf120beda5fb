"""Oracle estimator statistics -- TEST INFRASTRUCTURE ONLY.

Algorithm 1 ("Online Convergence Detection"): with N sampler outputs,
mu = mean, sigma^2 = (1/N) sum L_i^2 - mu^2 (population variance), and the
estimated relative error eps_hat = Phi^{-1}(1 - delta/2) * sigma / (sqrt(N) mu).
Sampling stops once eps_hat <= eps.  The mean and variance are accumulated
with Welford's recurrence (the same quantities, computed stably).
"""

from __future__ import annotations

import math
from statistics import NormalDist


def z_value(delta: float) -> float:
    return NormalDist().inv_cdf(1.0 - delta / 2.0)


def eps_hat(n: int, mean: float, m2: float, delta: float) -> float:
    if n == 0 or mean == 0.0:
        return math.inf
    sigma = math.sqrt(max(m2, 0.0) / n)
    return z_value(delta) * sigma / (math.sqrt(n) * abs(mean))


def direct_stats(xs):
    """Algorithm 1's formulas evaluated literally on a stored list."""
    n = len(xs)
    mu = sum(xs) / n
    var = sum(x * x for x in xs) / n - mu * mu
    return n, mu, var


def run_to_eps(sampler, eps: float, delta: float, batch: int, min_samples: int, budget: int):
    """Check after every batch of ``batch`` samples, from ``min_samples`` on.

    Returns (stats, converged).  Sample indices are 0, 1, 2, ... so the
    stopping point depends only on the outputs of the samples drawn so far.
    """
    from . import Stats
    st = Stats()
    done = 0
    while done < budget:
        cnt = min(batch, budget - done)
        sampler.run(done, cnt, st)
        done += cnt
        if done >= min_samples and eps_hat(st.n, st.mean, st.m2, delta) <= eps:
            return st, True
    return st, False
