"""Exact sampling-tree enumeration -- TEST INFRASTRUCTURE ONLY.

Walks every branch of the sampler's probability tree on a tiny graph, using
the oracle's own step distributions, with exact rational probabilities.
This gives the exact E[X] and E[X^2] of the sampler: by Theorem 2
("unbiasedness") E[X] must equal the number of embeddings whenever every
extendable candidate has positive probability, and by Theorem 1 the
variance vanishes when the weights are the exact extension counts.
"""

from __future__ import annotations

from fractions import Fraction


def enumerate_tree(sampler, literal_cv=None):
    """Returns dict with total probability, E[X], E[X^2] and the list of
    successful trajectories (each as a tuple of data vertices in order).

    literal_cv: when given, use the literal real-valued f_approx weights with
    this clustering-coefficient array (floats turned into exact fractions).
    """
    k = sampler.compiled["k"]
    out = {"p_total": Fraction(0), "ex": Fraction(0), "ex2": Fraction(0), "success": []}

    def dist(i, tau):
        if literal_cv is None:
            v, w = sampler.step_distribution(i, tau)
            return [(int(a), Fraction(int(b))) for a, b in zip(v, w)]
        v, w = sampler.step_distribution_literal(i, tau, literal_cv)
        return [(int(a), Fraction(float(b))) for a, b in zip(v, w)]

    def rec(i, tau, p):
        if i == k:
            out["p_total"] += p
            x = 1 / p
            out["ex"] += p * x
            out["ex2"] += p * x * x
            out["success"].append(tuple(tau))
            return
        cands = dist(i, tau)
        total = sum(w for _, w in cands)
        if total == 0:
            out["p_total"] += p
            return
        for v, w in cands:
            if w == 0:
                continue
            rec(i + 1, tau + [v], p * w / total)

    rec(0, [], Fraction(1))
    return out
