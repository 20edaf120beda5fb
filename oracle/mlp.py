"""Oracle for the learned proposal -- TEST INFRASTRUCTURE ONLY.

Plain numpy FP64 versions of what the library's learned-proposal kernels
compute: per-vertex features, training targets aggregated from sample
records, and the 8 -> 64 -> 64 -> 1 GELU network's forward pass and
parameter gradient.  GELU is the exact form a * Phi(a).

Parameter layout: W1[64][8], b1[64], W2[64][64] (output j, input i), b2[64],
w3[64], b3 -- 4801 values.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

H = 64
IN = 8
SIZES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / math.sqrt(2.0)))


def gelu_grad(a):
    return 0.5 * (1.0 + erf(a / math.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


def h_index(values) -> int:
    """Largest h such that at least h of the values are >= h."""
    v = sorted(values, reverse=True)
    h = 0
    for i, x in enumerate(v, start=1):
        if x >= i:
            h = i
        else:
            break
    return h


def features(g, tables) -> np.ndarray:
    """[n, 4]: log2(1 + d), log2(1 + S2), log2(1 + C_v * C(d, 2)),
    log2(1 + h-index of the neighbour degrees)."""
    n = g.n
    d = np.diff(g.off).astype(np.int64)
    out = np.zeros((n, 4), dtype=np.float64)
    out[:, 0] = np.log2(1.0 + d)
    out[:, 1] = np.log2(1.0 + tables.s2.astype(np.float64))
    tri = np.where(tables.trials > 0,
                   tables.hits.astype(np.float64) / np.maximum(tables.trials, 1).astype(np.float64) * 0.5 * d * (d - 1),
                   0.0)
    out[:, 2] = np.log2(1.0 + tri)
    for v in range(n):
        row = g.nbr[int(g.off[v]):int(g.off[v + 1])]
        out[v, 3] = math.log2(1.0 + h_index(d[row].tolist()))
    return out


def targets_from_records(recs, k: int, n: int):
    """sums[i][v], counts[i][v]: for each record and step i it reached, the
    product of the factors of the steps after i (0 if the sample failed),
    taken from the last step backwards."""
    sums = np.zeros((k, n), dtype=np.float64)
    counts = np.zeros((k, n), dtype=np.int64)
    for r in recs:
        steps = int(r["steps"])
        ok = int(r["fail_step"]) < 0
        prod = 1.0
        for i in range(k - 1, -1, -1):
            if i < steps:
                sums[i, int(r["v"][i])] += prod if ok else 0.0
                counts[i, int(r["v"][i])] += 1
            if ok and i > 0:
                prod = prod * (float(int(r["num"][i])) / float(int(r["den"][i])))
    return sums, counts


def inputs(feats, vtx, cls):
    x = np.zeros((len(vtx), IN), dtype=np.float64)
    x[:, :4] = feats[np.asarray(vtx, dtype=np.int64)]
    x[np.arange(len(vtx)), 4 + np.minimum(np.asarray(cls, dtype=np.int64), 3)] = 1.0
    return x


def forward(theta, x):
    p = unpack(theta)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = gelu(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(a2)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (a1, h1, a2, h2)


def loss(theta, x, target, weight, weight_sum):
    y, _ = forward(theta, x)
    return float(np.sum(weight * (y - target) ** 2) / weight_sum)


def grad(theta, x, target, weight, weight_sum):
    """Gradient of sum_r w_r (y_r - t_r)^2 / weight_sum, by the chain rule."""
    p = unpack(theta)
    y, (a1, h1, a2, h2) = forward(theta, x)
    dy = 2.0 * weight * (y - target) / weight_sum                     # [R]
    g = {"b3": np.array([dy.sum()]), "w3": h2.T @ dy}
    d2 = (dy[:, None] * p["w3"][None, :]) * gelu_grad(a2)              # [R, 64]
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * gelu_grad(a1)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(axis=0)
    return pack(g)
