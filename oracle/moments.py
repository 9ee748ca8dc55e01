"""Oracle for the joint moments of each unit up to fourth order: the
covariance, coskewness and cokurtosis that the joint plots compare between
the raw data and the fitted distribution models (Sec. 4.4, "Interactive
Joint Plots").

TEST INFRASTRUCTURE ONLY (see the package docstring).  Direct two-pass
float64 numpy: the mean of each unit first, then the centred products.

For a unit with voxels v and variables x_1 .. x_m (d = x - mean):
  M2[i, j]       = sum d_i d_j              i <= j
  M3[i, j, k]    = sum d_i d_j d_k          i <= j <= k
  M4[i, j, k, l] = sum d_i d_j d_k d_l      i <= j <= k <= l
each packed in lexicographic order of its index tuple (`tuples(m, r)`).
Coskewness and cokurtosis are these sums divided by n and the standard
deviations of the indices involved.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import combinations_with_replacement

import numpy as np

NONE_ID = 0xFFFFFFFF


def tuples(m: int, r: int):
    """Index tuples i1 <= ... <= ir over m variables, lexicographic."""
    return list(combinations_with_replacement(range(m), r))


@dataclass
class Moments:
    n: np.ndarray      # uint64 [U]
    mean: np.ndarray   # float64 [U, m]
    m2: np.ndarray     # float64 [U, P2]
    m3: np.ndarray     # float64 [U, P3]
    m4: np.ndarray     # float64 [U, P4]


def comoments(unit: np.ndarray, n_units: int, variables: np.ndarray) -> Moments:
    """Direct centred joint moments of orders 2, 3 and 4 of every unit."""
    u = np.asarray(unit, dtype=np.uint32).reshape(-1)
    m = variables.shape[0]
    x = np.asarray(variables, dtype=np.float32).reshape(m, -1).astype(np.float64)
    keep = u != NONE_ID
    u = u[keep].astype(np.int64)
    x = x[:, keep]
    U = int(n_units)
    cnt = np.bincount(u, minlength=U).astype(np.uint64)
    safe = np.maximum(cnt, 1).astype(np.float64)
    mean = np.stack([np.bincount(u, weights=x[j], minlength=U) / safe for j in range(m)], axis=1)
    mean[cnt == 0] = 0.0
    d = x - mean[u].T  # centred on the unit's own mean
    out = []
    for r in (2, 3, 4):
        cols = []
        for tup in tuples(m, r):
            p = d[tup[0]].copy()
            for k in tup[1:]:
                p *= d[k]
            cols.append(np.bincount(u, weights=p, minlength=U))
        out.append(np.stack(cols, axis=1))
    return Moments(cnt, mean, out[0], out[1], out[2])
