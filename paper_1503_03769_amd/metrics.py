"""Evaluation metric of section 4.1: the OSPA miss distance (Schuhmacher,
Vo and Vo, 2008) between estimated and true target positions, with the
paper's parameters p = 1 and cut-off c = 100 m.

For |X| = m <= |Y| = n:
  d(X, Y) = ( (min over injections pi of sum_i min(c, |x_i - y_pi(i)|)^p
              + c^p (n - m)) / n )^(1/p),
d(empty, empty) = 0, and the definition is symmetric.  The optimal
assignment is solved with scipy's Hungarian-method routine.
"""
import numpy as np
from scipy.optimize import linear_sum_assignment


def ospa(X, Y, c: float = 100.0, p: float = 1.0) -> float:
    X = np.asarray(X, dtype=np.float64).reshape(-1, 2)
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 2)
    m, n = X.shape[0], Y.shape[0]
    if m == 0 and n == 0:
        return 0.0
    if m > n:
        X, Y, m, n = Y, X, n, m
    if m == 0:
        return float(c)
    D = np.sqrt(((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1))
    D = np.minimum(D, c) ** p
    r, col = linear_sum_assignment(D)
    total = D[r, col].sum() + (c ** p) * (n - m)
    return float((total / n) ** (1.0 / p))


def positions(states):
    """(x, y) columns of [k, 4] CV states [x, vx, y, vy]."""
    s = np.asarray(states, dtype=np.float64).reshape(-1, 4)
    return s[:, [0, 2]]
