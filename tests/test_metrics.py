"""OSPA (section 4.1, p = 1, c = 100) against brute force over all
assignments, and its metric properties."""
import itertools
import math

import numpy as np

from paper_1503_03769_amd.metrics import ospa


def _brute(X, Y, c=100.0, p=1.0):
    X, Y = np.asarray(X).reshape(-1, 2), np.asarray(Y).reshape(-1, 2)
    if len(X) > len(Y):
        X, Y = Y, X
    m, n = len(X), len(Y)
    if n == 0:
        return 0.0
    best = math.inf
    for perm in itertools.permutations(range(n), m):
        s = sum(min(c, float(np.linalg.norm(X[i] - Y[perm[i]]))) ** p for i in range(m))
        best = min(best, s)
    return ((best + c ** p * (n - m)) / n) ** (1 / p)


def test_ospa_brute_force():
    rng = np.random.default_rng(0)
    for _ in range(60):
        m, n = rng.integers(0, 6), rng.integers(0, 7)
        X = rng.uniform(-150, 150, size=(m, 2))
        Y = rng.uniform(-150, 150, size=(n, 2))
        assert math.isclose(ospa(X, Y), _brute(X, Y), rel_tol=1e-12, abs_tol=1e-12)


def test_ospa_axioms():
    rng = np.random.default_rng(1)
    X = rng.uniform(-100, 100, size=(4, 2))
    Y = rng.uniform(-100, 100, size=(5, 2))
    Z = rng.uniform(-100, 100, size=(3, 2))
    assert ospa(X, X) == 0.0
    assert ospa(np.zeros((0, 2)), np.zeros((0, 2))) == 0.0
    assert ospa(np.zeros((0, 2)), Y) == 100.0
    assert math.isclose(ospa(X, Y), ospa(Y, X))
    assert ospa(X, Z) <= ospa(X, Y) + ospa(Y, Z) + 1e-12
    assert 0.0 <= ospa(X, Y) <= 100.0
