"""Pins of the 5-D coordinated-turn option of the oracle (state [x, vx, y,
vy, omega]; not in the paper, the textbook CT model): the noise-free
transition against a Runge-Kutta integration of the turn ODE, the omega = 0
case against the CV transition, speed conservation, the turn-rate noise and
birth spread, and the fifth component carried through resampling and the
exchange."""
import math

import numpy as np

from paper_1503_03769_amd.scenario import BASE_MODEL

CT = dict(BASE_MODEL, dim=5, sigma_w=0.01, birth_sigma_w=0.05, partitions=1, births_per_step=0,
          particles_per_target=200.0)


def _rk4_turn(x, T, steps=2000):
    """x' = vx, vx' = -w vy, y' = vy, vy' = w vx, w' = 0."""
    s = np.array(x, dtype=np.float64)

    def f(u):
        return np.array([u[1], -u[4] * u[3], u[3], u[4] * u[1], 0.0])

    h = T / steps
    for _ in range(steps):
        k1 = f(s)
        k2 = f(s + 0.5 * h * k1)
        k3 = f(s + 0.5 * h * k2)
        k4 = f(s + h * k3)
        s = s + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return s


def _state(orc, X, p, cap):
    st = orc.State(1, cap, 5)
    n = X.shape[1]
    st.X[:, :n] = X
    st.W[:n] = 1.0 / n
    st.n[0] = n
    return st


def test_noise_free_turn_matches_integration(orc):
    p = dict(CT, sigma_a=0.0, sigma_w=0.0, T=2.0)
    rng = np.random.default_rng(1)
    X = np.stack([rng.uniform(-500, 500, 8), rng.normal(0, 10, 8), rng.uniform(-500, 500, 8),
                  rng.normal(0, 10, 8), np.array([0.3, -0.2, 0.05, -0.05, 1e-3, -1e-7, 0.0, 0.7])])
    st = _state(orc, X, p, 64)
    orc.predict(p, st, 1, 9, 0)
    for i in range(8):
        ref = _rk4_turn(X[:, i], 2.0)
        np.testing.assert_allclose(st.X[:, i], ref, rtol=1e-9, atol=1e-9)


def test_zero_turn_rate_is_the_cv_model(orc):
    p5 = dict(CT, sigma_w=0.0)
    p4 = dict(BASE_MODEL, partitions=1, births_per_step=0, particles_per_target=200.0)
    rng = np.random.default_rng(2)
    X = np.stack([rng.uniform(-500, 500, 50), rng.normal(0, 10, 50), rng.uniform(-500, 500, 50),
                  rng.normal(0, 10, 50), np.zeros(50)])
    st5 = _state(orc, X, p5, 64)
    st4 = orc.State(1, 64)
    st4.X[:, :50] = X[:4]
    st4.W[:50] = 1.0 / 50
    st4.n[0] = 50
    orc.predict(p5, st5, 3, 9, 0)
    orc.predict(p4, st4, 3, 9, 0)
    assert np.array_equal(st5.X[:4, :50], st4.X[:, :50])
    assert np.all(st5.X[4, :50] == 0.0)


def test_turn_keeps_speed_and_noise_has_its_spread(orc):
    p = dict(CT, sigma_a=0.0, sigma_w=0.02, T=1.0)
    n = 20000
    rng = np.random.default_rng(3)
    X = np.stack([np.zeros(n), rng.normal(0, 10, n), np.zeros(n), rng.normal(0, 10, n), rng.normal(0, 0.1, n)])
    st = _state(orc, X, p, n + 8)
    orc.predict(p, st, 1, 4, 0)
    v0 = np.hypot(X[1], X[3])
    v1 = np.hypot(st.X[1, :n], st.X[3, :n])
    np.testing.assert_allclose(v1, v0, rtol=1e-12)
    dw = st.X[4, :n] - X[4]
    assert abs(dw.mean()) < 5 * 0.02 / math.sqrt(n)
    assert abs(dw.std() / 0.02 - 1) < 0.03


def test_birth_turn_rates_follow_the_birth_density(orc):
    p = dict(CT, births_per_step=20000)
    st = orc.State(1, 20300, 5)
    st.n[0] = 200
    orc.predict(p, st, 2, 5, 0)
    w = st.X[4, 200:20200]
    assert abs(w.mean()) < 5 * 0.05 / math.sqrt(20000)
    assert abs(w.std() / 0.05 - 1) < 0.03


def test_fifth_component_follows_resampling_and_exchange(orc):
    p = dict(CT, partitions=3, particles_per_target=600.0, exchange_fraction=0.2)
    K, cap = 3, 1024
    st = orc.State(K, cap, 5)
    rng = np.random.default_rng(4)
    for j in range(K):
        n = 300 + 50 * j
        st.n[j] = n
        sl = slice(j * cap, j * cap + n)
        st.X[:, sl] = rng.normal(size=(5, n))
        st.W[sl] = rng.uniform(0.1, 1.0, n) / n
    out, counts, _ = orc.resample(p, st, 6, 11, 0)
    # every child is a copy of its parent, all five components
    for j in range(K):
        parents = {tuple(st.X[:, j * cap + i]) for i in range(int(st.n[j]))}
        for c in range(int(out.n[j])):
            assert tuple(out.X[:, j * cap + c]) in parents
    before = sorted(tuple(np.r_[out.X[:, j * cap + i], out.W[j * cap + i]])
                    for j in range(K) for i in range(int(out.n[j])))
    orc.exchange(p, out, 6, 11, 0)
    after = sorted(tuple(np.r_[out.X[:, j * cap + i], out.W[j * cap + i]])
                   for j in range(K) for i in range(int(out.n[j])))
    assert before == after
