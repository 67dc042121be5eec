"""Pins of the oracle's update (Eqs 7-8, 10-15) and Step 3 sums (Eqs 16-18)
by identities and special cases that do not restate its code."""
import math

import numpy as np

from paper_1503_03769_amd.scenario import BASE_MODEL, make_scenario, random_particles


def _state(orc, K, cap, counts, seed, truth=None):
    st = orc.State(K, cap)
    X, W, n = random_particles(K, cap, counts, seed, truth=truth)
    st.X[:], st.W[:], st.n[:] = X, W, n
    return st


def _scenario(p, seed=5, steps=6):
    truth, Z = make_scenario(p, 4, steps, seed)
    k = max(range(1, steps + 1), key=lambda i: len(truth[i]))
    return truth[k], Z[k]


def test_mass_identity(orc):
    """Swapping the sums of Eq 8: sum_i w'_i = nu sum_i w_i + sum_p C/(kappa + C)."""
    p = dict(BASE_MODEL, partitions=3, clutter_rate=20.0)
    tr, Z = _scenario(p)
    st = _state(orc, 3, 700, [600, 333, 41], 9, truth=tr)
    W0 = st.W.copy()
    u = orc.update(p, st, Z)
    kap = orc.kappa(p)
    for j in range(3):
        sl = slice(j * 700, j * 700 + st.n[j])
        lhs = math.fsum(st.W[sl])
        rhs = (1 - p["p_D"]) * math.fsum(W0[sl]) + math.fsum(u["C"][j] / (kap + u["C"][j]))
        assert math.isclose(lhs, rhs, rel_tol=1e-12)
        assert math.isclose(u["mass"][j], lhs, rel_tol=1e-12)
        # Eq 16 in closed form, Eq 17
        assert np.allclose(u["dW"][j], u["C"][j] / (kap + u["C"][j]), rtol=1e-12, atol=1e-290)  # denormals aside
        assert math.isclose(u["dW0"][j], (1 - p["p_D"]) * math.fsum(W0[sl]), rel_tol=1e-12)


def test_no_measurements(orc):
    p = dict(BASE_MODEL, partitions=2)
    st = _state(orc, 2, 100, [80, 20], 3)
    W0 = st.W.copy()
    orc.update(p, st, np.zeros((0, 2)))
    assert np.array_equal(st.W[:80], (1 - p["p_D"]) * W0[:80])


def test_pd_zero_keeps_weights(orc):
    """p_D = 0: nothing is detected and the update is the identity, so predict
    followed by update scales every survivor weight by p_S."""
    p = dict(BASE_MODEL, partitions=1, p_D=0.0, births_per_step=0)
    tr, Z = _scenario(p)
    st = _state(orc, 1, 300, [250], 4, truth=tr)
    W0 = st.W.copy()
    orc.predict(p, st, 1, 3, 0)
    orc.update(p, st, Z)
    assert np.allclose(st.W[:250], p["p_S"] * W0[:250], rtol=1e-15, atol=0)


def test_heavy_clutter_limit(orc):
    p = dict(BASE_MODEL, partitions=1, clutter_rate=1e12)
    tr, Z = _scenario(dict(BASE_MODEL))
    st = _state(orc, 1, 300, [250], 4, truth=tr)
    W0 = st.W.copy()
    orc.update(p, st, Z)
    assert np.allclose(st.W[:250], (1 - p["p_D"]) * W0[:250], rtol=1e-6, atol=0)


def test_one_particle_one_measurement_no_clutter(orc):
    """kappa = 0, one particle and one measurement: the measurement term is
    exactly 1, so w' = (1 - p_D) w + 1."""
    p = dict(BASE_MODEL, partitions=1, clutter_rate=0.0)
    st = orc.State(1, 4)
    st.n[0] = 1
    st.X[:, 0] = [300.0, 1.0, -200.0, 2.0]
    st.W[0] = 0.37
    orc.update(p, st, np.array([[361.0, -0.58]]))
    assert math.isclose(st.W[0], (1 - p["p_D"]) * 0.37 + 1.0, rel_tol=1e-15)


def test_groups_are_independent(orc):
    """C is per group (each group sees all measurements, Eq 11): the update of
    group 0 does not depend on group 1's particles."""
    p2 = dict(BASE_MODEL, partitions=2)
    p1 = dict(BASE_MODEL, partitions=1)
    tr, Z = _scenario(p2)
    st = _state(orc, 2, 500, [400, 300], 12, truth=tr)
    one = orc.State(1, 500)
    one.X[:] = st.X[:, :500]
    one.W[:] = st.W[:500]
    one.n[0] = st.n[0]
    u2 = orc.update(p2, st, Z)
    u1 = orc.update(p1, one, Z)
    assert np.array_equal(u2["C"][0], u1["C"][0])
    assert np.array_equal(st.W[:400], one.W[:400])


def test_identical_particles_give_exact_local_estimate(orc):
    """A cloud of identical particles supporting a measurement has that
    particle's state as its Eq 18 estimate; two clouds give two labels."""
    p = dict(BASE_MODEL, partitions=1, clutter_rate=10.0, p_D=0.95)
    A = np.array([400.0, 3.0, 300.0, -2.0])
    B = np.array([-600.0, -1.0, 100.0, 4.0])
    st = orc.State(1, 400)
    st.n[0] = 400
    st.X[:, :200] = A[:, None]
    st.X[:, 200:] = B[:, None]
    st.W[:] = 1.0 / 200          # mass 2
    zA = [math.hypot(A[0], A[2]) + 3.0, math.atan2(A[2], A[0]) - 0.01]
    zB = [math.hypot(B[0], B[2]) - 5.0, math.atan2(B[2], B[0]) + 0.02]
    Z = np.array([[1500.0, 2.5], zA, zB, [100.0, -1.0]])
    u = orc.update(p, st, Z)
    e = orc.extract(p, 4, u)
    assert e["LT"][0] == 2
    assert list(np.nonzero(e["sel"][0])[0]) == [1, 2]
    assert np.allclose(e["zeta"][0, 1], A, rtol=1e-13)
    assert np.allclose(e["zeta"][0, 2], B, rtol=1e-13)
    f = orc.fuse(p, 4, e)
    assert list(f["label"]) == [1, 2] and list(f["votes"]) == [1, 1]
