"""Pins of the oracle's global-C reading of Eq 11 (global_cz = 1): the K
groups are K parts of one PHD, C_k(z) is summed over all of them before
Eq 12, and each group carries 1/K of the mass (initial mass, birth mass);
Step 3's LT is the run's total mass, rounded, in every group, and Step 5
gives every group round(N_total R_j) children of weight N_j / L'_j (the
non-proportional allocation of the DRNA scheme).

The pins do not restate the oracle's code: the update of K groups must equal
the single-group update of their union (a K = 1 filter, which is the
paper's per-group formula), the swapped-sum identity must hold with the
global denominator, and the mass splits, LT and child counts are checked on
hand-built cases whose answers follow from the reading alone."""
import math

import numpy as np

from paper_1503_03769_amd.scenario import BASE_MODEL, make_scenario, random_particles


def _scenario(p, seed=5, steps=6):
    truth, Z = make_scenario(p, 4, steps, seed)
    k = max(range(1, steps + 1), key=lambda i: len(truth[i]))
    return truth[k], Z[k]


def _groups(orc, K, cap, counts, seed, truth):
    st = orc.State(K, cap)
    X, W, n = random_particles(K, cap, counts, seed, truth=truth)
    st.X[:], st.W[:], st.n[:] = X, W, n
    return st


def _union(orc, st):
    """The particles of every group in one group (group order)."""
    K, cap = st.K, st.cap
    tot = int(st.n.sum())
    u = orc.State(1, tot)
    o = 0
    for j in range(K):
        sl = slice(j * cap, j * cap + int(st.n[j]))
        u.X[:, o:o + int(st.n[j])] = st.X[:, sl]
        u.W[o:o + int(st.n[j])] = st.W[sl]
        o += int(st.n[j])
    u.n[0] = tot
    return u


def test_update_of_groups_equals_update_of_their_union(orc):
    """With one C over all groups the K groups update exactly as one filter
    holding all their particles: every weight equals the K = 1 (textbook
    per-group) update of the union, and the groups' C_j add up to the
    union's C."""
    K, cap = 4, 500
    p = dict(BASE_MODEL, partitions=K, clutter_rate=30.0, global_cz=1)
    tr, Z = _scenario(p)
    st = _groups(orc, K, cap, [420, 77, 300, 5], 11, tr)
    un = _union(orc, st)
    ug = orc.update(p, st, Z)
    uu = orc.update(dict(p, partitions=1, global_cz=0), un, Z)
    o = 0
    for j in range(K):
        nj = int(st.n[j])
        np.testing.assert_allclose(st.W[j * cap:j * cap + nj], un.W[o:o + nj], rtol=1e-12, atol=0)
        o += nj
    np.testing.assert_allclose(ug["C"].sum(axis=0), uu["C"][0], rtol=1e-12, atol=1e-300)
    # the per-group reading differs on the same input (a wrong denominator
    # would not pass the comparison above)
    st2 = _groups(orc, K, cap, [420, 77, 300, 5], 11, tr)
    orc.update(dict(p, global_cz=0), st2, Z)
    assert not np.allclose(st2.W[:420], un.W[:420], rtol=1e-6)


def test_mass_identity_with_the_global_denominator(orc):
    """Swapping the sums of Eq 8 with D(z) = kappa + sum_j C_j(z):
    group j's new mass is nu sum_i w_i + sum_p C_j(z_p)/D(z_p), and Delta W^{j,p}
    (Eq 16) is C_j(z_p)/D(z_p)."""
    K, cap = 3, 600
    p = dict(BASE_MODEL, partitions=K, clutter_rate=20.0, global_cz=1)
    tr, Z = _scenario(p, seed=8)
    st = _groups(orc, K, cap, [590, 200, 333], 4, tr)
    W0 = st.W.copy()
    u = orc.update(p, st, Z)
    D = orc.kappa(p) + u["C"].sum(axis=0)
    for j in range(K):
        sl = slice(j * cap, j * cap + int(st.n[j]))
        rhs = (1 - p["p_D"]) * math.fsum(W0[sl]) + math.fsum(u["C"][j] / D)
        assert math.isclose(u["mass"][j], rhs, rel_tol=1e-12)
        assert math.isclose(math.fsum(st.W[sl]), rhs, rel_tol=1e-12)
        np.testing.assert_allclose(u["dW"][j], u["C"][j] / D, rtol=1e-12, atol=1e-290)


def test_one_group_is_the_per_group_filter(orc):
    """K = 1: the global and per-group readings are the same filter."""
    p = dict(BASE_MODEL, partitions=1, clutter_rate=10.0, births_per_step=300, particles_per_target=900.0)
    a = orc.OracleFilter(dict(p, global_cz=1), 4000, 3, 0)
    b = orc.OracleFilter(dict(p, global_cz=0), 4000, 3, 0)
    truth, Z = make_scenario(p, 3, 4, 21)
    for k in range(1, 5):
        oa, ob = a.step(k, Z[k]), b.step(k, Z[k])
        assert np.array_equal(oa["counts"], ob["counts"])
        assert list(oa["est"]["label"]) == list(ob["est"]["label"])
    assert np.array_equal(a.st.W, b.st.W) and np.array_equal(a.st.X, b.st.X)


def test_masses_are_split_over_the_groups(orc):
    """t = 0 and the births of Eq 6: the groups' initial weights add up to
    init_mass over all groups, and every birth weighs 1/K of what it weighs
    when each group carries the full birth mass (the same draws)."""
    K, cap = 4, 2000
    p = dict(BASE_MODEL, partitions=K, births_per_step=402, particles_per_target=4000.0, init_mass=2.0)
    g = orc.State(K, cap)
    orc.init(dict(p, global_cz=1), g, 5, 0)
    assert math.isclose(math.fsum(g.W), 2.0, rel_tol=1e-12)
    for j in range(K):
        assert math.isclose(math.fsum(g.W[j * cap:(j + 1) * cap]), 2.0 / K, rel_tol=1e-12)
    truth, Z = make_scenario(p, 3, 2, 9)
    for prop in (0, 1):
        q = dict(p, birth_proposal=prop, birth_alpha=0.1)
        a, b = orc.State(K, cap), orc.State(K, cap)
        orc.init(dict(q, global_cz=1), a, 5, 0)
        orc.init(dict(q, global_cz=0), b, 5, 0)
        n0 = a.n.copy()
        for s, gz in ((a, 1), (b, 0)):
            orc.predict(dict(q, global_cz=gz), s, 1, 5, 0)
            if prop == 1:
                orc.birth_from_measurements(dict(q, global_cz=gz), s, 1, 5, 0, Z[1])
        for j in range(K):
            sl = slice(j * cap + int(n0[j]), j * cap + int(a.n[j]))
            assert np.array_equal(a.X[:, sl], b.X[:, sl])
            np.testing.assert_allclose(a.W[sl], b.W[sl] / K, rtol=1e-15, atol=0)
        if prop == 0:
            tot = sum(math.fsum(a.W[j * cap + int(n0[j]):j * cap + int(a.n[j])]) for j in range(K))
            assert math.isclose(tot, p["birth_mass"], rel_tol=1e-12)


def test_target_number_and_child_counts_follow_the_total_mass(orc):
    """Step 3 and Step 5 read the run's total mass.  Four groups of masses
    0.1, 0.2, 0.3 and 0.6 (1.2 targets in all): LT = round(1.2) = 1 in every
    group (the groups' own masses would give 0, 0, 0, 1); every group draws
    round(1.2 R_j) children, each of weight N_j / L'_j, so the groups' masses
    stay 0.1, 0.2, 0.3 and 0.6."""
    K, cap, n = 4, 600, 500
    p = dict(BASE_MODEL, partitions=K, particles_per_target=4 * 250.0, births_per_step=0, global_cz=1)
    masses = [0.1, 0.2, 0.3, 0.6]
    M = 3
    dW = np.tile(np.array([0.05, 0.2, 0.1]), (K, 1))
    zn = np.ones((K, M, 4))
    e = orc.extract(p, M, dict(dW=dW, zeta_num=zn, mass=np.array(masses)))
    assert list(e["LT"]) == [1] * K
    assert all(list(np.nonzero(e["sel"][j])[0]) == [1] for j in range(K))
    e0 = orc.extract(dict(p, global_cz=0), M, dict(dW=dW, zeta_num=zn, mass=np.array(masses)))
    assert list(e0["LT"]) == [0, 0, 0, 1]
    st = orc.State(K, cap)
    st.n[:] = n
    for j in range(K):
        st.W[j * cap:j * cap + n] = masses[j] / n
        st.X[0, j * cap:j * cap + n] = np.linspace(10.0, 500.0, n)
        st.X[2, j * cap:j * cap + n] = 100.0
    out, counts, mq = orc.resample(p, st, 1, 5, 0)
    R_j = p["particles_per_target"] / K
    assert list(out.n) == [int(math.floor(1.2 * R_j + 0.5))] * K  # 300 children each
    for j in range(K):
        assert counts[j * cap:(j + 1) * cap].sum() == out.n[j]
        np.testing.assert_allclose(out.W[j * cap:j * cap + out.n[j]], mq[j] / out.n[j], rtol=0, atol=0)
        assert math.isclose(mq[j], masses[j], rel_tol=1e-12)
    out0, _, _ = orc.resample(dict(p, global_cz=0), st, 1, 5, 0)
    assert list(out0.n) == [int(math.floor(mj * R_j + 0.5)) for mj in masses]
