"""Pins of Step 3 (local estimation) and Step 4 (central fusion) on
hand-built cases, and of the grouped filter against the textbook filter of
section 2.2 at K = 1."""
import numpy as np

from paper_1503_03769_amd.scenario import BASE_MODEL, make_scenario


def _upd(dW, zeta_num, mass):
    return dict(dW=np.asarray(dW, float), zeta_num=np.asarray(zeta_num, float), mass=np.asarray(mass, float))


def test_extract_round_cap_and_ties(orc):
    p = dict(BASE_MODEL, partitions=3)
    M = 4
    dW = [[0.9, 0.2, 0.9, 0.0], [0.1, 0.3, 0.2, 0.4], [0.5, 0.5, 0.0, 0.0]]
    zn = np.ones((3, M, 4))
    e = orc.extract(p, M, _upd(dW, zn, [2.5, 7.0, 2.49]))
    assert list(e["LT"]) == [3, 4, 2]               # round = floor(x + 0.5), capped at M
    assert list(e["sel"][0]) == [1, 1, 1, 0]        # a zero-support label is never chosen
    assert list(e["sel"][1]) == [1, 1, 1, 1]
    assert list(e["sel"][2]) == [1, 1, 0, 0]
    e = orc.extract(p, M, _upd(dW, zn, [1.0, 1.0, 1.0]))
    assert list(e["sel"][0]) == [1, 0, 0, 0]        # tie between labels 0 and 2 goes to 0
    assert list(e["sel"][2]) == [1, 0, 0, 0]
    assert np.allclose(e["zeta"][0, 0], 1 / 0.9)     # Eq 18: numerator / Delta W


def test_fuse_majority_and_mean(orc):
    p = dict(BASE_MODEL, partitions=4)
    M = 3
    sel = np.zeros((4, M), dtype=np.int32)
    zeta = np.zeros((4, M, 4))
    sel[[0, 1, 2], 0] = 1                    # 3 of 4 groups: kept
    sel[[0, 3], 1] = 1                       # 2 of 4: not more than half, dropped
    sel[:, 2] = 1                            # all groups
    for j in range(4):
        zeta[j, :, :] = j + np.arange(4)[None, :] * 10
    f = orc.fuse(p, M, dict(sel=sel, zeta=zeta))
    assert list(f["label"]) == [0, 2]
    assert list(f["votes"]) == [3, 4]
    assert np.allclose(f["state"][0], np.mean([zeta[j, 0] for j in (0, 1, 2)], axis=0))
    assert np.allclose(f["state"][1], zeta[:, 2].mean(axis=0))


def test_fuse_single_group_keeps_all(orc):
    p = dict(BASE_MODEL, partitions=1)
    sel = np.array([[1, 0, 1]], dtype=np.int32)
    zeta = np.arange(12, dtype=float).reshape(1, 3, 4)
    f = orc.fuse(p, 3, dict(sel=sel, zeta=zeta))
    assert list(f["label"]) == [0, 2] and np.array_equal(f["state"], zeta[0, [0, 2]])


def test_grouped_filter_with_one_group_is_the_textbook_filter(orc):
    """Algorithm 1 with K = 1 reduces to the particle PHD filter of section 2.2
    (Eqs 5-8 and its resampling); both consume the same random streams."""
    p = dict(BASE_MODEL, partitions=1, particles_per_target=300.0, births_per_step=150)
    truth, Z = make_scenario(p, 3, 8, 77)
    cap = 4096
    seed, run = 21, 2
    g = orc.State(1, cap)
    orc.init(p, g, seed, run)
    for k in range(1, 9):
        t = g.copy()
        orc.predict(p, g, k, seed, run)
        orc.update(p, g, Z[k])
        Wupd, res = orc.textbook_step(p, t, k, seed, run, Z[k])
        n = int(g.n[0])
        assert int(t.n[0]) == n
        assert np.array_equal(t.X[:, :n], g.X[:, :n])          # Eq 5 / Eq 6 draws coincide
        assert np.allclose(Wupd[:n], g.W[:n], rtol=1e-13, atol=0)   # Eq 8 vs Eqs 12-15
        g, counts, mq = orc.resample(p, g, k, seed, run)
        L = int(g.n[0])
        assert int(res.n[0]) == L and int(counts.sum()) == L
        assert np.array_equal(res.X[:, :L], g.X[:, :L])
        assert np.allclose(res.W[:L], g.W[:L], rtol=1e-13, atol=0)
        orc.exchange(p, g, k, seed, run)                        # a no-op at K = 1
