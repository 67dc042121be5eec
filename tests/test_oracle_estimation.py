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
    (Eqs 5-8 and systematic resampling), written separately in the oracle
    with no particle reordering.  One step of each from the same state, at
    eight states of the grouped filter's run: the predicted survivors agree
    slot by slot, the births agree as a set (the same Philox draws; the
    grouped filter puts them in bearing order), every updated weight agrees,
    and both resamplings draw the same number of children with the same
    weight, each parent getting the floor or the ceiling of L w_i / sum w in
    both (so their counts differ by at most one)."""
    p = dict(BASE_MODEL, partitions=1, particles_per_target=300.0, births_per_step=150)
    truth, Z = make_scenario(p, 3, 8, 77)
    cap = 4096
    seed, run = 21, 2
    g = orc.State(1, cap)
    orc.init(p, g, seed, run)

    def key_order(X, W, n):
        return np.lexsort(np.vstack([W[:n], X[::-1, :n]]))

    for k in range(1, 9):
        t = g.copy()
        L0 = int(g.n[0])
        orc.predict(p, g, k, seed, run)
        orc.update(p, g, Z[k])
        Wupd, res = orc.textbook_step(p, t, k, seed, run, Z[k])
        n = int(g.n[0])
        assert int(t.n[0]) == n
        # Eq 5: survivors in place; Eq 6: the same births, in another order
        assert np.array_equal(t.X[:, :L0], g.X[:, :L0])
        og, ot = key_order(g.X, np.zeros(cap), n), key_order(t.X, np.zeros(cap), n)
        assert np.array_equal(t.X[:, ot], g.X[:, og])
        # Eq 8 against Eqs 12-15, particle by particle
        np.testing.assert_allclose(Wupd[ot], g.W[og], rtol=1e-13, atol=0)
        assert len(np.unique(g.X[0, :n])) == n  # states identify particles below
        parents_g = {x: i for i, x in enumerate(g.X[0, :n])}
        gr, counts_g, mq = orc.resample(p, g, k, seed, run)
        L = int(gr.n[0])
        assert int(res.n[0]) == L and int(counts_g.sum()) == L
        np.testing.assert_allclose(res.W[:L], gr.W[:L], rtol=1e-13, atol=0)
        # each parent's children in the textbook draw (children are copies)
        counts_t = np.zeros(n, dtype=np.int64)
        for x in res.X[0, :L]:
            counts_t[parents_g[x]] += 1
        assert counts_t.sum() == L
        # the grouped filter's counts follow its bearing order of the parents
        counts_by_slot = np.zeros(n, dtype=np.int64)
        for x in gr.X[0, :L]:
            counts_by_slot[parents_g[x]] += 1
        W = g.W[:n]
        ideal = L * W / W.sum()
        for c in (counts_t, counts_by_slot):
            assert np.all(c >= np.floor(ideal) - 1e-9) and np.all(c <= np.ceil(ideal) + 1e-9)
        assert np.abs(counts_t - counts_by_slot).max() <= 1
        orc.exchange(p, gr, k, seed, run)                       # a no-op at K = 1
        g = gr
