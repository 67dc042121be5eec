"""Pins of the learned-proposal oracle (oracle.mlp and the mixture births):
the hand-written gradient against central finite differences, the loss and
the births' proposal density against scipy's normal densities, the first Adam
step against its closed form, the simulated training pairs against the
distributions they are drawn from, and the mixture births' importance weights
(unbiased: the expected birth mass is m_b whatever the mixture)."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from paper_1503_03769_amd.scenario import BASE_MODEL


@pytest.fixture(scope="module")
def mlp():
    from oracle import mlp
    return mlp


def _params(mlp, hidden, seed, scale=0.5):
    rng = np.random.default_rng(seed)
    th = rng.normal(0.0, scale, mlp.n_params(hidden))
    d = mlp.unflatten(th, hidden)
    d["b4"][5::9] -= 1.5          # log-stds well inside the clip range
    return mlp.flatten(d, hidden)


def _pairs(orc, n, seed, p=BASE_MODEL):
    return orc.simulate_pairs(p, seed, 0, 0, n)


def test_gradient_matches_central_differences(orc, mlp):
    hidden = 6
    th = _params(mlp, hidden, 1)
    Z, X = _pairs(orc, 9, 5)
    loss, g = mlp.loss_and_grad(BASE_MODEL, th, Z, X, hidden)
    h = 1e-6
    fd = np.zeros_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        lp, _ = mlp.loss_and_grad(BASE_MODEL, th + e, Z, X, hidden)
        lm, _ = mlp.loss_and_grad(BASE_MODEL, th - e, Z, X, hidden)
        fd[i] = (lp - lm) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * max(1.0, np.max(np.abs(g))), np.max(np.abs(fd - g))


def test_gradient_is_zero_for_clipped_log_std(orc, mlp):
    hidden = 4
    d = mlp.unflatten(_params(mlp, hidden, 2), hidden)
    d["W4"][5, :] = 0.0
    d["b4"][5] = -20.0            # clipped at -12
    th = mlp.flatten(d, hidden)
    Z, X = _pairs(orc, 5, 6)
    _, g = mlp.loss_and_grad(BASE_MODEL, th, Z, X, hidden)
    G = mlp.unflatten(g, hidden)
    assert G["b4"][5] == 0.0 and np.all(G["W4"][5] == 0.0)


def test_constant_mixture_loss_against_scipy(orc, mlp):
    """With W4 = 0 the mixture is fixed by b4 (means offset from the measured
    position); the loss is then a plain mixture log-density."""
    hidden = 3
    rng = np.random.default_rng(3)
    d = mlp.unflatten(np.zeros(mlp.n_params(hidden)), hidden)
    b4 = rng.normal(0, 0.3, 36)
    for c in range(4):
        b4[9 * c + 5:9 * c + 9] = rng.uniform(-4.0, 0.5, 4)
    d["b4"] = b4
    th = mlp.flatten(d, hidden)
    Z, X = _pairs(orc, 50, 8)
    loss, _ = mlp.loss_and_grad(BASE_MODEL, th, Z, X, hidden)
    # state-space density via scipy, then the normalised-space loss
    reg = BASE_MODEL["region"]
    S = np.array([(reg[1] - reg[0]) / 2, BASE_MODEL["birth_sigma_v"], (reg[3] - reg[2]) / 2, BASE_MODEL["birth_sigma_v"]])
    px = Z[:, 0] * np.cos(Z[:, 1])
    py = Z[:, 0] * np.sin(Z[:, 1])
    logits = b4[0::9]
    pi = np.exp(logits) / np.exp(logits).sum()
    dens = np.zeros(len(Z))
    for c in range(4):
        mu = np.stack([px + S[0] * b4[9 * c + 1], np.full(len(Z), S[1] * b4[9 * c + 2]),
                       py + S[2] * b4[9 * c + 3], np.full(len(Z), S[3] * b4[9 * c + 4])], axis=1)
        sd = S * np.exp(b4[9 * c + 5:9 * c + 9])
        dens += pi[c] * np.prod(norm.pdf(X, loc=mu, scale=sd), axis=1)
    ref = -np.mean(np.log(dens) + np.log(S).sum())
    assert abs(loss - ref) <= 1e-10 * abs(ref), (loss, ref)


def test_mixture_table_density_against_scipy(orc, mlp):
    p = dict(BASE_MODEL, birth_proposal=2, birth_alpha=0.25)
    hidden = 8
    th = _params(mlp, hidden, 4, scale=0.3)
    Z = np.array([[600.0, 0.3], [1100.0, -2.5], [90.0, 3.0]])
    o, _ = mlp.forward(th, mlp.features(p, Z), hidden)
    t = mlp.mixture_table(p, Z, o)
    assert np.allclose(np.exp(t[:, :, 0]).sum(axis=1), 1.0, rtol=1e-14)
    rng = np.random.default_rng(9)
    for _ in range(20):
        pm = t[rng.integers(0, 3), rng.integers(0, 4)]
        x = pm[1:5] + pm[5:9] * rng.normal(size=4)
        mix = sum(np.exp(t[q, c, 0]) * np.prod(norm.pdf(x, loc=t[q, c, 1:5], scale=t[q, c, 5:9]))
                  for q in range(3) for c in range(4)) / 3
        inside = -1000 <= x[0] <= 1000 and -1000 <= x[2] <= 1000
        b = (1 / 4e6 if inside else 0.0) * norm.pdf(x[1], scale=10.0) * norm.pdf(x[3], scale=10.0)
        ref = 0.25 * b + 0.75 * mix
        got = orc.mixture_proposal_density(p, t, x)
        assert abs(got - ref) <= 1e-12 * ref, (got, ref)


def test_first_adam_step_is_a_signed_learning_rate(mlp):
    rng = np.random.default_rng(5)
    th = rng.normal(size=200)
    g = rng.normal(size=200) * 10.0 ** rng.uniform(-3, 2, 200)
    new, m, v = mlp.adam_step(th, g, np.zeros(200), np.zeros(200), 1, 1e-3)
    np.testing.assert_allclose(new - th, -1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-9)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_simulated_pairs_follow_the_models(orc):
    p = BASE_MODEL
    Z, X = orc.simulate_pairs(p, 11, 0, 0, 40000)
    n = len(Z)
    # positions uniform on [-1000, 1000]^2, velocities N(0, sigma_v^2)
    for d, (lo, hi) in ((0, (-1000, 1000)), (2, (-1000, 1000))):
        assert X[:, d].min() >= lo and X[:, d].max() <= hi
        assert abs(X[:, d].mean()) < 5 * 2000 / math.sqrt(12 * n)
        assert abs(X[:, d].var() / (2000 ** 2 / 12) - 1) < 0.03
    for d in (1, 3):
        assert abs(X[:, d].std() / p["birth_sigma_v"] - 1) < 0.02
    er = Z[:, 0] - np.hypot(X[:, 0], X[:, 2])
    et = np.angle(np.exp(1j * (Z[:, 1] - np.arctan2(X[:, 2], X[:, 0]))))
    assert abs(er.std() / p["sigma_r"] - 1) < 0.02 and abs(er.mean()) < 5 * p["sigma_r"] / math.sqrt(n)
    assert abs(et.std() / p["sigma_theta"] - 1) < 0.02
    assert np.all(Z[:, 1] >= -math.pi) and np.all(Z[:, 1] < math.pi)
    # pair i does not depend on where the batch starts
    Z2, X2 = orc.simulate_pairs(p, 11, 0, 123, 5)
    assert np.array_equal(Z2, Z[123:128]) and np.array_equal(X2, X[123:128])


def _table(mlp, p, Z, hidden=8, seed=6):
    th = _params(mlp, hidden, seed, scale=0.3)
    o, _ = mlp.forward(th, mlp.features(p, Z), hidden)
    return mlp.mixture_table(p, Z, o)


def test_mixture_birth_weights_are_unbiased(orc, mlp):
    p = dict(BASE_MODEL, birth_proposal=2, birth_alpha=0.2, partitions=1, births_per_step=400, birth_mass=0.1)
    Z = np.array([[700.0, 0.6], [300.0, -1.2], [1200.0, 2.0]])
    t = _table(mlp, p, Z)
    sums = []
    for step in range(1, 121):
        st = orc.State(1, 500)
        st.n[0] = 400
        orc.birth_from_mixture(p, st, step, 99, 0, t)
        sums.append(st.W[:400].sum())
    sums = np.array(sums)
    se = sums.std() / math.sqrt(len(sums))
    assert abs(sums.mean() - p["birth_mass"]) < 5 * se + 1e-4, (sums.mean(), se)


def test_mixture_births_draw_the_chosen_component(orc, mlp):
    """alpha = 0 and one measurement whose mixture has one component of weight
    ~1: the births are that Gaussian (moments), each weight gamma/(J q)."""
    p = dict(BASE_MODEL, birth_proposal=2, birth_alpha=0.0, partitions=1, births_per_step=4000)
    t = np.zeros((1, 4, 9))
    t[0, :, 0] = np.log([1 - 3e-12, 1e-12, 1e-12, 1e-12])
    t[0, :, 1:5] = [120.0, 3.0, -340.0, -7.0]
    t[0, :, 5:9] = [15.0, 9.0, 25.0, 11.0]
    st = orc.State(1, 4100)
    st.n[0] = 4000
    orc.birth_from_mixture(p, st, 2, 21, 0, t)
    X = st.X[:, :4000]
    n = 4000
    for d in range(4):
        assert abs(X[d].mean() - t[0, 0, 1 + d]) < 5 * t[0, 0, 5 + d] / math.sqrt(n)
        assert abs(X[d].std() / t[0, 0, 5 + d] - 1) < 0.05
    x0 = X[:, 0]
    q = np.prod(norm.pdf(x0, loc=t[0, 0, 1:5], scale=t[0, 0, 5:9]))
    gam = p["birth_mass"] / 4e6 * norm.pdf(x0[1], scale=10.0) * norm.pdf(x0[3], scale=10.0)
    assert abs(st.W[0] - gam / (4000 * q)) <= 1e-9 * st.W[0]


def test_mixture_births_without_measurements_are_the_birth_density(orc):
    p = dict(BASE_MODEL, birth_proposal=2, birth_alpha=0.3, partitions=2, births_per_step=100)
    st = orc.State(2, 200)
    st.n[:] = [50, 50]
    orc.birth_from_mixture(p, st, 3, 5, 0, np.zeros((0, 4, 9)))
    for j in range(2):
        np.testing.assert_allclose(st.W[j * 200:j * 200 + 50], p["birth_mass"] / 50, rtol=1e-14)


def test_oracle_training_reduces_the_loss(orc, mlp):
    """A few Adam steps of the FP64 oracle on a small net lower the loss."""
    hidden = 16
    rng = np.random.default_rng(0)
    th = mlp.flatten({k: rng.normal(0, math.sqrt(2.0 / (s[-1] if len(s) > 1 else 1)), s) * (len(s) > 1)
                      for k, s in mlp.shapes(hidden)}, hidden)
    Z, X = _pairs(orc, 512, 3)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0, _ = mlp.loss_and_grad(BASE_MODEL, th, Z, X, hidden)
    for t in range(1, 61):
        loss, g = mlp.loss_and_grad(BASE_MODEL, th, Z, X, hidden)
        th, m, v = mlp.adam_step(th, g, m, v, t, 1e-2)
    l1, _ = mlp.loss_and_grad(BASE_MODEL, th, Z, X, hidden)
    assert l1 < l0 - 1.0, (l0, l1)


def test_filter_with_a_hand_set_network_tracks_the_mass(orc, mlp):
    """A network with W4 = 0 proposes a fixed Gaussian around each measured
    position; the oracle filter with it follows the number of targets."""
    from paper_1503_03769_amd.scenario import make_scenario
    p = dict(BASE_MODEL, birth_proposal=2, birth_alpha=0.1, partitions=1, births_per_step=300,
             particles_per_target=300.0, clutter_rate=5.0)
    hidden = 4
    d = mlp.unflatten(np.zeros(mlp.n_params(hidden)), hidden)
    for c in range(4):
        d["b4"][9 * c + 5:9 * c + 9] = [math.log(20 / 1000), 0.0, math.log(20 / 1000), 0.0]
    th = mlp.flatten(d, hidden)
    truth, Z = make_scenario(p, 3, 25, 77)
    import oracle
    f = oracle.OracleFilter(p, 4096, 5, 0, mlp_theta=th, mlp_hidden=hidden)
    err = []
    for k in range(1, 26):
        out = f.step(k, Z[k])
        if k >= 10:
            err.append(abs(out["upd"]["mass"].sum() - len(truth[k])))
    assert np.mean(err) < 0.6, err
