"""GPU tests of the learned birth proposal against the FP64 oracle.

Tolerances (BF16 unit roundoff u = 2^-8, FP32 accumulation over 128 terms
gamma = 128 * 2^-24):
  * network outputs: first-order propagation of every rounding the GPU path
    makes, bounded with the oracle's own activations:
      E1 = u|h1| + |W1| e_f,  E_{l+1} = |W_{l+1}| E_l + gamma |W_{l+1}| |h_l| + u |h_{l+1}|,
      |o' - o| <= 1.1 (|W4| E3 + gamma |W4| |h3|) + 1e-6, and rms(o' - o) <= 2u rms(o);
  * loss: |L' - L| <= 1.5 mean_n sum_j |dL_n/do_j| bound(o_nj) + 1e-5;
  * gradient: each parameter tensor within 5% (about 13 u) of the oracle's in
    Frobenius norm, the whole vector at cosine >= 0.999;
  * simulated pairs: the oracle's FP64 pairs rounded to FP32, relative 1e-6;
  * births from given network outputs: as for the other birth proposals
    (states relative 1e-12 FP64 / 1e-6 FP32, weights through the update).
"""
import math

import numpy as np
import pytest

import oracle as orc
from oracle import mlp as omlp
from paper_1503_03769_amd.scenario import (BASE_MODEL, make_scenario, random_mixture_outputs, random_mlp_params)

from . import parity as P

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8
GAMMA = 128 * 2.0 ** -24


def _net(gpu, p=BASE_MODEL, batch=512, dataset=4096, seed=7, **kw):
    return gpu.Mlp(p, batch=batch, dataset=dataset, seed=seed, **kw)


def _output_bound(theta, F):
    """First-order bound on |o_gpu - o| (see the module docstring)."""
    Pm = omlp.unflatten(theta)
    o, (h1, h2, h3) = omlp.forward(theta, F)
    e_f = 1e-6 * (np.abs(F) + 1.0)
    E1 = U_BF16 * np.abs(h1) + e_f @ np.abs(Pm["W1"]).T
    A2, A3, A4 = np.abs(Pm["W2"]), np.abs(Pm["W3"]), np.abs(Pm["W4"])
    E2 = E1 @ A2.T + GAMMA * np.abs(h1) @ A2.T + U_BF16 * np.abs(h2)
    E3 = E2 @ A3.T + GAMMA * np.abs(h2) @ A3.T + U_BF16 * np.abs(h3)
    return o, 1.1 * (E3 @ A4.T + GAMMA * np.abs(h3) @ A4.T) + 1e-6


def test_simulated_pairs_match_oracle(gpu):
    print("mlp: simulated pairs", flush=True)
    net = _net(gpu, seed=0xABCD1234)
    net.simulate(run=3)
    zg, xg = net.read_dataset(0, 4096)
    zo, xo = orc.simulate_pairs(BASE_MODEL, 0xABCD1234, 3, 0, 4096)
    np.testing.assert_allclose(zg, zo.astype(np.float32), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(xg, xo.astype(np.float32), rtol=1e-6, atol=1e-5)
    zg2, _ = net.read_dataset(4000, 96)
    assert np.array_equal(zg2, zg[4000:4096])
    net.close()


@pytest.mark.parametrize("M", [1, 64, 200])
def test_forward_matches_oracle(gpu, M):
    print(f"mlp: forward M={M}", flush=True)
    theta = random_mlp_params(11)
    rng = np.random.default_rng(M)
    Z = np.stack([rng.uniform(0, 1500, M), rng.uniform(-math.pi, math.pi, M)], axis=1)
    net = _net(gpu)
    net.set_params(theta)
    og = net.forward(Z).astype(np.float64)
    o, bound = _output_bound(theta.astype(np.float64), omlp.features(BASE_MODEL, Z))
    err = np.abs(og - o)
    assert np.all(err <= bound), (err.max(), float((err / bound).max()))
    # and statistically: the roundings have random signs, so the rms error
    # stays within a small multiple of u times the rms output
    assert np.sqrt(np.mean(err ** 2)) <= 2 * U_BF16 * np.sqrt(np.mean(o ** 2)), np.sqrt(np.mean(err ** 2))
    net.close()


@pytest.mark.parametrize("n", [64, 300])
def test_loss_and_gradient_match_oracle(gpu, n):
    print(f"mlp: loss and gradient n={n}", flush=True)
    theta = random_mlp_params(12).astype(np.float64)
    Z, X = orc.simulate_pairs(BASE_MODEL, 99, 0, 0, n)
    Z = Z.astype(np.float32).astype(np.float64)
    X = X.astype(np.float32).astype(np.float64)
    net = _net(gpu)
    net.set_params(theta)
    lg, gg = net.loss_grad(Z, X)
    lo, go = omlp.loss_and_grad(BASE_MODEL, theta, Z, X)
    # loss bound from the output bound and the per-pair derivative
    F = omlp.features(BASE_MODEL, Z)
    o, bound = _output_bound(theta, F)
    _, g_o = omlp.nll_terms(BASE_MODEL, o, F, X)
    lbound = 1.5 * np.mean(np.sum(np.abs(g_o) * bound, axis=1)) + 1e-5
    assert abs(lg - lo) <= lbound, (lg, lo, lbound)
    gg = gg.astype(np.float64)
    cos = gg @ go / (np.linalg.norm(gg) * np.linalg.norm(go))
    assert cos >= 0.999, cos
    Gg, Go = omlp.unflatten(gg), omlp.unflatten(go)
    floor = 1e-3 * np.linalg.norm(go)
    for name in Gg:
        rel = np.linalg.norm(Gg[name] - Go[name]) / max(np.linalg.norm(Go[name]), floor)
        assert rel <= 0.05, (name, rel)
    net.close()


def test_adam_step(gpu):
    """One training step: the loss it reports is that of the first minibatch,
    and the parameters move by -lr g / (|g| + eps) (first Adam step), g the
    minibatch gradient; its signs agree with the oracle's gradient."""
    print("mlp: adam step", flush=True)
    theta = random_mlp_params(13)
    net = _net(gpu, batch=256, dataset=512, seed=5)
    net.simulate(run=0)
    z, x = net.read_dataset(0, 256)
    net.set_params(theta)
    l0, g = net.loss_grad(z, x)
    losses = net.train(1, lr=1e-3)
    assert losses[0] == np.float32(l0)
    new = net.get_params().astype(np.float64)
    g = g.astype(np.float64)
    step = -1e-3 * g / (np.abs(g) + 1e-8)
    # the new parameters are FP32: half an ulp of |theta| <= 4 is 2.4e-7
    np.testing.assert_allclose(new - theta.astype(np.float64), step, rtol=2e-3, atol=2.5e-7)
    assert net.steps() == 1
    _, go = omlp.loss_and_grad(BASE_MODEL, theta.astype(np.float64), z.astype(np.float64), x.astype(np.float64))
    big = np.abs(go) > 1e-2 * np.abs(go).max()
    assert np.mean(np.sign(g[big]) == np.sign(go[big])) >= 0.99
    net.close()


def test_training_lowers_the_loss(gpu):
    """Training on simulated pairs: the loss falls, and the oracle's FP64 loss
    of the trained network on fresh pairs agrees with the training loss."""
    print("mlp: training", flush=True)
    from paper_1503_03769_amd.proposal import train_proposal
    net, losses = train_proposal(BASE_MODEL, seed=21, steps=1500)
    first, last = float(np.mean(losses[:20])), float(np.mean(losses[-50:]))
    print(f"training loss {first:.3f} -> {last:.3f}", flush=True)
    assert np.all(np.isfinite(losses))
    assert last < first - 1.0, (first, last)
    theta = net.get_params().astype(np.float64)
    Z, X = orc.simulate_pairs(BASE_MODEL, 12345, 0, 0, 4000)
    lo, _ = omlp.loss_and_grad(BASE_MODEL, theta, Z, X)
    assert abs(lo - last) < 0.1, (lo, last)
    net.close()


def _births_case(gpu, prec, M_raw_seed=3, births=900):
    K, cap = 3, 4096
    p = dict(BASE_MODEL, partitions=K, births_per_step=births, birth_proposal=2, birth_alpha=0.1)
    truth, Z = make_scenario(p, 3, 4, 17)
    Zk = Z[4]
    raw = random_mixture_outputs(Zk.shape[0], M_raw_seed)
    X, W, n = P.cloud(K, cap, [2000, 700, 0], 13, truth[4], prec)
    return p, K, cap, Zk, raw, X, W, n


@pytest.mark.parametrize("prec,births", [("fp64", 900), ("fp32", 900), ("fp64", 3000), ("fp32", 3000)])
def test_births_from_given_outputs_match_oracle(gpu, prec, births):
    """300 births per group take the one-wavefront-per-birth kernel, 1000 the
    one-lane-per-birth kernel."""
    print(f"mlp: births from given outputs {prec} {births}", flush=True)
    p, K, cap, Zk, raw, X, W, n = _births_case(gpu, prec, births=births)
    f = P.make_filter(p, prec, cap)
    f.write_state(X, W, n, gpu.PHASE_READY)
    f.predict(4)
    f.set_birth_mixture(raw)
    f.update(Zk)
    Xg, Wg, ng = f.read_state()
    st = P.oracle_state(K, cap, X, W, n)
    orc.predict(p, st, 4, 1234, 0)
    orc.birth_from_mixture(p, st, 4, 1234, 0, omlp.mixture_table(p, Zk, raw.astype(np.float64)))
    births = st.copy()
    st.X[:] = P.as_storage(st.X, prec)
    st.W[:] = P.as_storage(st.W, prec)
    orc.update(p, st, Zk)
    assert np.array_equal(ng, st.n)
    rtol = 1e-12 if prec == "fp64" else 1e-6
    for j in range(K):
        sl = slice(j * cap, j * cap + int(st.n[j]))
        np.testing.assert_allclose(Xg[:, sl], births.X[:, sl], rtol=rtol, atol=1e-9 if prec == "fp64" else 1e-4)
    P.check_weights(Wg, st)
    f.close()


def test_births_without_measurements_use_the_birth_density(gpu):
    p = dict(BASE_MODEL, partitions=2, births_per_step=100, birth_proposal=2, birth_alpha=0.3,
             particles_per_target=200.0)
    f = P.make_filter(p, "fp64", 512)
    X, W, n = P.cloud(2, 512, [10, 10], 3, None, "fp64")
    f.write_state(X, W, n, gpu.PHASE_READY)
    f.predict(2)
    f.set_birth_mixture(np.zeros((0, 36), np.float32))
    f.update(np.zeros((0, 2)))
    Xg, Wg, ng = f.read_state()
    st = P.oracle_state(2, 512, X, W, n)
    orc.predict(p, st, 2, 1234, 0)
    orc.birth_from_mixture(p, st, 2, 1234, 0, np.zeros((0, 4, 9)))
    orc.update(p, st, np.zeros((0, 2)))
    P.check_states(Xg, Wg, ng, st, "fp64")
    f.close()


def test_attached_network_equals_its_outputs(gpu):
    """The product path (network run inside pphd_update) draws the same births
    as the same network's outputs handed in through set_birth_mixture."""
    print("mlp: attached network", flush=True)
    p, K, cap, Zk, _, X, W, n = _births_case(gpu, "fp32")
    net = _net(gpu)
    net.set_params(random_mlp_params(14, scale=0.5))
    out = net.forward(Zk)
    states = []
    for attached in (True, False):
        f = P.make_filter(p, "fp32", cap)
        f.write_state(X, W, n, gpu.PHASE_READY)
        f.predict(4)
        if attached:
            f.attach_mlp(net)
        else:
            f.set_birth_mixture(out)
        f.update(Zk)
        states.append(f.read_state())
        f.close()
    for a, b in zip(states[0], states[1]):
        assert np.array_equal(a, b)
    net.close()


def test_missing_network_is_an_error(gpu):
    p = dict(BASE_MODEL, partitions=1, births_per_step=10, birth_proposal=2, birth_alpha=0.1,
             particles_per_target=200.0)
    f = P.make_filter(p, "fp64", 512)
    f.init()
    f.predict(1)
    with pytest.raises(gpu.PphdError) as e:
        f.update(np.array([[500.0, 0.1]]))
    assert e.value.code == gpu.PPHD_ESTATE
    f.set_birth_mixture(np.zeros((2, 36), np.float32))
    with pytest.raises(gpu.PphdError) as e:
        f.update(np.array([[500.0, 0.1]]))   # outputs given for 2 measurements
    assert e.value.code == gpu.PPHD_EINVAL
    f.close()
    q = dict(p, birth_proposal=1)
    g = P.make_filter(q, "fp64", 512)
    net = _net(gpu)
    with pytest.raises(gpu.PphdError):
        g.attach_mlp(net)
    g.close()
    net.close()
