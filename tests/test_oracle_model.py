"""Pins of the oracle's model pieces: likelihood, clutter density, motion
model (against the matrices printed in section 4), births and t = 0."""
import json
import math
import os

import numpy as np
from scipy.stats import norm

from paper_1503_03769_amd.scenario import BASE_MODEL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_likelihood_is_product_of_gaussians(orc):
    """Away from the bearing cut the likelihood is the product of two normal
    densities (scipy), section 4 sensor model."""
    p = dict(BASE_MODEL)
    rng = np.random.default_rng(1)
    for _ in range(200):
        x, y = rng.uniform(-1000, 1000, 2)
        rho, phi = math.hypot(x, y), math.atan2(y, x)
        zr = rho + rng.normal(0, 15)
        zt = phi + rng.normal(0, 0.03)
        if abs(zt) >= math.pi:
            continue
        want = norm.pdf(zr, rho, p["sigma_r"]) * norm.pdf(zt, phi, p["sigma_theta"])
        got = orc.likelihood(p, zr, zt, x, y)
        assert math.isclose(got, want, rel_tol=1e-12, abs_tol=1e-300)


def test_likelihood_wraps_bearing(orc):
    """A target just below the negative x axis and a bearing just above it are
    close in angle although their bearings differ by almost 2 pi."""
    p = dict(BASE_MODEL)
    eps = 0.01
    x, y = -500 * math.cos(eps), -500 * math.sin(eps)      # bearing -pi + eps
    zt = math.pi - eps                                        # residual 2 pi - 2 eps ~ -2 eps
    got = orc.likelihood(p, 500.0, zt, x, y)
    want = norm.pdf(500.0, 500.0, p["sigma_r"]) * norm.pdf(2 * eps, 0, p["sigma_theta"])
    assert math.isclose(got, want, rel_tol=1e-9)


def test_kappa_uniform_clutter(orc):
    for lam in (0.0, 10.0, 50.0):
        p = dict(BASE_MODEL, clutter_rate=lam)
        assert math.isclose(orc.kappa(p), lam / (2000.0 * 2 * math.pi), rel_tol=1e-15)


def test_predict_without_noise_is_F_x(orc):
    """sigma_a = 0: the survivors move exactly by the printed F (T = 1)."""
    g = json.load(open(os.path.join(GOLDEN, "cv_model_T1.json")))
    F = np.array(g["F"], dtype=np.float64)
    p = dict(BASE_MODEL, sigma_a=0.0, T=g["T"], partitions=2, births_per_step=0)
    cap = 64
    st = orc.State(2, cap)
    rng = np.random.default_rng(2)
    st.n[:] = [40, 17]
    st.X[:] = rng.uniform(-100, 100, size=st.X.shape)
    st.W[:] = rng.uniform(0.1, 1, size=st.W.shape)
    X0, W0 = st.X.copy(), st.W.copy()
    orc.predict(p, st, 1, 7, 0)
    for j in range(2):
        for s in range(st.n[j]):
            g_ = j * cap + s
            assert np.array_equal(st.X[:, g_], F @ X0[:, g_])
            assert st.W[g_] == p["p_S"] * W0[g_]


def test_predict_noise_covariance_is_gamma_gamma_t(orc):
    """The increment x' - F x has covariance sigma_a^2 Gamma Gamma^T (Gamma as
    printed in section 4 at T = 1)."""
    g = json.load(open(os.path.join(GOLDEN, "cv_model_T1.json")))
    F, G = np.array(g["F"]), np.array(g["Gamma"])
    sa = 5.0
    p = dict(BASE_MODEL, sigma_a=sa, T=1.0, partitions=1, births_per_step=0)
    n = 100000
    st = orc.State(1, n)
    st.n[0] = n
    rng = np.random.default_rng(3)
    st.X[:] = rng.uniform(-10, 10, size=st.X.shape)
    X0 = st.X.copy()
    orc.predict(p, st, 2, 11, 0)
    inc = st.X - F @ X0
    cov = inc @ inc.T / n
    want = sa * sa * G @ G.T
    se = np.sqrt((want ** 2 + np.outer(np.diag(want), np.diag(want))) / n)  # std. error of a covariance
    assert np.all(np.abs(cov - want) <= 6 * se + 1e-9), (cov, want)


def test_births_mass_region_and_split(orc):
    p = dict(BASE_MODEL, partitions=3, births_per_step=100, birth_mass=0.1)
    cap = 200
    st = orc.State(3, cap)
    st.n[:] = [5, 0, 10]
    st.W[:] = 0.5
    orc.predict(p, st, 4, 5, 0)
    Js = [orc.births_in_partition(p, j) for j in range(3)]
    assert Js == [34, 33, 33]                       # J split equally, first J mod K get one more
    assert list(st.n) == [5 + 34, 0 + 33, 10 + 33]
    for j, ns in enumerate([5, 0, 10]):
        b = slice(j * cap + ns, j * cap + ns + Js[j])
        assert math.isclose(st.W[b].sum(), p["birth_mass"], rel_tol=1e-14)
        assert np.all((st.X[0, b] >= -1000) & (st.X[0, b] <= 1000))
        assert np.all((st.X[2, b] >= -1000) & (st.X[2, b] <= 1000))


def test_init_equal_weights(orc):
    p = dict(BASE_MODEL, partitions=4, particles_per_target=1000.0, init_mass=1.0)
    cap = 300
    st = orc.State(4, cap)
    orc.init(p, st, 1, 0)
    assert list(st.n) == [250] * 4
    for j in range(4):
        w = st.W[j * cap:j * cap + 250]
        assert np.all(w == 1.0 / 250)


def test_gaussian_birth_density_moments(orc):
    """birth_density 1: births follow N(x_bar, diag(std^2)) of section 4 and
    each carries m_b / J_j."""
    from paper_1503_03769_amd.scenario import PAPER_MODEL
    p = dict(PAPER_MODEL, partitions=1, births_per_step=20000, particles_per_target=100.0)
    st = orc.State(1, 20200)
    st.n[0] = 100
    orc.predict(p, st, 3, 5, 0)
    X = st.X[:, 100:20100]
    W = st.W[100:20100]
    assert np.allclose(W, p["birth_mass"] / 20000, rtol=1e-15)
    mean, std = np.array(p["birth_mean"]), np.array(p["birth_std"])
    n = X.shape[1]
    for d in range(4):
        assert abs(X[d].mean() - mean[d]) < 5 * std[d] / np.sqrt(n)
        assert abs(X[d].std() / std[d] - 1) < 0.03
    # the four coordinates are independent
    c = np.corrcoef(X)
    assert np.all(np.abs(c - np.eye(4)) < 0.05)
