"""Pins of the measurement-driven birth proposal (Eq 6 with p_k(.|Z_k)):
its density integrates to one, its importance weights are unbiased (the
expected birth mass is m_b whatever the proposal), and without measurements
it reduces to the birth density itself."""
import math

import numpy as np
import pytest

from paper_1503_03769_amd.scenario import BASE_MODEL


def _p(**kw):
    d = dict(BASE_MODEL, birth_proposal=1, birth_alpha=0.0)
    d.update(kw)
    return d


@pytest.mark.parametrize("r_p,theta_p", [(700.0, 0.6), (8.0, -2.0), (1500.0, 3.1)])
def test_component_density_integrates_to_one(orc, r_p, theta_p):
    """Quadrature of q_p in polar coordinates (rho drho dphi), over windows
    around bearing theta_p and, for small r_p, theta_p + pi (negative draws)."""
    p = _p(region=(-5000.0, 5000.0, -5000.0, 5000.0))
    Z = np.array([[r_p, theta_p]])
    sr, st = p["sigma_r"], p["sigma_theta"]
    total = 0.0
    rho = np.linspace(max(1e-3, r_p - 9 * sr), r_p + 9 * sr, 241) if r_p > 10 * sr else np.linspace(1e-4, r_p + 9 * sr, 481)
    for c in (theta_p, theta_p + math.pi):
        phi = np.linspace(c - 9 * st, c + 9 * st, 161)
        vals = np.array([[orc.birth_proposal_density(p, Z, r * math.cos(f), r * math.sin(f)) * r for f in phi] for r in rho])
        total += np.trapezoid(np.trapezoid(vals, phi, axis=1), rho)
    assert abs(total - 1.0) < 2e-4, total


def test_weights_are_unbiased(orc):
    """E_q[gamma/(J q)] summed over the J births is m_b (Eq 6 importance weights)."""
    p = _p(birth_alpha=0.2, partitions=1, births_per_step=400, birth_mass=0.1)
    Z = np.array([[700.0, 0.6], [300.0, -1.2], [1200.0, 2.0], [50.0, 0.1]])
    sums = []
    for step in range(1, 151):
        st = orc.State(1, 500)
        st.n[0] = 400                     # all slots reserved for births
        orc.birth_from_measurements(p, st, step, 99, 0, Z)
        sums.append(st.W[:400].sum())
    sums = np.array(sums)
    se = sums.std() / math.sqrt(len(sums))
    assert abs(sums.mean() - p["birth_mass"]) < 5 * se + 1e-4, (sums.mean(), se)


def test_no_measurements_is_the_birth_density(orc):
    p = _p(birth_alpha=0.3, partitions=2, births_per_step=100)
    st = orc.State(2, 200)
    st.n[:] = [50, 50]
    orc.birth_from_measurements(p, st, 3, 5, 0, np.zeros((0, 2)))
    for j in range(2):
        w = st.W[j * 200:j * 200 + 50]
        assert np.allclose(w, p["birth_mass"] / 50, rtol=1e-15)
        x, y = st.X[0, j * 200:j * 200 + 50], st.X[2, j * 200:j * 200 + 50]
        assert np.all((x >= -1000) & (x <= 1000) & (y >= -1000) & (y <= 1000))


def test_mixture_places_births_near_measurements(orc):
    p = _p(birth_alpha=0.1, partitions=1, births_per_step=2000)
    Z = np.array([[800.0, 0.5]])
    st = orc.State(1, 2100)
    st.n[0] = 2000
    orc.birth_from_measurements(p, st, 1, 7, 0, Z)
    x, y = st.X[0, :2000], st.X[2, :2000]
    near = np.hypot(x - 800 * math.cos(0.5), y - 800 * math.sin(0.5)) < 100
    frac = near.mean()
    assert 0.85 < frac < 0.95, frac            # ~ (1 - alpha) of the draws
