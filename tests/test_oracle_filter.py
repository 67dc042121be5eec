"""Whole-filter pin of the oracle: the PHD's integral is the expected number
of targets (section 2.1), so after a burn-in the group mass of the updated
PHD follows the true target count; with K groups every group carries the
full count (each sees every measurement, section 3)."""
import numpy as np
import pytest

from paper_1503_03769_amd.scenario import BASE_MODEL, make_scenario


@pytest.mark.parametrize("K", [1, 4])
def test_mass_tracks_true_count(orc, K):
    # targets appear inside a 200 m square 700 m from the sensor, which the
    # (uniform) birth density covers, so the filter can pick them up
    box = (400.0, 600.0, 400.0, 600.0)
    p = dict(BASE_MODEL, partitions=K, particles_per_target=400.0 * K, births_per_step=400 * K,
             clutter_rate=10.0, region=box, birth_sigma_v=3.0, sigma_a=1.0)
    steps = 40
    errs = []
    for run in range(2):
        truth, Z = make_scenario(p, 3, steps, 900 + run, start_box=(450.0, 550.0, 450.0, 550.0),
                                 start_sigma_v=2.0)
        f = orc.OracleFilter(p, 6000, 31 + run, run)
        for k in range(1, steps + 1):
            out = f.step(k, Z[k])
            if k > 5:
                for j in range(K):
                    errs.append(out["upd"]["mass"][j] - len(truth[k]))
    errs = np.array(errs)
    # mass follows the count: small bias and spread well below one target
    assert abs(errs.mean()) < 0.35, errs.mean()
    assert np.sqrt(np.mean(errs ** 2)) < 0.8, np.sqrt(np.mean(errs ** 2))


def test_thread_count_does_not_change_results(orc):
    """The oracle runs its independent groups one per thread; one thread and
    four threads give the same filter bit for bit."""
    p = dict(BASE_MODEL, partitions=6, particles_per_target=600.0 * 6, births_per_step=1200, clutter_rate=20.0,
             birth_proposal=1, birth_alpha=0.1)
    truth, Z = make_scenario(p, 3, 4, 17)
    outs = []
    before = orc.threads()
    try:
        for nt in (1, 4):
            orc.set_threads(nt)
            f = orc.OracleFilter(p, 1500, 8, 2)
            for k in range(1, 5):
                out = f.step(k, Z[k])
            outs.append((f.st.X.copy(), f.st.W.copy(), f.st.n.copy(), out["upd"]["C"].copy()))
    finally:
        orc.set_threads(before)
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
