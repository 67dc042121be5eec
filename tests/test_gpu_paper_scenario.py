"""The paper's accuracy comparison in its own setting (section 4; Table 1 at
r = 0): the distributed filter with K = 4 groups of N/K particles tracks as
well as the standard filter with N particles, and both beat the standard
filter with only N/K particles.  60 paired Monte Carlo runs (the same tracks
for the three methods), run as GPU batches.  At r = 10 the order of the
N/K filter holds, and the count errors are mostly misses from a low mass."""
import pytest

from paper_1503_03769_amd.paper_table import run_config

pytestmark = pytest.mark.gpu


def test_distributed_filter_matches_full_filter(gpu):
    res = {m: run_config(m, 0.0, 60, 50)["mean_ospa"] for m in ("PHD", "DCPPHD", "partPHD")}
    print(res, flush=True)
    assert abs(res["DCPPHD"] - res["PHD"]) < 0.05 * res["PHD"], res
    assert res["partPHD"] > res["DCPPHD"] and res["partPHD"] > res["PHD"], res


def test_clutter_keeps_the_order_and_the_mass_runs_low(gpu):
    """r = 10: the filter with only N/K particles stays the least accurate.
    With p_D = 1 and clutter every detected target adds C/(kappa + C) < 1 to
    the updated mass (Eqs 12-15), so the mass runs below the number of
    targets and Step 3's round(mass) misses targets far more often than it
    adds one: the count errors behind the larger OSPA with clutter."""
    import numpy as np

    from paper_1503_03769_amd import pphd
    from paper_1503_03769_amd.scenario import PAPER_MODEL, make_paper_scenario

    res = {m: run_config(m, 10.0, 60, 50)["mean_ospa"] for m in ("PHD", "DCPPHD", "partPHD")}
    print(res, flush=True)
    assert res["partPHD"] > res["DCPPHD"] and res["partPHD"] > res["PHD"], res
    p = dict(PAPER_MODEL, clutter_rate=10.0, partitions=1, particles_per_target=800.0, births_per_step=800)
    bias, low, high = [], 0, 0
    for i in range(12):
        truth, Z = make_paper_scenario(p, 50, 77000 + i)
        f = pphd.Filter(p, pphd.PPHD_FP64, 8192, max(z.shape[0] for z in Z[1:]) + 1, 4242, i)
        f.init()
        for k in range(1, 51):
            f.predict(k)
            f.update(Z[k])
            u = f.read_update()
            f.resample(k)
            f.exchange(k)
            n = truth[k].shape[0]
            if n == 0:
                continue
            mass = float(u["mass"].sum())
            bias.append(mass - n)
            low += int(u["LT"][0]) < n
            high += int(u["LT"][0]) > n
        f.close()
    print(f"mean(mass - n) {np.mean(bias):+.3f}; round(mass) low in {low}, high in {high} of {len(bias)} scans",
          flush=True)
    assert np.mean(bias) < -0.1 and low > 2 * high


def test_paper_model_fp64_update_matches_oracle(gpu):
    """Step 2 at the section-4 sensor (sigma_theta = 0.05 rad, K = 4, r = 10)
    in FP64 against the oracle, element by element.  Half of every group sits
    around the targets of scan 18 (bearings -0.83 to -1.04 rad, ranges over
    60 m); the other half sits at bearing about -3.0 rad.  One extra
    measurement at bearing 1.5 rad is more than pi/2 from every particle.  Its
    residual against the -3.0 rad part needs the 2 pi wrap (|1.5 + 3.0| > pi)
    and wraps to about 1.78 rad, closer than the 2 rad or more that separate
    it from the other half, so C of that measurement rests on the wrapped
    pairs.  Their terms, near 2^-900, are representable in double: exactly the
    pairs a wrap-free evaluation would lose."""
    import math

    import numpy as np

    import oracle as orc
    from paper_1503_03769_amd import pphd
    from paper_1503_03769_amd.scenario import PAPER_MODEL, make_paper_scenario
    from tests import parity as P

    K, cap = 4, 1024
    p = dict(PAPER_MODEL, clutter_rate=10.0)
    truth, Zs = make_paper_scenario(p, 30, 1234)
    k = 18
    rng = np.random.default_rng(5)
    counts = [700, 650, 720, 600]
    X = np.zeros((4, K * cap))
    W = np.zeros(K * cap)
    for j, nj in enumerate(counts):
        near = nj // 2
        idx = rng.integers(0, len(truth[k]), near)
        sl = slice(j * cap, j * cap + near)
        X[0, sl] = truth[k][idx, 0] + rng.normal(0, 4, near)
        X[1, sl] = truth[k][idx, 1] + rng.normal(0, 1, near)
        X[2, sl] = truth[k][idx, 2] + rng.normal(0, 4, near)
        X[3, sl] = truth[k][idx, 3] + rng.normal(0, 1, near)
        far = nj - near
        r = rng.uniform(90, 110, far)
        b = rng.normal(-3.0, 0.02, far)
        sl = slice(j * cap + near, j * cap + nj)
        X[0, sl], X[2, sl] = r * np.cos(b), r * np.sin(b)
        X[1, sl], X[3, sl] = rng.normal(0, 1, far), rng.normal(0, 1, far)
        W[j * cap:j * cap + nj] = np.exp(rng.uniform(-3, 0, nj)) * 1e-3
    n = np.array(counts, dtype=np.int32)
    Z = np.vstack([Zs[k], [[100.0, 1.5]]])
    phi = np.concatenate([np.arctan2(X[2, j * cap:j * cap + c], X[0, j * cap:j * cap + c])
                          for j, c in enumerate(counts)])
    gap = np.abs((1.5 - phi + math.pi) % (2 * math.pi) - math.pi)
    assert gap.min() > 0.5 * math.pi
    # the wrapped pairs (raw residual beyond pi) are the closest ones
    wrapped = np.abs(1.5 - phi) > math.pi
    assert wrapped.any() and gap[~wrapped].min() > gap[wrapped].max() + 0.1
    print(f"paper model FP64 update: M = {Z.shape[0]}, wrapped gap to the extra measurement "
          f"{gap[wrapped].min():.3f}..{gap[wrapped].max():.3f} rad, others from {gap[~wrapped].min():.3f} rad",
          flush=True)
    f = P.make_filter(p, "fp64", cap, max_meas=64)
    f.write_state(X, W, n, pphd.PHASE_PREDICTED)
    f.update(Z)
    Xg, Wg, ng = f.read_state()
    ug = f.read_update()
    lg = f.read_local()
    est_g, _ = f.extract()
    st = P.oracle_state(K, cap, X, W, n)
    uo = orc.update(p, st, Z)
    eo = orc.extract(p, Z.shape[0], uo)
    fo = orc.fuse(p, Z.shape[0], eo)
    # the extra measurement's C lives on the wrapped pairs alone, far above
    # the 1e-300 floor of the FP64 comparison
    assert np.all(uo["C"][:, -1] > 1e-290), uo["C"][:, -1]
    P.check_cz(ug["C"], uo["C"], orc.kappa(p), "fp64")
    P.check_weights(Wg, st)
    np.testing.assert_allclose(ug["mass"], uo["mass"], rtol=1e-9)
    np.testing.assert_allclose(ug["dW"], uo["dW"], rtol=0, atol=1e-12)
    P.check_selection(lg["sel"], lg["zeta"], ug["mass"], ug["LT"], uo, eo, tol=1e-9)
    assert list(est_g["label"]) == list(fo["label"])
    assert list(est_g["votes"]) == list(fo["votes"])
    if len(fo["label"]):
        np.testing.assert_allclose(est_g["state"], fo["state"], rtol=1e-9, atol=1e-9)
    f.close()
