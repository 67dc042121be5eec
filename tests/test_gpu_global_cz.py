"""The global-C reading of Eq 11 (global_cz = 1) on the GPU against the
oracle: one C(z) summed over every group of the run before Eq 12, the groups
splitting the PHD mass, LT from the run's total mass and every group drawing
round(N_total R_j) children.

Step 2-4 parity element by element (each group's own C_j, every weight, the
group masses, Delta W, LT and label sets, fused estimates) in FP32 at the
benchmark's shape (64 groups, lambda 50) and in FP64, and a free-running
FP64 filter over 20 steps (init, births, resampling and exchange included)."""
import numpy as np
import pytest

import oracle as orc
from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.scenario import BASE_MODEL, WORKLOADS, make_scenario, workload_seed
from tests import parity as P

pytestmark = pytest.mark.gpu

CASES = [
    # prec, K, counts range, lambda, targets, label
    ("fp32", 64, (12000, 17000), 50.0, 10, "FP32, 64 groups, lambda 50"),
    ("fp64", 4, (3000, 5000), 20.0, 5, "FP64, 4 groups, lambda 20"),
    ("fp64", 3, (500, 900), 0.0, 3, "FP64, 3 groups, no clutter"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[-1] for c in CASES])
def test_global_update_matches_oracle(gpu, case):
    prec, K, (lo, hi), lam, ntg, label = case
    print(f"global C update: {label}", flush=True)
    p = dict(BASE_MODEL, partitions=K, clutter_rate=lam, global_cz=1, births_per_step=0)
    truth, Zs = make_scenario(p, ntg, 8, 77 + K)
    k = max(range(1, 9), key=lambda i: len(truth[i]))
    Z = Zs[k]
    counts = [int(c) for c in np.random.default_rng(K).integers(lo, hi, K)]
    counts[K // 2] = 0 if K > 3 else counts[K // 2]
    cap = max(counts) + 256
    X, W, n = P.cloud(K, cap, counts, 5 + K, truth[k], prec)
    # the groups split the mass: each group's weights are 1/K of a full PHD's
    W = P.as_storage(W / K, prec)
    f = P.make_filter(p, prec, cap, max_meas=128)
    f.write_state(X, W, n, pphd.PHASE_PREDICTED)
    f.update(Z)
    Xg, Wg, ng = f.read_state()
    ug = f.read_update()
    lg = f.read_local()
    est_g, mass_g = f.extract()
    st = P.oracle_state(K, cap, X, W, n)
    uo = orc.update(p, st, Z)
    eo = orc.extract(p, Z.shape[0], uo)
    fo = orc.fuse(p, Z.shape[0], eo)
    kappa = orc.kappa(p)
    # each group's own C_j (Eq 11); the comparison scale is the global
    # denominator kappa + sum_j C_j that enters Eq 12
    D = kappa + uo["C"].sum(axis=0)
    if prec == "fp32":
        err_c = float((np.abs(ug["C"] - uo["C"]) / np.maximum(D, 1e-300)).max()) if Z.shape[0] else 0.0
        assert err_c <= 1e-5, err_c
    else:
        ec = P.check_cz(ug["C"], uo["C"], kappa, prec)
        err_c = ec
    ew = P.check_weights(Wg, st)
    np.testing.assert_allclose(ug["mass"], uo["mass"], rtol=1e-6 if prec == "fp32" else 1e-9, atol=1e-300)
    np.testing.assert_allclose(ug["dW"], uo["dW"], rtol=0, atol=1e-5 if prec == "fp32" else 1e-12)
    P.check_selection(lg["sel"], lg["zeta"], ug["mass"], ug["LT"], uo, eo, run_total=True)
    if np.array_equal(lg["sel"], eo["sel"]):
        assert list(est_g["label"]) == list(fo["label"])
        assert list(est_g["votes"]) == list(fo["votes"])
        if len(fo["label"]):
            scale = max(1.0, float(np.abs(fo["state"]).max()))
            assert np.all(np.abs(est_g["state"] - fo["state"]) <= 1e-5 * scale)
    # the groups' masses add up to the expected target number
    print(f"  M = {Z.shape[0]}, max C err {err_c:.2e}, max weight err {ew:.2e}, total mass "
          f"{ug['mass'].sum():.3f}, LT {list(ug['LT'][:8])}, fused {len(est_g)}", flush=True)
    f.close()


def test_global_fp64_run_matches_oracle(gpu):
    """Free-running FP64 filter with one C over 4 groups: group sizes, masses,
    fused estimates every step and the final particle set agree with the
    oracle."""
    print("global C, FP64 run of 20 steps", flush=True)
    K = 4
    box = (400.0, 600.0, 400.0, 600.0)
    p = dict(BASE_MODEL, partitions=K, particles_per_target=400.0 * K, births_per_step=400 * K,
             region=box, birth_sigma_v=3.0, sigma_a=1.0, global_cz=1)
    cap, steps, seed = 6000, 20, 4321
    truth, Z = make_scenario(p, 3, steps, seed, start_box=(450.0, 550.0, 450.0, 550.0), start_sigma_v=2.0)
    f = P.make_filter(p, "fp64", cap, max_meas=256, seed=seed, run=3)
    f.init()
    o = orc.OracleFilter(p, cap, seed, 3)
    for k in range(1, steps + 1):
        f.predict(k)
        f.update(Z[k])
        ug = f.read_update()
        est_g, _ = f.extract()
        f.resample(k)
        f.exchange(k)
        out = o.step(k, Z[k])
        np.testing.assert_allclose(ug["mass"], out["upd"]["mass"], rtol=1e-9, atol=1e-300)
        assert list(ug["LT"]) == list(out["ext"]["LT"]), k
        assert list(est_g["label"]) == list(out["est"]["label"]), k
        if len(est_g):
            np.testing.assert_allclose(est_g["state"], out["est"]["state"], rtol=1e-9, atol=1e-9)
        Xg, Wg, ng = f.read_state()
        assert np.array_equal(ng, o.st.n), (k, ng, o.st.n)
        print(f"  step {k}: total mass {ug['mass'].sum():.4f}, sizes {list(ng)}, fused {len(est_g)}", flush=True)
    P.check_states(Xg, Wg, ng, o.st, "fp64", rtol=1e-9)
    f.close()


def test_global_batch_equals_single_filters(gpu):
    """Three runs of 4 groups each with one C per run, as one batch: every
    run's weights after a step equal the same run filtered alone (the sum
    over groups stays inside each run)."""
    print("global C batch of 3 runs", flush=True)
    p = dict(BASE_MODEL, partitions=4, global_cz=1, births_per_step=800, particles_per_target=2000.0)
    runs = [dict(partitions=4, births_per_step=800, clutter_rate=lam, particles_per_target=2000.0, run_id=r)
            for r, lam in enumerate((10.0, 40.0, 25.0))]
    cap, Mx = 2048, 128
    scen = [make_scenario(dict(p, clutter_rate=r["clutter_rate"]), 4, 3, 90 + i) for i, r in enumerate(runs)]
    b = pphd.Batch(p, runs, pphd.PPHD_FP32, cap, Mx, 55, apply_tuning=False)
    singles = [pphd.Filter(dict(p, clutter_rate=r["clutter_rate"]), pphd.PPHD_FP32, cap, Mx, 55, r["run_id"],
                           apply_tuning=False)
               for r in runs]
    b.init()
    for f in singles:
        f.init()
    for k in (1, 2):
        b.predict(k)
        b.update([scen[i][1][k] for i in range(3)])
        for i, f in enumerate(singles):
            f.predict(k)
            f.update(scen[i][1][k])
        Xb, Wb, nb = b.read_state()
        for i, f in enumerate(singles):
            Xs, Ws, ns = f.read_state()
            assert np.array_equal(nb[i * 4:(i + 1) * 4], ns)
            for j in range(4):
                sb = slice((i * 4 + j) * cap, (i * 4 + j) * cap + int(ns[j]))
                ss = slice(j * cap, j * cap + int(ns[j]))
                assert np.array_equal(Wb[sb], Ws[ss]), (k, i, j)
                assert np.array_equal(Xb[:, sb], Xs[:, ss]), (k, i, j)
        b.resample(k)
        b.exchange(k)
        for f in singles:
            f.resample(k)
            f.exchange(k)
    b.close()
    for f in singles:
        f.close()
