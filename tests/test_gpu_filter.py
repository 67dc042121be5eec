"""Whole-step parity of the HIP path: the FP64 filter against the oracle over a
full run, the full-size FP32 launch configuration on sampled groups, and
determinism."""
import numpy as np
import pytest

import oracle as orc
from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.scenario import BASE_MODEL, WORKLOADS, make_scenario, random_particles, workload_seed
from tests import parity as P

pytestmark = pytest.mark.gpu


def _run_both(p, prec, cap, steps, n_targets, seed, max_meas=256, start_box=None):
    kw = {} if start_box is None else dict(start_box=start_box, start_sigma_v=2.0)
    truth, Z = make_scenario(p, n_targets, steps, seed, **kw)
    f = P.make_filter(p, prec, cap, max_meas=max_meas, seed=seed, run=3)
    f.init()
    o = orc.OracleFilter(p, cap, seed, 3)
    for k in range(1, steps + 1):
        print(f"  step {k}", flush=True)
        f.predict(k)
        f.update(Z[k])
        ug = f.read_update()
        est_g, _ = f.extract()
        f.resample(k)
        f.exchange(k)
        out = o.step(k, Z[k])
        yield k, f, o, ug, est_g, out


@pytest.mark.parametrize("name,K,steps", [("plain_fp64_3tgt", 1, 50), ("four_groups_fp64", 4, 20)])
def test_fp64_run_matches_oracle(gpu, name, K, steps):
    """Free-running FP64 filter: every step's masses, estimates, group sizes
    and the final particle set agree with the oracle."""
    print(f"end-to-end {name}", flush=True)
    if name == "plain_fp64_3tgt":
        w = WORKLOADS[name]
        p, cap, ntg, box = w["model"], w["cap"], w["n_targets"], None
        seed = workload_seed(w["config_index"], 0)
    else:
        box = (400.0, 600.0, 400.0, 600.0)
        p = dict(BASE_MODEL, partitions=K, particles_per_target=400.0 * K, births_per_step=400 * K,
                 region=box, birth_sigma_v=3.0, sigma_a=1.0)
        cap, ntg, seed = 6000, 3, 4321
        box = (450.0, 550.0, 450.0, 550.0)
    for k, f, o, ug, est_g, out in _run_both(p, "fp64", cap, steps, ntg, seed, start_box=box):
        np.testing.assert_allclose(ug["mass"], out["upd"]["mass"], rtol=1e-9, atol=1e-300)
        assert list(est_g["label"]) == list(out["est"]["label"]), k
        if len(est_g):
            np.testing.assert_allclose(est_g["state"], out["est"]["state"], rtol=1e-9, atol=1e-9)
        Xg, Wg, ng = f.read_state()
        assert np.array_equal(ng, o.st.n), (k, ng, o.st.n)
    P.check_states(Xg, Wg, ng, o.st, "fp64", rtol=1e-9)
    f.close()


def test_full_size_fp32_sampled_groups(gpu):
    """The benchmark's launch configuration (64 groups, ~16k particles each,
    ~60 measurements): C, weights and masses of sampled groups against the
    oracle run on those groups alone; the mass identity on every group."""
    w = WORKLOADS["large_fp32_10tgt_k64"]
    p, cap, K = w["model"], w["cap"], 64
    truth, Z = make_scenario(p, w["n_targets"], 12, workload_seed(w["config_index"], 0))
    k = max(range(1, 13), key=lambda i: len(truth[i]))
    tk, zk = truth[k], Z[k]
    rng = np.random.default_rng(5)
    counts = rng.integers(15000, 17500, size=K).astype(np.int32)
    counts[7] = 0
    X, W, n = P.cloud(K, cap, counts, 61, tk, "fp32")
    f = P.make_filter(p, "fp32", cap, max_meas=w["max_meas"])
    f.write_state(X, W, n, pphd.PHASE_PREDICTED)
    f.update(zk)
    Xg, Wg, ng = f.read_state()
    ug = f.read_update()
    kappa = orc.kappa(p)
    # identity on every group: sum w' = nu sum w + sum_p C/(kappa + C)
    for j in range(K):
        sl = slice(j * cap, j * cap + int(n[j]))
        rhs = (1 - p["p_D"]) * W[sl].sum() + (ug["C"][j] / (kappa + ug["C"][j])).sum()
        assert abs(ug["mass"][j] - rhs) <= 1e-5 * max(rhs, 1e-12)
    p1 = dict(p, partitions=1)
    for j in (0, 7, 33, 63):
        print(f"  group {j}", flush=True)
        st = orc.State(1, cap)
        st.X[:] = X[:, j * cap:(j + 1) * cap]
        st.W[:] = W[j * cap:(j + 1) * cap]
        st.n[0] = n[j]
        uo = orc.update(p1, st, zk)
        P.check_cz(ug["C"][j:j + 1], uo["C"], kappa, "fp32")
        sub = orc.State(1, cap)
        sub.W[:] = st.W
        sub.n[0] = n[j]
        P.check_weights(Wg[j * cap:(j + 1) * cap], sub)
        assert abs(ug["mass"][j] - uo["mass"][0]) <= 1e-6 * max(uo["mass"][0], 1e-300)
    f.close()


def test_full_size_resample_exact(gpu):
    """Resampling counts at the benchmark's size, every group, exact."""
    w = WORKLOADS["large_fp32_10tgt_k64"]
    p, cap, K = w["model"], w["cap"], 64
    rng = np.random.default_rng(9)
    counts = rng.integers(14000, 17000, size=K).astype(np.int32)
    X, W, n = P.cloud(K, cap, counts, 71, None, "fp32")
    f = P.make_filter(p, "fp32", cap, max_meas=w["max_meas"])
    f.set_record_counts(True)
    f.write_state(X, W, n, pphd.PHASE_UPDATED)
    f.resample(5)
    cg, mqg, clamped = f.read_resample()
    Xg, Wg, ng = f.read_state()
    st = P.oracle_state(K, cap, X, W, n)
    out, co, mqo = orc.resample(p, st, 5, 1234, 0)
    assert np.array_equal(ng, out.n)
    for j in range(K):
        sl = slice(j * cap, j * cap + int(n[j]))
        assert np.array_equal(cg[sl], co[sl]), f"group {j}: counts differ"
    for j in range(0, K, 9):
        sl = slice(j * cap, j * cap + int(out.n[j]))
        assert np.array_equal(Xg[:, sl], out.X[:, sl])
    f.close()


def test_runs_are_deterministic(gpu):
    """No floating-point atomics: two runs give bit-identical particle sets."""
    p = dict(BASE_MODEL, partitions=8, particles_per_target=2.0e4, births_per_step=4000, clutter_rate=50.0)
    truth, Z = make_scenario(p, 6, 5, 3)
    res = []
    for _ in range(2):
        f = P.make_filter(p, "fp32", 8192, max_meas=512, seed=77)
        f.init()
        for k in range(1, 6):
            f.predict(k)
            f.update(Z[k])
            f.extract()
            f.resample(k)
            f.exchange(k)
        res.append(f.read_state())
        f.close()
    (Xa, Wa, na), (Xb, Wb, nb) = res
    assert np.array_equal(na, nb)
    for j in range(8):
        sl = slice(j * 8192, j * 8192 + int(na[j]))     # slots beyond the count are unspecified
        assert np.array_equal(Xa[:, sl], Xb[:, sl]) and np.array_equal(Wa[sl], Wb[sl])


def test_device_extract_fuses_with_the_resampling_scatter(gpu):
    """pphd_extract_device right after an update launches the resampling's
    parent scatter with the fusion in its first workgroups; pphd_resample
    then skips the scatter.  Against host extraction (k_fuse alone, the
    scatter at pphd_resample): the same estimates and bit-identical particle
    sets every step.  Also a second device extraction in the same step (the
    fusion alone, the scatter not repeated) and a state written between the
    extraction and the resampling (which must scatter the written state)."""
    import torch

    p = dict(BASE_MODEL, partitions=16, particles_per_target=2.0e4, births_per_step=3000, clutter_rate=50.0,
             birth_proposal=1, birth_alpha=0.1)
    truth, Z = make_scenario(p, 6, 7, 5)
    cap, Mx = 8192, 512
    host = P.make_filter(p, "fp32", cap, max_meas=Mx, seed=41)
    dev = P.make_filter(p, "fp32", cap, max_meas=Mx, seed=41)
    out = torch.zeros((Mx * 40 + 7) // 8, dtype=torch.float64, device="cuda")
    nout = torch.zeros(1, dtype=torch.int32, device="cuda")
    host.init()
    dev.init()
    for k in range(1, 8):
        print(f"  step {k}", flush=True)
        for f in (host, dev):
            f.predict(k)
            f.update(Z[k])
        est_h, _ = host.extract()
        dev.extract_device(out, nout, Mx)
        if k == 3:
            dev.extract_device(out, nout, Mx)       # the fusion again, no second scatter
        if k == 5:
            # a written state replaces the one the extraction scattered
            for f in (host, dev):
                X, W, n = f.read_state()
                W = (W * 0.5).astype(W.dtype)
                f.write_state(X, W, n, pphd.PHASE_UPDATED)
        torch.cuda.synchronize()
        n_d = int(nout.cpu()[0])
        recs = np.frombuffer(out.cpu().numpy().tobytes(), dtype=pphd.ESTIMATE_DTYPE)[:min(n_d, Mx)]
        assert n_d == len(est_h), (k, n_d, len(est_h))
        assert list(recs["label"]) == list(est_h["label"]) and list(recs["votes"]) == list(est_h["votes"])
        assert np.array_equal(recs["state"], est_h["state"]), k
        for f in (host, dev):
            f.resample(k)
            f.exchange(k)
        Xa, Wa, na = host.read_state()
        Xb, Wb, nb = dev.read_state()
        assert np.array_equal(na, nb), k
        for j in range(16):
            sl = slice(j * cap, j * cap + int(na[j]))
            assert np.array_equal(Xa[:, sl], Xb[:, sl]) and np.array_equal(Wa[sl], Wb[sl]), (k, j)
    host.close()
    dev.close()


@pytest.mark.parametrize("pt_cz,pt_weight", [(4, 4), (4, 8), (16, 4), (8, 16)])
def test_tile_shapes_against_the_oracle(gpu, pt_cz, pt_weight):
    """The two passes' tile shapes, equal (the second pass then splits its
    heavy tiles from the first pass's kept counts) and unequal: C(z),
    weights, masses and the local estimates against the oracle, with
    clutter (lambda 50) and several hundred particles per group past the
    last whole tile."""
    K, lam = 6, 50.0
    p = dict(BASE_MODEL, partitions=K, clutter_rate=lam, births_per_step=0)
    truth, Z = make_scenario(p, 10, 8, 314)
    k = max(range(1, 9), key=lambda i: len(truth[i]))
    tk, zk = truth[k], Z[k]
    counts = [5000, 4097, 3333, 1, 2600, 4999]
    cap = 5120
    X, W, n = P.cloud(K, cap, counts, 27, tk, "fp32", spread=60.0)
    f = P.make_filter(p, "fp32", cap, max_meas=128)
    f.set_tuning(pt_cz, pt_weight, 16)
    f.write_state(X, W, n, pphd.PHASE_PREDICTED)
    f.update(zk)
    Xg, Wg, ng = f.read_state()
    ug = f.read_update()
    lg = f.read_local()
    st = P.oracle_state(K, cap, X, W, n)
    uo = orc.update(p, st, zk)
    eo = orc.extract(p, zk.shape[0], uo)
    kappa = orc.kappa(p)
    print(f"  M = {zk.shape[0]}", flush=True)
    P.check_cz(ug["C"], uo["C"], kappa, "fp32")
    P.check_weights(Wg, st)
    np.testing.assert_allclose(ug["mass"], uo["mass"], rtol=1e-6, atol=1e-300)
    P.check_selection(lg["sel"], lg["zeta"], ug["mass"], ug["LT"], uo, eo)
    f.close()
