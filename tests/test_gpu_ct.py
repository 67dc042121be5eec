"""GPU tests of the 5-D coordinated-turn option (state [x, vx, y, vy, omega]):
a free-running FP64 run against the oracle, and a batch with the learned
proposal (the dense-stress combination) equal to its runs filtered alone."""
import numpy as np
import pytest

import oracle as orc
from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.scenario import BASE_MODEL, make_scenario, random_mlp_params
from tests import parity as P

pytestmark = pytest.mark.gpu

CT = dict(BASE_MODEL, dim=5, sigma_w=0.01, birth_sigma_w=0.02)


def test_ct_run_matches_oracle(gpu):
    print("ct end-to-end fp64", flush=True)
    K, cap, steps, seed = 3, 6000, 15, 2468
    box = (400.0, 600.0, 400.0, 600.0)
    p = dict(CT, partitions=K, particles_per_target=400.0 * K, births_per_step=400 * K, region=box,
             birth_sigma_v=3.0, sigma_a=1.0)
    truth, Z = make_scenario(p, 3, steps, seed, start_box=(450.0, 550.0, 450.0, 550.0), start_sigma_v=2.0)
    f = P.make_filter(p, "fp64", cap, seed=seed, run=2)
    f.init()
    o = orc.OracleFilter(p, cap, seed, 2)
    for k in range(1, steps + 1):
        f.predict(k)
        f.update(Z[k])
        ug = f.read_update()
        est_g, _ = f.extract()
        f.resample(k)
        f.exchange(k)
        out = o.step(k, Z[k])
        np.testing.assert_allclose(ug["mass"], out["upd"]["mass"], rtol=1e-9, atol=1e-300)
        assert list(est_g["label"]) == list(out["est"]["label"]), k
        Xg, Wg, ng = f.read_state()
        assert np.array_equal(ng, o.st.n), (k, ng, o.st.n)
    assert Xg.shape[0] == 5
    P.check_states(Xg, Wg, ng, o.st, "fp64", rtol=1e-9)
    f.close()


def test_ct_batch_with_learned_proposal_equals_singles(gpu):
    """Turn-rate state, learned births, three runs in one batch: each run's
    particles and estimates equal the same run filtered alone."""
    print("ct batch + learned proposal", flush=True)
    runs = [dict(partitions=2, births_per_step=600, clutter_rate=30.0, particles_per_target=1200.0, run_id=1),
            dict(partitions=1, births_per_step=300, clutter_rate=80.0, particles_per_target=900.0, run_id=2),
            dict(partitions=3, births_per_step=900, clutter_rate=10.0, particles_per_target=1500.0, run_id=3)]
    p = dict(CT, birth_proposal=2, birth_alpha=0.1)
    cap, maxm, seed, steps = 8192, 128, 97, 5
    net = pphd.Mlp(p, batch=512, dataset=4096, seed=3)
    net.set_params(random_mlp_params(21, scale=0.5))
    scen = [make_scenario(dict(p, clutter_rate=r["clutter_rate"]), 3, steps, 50 + i) for i, r in enumerate(runs)]
    b = pphd.Batch(p, runs, pphd.PPHD_FP32, cap, maxm, seed, apply_tuning=False)
    b.attach_mlp(net)
    singles = []
    for r in runs:
        q = dict(p, partitions=r["partitions"], births_per_step=r["births_per_step"],
                 clutter_rate=r["clutter_rate"], particles_per_target=r["particles_per_target"])
        f = pphd.Filter(q, pphd.PPHD_FP32, cap, maxm, seed, r["run_id"], apply_tuning=False)
        f.attach_mlp(net)
        singles.append(f)
    b.init()
    for f in singles:
        f.init()
    for k in range(1, steps + 1):
        b.predict(k)
        b.update([Z[k] for _, Z in scen])
        est_b, _ = b.extract()
        b.resample(k)
        b.exchange(k)
        for i, f in enumerate(singles):
            f.predict(k)
            f.update(scen[i][1][k])
            est_s, _ = f.extract()
            f.resample(k)
            f.exchange(k)
            assert est_b[i].tobytes() == est_s.tobytes(), (k, i)
    Xb, Wb, nb = b.read_state()
    assert Xb.shape[0] == 5
    for i, f in enumerate(singles):
        g0, K = int(b.run_g0[i]), runs[i]["partitions"]
        Xs, Ws, ns = f.read_state()
        assert np.array_equal(nb[g0:g0 + K], ns)
        for j in range(K):
            n = int(ns[j])
            assert np.array_equal(Xb[:, (g0 + j) * cap:(g0 + j) * cap + n], Xs[:, j * cap:j * cap + n])
            assert np.array_equal(Wb[(g0 + j) * cap:(g0 + j) * cap + n], Ws[j * cap:j * cap + n])
        f.close()
    b.close()
    net.close()
