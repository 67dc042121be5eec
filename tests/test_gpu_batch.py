"""GPU tests of the batched form: many independent runs in one set of
launches per stage.

A run inside a batch draws the same Philox numbers as the same run filtered
alone (same seed and run id) and goes through the same arithmetic in the same
order, so its particles, weights, counts and fused estimates must equal the
single filter's bit for bit.  The single filter is checked against the oracle
elsewhere; here one batched run is also checked against the oracle directly,
and the captured HIP-graph step must reproduce the eagerly launched one.
"""
import numpy as np
import pytest

import oracle as orc
from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.scenario import BASE_MODEL, make_scenario

from . import parity as P

pytestmark = pytest.mark.gpu

RUNS = [
    dict(partitions=1, births_per_step=300, clutter_rate=10.0, particles_per_target=800.0, run_id=3),
    dict(partitions=3, births_per_step=500, clutter_rate=40.0, particles_per_target=1500.0, run_id=7),
    dict(partitions=2, births_per_step=101, clutter_rate=25.0, particles_per_target=400.0, run_id=11),
    dict(partitions=1, births_per_step=50, clutter_rate=60.0, particles_per_target=2000.0, run_id=12),
]
TARGETS = [2, 4, 1, 3]
CAP, MAXM, SEED = 8192, 128, 4321


def _model(prop):
    return dict(BASE_MODEL, birth_proposal=prop, birth_alpha=0.1 if prop else 1.0)


def _single(p, r, prec):
    q = dict(p, partitions=r["partitions"], births_per_step=r["births_per_step"], clutter_rate=r["clutter_rate"],
             particles_per_target=r["particles_per_target"])
    # (the library's default shapes on both sides: a tuned tile shape changes
    # the FP32 summation order, and the batch and single filters fall in
    # different buckets of the tuning table)
    return q, pphd.Filter(q, P.PREC[prec], CAP, MAXM, SEED, r["run_id"], apply_tuning=False)


def _scenarios(p, steps):
    out = []
    for i, r in enumerate(RUNS):
        truth, Z = make_scenario(dict(p, clutter_rate=r["clutter_rate"]), TARGETS[i], steps, 900 + i)
        out.append((truth, Z))
    return out


def _run_slices(b, r):
    g0 = int(b.run_g0[r])
    return g0, int(RUNS[r]["partitions"])


def _assert_run_equal(bstate, sstate, g0, K):
    Xb, Wb, nb = bstate
    Xs, Ws, ns = sstate
    assert np.array_equal(nb[g0:g0 + K], ns)
    for j in range(K):
        n = int(ns[j])
        sb = slice((g0 + j) * CAP, (g0 + j) * CAP + n)
        ss = slice(j * CAP, j * CAP + n)
        assert np.array_equal(Xb[:, sb], Xs[:, ss])
        assert np.array_equal(Wb[sb], Ws[ss])


@pytest.mark.parametrize("prec,prop", [("fp32", 1), ("fp64", 0), ("fp64", 1)])
def test_batched_runs_equal_single_filters(gpu, prec, prop):
    print(f"batch vs single {prec} proposal {prop}", flush=True)
    p = _model(prop)
    steps = 8
    sc = _scenarios(p, steps)
    b = pphd.Batch(p, RUNS, P.PREC[prec], CAP, MAXM, SEED, apply_tuning=False)
    singles = [_single(p, r, prec)[1] for r in RUNS]
    b.init()
    for f in singles:
        f.init()
    for k in range(1, steps + 1):
        b.predict(k)
        b.update([Z[k] for _, Z in sc])
        est_b, mass_b = b.extract()
        b.resample(k)
        b.exchange(k)
        for r, f in enumerate(singles):
            f.predict(k)
            f.update(sc[r][1][k])
            est_s, mass_s = f.extract()
            f.resample(k)
            f.exchange(k)
            g0, K = _run_slices(b, r)
            assert np.array_equal(mass_b[g0:g0 + K], mass_s)
            assert est_b[r].tobytes() == est_s.tobytes(), (k, r)
    sb = b.read_state()
    for r, f in enumerate(singles):
        g0, K = _run_slices(b, r)
        _assert_run_equal(sb, f.read_state(), g0, K)
        f.close()
    b.close()


def test_batched_run_first_step_matches_oracle(gpu):
    """Run 1 (three groups) of an FP64 batch after one predict + update: the
    predicted particles and updated weights against the oracle."""
    p = _model(0)
    sc = _scenarios(p, 2)
    b = pphd.Batch(p, RUNS, pphd.PPHD_FP64, CAP, MAXM, SEED)
    b.init()
    b.predict(1)
    X0, W0, n0 = b.read_state()
    b.update([Z[1] for _, Z in sc])
    X1, W1, n1 = b.read_state()
    r = 1
    q, f = _single(p, RUNS[r], "fp64")
    f.close()
    g0, K = _run_slices(b, r)
    st = orc.State(K, CAP)
    orc.init(q, st, SEED, RUNS[r]["run_id"])
    orc.predict(q, st, 1, SEED, RUNS[r]["run_id"])
    sl = slice(g0 * CAP, (g0 + K) * CAP)
    P.check_states(X0[:, sl], W0[sl], n0[g0:g0 + K], st, "fp64")
    orc.update(q, st, sc[r][1][1])
    P.check_weights(W1[sl], st)
    b.close()


def test_captured_step_equals_eager_batch(gpu):
    """Whole steps replayed from the captured graphs (measurement buffers
    refilled on the stream between replays) equal the eagerly launched batch."""
    import torch
    print("batch graph", flush=True)
    p = _model(1)
    steps = 6
    sc = _scenarios(p, steps)
    nr = len(RUNS)
    zcap = nr * MAXM
    dz = torch.zeros((zcap, 2), dtype=torch.float64, device="cuda")
    dwin = torch.zeros((nr, 2), dtype=torch.int32, device="cuda")
    dout = torch.zeros((nr * MAXM * 40,), dtype=torch.uint8, device="cuda")
    dn = torch.zeros(nr, dtype=torch.int32, device="cuda")
    eager = pphd.Batch(p, RUNS, pphd.PPHD_FP32, CAP, MAXM, SEED)
    graph = pphd.Batch(p, RUNS, pphd.PPHD_FP32, CAP, MAXM, SEED)
    eager.init()
    graph.init()
    graph.capture(dz, zcap, dwin, dout, MAXM, dn, 1)
    for k in range(1, steps + 1):
        z, win = pphd.Batch.pack([Z[k] for _, Z in sc])
        eager.predict(k)
        eager.update([Z[k] for _, Z in sc])
        est_e, _ = eager.extract()
        eager.resample(k)
        eager.exchange(k)
        dz[:z.shape[0]].copy_(torch.from_numpy(z))
        dwin.copy_(torch.from_numpy(win))
        graph.launch()
        torch.cuda.synchronize()
        n = dn.cpu().numpy()
        raw = dout.cpu().numpy()
        for r in range(nr):
            recs = np.frombuffer(raw[r * MAXM * 40:(r * MAXM + int(n[r])) * 40].tobytes(), dtype=pphd.ESTIMATE_DTYPE)
            assert recs.tobytes() == est_e[r].tobytes(), (k, r)
    Xe, We, ne = eager.read_state()
    Xg, Wg, ng = graph.read_state()
    assert np.array_equal(ne, ng)
    for g in range(eager.K):
        sl = slice(g * CAP, g * CAP + int(ne[g]))
        assert np.array_equal(Xe[:, sl], Xg[:, sl]) and np.array_equal(We[sl], Wg[sl])
    eager.close()
    graph.close()


def test_batch_argument_errors(gpu):
    p = _model(0)
    b = pphd.Batch(p, RUNS, pphd.PPHD_FP32, CAP, MAXM, SEED)
    b.init()
    b.predict(1)
    z = np.zeros((10, 2))
    bad = np.array([[0, 5], [5, 5], [8, 5], [0, 0]], dtype=np.int32)   # run 2 runs past the set
    with pytest.raises(pphd.PphdError) as e:
        pphd.pphd_batch_update(b.h, z.ctypes.data, 10, bad.ctypes.data, 0)
    assert e.value.code == pphd.PPHD_EINVAL
    with pytest.raises(pphd.PphdError) as e:
        pphd.pphd_update(b.h, z.ctypes.data, 10, 0)
    assert e.value.code == pphd.PPHD_EINVAL
    q = pphd.Batch(dict(p, birth_proposal=2, birth_alpha=0.1), RUNS, pphd.PPHD_FP32, CAP, MAXM, SEED)
    q.init()
    q.predict(1)
    with pytest.raises(pphd.PphdError) as e:      # no network attached
        q.update([np.zeros((0, 2))] * len(RUNS))
    assert e.value.code == pphd.PPHD_ESTATE
    q.close()
    b.close()


def test_large_uneven_batch_matches_oracle_on_sampled_runs(gpu):
    """520 one-group FP32 runs of two sizes (the flat work lists of unlike
    runs), 300 births each: every run has two birth tiles split into chunks,
    1040 in all over the 1024-workgroup grid, so many workgroups finalize two
    of them in turn.  After one predict + update, sampled runs against the
    oracle."""
    print("large uneven batch", flush=True)
    p = _model(0)
    runs = [dict(partitions=1, births_per_step=300, clutter_rate=20.0,
                 particles_per_target=150.0 if i % 2 else 300.0, run_id=i) for i in range(520)]
    cap, maxm, seed = 1024, 64, 97
    Zs = [make_scenario(dict(p, clutter_rate=20.0), 2, 2, 4000 + i)[1] for i in range(len(runs))]
    b = pphd.Batch(p, runs, pphd.PPHD_FP32, cap, maxm, seed)
    b.init()
    b.predict(1)
    X0, W0, n0 = b.read_state()
    b.update([Z[1] for Z in Zs])
    X1, W1, n1 = b.read_state()
    for r in (0, 1, 257, 518, 519):
        q = dict(p, partitions=1, births_per_step=300, clutter_rate=20.0,
                 particles_per_target=runs[r]["particles_per_target"])
        g0 = int(b.run_g0[r])
        st = orc.State(1, cap)
        orc.init(q, st, seed, r)
        orc.predict(q, st, 1, seed, r)
        sl = slice(g0 * cap, (g0 + 1) * cap)
        P.check_states(X0[:, sl], W0[sl], n0[g0:g0 + 1], st, "fp32")
        st.X[:] = X0[:, sl]
        st.W[:] = W0[sl]
        orc.update(q, st, Zs[r][1])
        P.check_weights(W1[sl], st)
    b.close()
