"""Stage parity of the HIP path against the oracle, one stage at a time, on
identical seeded inputs (loaded into both sides from the generator, rounded
to the GPU's storage precision first)."""
import math

import numpy as np
import pytest

import oracle as orc
from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.scenario import BASE_MODEL, WORKLOADS, make_scenario
from tests import parity as P

pytestmark = pytest.mark.gpu


def _scen(params, seed=11, steps=8, n=5):
    truth, Z = make_scenario(params, n, steps, seed)
    k = max(range(1, steps + 1), key=lambda i: (len(truth[i]), len(Z[i])))
    return truth[k], Z[k]


PREDICT_CASES = [
    ("fp64", 1, [3000], 500, 8192),
    ("fp64", 3, [3000, 1234, 0], 100, 5000),
    ("fp32", 4, [9000, 4097, 1, 0], 77, 12000),
    # more births per group than one workgroup orders in registers (8192 in
    # FP32, 4096 in FP64): the multi-launch bearing order
    ("fp32", 2, [2000, 500], 20000, 13000),
    ("fp64", 1, [300], 5000, 6000),
]


@pytest.mark.parametrize("prec,K,counts,J,cap", PREDICT_CASES)
def test_predict_and_birth(gpu, prec, K, counts, J, cap):
    print(f"predict {prec} K={K} counts={counts} J={J}", flush=True)
    p = dict(BASE_MODEL, partitions=K, births_per_step=J)
    X, W, n = P.cloud(K, cap, counts, 5, None, prec)
    f = P.make_filter(p, prec, cap)
    f.write_state(X, W, n, pphd.PHASE_READY)
    f.predict(9)
    Xg, Wg, ng = f.read_state()
    st = P.oracle_state(K, cap, X, W, n)
    orc.predict(p, st, 9, 1234, 0)
    P.check_states(Xg, Wg, ng, st, prec)
    f.close()


UPDATE_CASES = [
    # prec, K, counts, clutter, p_D, n_targets, max_meas, label
    ("fp64", 1, [3500], 10.0, 0.95, 3, 256, "one group, FP64 (3 targets, lambda 10)"),
    ("fp64", 3, [2500, 700, 0], 10.0, 0.95, 4, 256, "three groups with an empty one"),
    ("fp32", 4, [10000, 4097, 1, 0], 50.0, 0.95, 6, 512, "FP32, several tiles and ragged tails"),
    ("fp32", 2, [5000, 3000], 0.0, 1.0, 4, 256, "no clutter (kappa = 0), p_D = 1"),
    ("fp32", 2, [3000, 2000], 50.0, 0.0, 4, 256, "p_D = 0"),
    ("fp64", 2, [3000, 2000], 50.0, 0.95, 4, 64, "measurement count at max_meas"),
]


@pytest.mark.parametrize("case", UPDATE_CASES, ids=[c[-1] for c in UPDATE_CASES])
def test_update_extract(gpu, case):
    prec, K, counts, lam, pD, ntg, max_meas, label = case
    print(f"update {label}", flush=True)
    cap = max(counts) + 512
    p = dict(BASE_MODEL, partitions=K, clutter_rate=lam, p_D=pD)
    # with kappa = 0 every measurement must lie within FP64 range of some
    # particle, or the oracle's C underflows to 0 and Eq 12 becomes 0/0
    truth, Z = _scen(dict(p, clutter_rate=lam if lam == 0.0 else max(lam, 10.0)), n=ntg)
    if max_meas == 64:
        rng = np.random.default_rng(4)
        extra = np.column_stack([rng.uniform(0, 2000, 64), rng.uniform(-math.pi, math.pi, 64)])
        Z = np.vstack([Z, extra])[:64]
    X, W, n = P.cloud(K, cap, counts, 21, truth, prec)
    f = P.make_filter(p, prec, cap, max_meas=max_meas)
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
    assert np.array_equal(ng, n)
    kappa = orc.kappa(p)
    ec = P.check_cz(ug["C"], uo["C"], kappa, prec)
    ew = P.check_weights(Wg, st)
    np.testing.assert_allclose(ug["mass"], uo["mass"], rtol=1e-6, atol=1e-300)
    np.testing.assert_allclose(mass_g, uo["mass"], rtol=1e-6, atol=1e-300)
    np.testing.assert_allclose(ug["dW"], uo["dW"], rtol=0, atol=1e-5)
    P.check_selection(lg["sel"], lg["zeta"], ug["mass"], ug["LT"], uo, eo)
    if np.array_equal(lg["sel"], eo["sel"]):
        assert list(est_g["label"]) == list(fo["label"])
        assert list(est_g["votes"]) == list(fo["votes"])
        if len(fo["label"]):
            scale = max(1.0, float(np.abs(fo["state"]).max()))
            assert np.all(np.abs(est_g["state"] - fo["state"]) <= 1e-5 * scale)
    print(f"  max C err {ec:.2e}, max weight err {ew:.2e}", flush=True)
    f.close()


RESAMPLE_CASES = [
    ("fp64", 1, [3500], 1000.0, 500, 8192, "one group FP64"),
    ("fp32", 5, [9000, 5000, 1, 0, 2048], 5000.0, 250, 12000, "FP32 ragged groups"),
    ("fp32", 2, [4000, 4000], 4000.0, 100, 6000, "clamped to capacity"),
    ("fp64", 2, [2048, 1000], 1000.0, 0, 4096, "equal weights"),
]


@pytest.mark.parametrize("case", RESAMPLE_CASES, ids=[c[-1] for c in RESAMPLE_CASES])
def test_resample_counts_exact(gpu, case):
    prec, K, counts, R, J, cap, label = case
    print(f"resample {label}", flush=True)
    p = dict(BASE_MODEL, partitions=K, particles_per_target=R, births_per_step=J)
    X, W, n = P.cloud(K, cap, counts, 33, None, prec)
    if label == "equal weights":
        W[:] = 1.0 / 1024
    if label == "clamped to capacity":
        W = P.as_storage(W * 10.0, prec)   # mass ~ 13: round(N R_j) far above cap - J_j
    f = P.make_filter(p, prec, cap)
    f.set_record_counts(True)
    f.write_state(X, W, n, pphd.PHASE_UPDATED)
    f.resample(6)
    Xg, Wg, ng = f.read_state()
    cg, mqg, clamped = f.read_resample()
    st = P.oracle_state(K, cap, X, W, n)
    out, co, mqo = orc.resample(p, st, 6, 1234, 0)
    assert np.array_equal(ng, out.n)
    for j in range(K):
        sl = slice(j * cap, j * cap + int(n[j]))
        assert np.array_equal(cg[sl], co[sl]), f"group {j}: counts differ"
    assert np.array_equal(mqg, mqo)
    for j in range(K):
        sl = slice(j * cap, j * cap + int(out.n[j]))
        assert np.array_equal(Xg[:, sl], out.X[:, sl])
        assert np.array_equal(Wg[sl], P.as_storage(out.W[sl], prec))
    if label == "clamped to capacity":
        assert clamped == K
    else:
        assert clamped == 0
    f.close()


@pytest.mark.parametrize("prec,K,counts", [("fp32", 5, [3000, 120, 2500, 999, 3999]),
                                           ("fp64", 3, [50, 50, 50]), ("fp64", 1, [700])])
def test_exchange_exact(gpu, prec, K, counts):
    print(f"exchange {prec} K={K}", flush=True)
    cap = 4200
    p = dict(BASE_MODEL, partitions=K, births_per_step=0)
    X, W, n = P.cloud(K, cap, counts, 44, None, prec)
    f = P.make_filter(p, prec, cap)
    f.write_state(X, W, n, pphd.PHASE_RESAMPLED)
    f.exchange(3)
    Xg, Wg, ng = f.read_state()
    st = P.oracle_state(K, cap, X, W, n)
    orc.exchange(p, st, 3, 1234, 0)
    assert np.array_equal(ng, st.n)
    for j in range(K):
        sl = slice(j * cap, j * cap + int(n[j]))
        assert np.array_equal(Xg[:, sl], st.X[:, sl])
        assert np.array_equal(Wg[sl], st.W[sl])
    f.close()


@pytest.mark.parametrize("prec,K,J,counts,cap", [("fp64", 3, 900, [2000, 700, 0], 4096),
                                                 ("fp32", 3, 900, [2000, 700, 0], 4096),
                                                 ("fp32", 2, 18000, [1500, 300], 11000),
                                                 ("fp64", 1, 5000, [800], 6000),
                                                 ("fp32", 1100, 330000, [300] * 1100, 1024),
                                                 ("fp32", 2, 6000, [1500, 300], 8192),
                                                 ("fp32", 64, 50000, [14000 + 37 * j for j in range(64)], 32768)])
def test_measurement_driven_births(gpu, prec, K, J, counts, cap):
    """Eq 6 with p_k(.|Z_k): predict reserves the birth slots, update draws
    them from the measurement-driven mixture and then updates all weights.
    In FP32 up to 1152 births per group of this proposal are drawn, ordered
    and weighted in one workgroup each (the second and fifth cases); the
    first case (FP64)
    and the last (3000 per group) draw and order them there and weight them
    in their own kernel; the third and fourth cases order their births in
    several launches.  In
    the fifth, 1100 groups of 300 survivors and 300 births, each workgroup of
    the second pass takes two birth tiles split into chunks, whose sums meet
    in LDS buffers used in turn.  The seventh has the birth share of the
    64-group benchmark workload: about 781 births per group of some 14 000
    survivors, drawn, ordered and weighted in one workgroup each."""
    print(f"measurement-driven births {prec} K={K} J={J}", flush=True)
    p = dict(BASE_MODEL, partitions=K, births_per_step=J, birth_proposal=1, birth_alpha=0.1)
    truth, Z = _scen(p, n=4)
    X, W, n = P.cloud(K, cap, counts, 13, truth, prec)
    f = P.make_filter(p, prec, cap)
    f.write_state(X, W, n, pphd.PHASE_READY)
    f.predict(4)
    f.update(Z)
    Xg, Wg, ng = f.read_state()
    st = P.oracle_state(K, cap, X, W, n)
    orc.predict(p, st, 4, 1234, 0)
    orc.birth_from_measurements(p, st, 4, 1234, 0, Z)
    births = st.copy()
    # the GPU stores the drawn births at its storage precision before updating
    st.X[:] = P.as_storage(st.X, prec)
    st.W[:] = P.as_storage(st.W, prec)
    orc.update(p, st, Z)
    assert np.array_equal(ng, st.n)
    rtol = 1e-12 if prec == "fp64" else 1e-6
    for j in range(K):
        sl = slice(j * cap, j * cap + int(st.n[j]))
        np.testing.assert_allclose(Xg[:, sl], births.X[:, sl], rtol=rtol, atol=1e-9 if prec == "fp64" else 1e-4)
    P.check_weights(Wg, st)
    f.close()


def test_no_clutter_far_measurement_keeps_unit_mass(gpu):
    """kappa = 0 and p_D = 1: each measurement hands exactly one unit of mass
    to the particles (the sum over i of the Eq 12 terms is C/C = 1), even for
    a measurement so far from every particle that its C underflows double
    precision -- the integer-shift scaling of the first pass keeps it."""
    p = dict(BASE_MODEL, partitions=2, clutter_rate=0.0, p_D=1.0)
    cap = 4096
    X, W, n = P.cloud(2, cap, [3000, 2500], 8, None, "fp32")
    X[0, :] = np.clip(X[0, :], -900, -500)            # particles only in x < -500
    Z = np.array([[1900.0, 0.01], [1950.0, 0.5], [600.0, 3.0]])   # far to the east / north-west
    for prec in ("fp32", "fp64"):
        f = P.make_filter(p, prec, cap)
        f.write_state(P.as_storage(X, prec), P.as_storage(W, prec), n, pphd.PHASE_PREDICTED)
        f.update(Z)
        u = f.read_update()
        np.testing.assert_allclose(u["mass"], [3.0, 3.0], rtol=1e-5)
        assert np.all(np.isfinite(f.read_state()[1]))
        f.close()


def test_call_order_and_argument_errors(gpu):
    p = dict(BASE_MODEL, partitions=2)
    f = P.make_filter(p, "fp32", 4096, max_meas=8)
    with pytest.raises(pphd.PphdError) as e:
        f.predict(1)
    assert e.value.code == pphd.PPHD_ESTATE
    f.init()
    with pytest.raises(pphd.PphdError) as e:
        f.resample(1)
    assert e.value.code == pphd.PPHD_ESTATE
    f.predict(1)
    with pytest.raises(pphd.PphdError) as e:
        f.update(np.zeros((9, 2)))
    assert e.value.code == pphd.PPHD_EINVAL
    f.update(np.zeros((0, 2)))
    f.resample(1)
    f.exchange(1)
    f.close()


def test_gaussian_birth_density_matches_oracle(gpu):
    """birth_density 1 (the section-4 Gaussian birth intensity): init and
    predict with births against the oracle, FP64."""
    from paper_1503_03769_amd.scenario import PAPER_MODEL
    K, cap = 4, 2048
    p = dict(PAPER_MODEL)
    f = P.make_filter(p, "fp64", cap, max_meas=64)
    f.init()
    f.predict(1)
    Xg, Wg, ng = f.read_state()
    st = orc.State(K, cap)
    orc.init(p, st, 1234, 0)
    orc.predict(p, st, 1, 1234, 0)
    P.check_states(Xg, Wg, ng, st, "fp64")
    f.close()


def test_exchange_exact_many_groups(gpu):
    """A run of more groups than one workgroup holds per stratum (1100 > 1024)
    takes the two-launch exchange; it must equal the oracle's exactly."""
    K, cap = 1100, 128
    print(f"exchange fp32 K={K}", flush=True)
    rng = np.random.default_rng(12)
    counts = [int(c) for c in rng.integers(40, 120, K)]
    p = dict(BASE_MODEL, partitions=K, births_per_step=0)
    X, W, n = P.cloud(K, cap, counts, 45, None, "fp32")
    f = P.make_filter(p, "fp32", cap)
    f.write_state(X, W, n, pphd.PHASE_RESAMPLED)
    f.exchange(5)
    Xg, Wg, ng = f.read_state()
    st = P.oracle_state(K, cap, X, W, n)
    orc.exchange(p, st, 5, 1234, 0)
    assert np.array_equal(ng, st.n)
    for j in range(K):
        sl = slice(j * cap, j * cap + int(n[j]))
        assert np.array_equal(Xg[:, sl], st.X[:, sl]) and np.array_equal(Wg[sl], st.W[sl])
    f.close()
