"""Oracle parity of Step 2 (Eqs 7, 11-18; section 3.1 Steps 2-4) at the
measurement counts the workloads reach: more than one 64-lane chunk of
measurements (lambda 80-100, M in (64, 128]) and about 250 (lambda 200, the
dense-stress shape), over 64 and 256 groups.

Each case predicts survivors on the GPU, lets the update draw the births of
the measurement-driven or learned proposal (fewer than 16 wave tiles of
births per group, so birth tiles are split into measurement chunks), and
compares with the oracle element by element: C_j(z), every weight, the
closed-form Delta W, masses, LT and label sets, and the fused labels, votes
and states.  The oracle's input is the GPU's predicted survivors (already
checked against the oracle's predict) plus the oracle's own births rounded
to the storage precision, so the comparison sees only the update.

Some measurement sets are padded with clutter in one bearing frame so that
the frame-A / frame-B split of the bearing-frame passes falls inside a later
64-measurement chunk rather than the first."""
import math

import numpy as np
import pytest

import oracle as orc
from oracle import mlp as omlp
from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.scenario import BASE_MODEL, make_scenario, random_mixture_outputs
from tests import parity as P

pytestmark = pytest.mark.gpu


def _frame_padded(Z, nA, nB, seed):
    """Z plus uniform clutter so that exactly nA measurements have |bearing|
    <= pi/2 (frame A) and nB do not (frame B); shuffled."""
    rng = np.random.default_rng(seed)
    inA = np.abs(Z[:, 1]) <= 0.5 * math.pi
    addA, addB = max(0, nA - int(inA.sum())), max(0, nB - int((~inA).sum()))
    ra = np.column_stack([rng.uniform(0, 2000, addA), rng.uniform(-0.5 * math.pi, 0.5 * math.pi, addA)])
    sb = rng.uniform(0.5 * math.pi + 1e-6, math.pi, addB) * rng.choice([-1.0, 1.0], addB)
    rb = np.column_stack([rng.uniform(0, 2000, addB), sb])
    out = np.vstack([Z, ra, rb])
    return np.ascontiguousarray(out[rng.permutation(out.shape[0])])


def _cloud5(K, cap, counts, seed, truth, prec, dim):
    X, W, n = P.cloud(K, cap, counts, seed, truth, prec)
    if dim == 5:
        rng = np.random.default_rng(seed + 1)
        om = np.zeros((1, K * cap))
        om[0] = rng.normal(0.0, 0.02, K * cap)
        X = np.vstack([X, P.as_storage(om, prec)])
    return X, W, n


def _run_case(prec, K, counts, lam, n_targets, births, proposal, seed, max_meas, frames=None, dim=4):
    p = dict(BASE_MODEL, partitions=K, clutter_rate=lam, births_per_step=births, birth_proposal=proposal,
             birth_alpha=0.1)
    if dim == 5:
        p.update(dim=5, sigma_w=0.01, birth_sigma_w=0.02)
    truth, Zs = make_scenario(p, n_targets, 6, seed, turn_sigma=0.02 if dim == 5 else 0.0)
    k = max(range(1, 7), key=lambda i: len(Zs[i]))
    Z = Zs[k]
    if frames is not None:
        Z = _frame_padded(Z, frames[0], frames[1], seed)
    M = Z.shape[0]
    nA = int((np.abs(Z[:, 1]) <= 0.5 * math.pi).sum())
    print(f"  M reached = {M} (frame A {nA}, frame B {M - nA}), K = {K}, births/group = {births // K}, "
          f"{prec}, dim {dim}", flush=True)
    assert M <= max_meas
    cap = int(max(counts)) + births // K + 512
    X, W, n = _cloud5(K, cap, counts, seed + 7, truth[k], prec, dim)
    f = P.make_filter(p, prec, cap, max_meas=max_meas, seed=4321, run=5)
    f.write_state(X, W, n, pphd.PHASE_READY)
    f.predict(k)
    raw = None
    if proposal == 2:
        raw = random_mixture_outputs(M, seed + 3)
        f.set_birth_mixture(raw)
    # the GPU's predicted survivors against the oracle's predict
    Xp, Wp, npred = f.read_state()
    st = P.oracle_state(K, cap, X, W, n) if dim == 4 else _state5(K, cap, X, W, n)
    orc.predict(p, st, k, 4321, 5)
    assert np.array_equal(npred, st.n)
    rtol = 1e-12 if prec == "fp64" else 1e-6
    for j in range(K):
        sl = slice(j * cap, j * cap + int(n[j]))
        np.testing.assert_allclose(Xp[:, sl], st.X[:, sl], rtol=rtol, atol=1e-9 if prec == "fp64" else 1e-4)
    # the update's input on the oracle side: the GPU's survivors, the
    # oracle's births at the storage precision
    if proposal == 1:
        orc.birth_from_measurements(p, st, k, 4321, 5, Z)
    else:
        orc.birth_from_mixture(p, st, k, 4321, 5, omlp.mixture_table(p, Z, raw.astype(np.float64)))
    born = st.copy()
    for j in range(K):
        sl = slice(j * cap, j * cap + int(n[j]))
        st.X[:, sl] = Xp[:, sl]
        st.W[sl] = Wp[sl]
    st.X[:] = P.as_storage(st.X, prec)
    st.W[:] = P.as_storage(st.W, prec)
    f.update(Z)
    Xg, Wg, ng = f.read_state()
    ug = f.read_update()
    lg = f.read_local()
    est_g, mass_g = f.extract()
    assert np.array_equal(ng, st.n)
    # births drawn on the GPU against the oracle's draw
    for j in range(K):
        sl = slice(j * cap + int(n[j]), j * cap + int(st.n[j]))
        np.testing.assert_allclose(Xg[:, sl], born.X[:, sl], rtol=rtol, atol=1e-9 if prec == "fp64" else 1e-4)
    uo = orc.update(p, st, Z)
    eo = orc.extract(p, M, uo)
    fo = orc.fuse(p, M, eo)
    kappa = orc.kappa(p)
    ec = P.check_cz(ug["C"], uo["C"], kappa, prec)
    ew = P.check_weights(Wg, st)
    np.testing.assert_allclose(ug["mass"], uo["mass"], rtol=1e-6, atol=1e-300)
    np.testing.assert_allclose(mass_g, uo["mass"], rtol=1e-6, atol=1e-300)
    np.testing.assert_allclose(ug["dW"], uo["dW"], rtol=0, atol=1e-5)
    P.check_selection(lg["sel"], lg["zeta"], ug["mass"], ug["LT"], uo, eo)
    fused = np.array_equal(lg["sel"], eo["sel"])
    if fused:
        assert list(est_g["label"]) == list(fo["label"])
        assert list(est_g["votes"]) == list(fo["votes"])
        if len(fo["label"]):
            scale = max(1.0, float(np.abs(fo["state"]).max()))
            assert np.all(np.abs(est_g["state"] - fo["state"]) <= 1e-5 * scale)
    print(f"  max C err {ec:.2e}, max weight err {ew:.2e}, labels {int(lg['sel'].sum())}, "
          f"fused {len(est_g)} (compared: {fused})", flush=True)
    f.close()


def _state5(K, cap, X, W, n):
    st = orc.State(K, cap, X.shape[0])
    st.X[:] = X
    st.W[:] = W
    st.n[:] = n
    return st


def _counts(K, lo, hi, seed):
    return [int(c) for c in np.random.default_rng(seed).integers(lo, hi, K)]


DENSE_CASES = [
    # prec, K, count range, lambda, targets, births, proposal, seed, max_meas, frames (nA, nB), dim, label
    ("fp32", 64, (2000, 3200), 90.0, 10, 64 * 300, 1, 31, 192, None, 4,
     "64 groups, lambda 90 (second 64-measurement chunk)"),
    ("fp32", 64, (2000, 3200), 80.0, 10, 64 * 300, 1, 32, 192, (70, 45), 4,
     "64 groups, frame split inside the second chunk (70 A + 45 B)"),
    ("fp64", 8, (2500, 3500), 100.0, 8, 8 * 400, 1, 33, 192, (100, 20), 4,
     "FP64, 8 groups, frame split at 100"),
    ("fp32", 256, (800, 1300), 200.0, 50, 256 * 150, 1, 34, 320, None, 4,
     "256 groups, lambda 200 (about 250 measurements)"),
    ("fp32", 256, (800, 1300), 200.0, 50, 256 * 120, 1, 35, 384, (190, 70), 4,
     "256 groups, frame split at 190 (third chunk)"),
    ("fp32", 256, (800, 1300), 200.0, 50, 256 * 150, 2, 36, 320, None, 5,
     "dense-stress combination: CT 5-D, learned-mixture births, 256 groups, lambda 200"),
]


@pytest.mark.parametrize("case", DENSE_CASES, ids=[c[-1] for c in DENSE_CASES])
def test_update_above_64_measurements(gpu, case):
    prec, K, rng_c, lam, ntg, J, prop, seed, maxm, frames, dim, label = case
    print(f"dense update: {label}", flush=True)
    _run_case(prec, K, _counts(K, rng_c[0], rng_c[1], seed), lam, ntg, J, prop, seed, maxm, frames, dim)


def test_fusion_majority_over_many_groups(gpu):
    """Step 4 at 256 groups: fused labels, votes and states of the GPU's own
    label sets and local estimates against the oracle's fusion of the same
    sets (so the comparison is exact even where a label set is a near tie)."""
    print("fusion at 256 groups", flush=True)
    K, cap = 256, 1024
    p = dict(BASE_MODEL, partitions=K, clutter_rate=150.0, births_per_step=0, particles_per_target=800.0 * K)
    truth, Zs = make_scenario(p, 30, 4, 77)
    Z = Zs[4]
    X, W, n = P.cloud(K, cap, _counts(K, 600, 1000, 78), 79, truth[4], "fp32")
    # spread the group masses over [0.5, 2] times: label sets differ between groups
    scale = np.repeat(np.random.default_rng(80).uniform(0.5, 2.0, K), cap)
    W = P.as_storage(W * scale * 30.0, "fp32")
    f = P.make_filter(p, "fp32", cap, max_meas=320)
    f.write_state(X, W, n, pphd.PHASE_PREDICTED)
    f.update(Z)
    lg = f.read_local()
    est_g, _ = f.extract()
    M = Z.shape[0]
    fo = orc.fuse(p, M, dict(sel=lg["sel"].astype(np.int32), zeta=lg["zeta"]))
    votes = lg["sel"].sum(axis=0)
    print(f"  M = {M}, labels per group {lg['sel'].sum(axis=1).min()}..{lg['sel'].sum(axis=1).max()}, "
          f"votes {votes.min()}..{votes.max()}, fused {len(fo['label'])}", flush=True)
    # both outcomes of the strict majority rule occur
    assert np.any(2 * votes > K) and np.any((votes > 0) & (2 * votes <= K))
    assert list(est_g["label"]) == list(fo["label"])
    assert list(est_g["votes"]) == list(fo["votes"])
    np.testing.assert_allclose(est_g["state"], fo["state"], rtol=1e-10, atol=1e-7)
    f.close()
