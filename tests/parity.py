"""Shared helpers of the GPU parity tests: build matching inputs for the GPU
filter and the oracle, and the tolerances.

Tolerances (relative error at most 1e-5 on weights and C(z), exact on
resampling counts):
  * C_j(z):  FP64 storage: |C' - C| <= 1e-5 C (where C > 1e-300);
             FP32 storage: |C' - C| <= 1e-5 (kappa + C), the quantity that
             enters the weight update -- a clutter measurement far from every
             particle has C ~ 1e-200 that no FP32 likelihood can resolve.
  * weights: |w' - w| <= 1e-5 max(w, 1e-3 mean_j(w)).
  * mass:    relative 1e-6.
  * predicted states: relative 1e-12 (FP64) / 1e-6 (FP32), absolute floor for
    values near zero.
  * counts, copied states and integer decisions: exact (decisions that depend
    on a floating-point tie within the tolerance are compared for validity).
"""
import numpy as np

import oracle as orc
from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.scenario import random_particles

PREC = {"fp64": pphd.PPHD_FP64, "fp32": pphd.PPHD_FP32}


def as_storage(a, prec):
    return a.astype(np.float32).astype(np.float64) if prec == "fp32" else a.copy()


def make_filter(params, prec, cap, max_meas=256, seed=1234, run=0):
    return pphd.Filter(params, PREC[prec], cap, max_meas, seed, run)


def oracle_state(K, cap, X, W, n):
    st = orc.State(K, cap)
    st.X[:] = X
    st.W[:] = W
    st.n[:] = n
    return st


def cloud(K, cap, counts, seed, truth, prec, spread=30.0):
    X, W, n = random_particles(K, cap, counts, seed, truth=truth, spread=spread)
    return as_storage(X, prec), as_storage(W, prec), n


def check_states(Xg, Wg, ng, st, prec, rtol=None):
    K, cap = st.K, st.cap
    assert np.array_equal(ng, st.n), (ng, st.n)
    if rtol is None:
        rtol = 1e-12 if prec == "fp64" else 1e-6
    atol = 1e-9 if prec == "fp64" else 1e-4
    for j in range(K):
        sl = slice(j * cap, j * cap + int(st.n[j]))
        np.testing.assert_allclose(Xg[:, sl], st.X[:, sl], rtol=rtol, atol=atol)
        np.testing.assert_allclose(Wg[sl], st.W[sl], rtol=rtol, atol=0)


def check_weights(Wg, st):
    K, cap = st.K, st.cap
    worst = 0.0
    for j in range(K):
        n = int(st.n[j])
        if n == 0:
            continue
        sl = slice(j * cap, j * cap + n)
        w, g = st.W[sl], Wg[sl]
        floor = 1e-3 * w.mean()
        err = np.abs(g - w) / np.maximum(w, floor)
        worst = max(worst, float(err.max()))
    assert worst <= 1e-5, f"weight relative error {worst:.3e} > 1e-5"
    return worst


def check_cz(Cg, Co, kappa, prec):
    if Co.size == 0:
        return 0.0
    if prec == "fp64":
        mask = Co > 1e-300
        err = np.where(mask, np.abs(Cg - Co) / np.where(mask, Co, 1.0), 0.0)
        assert np.all(np.abs(Cg[~mask]) < 1e-290)
    else:
        denom = kappa + Co
        mask = denom > 0
        err = np.where(mask, np.abs(Cg - Co) / np.where(mask, denom, 1.0), 0.0)
        # kappa = 0 and no support at all: both sides must report zero
        assert np.all(Cg[~mask] == 0.0)
    worst = float(err.max())
    assert worst <= 1e-5, f"C(z) error {worst:.3e} > 1e-5"
    return worst


def check_selection(sel_g, zeta_g, mass_g, LT_g, upd_o, ext_o, tol=1e-5, run_total=False):
    """Local estimates: LT and the label sets must agree except where the
    oracle's own numbers sit within the tolerance of a rounding or ranking
    boundary; common labels' estimates agree to 1e-5 of the state scale.
    run_total: LT follows the total mass of the groups (one run whose groups
    split one PHD) instead of each group's own."""
    K, M = upd_o["dW"].shape
    total = float(np.sum(upd_o["mass"]))
    for j in range(K):
        m = total if run_total else upd_o["mass"][j]
        near_half = abs((m - np.floor(m)) - 0.5) < tol * max(1.0, m)
        if not near_half:
            assert LT_g[j] == ext_o["LT"][j], (j, LT_g[j], ext_o["LT"][j], m)
        a = set(np.nonzero(sel_g[j])[0])
        b = set(np.nonzero(ext_o["sel"][j])[0])
        if a != b and not near_half:
            dW = upd_o["dW"][j]
            chosen = sorted(b, key=lambda p: (-dW[p], p))
            cut = dW[chosen[-1]] if chosen else 0.0
            for p in a ^ b:
                assert abs(dW[p] - cut) <= tol, (j, p, dW[p], cut)
        for p in a & b:
            z_o = ext_o["zeta"][j, p]
            z_g = zeta_g[j, p]
            scale = max(1.0, float(np.abs(z_o).max()))
            assert np.all(np.abs(z_g - z_o) <= tol * scale), (j, p, z_g, z_o)
