"""End-to-end parity of the FP32 filter in distribution.

The FP32 GPU filter and the FP64 oracle run the same Monte Carlo runs of a
reduced benchmark workload (64 groups, 1e4 particles per target over all
groups, 5000 births per step from the measurement-driven proposal, clutter
rate 50, 10 targets, 20 steps): the same truth tracks and measurement sets
and the same Philox streams per run.  Once one resampling count differs
(FP32 against FP64 weights) the two trajectories are different samples of
the same filter, so they are compared as distributions: for the total PHD
mass after each update (its integral is the expected target number, section
2.1), the number of fused estimates, and the OSPA (p = 1, c = 100, section
4.1), the mean over runs of the paired difference GPU - oracle must lie
within 3 standard errors of zero (time-averaged over steps 6-20) and within
4 standard errors at every step (20 steps x 3 quantities).  A bias the
single-step tolerances let through (a weight 1e-5 off in the same direction
every step) would build up and fail this."""
import numpy as np
import pytest

import oracle as orc
from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.metrics import ospa, positions
from paper_1503_03769_amd.scenario import BASE_MODEL, make_scenario

pytestmark = pytest.mark.gpu

K, RUNS, STEPS, BURN = 64, 16, 20, 5
P = dict(BASE_MODEL, partitions=K, particles_per_target=1e4, births_per_step=5000, clutter_rate=50.0,
         birth_proposal=1, birth_alpha=0.1)
CAP, MAXM, SEED = 4096, 160, 777


def _paired_runs():
    out = {"gpu": np.zeros((3, RUNS, STEPS)), "orc": np.zeros((3, RUNS, STEPS))}
    for r in range(RUNS):
        truth, Z = make_scenario(P, 10, STEPS, 9100 + r)
        assert max(z.shape[0] for z in Z[1:]) <= MAXM
        f = pphd.Filter(P, pphd.PPHD_FP32, CAP, MAXM, SEED, r)
        o = orc.OracleFilter(P, CAP, SEED, r)
        f.init()
        for k in range(1, STEPS + 1):
            f.predict(k)
            f.update(Z[k])
            mass_g = float(f.read_update()["mass"].sum())
            est_g, _ = f.extract()
            f.resample(k)
            f.exchange(k)
            res = o.step(k, Z[k])
            mass_o = float(res["upd"]["mass"].sum())
            for side, mass, st in (("gpu", mass_g, est_g["state"]), ("orc", mass_o, res["est"]["state"])):
                out[side][0, r, k - 1] = mass
                out[side][1, r, k - 1] = len(st)
                out[side][2, r, k - 1] = ospa(positions(st), positions(truth[k]))
        f.close()
        print(f"  run {r}: mean mass GPU {out['gpu'][0, r, BURN:].mean():.3f} oracle "
              f"{out['orc'][0, r, BURN:].mean():.3f}, OSPA GPU {out['gpu'][2, r, BURN:].mean():.2f} oracle "
              f"{out['orc'][2, r, BURN:].mean():.2f}", flush=True)
    return out


def test_fp32_filter_matches_oracle_in_distribution(gpu):
    print(f"statistical parity: {RUNS} runs x {STEPS} steps, {K} groups, oracle threads {orc.threads()}",
          flush=True)
    out = _paired_runs()
    names = ("total mass", "fused estimates", "OSPA")
    for q, name in enumerate(names):
        g, o = out["gpu"][q], out["orc"][q]
        # time-averaged per run, then paired over runs
        d = g[:, BURN:].mean(axis=1) - o[:, BURN:].mean(axis=1)
        se = d.std(ddof=1) / np.sqrt(RUNS)
        slack = 1e-3 * max(abs(o[:, BURN:].mean()), 1e-3)  # identical trajectories give se = 0
        print(f"  {name}: GPU {g[:, BURN:].mean():.4f} oracle {o[:, BURN:].mean():.4f} "
              f"paired difference {d.mean():+.4f} (standard error {se:.4f})", flush=True)
        assert abs(d.mean()) <= 3.0 * se + slack, (name, d.mean(), se)
        for k in range(STEPS):
            dk = g[:, k] - o[:, k]
            sek = dk.std(ddof=1) / np.sqrt(RUNS)
            slk = 1e-3 * max(abs(o[:, k].mean()), 1e-3)
            assert abs(dk.mean()) <= 4.0 * sek + slk, (name, k + 1, dk.mean(), sek)
