"""What the trained proposal network gains: the same filter, the same
scenario (10 targets, clutter rate 50, 16 groups, 2e5 particles at 10
targets of which 2000 births per step) and the same particle budget, with
births drawn from the birth density itself (uniform over the region) or from
the trained network's mixtures (Eq 6 weights keep both unbiased).  Mean OSPA
over steps 1-40 (track initiation included) on four seeded scenarios; the
network is trained on the GPU first."""
import numpy as np
import pytest

from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.proposal import train_proposal
from paper_1503_03769_amd.runs import run_ospa
from paper_1503_03769_amd.scenario import WORKLOADS, make_scenario, workload_seed

pytestmark = pytest.mark.gpu


def test_learned_proposal_beats_uniform_birth(gpu):
    w = WORKLOADS["learned_fp32_10tgt"]
    p = w["model"]
    print("learned gain: training", flush=True)
    net, losses = train_proposal(p, seed=1)
    print(f"training loss {losses[:20].mean():.3f} -> {losses[-50:].mean():.3f}", flush=True)
    res = {}
    for name, prop in (("uniform", 0), ("learned", 2)):
        q = dict(p, birth_proposal=prop)
        vals = []
        for run in range(4):
            seed = workload_seed(w["config_index"], run)
            truth, Z = make_scenario(q, w["n_targets"], 40, seed)
            d, n = run_ospa(q, pphd.PPHD_FP32, w["cap"], w["max_meas"], truth, Z, seed, run,
                            net=net if prop == 2 else None)
            vals.append(d.mean())
            print(f"{name} run {run}: mean OSPA {d.mean():.2f} m (steps 1-10 {d[:10].mean():.2f}, "
                  f"11-40 {d[10:].mean():.2f}), particles {n.mean():.0f}", flush=True)
        res[name] = float(np.mean(vals))
    net.close()
    print(res, flush=True)
    assert res["learned"] < 0.9 * res["uniform"], res
