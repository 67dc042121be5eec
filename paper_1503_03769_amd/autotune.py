"""Tile-shape autotuner for the two likelihood passes of pphd_update.

For every tile shape (particles per thread of the C(z) pass and of the weight
pass, measurements per wavefront) it runs the named workload (a single filter
or a batch of runs) from t = 0 and
averages the passes' HIP-event times (C(z) pass + weight pass + k_wfinal
where it runs) over a
window of steady-state steps.  The fastest shape is written to tuning.json
next to this file, keyed by storage precision (and "_batch" for batches);
`pphd.Filter` and `pphd.Batch` apply it by default.  The shape changes only floating-point summation order.

    python -m paper_1503_03769_amd.autotune [--workload NAME] [--steps A B]
"""
import argparse
import itertools
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_PATH = os.path.join(HERE, "tuning.json")

SHAPES = {"fp32": [4, 8, 16], "fp64": [2, 4, 8]}
MEAS_PER_WAVE = [8, 16, 32, 64, 128, 256]


def tune(workload: str, first: int, last: int, verbose: bool = True, meas_per_wave=None):
    import torch

    from . import pphd
    from .scenario import WORKLOADS, make_scenario, workload_seed

    from .scenario import batch_runs

    w = WORKLOADS[workload]
    p = w["model"]
    prec_name = w["precision"]
    prec = pphd.PPHD_FP32 if prec_name == "fp32" else pphd.PPHD_FP64
    seed = workload_seed(w["config_index"], 0)
    if w.get("batch"):
        runs, targets = batch_runs(w["n_runs"], seed)
        scen = [make_scenario(dict(p, clutter_rate=r["clutter_rate"]), targets[i], last, seed + 7919 * (i + 1))
                for i, r in enumerate(runs)]
        packs = [None] + [pphd.Batch.pack([scen[i][1][k] for i in range(len(runs))]) for k in range(1, last + 1)]
        zdev = [None] + [(torch.from_numpy(z).cuda(), torch.from_numpy(win).cuda()) for z, win in packs[1:]]

        def make():
            return pphd.Batch(p, runs, prec, w["cap"], w["max_meas"], seed, apply_tuning=False)

        def update(f, k):
            f.update_device(zdev[k][0], zdev[k][0].shape[0], zdev[k][1])
    else:
        truth, Z = make_scenario(p, w["n_targets"], last, seed)
        zdev = [None] + [torch.from_numpy(np.ascontiguousarray(Z[k])).cuda() for k in range(1, last + 1)]

        def make():
            return pphd.Filter(p, prec, w["cap"], w["max_meas"], seed, 0, apply_tuning=False)

        def update(f, k):
            f.update(zdev[k])
    results = []
    for pt1, pt2, mz in itertools.product(SHAPES[prec_name], SHAPES[prec_name], meas_per_wave or MEAS_PER_WAVE):
        f = make()
        f.set_tuning(pt1, pt2, mz)
        f.init()
        for k in range(1, last + 1):
            if k == first:
                f.set_timing(True)
            f.predict(k)
            update(f, k)
            f.resample(k)
            f.exchange(k)
        t = f.read_timing()
        f.close()
        n = max(t["cz"][1], 1)
        us = 1e3 * (t["cz"][0] + t["weight"][0] + t["wfinal"][0]) / n
        results.append((us, pt1, pt2, mz))
        if verbose:
            print(f"pt_cz={pt1:2d} pt_weight={pt2:2d} meas_per_wave={mz:3d}: {us:8.2f} us per update "
                  f"(cz {1e3 * t['cz'][0] / n:6.2f}, weight {1e3 * t['weight'][0] / n:6.2f})", flush=True)
    results.sort()
    us, pt1, pt2, mz = results[0]
    return dict(pt_cz=pt1, pt_weight=pt2, meas_per_wave=mz, passes_us=us, workload=workload,
                steps=[first, last]), results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="large_fp32_10tgt_k64")
    ap.add_argument("--steps", type=int, nargs=2, default=[20, 40])
    ap.add_argument("--out", default=TUNING_PATH)
    ap.add_argument("--meas-per-wave", type=int, nargs="+", default=None,
                    help="the measurement chunks to try (the bearing-frame passes of workloads with clutter "
                         "take all of a run's measurements per wavefront and ignore it)")
    args = ap.parse_args()
    best, _ = tune(args.workload, args.steps[0], args.steps[1], meas_per_wave=args.meas_per_wave)
    data = {}
    if os.path.exists(args.out):
        with open(args.out) as fh:
            data = json.load(fh)
    from .scenario import WORKLOADS
    w = WORKLOADS[args.workload]
    data[w["precision"] + ("_batch" if w.get("batch") else "")] = best
    with open(args.out, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(json.dumps(best), flush=True)


if __name__ == "__main__":
    sys.exit(main())
