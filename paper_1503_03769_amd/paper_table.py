"""The paper's comparison (section 4.1, Table 1) in the section-4 setting:
the standard particle PHD filter with N particles ("PHD", K = 1), the
distributed filter with K = 4 groups ("DCPPHD", N/K particles per group) and
the standard filter with N/K particles ("partPHD"), plus the distributed
filter with one C(z) summed over its 4 groups ("DCPPHD-gC", the groups
splitting the PHD mass), at clutter rates
r = 0, 10, 20, each over Monte Carlo runs of seeded 5-track scenarios.  The
runs of one configuration go through the GPU as one batch (one set of
launches per stage for all runs).  Mean OSPA (p = 1, c = 100) over runs and
scans, the standard deviation of the per-run means, and the GPU time per
scan of the whole batch.

    python -m paper_1503_03769_amd.paper_table [--runs 100] [--steps 50]
"""
import argparse
import json
import sys
import time

import numpy as np

from . import pphd
from .metrics import ospa, positions
from .scenario import PAPER_MODEL, make_paper_scenario

# particles per target over all groups (R), births per scan (J) and groups (K)
METHODS = {
    "PHD": dict(partitions=1, particles_per_target=800.0, births_per_step=800),
    "DCPPHD": dict(partitions=4, particles_per_target=800.0, births_per_step=800),
    "partPHD": dict(partitions=1, particles_per_target=200.0, births_per_step=200),
    "DCPPHD-gC": dict(partitions=4, particles_per_target=800.0, births_per_step=800),
}
# model fields of a method beyond its run table
MODEL_FIELDS = {"DCPPHD-gC": dict(global_cz=1)}


def run_config(method: str, clutter: float, n_runs: int, steps: int, seed0: int = 77000,
               precision=pphd.PPHD_FP64):
    import torch
    p = dict(PAPER_MODEL, clutter_rate=float(clutter), **MODEL_FIELDS.get(method, {}))
    m = METHODS[method]
    runs = [dict(m, clutter_rate=float(clutter), run_id=i) for i in range(n_runs)]
    scen = [make_paper_scenario(p, steps, seed0 + i) for i in range(n_runs)]
    max_meas = max(max(z.shape[0] for z in Z[1:]) for _, Z in scen)
    b = pphd.Batch(p, runs, precision, 8192, max(max_meas, 1), 4242)
    b.init()
    d = np.zeros((n_runs, steps))
    gpu_s = 0.0
    for k in range(1, steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.predict(k)
        b.update([Z[k] for _, Z in scen])
        est, _ = b.extract()
        b.resample(k)
        b.exchange(k)
        torch.cuda.synchronize()
        gpu_s += time.perf_counter() - t0
        for r in range(n_runs):
            d[r, k - 1] = ospa(positions(est[r]["state"]), positions(scen[r][0][k]))
    b.close()
    per_run = d.mean(axis=1)
    return dict(method=method, r=clutter, runs=n_runs, mean_ospa=float(d.mean()),
                std_of_run_means=float(per_run.std()), ms_per_scan=1e3 * gpu_s / steps)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=100)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    rows = []
    for r in (0.0, 10.0, 20.0):
        for method in METHODS:
            row = run_config(method, r, args.runs, args.steps)
            rows.append(row)
            print(f"{method:9s} r={r:4.0f}: mean OSPA {row['mean_ospa']:7.3f}  std(run means) "
                  f"{row['std_of_run_means']:6.3f}  {row['ms_per_scan']:7.3f} ms/scan ({args.runs} runs)",
                  flush=True)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(rows, fh, indent=1)


if __name__ == "__main__":
    sys.exit(main())
