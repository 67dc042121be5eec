"""Whole filter runs on one scenario, scored by OSPA (section 4.1): the loop
the benchmark and the proposal comparison share.  Every stage runs in the
library; this module only sequences the calls and scores the estimates."""
import numpy as np

from . import pphd
from .metrics import ospa, positions


def run_ospa(params: dict, precision: int, cap: int, max_meas: int, truth, Z, seed: int, run: int = 0,
             net=None, steps=None):
    """Runs steps 1..steps of the scenario and returns the OSPA of the fused
    estimates at every step (index k-1 for step k) and the particle count
    after each predict (births included)."""
    steps = len(Z) - 1 if steps is None else steps
    f = pphd.Filter(params, precision, cap, max_meas, seed, run)
    if net is not None:
        f.attach_mlp(net)
    f.init()
    d, counts = [], []
    for k in range(1, steps + 1):
        f.predict(k)
        counts.append(int(f.read_counts().sum()))
        f.update(Z[k])
        est, _ = f.extract()
        d.append(ospa(positions(est["state"]), positions(truth[k])))
        f.resample(k)
        f.exchange(k)
    f.close()
    return np.array(d), np.array(counts)
