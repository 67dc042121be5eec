"""Training recipe of the learned birth proposal (include/pphd_mlp.h).

Every step runs in the library's kernels: the simulated (z, x) pairs, the
forward and backward passes and the Adam steps.  This module only fixes the
schedule: 2^20 pairs (about 1e6) drawn from the birth density and the sensor
model, minibatches of 4096, Adam with the step size held for the first 60% of
the steps and then cut by 10x twice.
"""
from . import pphd

DATASET = 1 << 20
BATCH = 4096
STEPS = 3000
LR = 2e-3


def schedule(steps, lr=LR):
    a = int(0.6 * steps)
    b = int(0.85 * steps)
    return [(a, lr), (b - a, 0.1 * lr), (steps - b, 0.01 * lr)]


def train_proposal(params: dict, seed: int = 1, steps: int = STEPS, batch: int = BATCH, dataset: int = DATASET,
                   lr: float = LR, init_id: int = 0, stream=None):
    """Returns (network, per-step minibatch losses)."""
    import numpy as np
    net = pphd.Mlp(params, batch=batch, dataset=dataset, seed=seed, lr=lr, stream=stream)
    net.init_params(init_id)
    net.simulate(run=0)
    losses = [net.train(n, lr=r) for n, r in schedule(steps, lr) if n > 0]
    return net, np.concatenate(losses)
