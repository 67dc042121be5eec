"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module simulates the *world* the filter observes -- target trajectories,
detections and clutter -- and defines the named workloads.  It contains none
of the filter's arithmetic (no likelihood, weight, resampling or exchange), and
it draws its randomness from numpy's PCG64, never from the filter's Philox
streams.

Workload recipe (the paper's truth tracks are not available, so a seeded
generator stands in for them):
  * target i of n appears at step b_i = 1 + floor(u T/10) and disappears after
    step T - floor(u' T/10), so most targets are present for most of the run;
  * its initial position is uniform in [-800, 800]^2, its velocity N(0, 10^2 I),
    and it moves with the constant-velocity model of section 4 (acceleration
    noise sigma_a on each axis); at the edge of the surveillance square
    [-1000, 1000]^2 it is reflected (position mirrored, velocity component
    negated), so it stays in view;
  * each live target is detected with probability p_D; a detection is
    [range, bearing] + N(0, diag(sigma_r^2, sigma_theta^2)) with the bearing
    wrapped into [-pi, pi);
  * clutter is Poisson(lambda) points uniform over [r_min, r_max] x [th_min, th_max);
  * each measurement set is shuffled.
"""
import math

import numpy as np

BASE_MODEL = dict(
    T=1.0, sigma_a=5.0, sensor_x=0.0, sensor_y=0.0, sigma_r=10.0, sigma_theta=0.02,
    p_S=0.99, p_D=0.95, clutter_rate=10.0, r_min=0.0, r_max=2000.0,
    th_min=-math.pi, th_max=math.pi, birth_mass=0.1,
    region=(-1000.0, 1000.0, -1000.0, 1000.0), birth_sigma_v=10.0, init_mass=1.0,
    particles_per_target=1000.0, exchange_fraction=0.1, partitions=1, births_per_step=500,
    birth_proposal=0, birth_alpha=1.0,
)

# Named workloads.  "precision" is the GPU path's storage type; the oracle is FP64.
# Births use the measurement-driven proposal of Eq 6 (a 0.1 share of the
# birth density itself keeps the importance weights bounded).
WORKLOADS = {
    # 3 targets, 50 steps, one group, FP64 everywhere.
    "plain_fp64_3tgt": dict(
        model=dict(BASE_MODEL, clutter_rate=10.0, particles_per_target=1000.0,
                   births_per_step=500, partitions=1, birth_proposal=1, birth_alpha=0.1),
        n_targets=3, steps=50, cap=16384, precision="fp64", max_meas=256, config_index=1),
    # 10 targets, 100 steps, 64 groups with exchange and fusion, FP32 storage.
    "large_fp32_10tgt_k64": dict(
        model=dict(BASE_MODEL, clutter_rate=50.0, particles_per_target=1.0e5,
                   births_per_step=50000, partitions=64, birth_proposal=1, birth_alpha=0.1),
        n_targets=10, steps=100, cap=32768, precision="fp32", max_meas=512, config_index=2),
    # 10 targets, 16 groups, 2e5 particles at 10 targets (R = 1.98e4 per
    # target, J = 2000 births, 1% of the budget): the learned birth proposal
    # against uniform birth at the same particle budget.
    "learned_fp32_10tgt": dict(
        model=dict(BASE_MODEL, clutter_rate=50.0, particles_per_target=1.98e4,
                   births_per_step=2000, partitions=16, birth_proposal=2, birth_alpha=0.1),
        n_targets=10, steps=100, cap=32768, precision="fp32", max_meas=512, config_index=4),
    # 256 independent runs in one batch (see batch_runs): 1e4-2e5 particles,
    # clutter rate 10-100 and 1-12 targets each, one group per run.
    "batch_fp32_256runs": dict(
        model=dict(BASE_MODEL, birth_proposal=1, birth_alpha=0.1),
        n_runs=256, steps=40, cap=300000, precision="fp32", max_meas=192, config_index=3,
        batch=True),
    # Dense stress: 16 runs of 50 targets each in one batch, clutter rate 200,
    # the 5-D coordinated-turn state (truth targets turn at rates N(0, 0.02^2)),
    # K = 256 groups per run, 4e6 particles at 50 targets plus 2e5 births,
    # learned birth proposal.
    "dense_ct_fp32_16runs": dict(
        model=dict(BASE_MODEL, dim=5, sigma_w=0.01, birth_sigma_w=0.02, clutter_rate=200.0,
                   particles_per_target=8.0e4, births_per_step=200000, partitions=256, birth_proposal=2,
                   birth_alpha=0.1),
        n_runs=16, n_targets=50, steps=30, cap=32768, precision="fp32", max_meas=320, config_index=5,
        batch=True, turn_sigma=0.02),
}


# Section 4 of the paper: 5 tracks over 50 scans, survival 0.9, detection 1,
# Gaussian birth intensity N([0, 3, 0, -3], diag(10, 1, 10, 1)), clutter over
# bearing [-pi/2, pi/2] x range [0, 200] m, range-bearing noise 5 m / 0.05 rad
# (read as standard deviations), 200 particles per target and group, K = 4.
# Values the paper leaves open: birth mass 0.1 per scan, initial mass 0.1,
# acceleration noise 0.5 m/s^2 on both axes (the printed noise matrix does not
# fit this state), 200 births per group and scan.
PAPER_MODEL = dict(
    BASE_MODEL, sigma_a=0.5, sigma_r=5.0, sigma_theta=0.05, p_S=0.9, p_D=1.0, clutter_rate=10.0,
    r_min=0.0, r_max=200.0, th_min=-math.pi / 2, th_max=math.pi / 2, birth_mass=0.1, init_mass=0.1,
    region=(-100.0, 300.0, -300.0, 100.0), birth_density=1, birth_mean=(0.0, 3.0, 0.0, -3.0),
    birth_std=(math.sqrt(10.0), 1.0, math.sqrt(10.0), 1.0), partitions=4, particles_per_target=800.0,
    births_per_step=800, birth_proposal=0, birth_alpha=1.0,
)


def make_paper_scenario(model: dict, steps: int, seed: int, n_targets: int = 5):
    """Tracks in the paper's setting: target i appears at scan 1 + floor(20u),
    drawn from the Gaussian birth intensity, moves with the CV model and
    leaves after 20 + floor(20u') scans (or at the end); every target is
    detected (p_D = 1 in the paper, but model["p_D"] is honoured); clutter is
    Poisson(model["clutter_rate"]) uniform over the clutter region.  Returns
    (truth, Z) like make_scenario."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T, sa = model["T"], model["sigma_a"]
    mean = np.asarray(model["birth_mean"], dtype=np.float64)
    std = np.asarray(model["birth_std"], dtype=np.float64)
    births = [1 + int(math.floor(rng.uniform() * 20)) for _ in range(n_targets)]
    lives = [20 + int(math.floor(rng.uniform() * 20)) for _ in range(n_targets)]
    states = [None] * n_targets
    truth = [np.zeros((0, 4))]
    Z = [np.zeros((0, 2))]
    for k in range(1, steps + 1):
        alive = []
        for i in range(n_targets):
            if k < births[i] or k > births[i] + lives[i]:
                continue
            if k == births[i]:
                states[i] = mean + std * rng.normal(size=4)
            else:
                states[i] = _cv_step(rng, states[i], T, sa)
            alive.append(states[i].copy())
        tk = np.array(alive).reshape(-1, 4)
        meas = []
        for st in tk:
            if rng.uniform() < model["p_D"]:
                dx, dy = st[0] - model["sensor_x"], st[2] - model["sensor_y"]
                r = math.hypot(dx, dy) + rng.normal(0, model["sigma_r"])
                th = math.atan2(dy, dx) + rng.normal(0, model["sigma_theta"])
                th = (th + math.pi) % (2 * math.pi) - math.pi
                meas.append((r, th))
        for _ in range(rng.poisson(model["clutter_rate"])):
            meas.append((rng.uniform(model["r_min"], model["r_max"]),
                         rng.uniform(model["th_min"], model["th_max"])))
        zk = np.array(meas, dtype=np.float64).reshape(-1, 2)
        if zk.shape[0] > 1:
            zk = zk[rng.permutation(zk.shape[0])]
        truth.append(tk)
        Z.append(np.ascontiguousarray(zk))
    return truth, Z


def batch_runs(n_runs: int, seed: int):
    """Run table of a batch and the number of targets of each run: particle
    budget N uniform in [1e4, 2e5], clutter rate uniform in [10, 100], 1-12
    targets; a fifth of the budget is births, the rest R = 0.8 N / targets
    particles per target; one group per run; run r has Philox run word r."""
    rng = np.random.Generator(np.random.PCG64(seed))
    runs, targets = [], []
    for r in range(n_runs):
        N = rng.uniform(1e4, 2e5)
        lam = rng.uniform(10.0, 100.0)
        n = int(rng.integers(1, 13))
        runs.append(dict(partitions=1, births_per_step=int(round(0.2 * N)), clutter_rate=float(lam),
                         particles_per_target=0.8 * N / n, run_id=r))
        targets.append(n)
    return runs, targets


def workload_runs(w: dict, seed: int):
    """Run table and target counts of a batch workload: random budgets for
    the many-run batch (batch_runs), identical runs (the model's own values,
    run word r) otherwise."""
    if "n_targets" not in w:
        return batch_runs(w["n_runs"], seed)
    p = w["model"]
    runs = [dict(partitions=int(p["partitions"]), births_per_step=int(p["births_per_step"]),
                 clutter_rate=float(p["clutter_rate"]), particles_per_target=float(p["particles_per_target"]),
                 run_id=r) for r in range(w["n_runs"])]
    return runs, [int(w["n_targets"])] * w["n_runs"]


def workload_seed(config_index: int, run: int) -> int:
    return 0x5EED0000 + 1000 * int(config_index) + int(run)


def _cv_step(rng, s, T, sigma_a):
    a = rng.normal(0.0, sigma_a, size=2)
    x, vx, y, vy = s
    return np.array([x + T * vx + 0.5 * T * T * a[0], vx + T * a[0],
                     y + T * vy + 0.5 * T * T * a[1], vy + T * a[1]])


def _ct_step(rng, s, T, sigma_a, w):
    """Coordinated turn at the constant rate w plus CV acceleration noise."""
    a = rng.normal(0.0, sigma_a, size=2)
    x, vx, y, vy = s
    if w != 0.0:
        sn, cs = math.sin(w * T), math.cos(w * T)
        fa, fb = sn / w, (1.0 - cs) / w
    else:
        sn, cs, fa, fb = 0.0, 1.0, T, 0.0
    return np.array([x + fa * vx - fb * vy + 0.5 * T * T * a[0], cs * vx - sn * vy + T * a[0],
                     y + fb * vx + fa * vy + 0.5 * T * T * a[1], sn * vx + cs * vy + T * a[1]])


def _reflect(s, lo, hi, ip, iv):
    while not (lo <= s[ip] <= hi):
        if s[ip] > hi:
            s[ip] = 2 * hi - s[ip]
        else:
            s[ip] = 2 * lo - s[ip]
        s[iv] = -s[iv]
    return s


def make_scenario(model: dict, n_targets: int, steps: int, seed: int, start_box=(-800.0, 800.0, -800.0, 800.0),
                  start_sigma_v=10.0, surveillance=(-1000.0, 1000.0, -1000.0, 1000.0), turn_sigma=0.0):
    """Returns (truth, Z): truth[k] is an array [n_alive, 4] and Z[k] an array
    [M_k, 2] of (range, bearing) for k = 1..steps (index 0 is unused).
    start_box / start_sigma_v: where targets appear and their velocity spread;
    surveillance: the square targets are reflected at; turn_sigma > 0: each
    target turns at a constant rate drawn from N(0, turn_sigma^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    turns = rng.normal(0.0, turn_sigma, size=n_targets) if turn_sigma > 0 else np.zeros(n_targets)
    T, sa = model["T"], model["sigma_a"]
    xmin, xmax, ymin, ymax = surveillance
    births = [1 + int(math.floor(rng.uniform() * steps / 10)) for _ in range(n_targets)]
    deaths = [steps - int(math.floor(rng.uniform() * steps / 10)) for _ in range(n_targets)]
    states = [None] * n_targets
    truth = [np.zeros((0, 4))]
    Z = [np.zeros((0, 2))]
    for k in range(1, steps + 1):
        alive = []
        for i in range(n_targets):
            if k < births[i] or k > deaths[i]:
                continue
            if k == births[i]:
                states[i] = np.array([rng.uniform(start_box[0], start_box[1]), rng.normal(0, start_sigma_v),
                                      rng.uniform(start_box[2], start_box[3]), rng.normal(0, start_sigma_v)])
            else:
                if turn_sigma > 0:
                    states[i] = _ct_step(rng, states[i], T, sa, float(turns[i]))
                else:
                    states[i] = _cv_step(rng, states[i], T, sa)
                states[i] = _reflect(states[i], xmin, xmax, 0, 1)
                states[i] = _reflect(states[i], ymin, ymax, 2, 3)
            alive.append(states[i].copy())
        tk = np.array(alive).reshape(-1, 4)
        meas = []
        for s in tk:
            if rng.uniform() < model["p_D"]:
                dx, dy = s[0] - model["sensor_x"], s[2] - model["sensor_y"]
                r = math.hypot(dx, dy) + rng.normal(0, model["sigma_r"])
                th = math.atan2(dy, dx) + rng.normal(0, model["sigma_theta"])
                th = (th + math.pi) % (2 * math.pi) - math.pi
                meas.append((r, th))
        nc = rng.poisson(model["clutter_rate"])
        for _ in range(nc):
            meas.append((rng.uniform(model["r_min"], model["r_max"]),
                         rng.uniform(model["th_min"], model["th_max"])))
        zk = np.array(meas, dtype=np.float64).reshape(-1, 2)
        if zk.shape[0] > 1:
            zk = zk[rng.permutation(zk.shape[0])]
        truth.append(tk)
        Z.append(np.ascontiguousarray(zk))
    return truth, Z


def bf16_representable(a):
    """float32 values rounded to the nearest BF16 value (ties to even)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def random_mlp_params(seed, scale=1.0, hidden=128):
    """Random network parameters in the flat layout of the learned proposal
    (uniform He-style magnitudes; output log-std biases offset to about
    exp(-3) so the mixtures are moderately narrow), BF16-representable."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, n_out in ((2, hidden), (hidden, hidden), (hidden, hidden), (hidden, 36)):
        a = scale * math.sqrt(6.0 / fan_in) * (0.2 if n_out == 36 else 1.0)
        parts.append(rng.uniform(-a, a, size=n_out * fan_in))
        b = rng.normal(0.0, 0.05, size=n_out)
        if n_out == 36:
            b[5::9] -= 3.0
            b[7::9] -= 3.0
        parts.append(b)
    return bf16_representable(np.concatenate(parts))


def random_mixture_outputs(M, seed):
    """Random network outputs [M, 36] (float32): logits N(0, 1), mean offsets
    N(0, 0.02^2) (normalised units), position log-stds N(-4.5, 0.3^2),
    velocity log-stds N(0, 0.3^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    o = np.zeros((M, 4, 9))
    o[:, :, 0] = rng.normal(0, 1, (M, 4))
    o[:, :, 1:5] = rng.normal(0, 0.02, (M, 4, 4))
    o[:, :, 5] = rng.normal(-4.5, 0.3, (M, 4))
    o[:, :, 7] = rng.normal(-4.5, 0.3, (M, 4))
    o[:, :, 6] = rng.normal(0, 0.3, (M, 4))
    o[:, :, 8] = rng.normal(0, 0.3, (M, 4))
    return o.reshape(M, 36).astype(np.float32)


def random_particles(K, cap, counts, seed, truth=None, spread=30.0, dtype=np.float64):
    """A synthetic particle cloud in the [4][K*cap] layout: part of every
    partition is scattered around the given truth states, the rest uniform over
    the surveillance square; weights are positive with a few orders of
    magnitude of spread.  Returns (X, W, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.zeros((4, K * cap), dtype=np.float64)
    W = np.zeros(K * cap, dtype=np.float64)
    n = np.asarray(counts, dtype=np.int32).copy()
    for j in range(K):
        nj = int(n[j])
        base = j * cap
        pos = rng.uniform(-1000, 1000, size=(nj, 2))
        vel = rng.normal(0, 10, size=(nj, 2))
        if truth is not None and len(truth) > 0 and nj > 0:
            near = rng.uniform(size=nj) < 0.6
            idx = rng.integers(0, len(truth), size=nj)
            pos[near, 0] = truth[idx[near], 0] + rng.normal(0, spread, size=near.sum())
            pos[near, 1] = truth[idx[near], 2] + rng.normal(0, spread, size=near.sum())
            vel[near, 0] = truth[idx[near], 1] + rng.normal(0, 3, size=near.sum())
            vel[near, 1] = truth[idx[near], 3] + rng.normal(0, 3, size=near.sum())
        X[0, base:base + nj] = pos[:, 0]
        X[1, base:base + nj] = vel[:, 0]
        X[2, base:base + nj] = pos[:, 1]
        X[3, base:base + nj] = vel[:, 1]
        W[base:base + nj] = np.exp(rng.uniform(-3, 0, size=nj)) * 1e-3
    if dtype == np.float32:
        X = X.astype(np.float32).astype(np.float64)
        W = W.astype(np.float32).astype(np.float64)
    return X, W, n
