"""Benchmark of the distributed particle PHD filter step on one MI355X.

One step = the whole per-step recursion through the C ABI on one stream:
predict (+births) -> update (C(z) pass, combine, weight pass, finalize) ->
extract (fusion, estimates to device memory) -> resample -> exchange.
All measurement sets are resident in device memory before timing starts.

Prints one JSON line:
  value        particle x measurement updates per second (sum over timed steps
               of N_k * M_k, divided by the timed wall time)
  steps_per_s  filter steps per second
  steps_per_s_pcie  the same steps with every Z_k uploaded from host memory
               through pphd_update and the fused estimates downloaded with
               pphd_extract (PCIe included; not the headline)
  roofline     the dominant kernel against HBM bandwidth
  variants     the same workload in FP64 storage, and with births drawn from
               the birth density itself (uniform births, proposal 0)
  cpu_baseline the FP64 oracle on the host for a bounded sample of the run,
               on all the host cores the process may use and on one thread
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# HBM peak of the MI355X (bytes/s).
HBM_PEAK_GBS = 8000.0
# Wave tile of the frame passes (64 lanes x 4 particles per lane, the tuned shape).
PASS_TILE = 256
BIRTH_PROPOSALS = {0: "birth density (uniform over the region)", 1: "measurement-driven mixture",
                   2: "learned per-measurement mixtures"}
# Kernel sources a stored counter summary was taken on.
KERNEL_SOURCES = ("paper_1503_03769_amd/csrc/kernels.h", "paper_1503_03769_amd/csrc/pphd.hip")


def pass_bytes(counts, Mg, esz, tile=PASS_TILE):
    """Algorithmic HBM bytes of one launch of each likelihood pass, from the
    particle count and the measurement count of every group.
      first pass:  per particle the geometry (scaled range, two frame bearings,
                   log2 weight: 4 doubles) and the weight; per tile and
                   measurement the partial sum (8 bytes), per tile the
                   weight total and the partials' exponent (8 + 4 bytes);
      second pass: per particle the geometry (3 doubles), the weight and the
                   four CV components read, the new weight and its bearing
                   bucket (4 bytes) written; per 256-slot tile the bucket
                   counts (64 x 4 bytes), weight sum and maximum (16 bytes).
    The measurement rows a tile reads are shared by every tile of the run and
    are not counted."""
    counts = np.asarray(counts, dtype=np.int64)
    Mg = np.asarray(Mg, dtype=np.int64)
    n = int(counts.sum())
    tiles = -(-counts // tile)
    cz = n * (32 + esz) + int((tiles * (8 * Mg + 12)).sum())
    weight = n * (28 + 6 * esz) + int((-(-counts // 256)).sum()) * 272
    return cz, weight


def step_bytes(counts, births, esz, dim=4):
    """Algorithmic HBM bytes of one launch of the per-particle kernels around
    the passes, from each group's particle count after the births and its
    births:
      birth_order (births drawn, ordered and weighed, with the survivors'
                   prediction in the same launch): per survivor the state and
                   weight read and written ((dim + 1) values each way) and its
                   four FP64 geometry values written; per birth its state,
                   weight and geometry written;
      rs_expand   (the systematic expansion, with the ring exchange fused):
                   per parent its state and weight read, per child the same
                   written (the children number about as many as the
                   parents), and one 8-byte tile sum per 256 parents."""
    counts = np.asarray(counts, dtype=np.int64)
    births = np.asarray(births, dtype=np.int64)
    rec = (dim + 1) * esz
    surv = int((counts - births).clip(min=0).sum())
    front = surv * (2 * rec + 32) + int(births.sum()) * (rec + 32)
    expand = int(counts.sum()) * 2 * rec + int((-(-counts // 256)).sum()) * 8
    return front, expand


def source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel_class, workload):
    """HBM bytes per launch of the dominant pass from the committed counter
    summary (profiles/traffic_<class>_<workload>.txt: FETCH_SIZE and
    WRITE_SIZE per dispatch, scaled by a plain copy's counters), or None when
    there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_class}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash():
        return None
    return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=90)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large_fp32_10tgt_k64")
    ap.add_argument("--run", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="bound on the oracle's CPU-baseline sample (0 = skip)")
    ap.add_argument("--no-timing-pass", action="store_true",
                    help="skip the HIP-event pass (for profiler runs)")
    ap.add_argument("--no-pcie", action="store_true",
                    help="skip the pass with host measurement sets and host estimates (for profiler runs)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP64 and uniform-birth variants of the workload and the default-shape pass")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch workloads: skip the run-by-run comparison pass (for profiler runs)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding the groups over "
              "several GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1503_03769_amd import pphd
    from paper_1503_03769_amd.metrics import ospa, positions
    from paper_1503_03769_amd.scenario import WORKLOADS, make_scenario, workload_seed

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy_mib > 0:
        nel = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = WORKLOADS[args.workload]
    if w.get("batch"):
        line = bench_batch(args, w)
        print(json.dumps(line), flush=True)
        return
    p = w["model"]
    prec = pphd.PPHD_FP32 if w["precision"] == "fp32" else pphd.PPHD_FP64
    total = args.warmup + args.steps
    seed = workload_seed(w["config_index"], args.run)
    truth, Z = make_scenario(p, w["n_targets"], max(total, w["steps"]), seed)
    Ms = [Z[k].shape[0] for k in range(len(Z))]
    assert max(Ms) <= w["max_meas"]
    # measurement sets resident in HBM before timing
    offs = np.concatenate([[0], np.cumsum(Ms)])
    zall = torch.from_numpy(np.concatenate([Z[k] for k in range(len(Z))]).reshape(-1, 2)).cuda()
    cap_est = w["max_meas"]
    est_dev = torch.zeros((total + 1, cap_est * 40), dtype=torch.uint8, device="cuda")
    nest_dev = torch.zeros(total + 1, dtype=torch.int32, device="cuda")

    # learned birth proposal: train the network first (outside the timed region)
    net, mlp_info = None, None
    if int(p.get("birth_proposal", 0)) == 2:
        from paper_1503_03769_amd.proposal import train_proposal
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net, losses = train_proposal(p, seed=1)
        torch.cuda.synchronize()
        mlp_info = {"train_s": time.perf_counter() - t0, "train_steps": int(len(losses)),
                    "final_loss": float(np.mean(losses[-50:])), "pairs": 1 << 20}

    def make(q=p, pr=prec, tuned=True):
        f = pphd.Filter(q, pr, w["cap"], w["max_meas"], seed, args.run, apply_tuning=tuned)
        if net is not None and int(q.get("birth_proposal", 0)) == 2:
            f.attach_mlp(net)
        return f

    def step(f, k):
        f.predict(k)
        f.update(zall[offs[k]:offs[k + 1]])
        f.extract_device(est_dev[k], nest_dev[k:k + 1], cap_est)
        f.resample(k)
        f.exchange(k)

    def step_pcie(f, k):
        # Z_k from host memory (copied through the library's pinned staging),
        # the fused estimates back to host memory (a synchronising download)
        f.predict(k)
        f.update(Z[k])
        f.extract()
        f.resample(k)
        f.exchange(k)

    def timed(q=p, pr=prec, one=step, tuned=True):
        f = make(q, pr, tuned)
        f.init()
        for k in range(1, args.warmup + 1):
            one(f, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.warmup + 1, total + 1):
            one(f, k)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        f.close()
        return el

    def counted(q, pr):
        """particle x measurement pairs of the timed steps (the same run,
        bit-identical, with the particle counts read after every predict)"""
        f = make(q, pr)
        f.init()
        n_pairs = 0
        for k in range(1, total + 1):
            f.predict(k)
            f.update(zall[offs[k]:offs[k + 1]])
            # (the counts after the update are the predicted ones: the update
            # changes weights only; read here, the predict still rides in the
            # update's first launch as in the timed pass)
            if k > args.warmup:
                n_pairs += int(f.read_counts().sum()) * Ms[k]
            f.extract_device(est_dev[k], nest_dev[k:k + 1], cap_est)
            f.resample(k)
            f.exchange(k)
        f.close()
        return n_pairs

    def run_ospa():
        nest = nest_dev.cpu().numpy()
        raw = est_dev.cpu().numpy()
        d = []
        for k in range(args.warmup + 1, total + 1):
            recs = np.frombuffer(raw[k].tobytes(), dtype=pphd.ESTIMATE_DTYPE)[:min(int(nest[k]), cap_est)]
            d.append(ospa(positions(recs["state"]), positions(truth[k])))
        return float(np.mean(d))

    # ---- pass A: timed ------------------------------------------------------
    elapsed = timed()
    ms_per_step = elapsed * 1e3 / args.steps
    probe = make()
    shape = probe.tuning
    probe.close()
    # the same steps with the library's default launch shape
    elapsed_default = timed(tuned=False) if shape and not args.no_variants else None
    # ---- the same steps with host measurement sets and host estimates -------
    elapsed_pcie = timed(one=step_pcie) if not args.no_pcie else None

    # ---- pass B: same run, per-kernel HIP-event times and particle counts ----
    K_ = int(p["partitions"])
    J_ = int(p["births_per_step"])
    births_per_group = np.array([J_ // K_ + (1 if j < J_ % K_ else 0) for j in range(K_)])
    kern = {}
    pairs = []
    parts = []
    pbytes = []
    esz = 4 if prec == pphd.PPHD_FP32 else 8
    if not args.no_timing_pass:
        g = make()
        g.init()
        for k in range(1, total + 1):
            if k == args.warmup + 1:
                g.set_timing(True)
            g.predict(k)
            g.update(zall[offs[k]:offs[k + 1]])
            if k > args.warmup:
                n = g.read_counts()
                pairs.append(int(n.sum()) * Ms[k])
                parts.append(int(n.sum()))
                pbytes.append(pass_bytes(n, np.full(len(n), Ms[k]), esz)
                              + step_bytes(n, births_per_group, esz, int(p.get("dim", 4))))
            g.extract_device(est_dev[k], nest_dev[k:k + 1], cap_est)
            g.resample(k)
            g.exchange(k)
        kern = g.read_timing()
        g.close()

    # estimates of the timed run -> OSPA against the truth
    ospa_mean = run_ospa()
    # ---- variants of the same workload: FP64 storage, uniform births -------
    variants = {}
    if not args.no_variants:
        vlist = []
        if prec == pphd.PPHD_FP32:
            vlist.append(("fp64", p, pphd.PPHD_FP64, "FP64 storage and likelihoods (the same run)"))
        if int(p.get("birth_proposal", 0)) != 0:
            vlist.append(("uniform_births", dict(p, birth_proposal=0), prec,
                          "births drawn from the birth density itself (uniform position, weight m_b/J_j)"))
        for name, q, pr, what in vlist:
            el = timed(q, pr)
            n_pairs = counted(q, pr)
            variants[name] = {"value": n_pairs / el, "unit": "pair-updates/s", "ms_per_step": el * 1e3 / args.steps,
                              "steps_per_s": args.steps / el, "dtype": "f64" if pr == pphd.PPHD_FP64 else "f32",
                              "birth_proposal": int(q.get("birth_proposal", 0)), "ospa_mean": run_ospa(),
                              "what": what}

    value = float(sum(pairs)) / elapsed if pairs else None
    line = {
        "metric": "particle x measurement updates/sec (also filter steps/sec and OSPA) at 1 GPU",
        "value": value,
        "unit": "pair-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "steps_per_s": 1e3 / ms_per_step,
        "steps_per_s_pcie": args.steps / elapsed_pcie if elapsed_pcie else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == pphd.PPHD_FP32 else "f64",
        "data": "synthetic (seeded truth tracks, detections and Poisson clutter)",
        "config": {
            "workload": args.workload,
            "birth_proposal": int(p.get("birth_proposal", 0)),
            "birth_proposal_name": BIRTH_PROPOSALS[int(p.get("birth_proposal", 0))],
            "partitions": int(p["partitions"]),
            "targets": int(w["n_targets"]),
            "clutter_rate": float(p["clutter_rate"]),
            "births_per_step": int(p["births_per_step"]),
            "particles_per_target": float(p["particles_per_target"]),
            "mean_particles": float(np.mean(parts)) if parts else None,
            "mean_measurements": float(np.mean([Ms[k] for k in range(args.warmup + 1, total + 1)])),
            "parallelism": f"{int(p['partitions'])} particle partitions on one GPU",
        },
        "ospa_mean": ospa_mean,
        "ospa_params": {"p": 1, "c": 100.0},
        "tuning": tuning_record(pphd, shape, elapsed, elapsed_default, args.steps, False, prec,
                                int(p["partitions"]), w["cap"],
                                float(p["clutter_rate"]) + 10.0),
    }
    if variants:
        line["variants"] = variants
    if kern:
        per = {name: {"avg_us": 1e3 * ms / max(n, 1), "launches": n} for name, (ms, n) in kern.items() if n}
        line["kernels"] = per
        # dominant kernel: the larger of the two likelihood passes
        line["roofline"] = roofline(pphd, kern, np.mean(pbytes, axis=0), args.workload)
    if mlp_info is not None:
        # the same run with births from the birth density itself, same budget
        from paper_1503_03769_amd.runs import run_ospa
        d, _ = run_ospa(dict(p, birth_proposal=0), prec, w["cap"], w["max_meas"], truth, Z, seed, args.run,
                        steps=total)
        mlp_info["ospa_mean_uniform_birth"] = float(np.mean(d[args.warmup:total]))
        line["learned_proposal"] = mlp_info
    if args.cpu_seconds > 0:
        # with the learned proposal the oracle runs the trained network in FP64
        theta = net.get_params().astype(np.float64) if mlp_info is not None else None
        line["cpu_baseline"] = cpu_baseline(p, w, truth, Z, seed, args.run, args.cpu_seconds, theta)
    print(json.dumps(line), flush=True)


ROOF_CLASSES = ("cz", "weight", "birth_order", "rs_expand")
ROOF_KERNELS = {"cz": "k_cz_frames", "weight": "k_weight_frames", "birth_order": "k_birth_draw_sort",
                "rs_expand": "k_rs_expand"}


def roofline(pphd, kern, bytes_per_launch, workload):
    """The longest of the per-particle kernels (the two likelihood passes, the
    births' launch that also predicts the survivors, the resampling expansion
    that also exchanges) against HBM bandwidth: algorithmic bytes per launch
    over its average duration.  The passes skip, per tile, the measurements
    whose terms are exactly zero, so their floor too is moving their
    particles' data.  Every class's figures are listed under "kernels"."""
    rows = {}
    for i, c in enumerate(ROOF_CLASSES):
        if c not in kern or not kern[c][1]:
            continue
        if c == "birth_order" and kern.get("predict", (0, 0))[1]:
            continue  # the prediction had a launch of its own: these bytes do not describe that launch
        ms, n = kern[c]
        avg_s = ms / 1e3 / n
        B = float(bytes_per_launch[i])
        rows[c] = (avg_s, B)
    dom = max(rows, key=lambda c: rows[c][0])
    avg_s, B = rows[dom]
    achieved = B / avg_s / 1e9
    return {
        "kernel": ROOF_KERNELS[dom],
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": stored_traffic(dom, workload),
        "avg_launch_us": avg_s * 1e6,
        "bytes_per_launch": B,
        "others": {ROOF_KERNELS[c]: {"avg_launch_us": a * 1e6, "bytes_per_launch": b, "GB_s": b / a / 1e9,
                                     "frac": b / a / 1e9 / HBM_PEAK_GBS, "traffic": stored_traffic(c, workload)}
                   for c, (a, b) in rows.items() if c != dom},
    }


def bench_batch(args, w):
    """Independent runs in one batch: every step is one replay of the captured
    HIP graph (all stages of all runs); the runs' measurement sets sit in HBM
    and are copied into the graph's input buffers on the stream."""
    import torch

    from paper_1503_03769_amd import pphd
    from paper_1503_03769_amd.metrics import ospa, positions
    from paper_1503_03769_amd.scenario import make_scenario, workload_runs, workload_seed

    p = w["model"]
    prec = pphd.PPHD_FP32 if w["precision"] == "fp32" else pphd.PPHD_FP64
    total = args.warmup + args.steps
    seed = workload_seed(w["config_index"], args.run)
    runs, targets = workload_runs(w, seed)
    R, Mx, cap = len(runs), w["max_meas"], w["cap"]
    scen = [make_scenario(dict(p, clutter_rate=r["clutter_rate"]), targets[i], total, seed + 7919 * (i + 1),
                          turn_sigma=w.get("turn_sigma", 0.0))
            for i, r in enumerate(runs)]
    net, mlp_info = None, None
    if int(p.get("birth_proposal", 0)) == 2:
        from paper_1503_03769_amd.proposal import train_proposal
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net, losses = train_proposal(p, seed=1)
        torch.cuda.synchronize()
        mlp_info = {"train_s": time.perf_counter() - t0, "train_steps": int(len(losses)),
                    "final_loss": float(np.mean(losses[-50:])), "pairs": 1 << 20}

    def make_batch(tuned=True):
        bb = pphd.Batch(p, runs, prec, cap, Mx, seed, apply_tuning=tuned)
        if net is not None:
            bb.attach_mlp(net)
        return bb
    packs = [pphd.Batch.pack([scen[i][1][k] for i in range(R)]) for k in range(total + 1)]
    Ms = np.array([[scen[i][1][k].shape[0] for i in range(R)] for k in range(total + 1)])
    assert Ms.max() <= Mx
    zdev = [torch.from_numpy(z).cuda() for z, _ in packs]
    wdev = [torch.from_numpy(win).cuda() for _, win in packs]
    dz = torch.zeros((R * Mx, 2), dtype=torch.float64, device="cuda")
    dwin = torch.zeros((R, 2), dtype=torch.int32, device="cuda")
    dout = torch.zeros((R * Mx * 40,), dtype=torch.uint8, device="cuda")
    dn = torch.zeros(R, dtype=torch.int32, device="cuda")

    def fill(k):
        n = zdev[k].shape[0]
        if n:
            dz[:n].copy_(zdev[k])
        dwin.copy_(wdev[k])

    # ---- pass A: timed graph replays ----------------------------------------
    def replayed(tuned=True):
        bb = make_batch(tuned)
        bb.init()
        bb.capture(dz, R * Mx, dwin, dout, Mx, dn, 1)
        for k in range(1, args.warmup + 1):
            fill(k)
            bb.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.warmup + 1, total + 1):
            fill(k)
            bb.launch()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        shape = bb.tuning
        bb.close()
        return el, shape

    elapsed, shape = replayed()
    # the same replays with the library's default launch shape
    elapsed_default = replayed(tuned=False)[0] if shape and not args.no_variants else None

    kern, pairs, parts, ospas, pbytes = {}, [], [], [], []
    esz = 4 if prec == pphd.PPHD_FP32 else 8
    group_run = np.repeat(np.arange(R), [int(r["partitions"]) for r in runs])  # run of every group
    group_births = np.concatenate([[int(r["births_per_step"]) // int(r["partitions"])
                                    + (1 if j < int(r["births_per_step"]) % int(r["partitions"]) else 0)
                                    for j in range(int(r["partitions"]))] for r in runs])
    # ---- pass B: eager batch, per-kernel HIP-event times, counts, estimates --
    g = make_batch()
    g.init()
    pairs, parts = [], []
    est_hist = torch.zeros((total + 1, R * Mx * 40), dtype=torch.uint8, device="cuda")
    n_hist = torch.zeros((total + 1, R), dtype=torch.int32, device="cuda")
    for k in range(1, total + 1):
        if k == args.warmup + 1 and not args.no_timing_pass:
            g.set_timing(True)
        g.predict(k)
        g.update_device(zdev[k], zdev[k].shape[0], wdev[k])
        if k > args.warmup:
            n = g.read_counts()
            pairs.append(int(np.dot(n, Ms[k][group_run])))
            parts.append(int(n.sum()))
            pbytes.append(pass_bytes(n, Ms[k][group_run], esz) + step_bytes(n, group_births, esz, int(p.get("dim", 4))))
        g.extract_device(est_hist[k], n_hist[k], Mx)
        g.resample(k)
        g.exchange(k)
    kern = g.read_timing() if not args.no_timing_pass else {}
    g.close()
    del g
    nh = n_hist.cpu().numpy()
    eh = est_hist.cpu().numpy()
    for k in range(args.warmup + 1, total + 1):
        for r in range(R):
            recs = np.frombuffer(eh[k, r * Mx * 40:(r * Mx + min(int(nh[k, r]), Mx)) * 40].tobytes(),
                                 dtype=pphd.ESTIMATE_DTYPE)
            ospas.append(ospa(positions(recs["state"]), positions(scen[r][0][k])))

    # ---- pass C: the same runs as separate filters, one after another, over
    # the same steps (the timed window is the same as pass A's) ---------------
    singles = []
    for r in (runs if not args.no_sequential else []):
        q = dict(p, partitions=r["partitions"], births_per_step=r["births_per_step"],
                 clutter_rate=r["clutter_rate"], particles_per_target=r["particles_per_target"])
        f = pphd.Filter(q, prec, cap, Mx, seed, r["run_id"])
        if net is not None:
            f.attach_mlp(net)
        singles.append(f)
    zsets = [[torch.from_numpy(np.ascontiguousarray(scen[i][1][k])).cuda() for k in range(total + 1)]
             for i in range(R)] if singles else []
    one = torch.zeros(Mx * 40, dtype=torch.uint8, device="cuda")
    n1 = torch.zeros(1, dtype=torch.int32, device="cuda")

    def seq_step(k):
        for i, f in enumerate(singles):
            f.predict(k)
            f.update(zsets[i][k])
            f.extract_device(one, n1, Mx)
            f.resample(k)
            f.exchange(k)

    seq_ms = None
    if singles:
        for f in singles:
            f.init()
        for k in range(1, args.warmup + 1):
            seq_step(k)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(args.warmup + 1, total + 1):
            seq_step(k)
        torch.cuda.synchronize()
        seq_ms = (time.perf_counter() - t1) * 1e3 / args.steps
    for f in singles:
        f.close()

    ms_per_step = elapsed * 1e3 / args.steps
    value = float(sum(pairs)) / elapsed
    line = {
        "metric": "particle x measurement updates/sec (also filter steps/sec and OSPA) at 1 GPU",
        "value": value,
        "unit": "pair-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "steps_per_s": 1e3 / ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == pphd.PPHD_FP32 else "f64",
        "data": "synthetic (seeded truth tracks, detections and Poisson clutter per run)",
        "timed": "the captured step replayed once per step, inputs copied into its buffers on the stream",
        "config": {
            "workload": args.workload,
            "runs": R,
            "state_dim": int(p.get("dim", 4)),
            "groups_per_run": sorted({int(r["partitions"]) for r in runs}),
            "clutter_rates": [float(min(r["clutter_rate"] for r in runs)), float(max(r["clutter_rate"] for r in runs))],
            "targets": [int(min(targets)), int(max(targets))],
            "birth_proposal": int(p.get("birth_proposal", 0)),
            "mean_particles_per_run": float(np.mean(parts)) / R,
            "mean_measurements_per_run": float(Ms[args.warmup + 1:].mean()),
            "launch": "one HIP-graph replay per step (every stage of every run)",
        },
        "ospa_mean": float(np.mean(ospas)),
        "ospa_params": {"p": 1, "c": 100.0},
        "tuning": tuning_record(pphd, shape, elapsed, elapsed_default, args.steps, True, prec,
                                sum(int(r["partitions"]) for r in runs), cap,
                                float(np.mean([r["clutter_rate"] for r in runs])) + 10.0),
        "sequential_single_filters_ms_per_step": seq_ms,
        "speedup_vs_sequential": seq_ms / ms_per_step if seq_ms else None,
    }
    if kern:
        per = {name: {"avg_us": 1e3 * ms / max(n, 1), "launches": n} for name, (ms, n) in kern.items() if n}
        line["kernels"] = per
        line["roofline"] = roofline(pphd, kern, np.mean(pbytes, axis=0), args.workload)
    if mlp_info is not None:
        line["learned_proposal"] = mlp_info
    if args.cpu_seconds > 0:
        r = runs[0]
        # a run with many groups is sampled as 4 of its groups (same particles
        # and births per group) so that one oracle step fits the time budget
        Ks = min(int(r["partitions"]), 4)
        f = Ks / float(r["partitions"])
        q = dict(p, partitions=Ks, births_per_step=int(round(r["births_per_step"] * f)),
                 clutter_rate=r["clutter_rate"], particles_per_target=r["particles_per_target"] * f)
        theta = net.get_params().astype(np.float64) if net is not None else None
        cb = cpu_baseline(q, dict(w, cap=cap), scen[0][0], scen[0][1], seed, r["run_id"], args.cpu_seconds, theta)
        what = "run 0 of the batch" if Ks == r["partitions"] else \
            f"{Ks} of the {r['partitions']} groups of run 0 (same particles and births per group)"
        cb["sample"] = what + " from t = 0, " + cb["sample"].split(", ", 1)[-1]
        line["cpu_baseline"] = cb
    return line


def tuning_record(pphd, shape, elapsed, elapsed_default, steps, batch, prec, groups, cap, meas):
    """The autotuned launch shape the run used (pphd.lookup_tuning: its
    bucket, else the nearest of the same kind) and the measured gain over the
    library's default shape on the same steps."""
    rec = {"bucket": pphd.tuning_bucket(prec, batch, groups, cap, meas), "shape": None, "gain_vs_default": None}
    if shape:
        rec["shape"] = {k: shape[k] for k in ("pt_cz", "pt_weight", "pass_workgroups", "rs_tiles", "meas_per_wave")
                        if k in shape}
        rec["tuned_on"] = shape.get("workload")
        if elapsed_default:
            rec["ms_per_step_default_shape"] = elapsed_default * 1e3 / steps
            rec["gain_vs_default"] = elapsed_default / elapsed
    return rec


def host_cpu():
    """The host's CPU model name (with the family, model and stepping numbers
    /proc/cpuinfo gives, since a virtual machine may shorten the name),
    logical CPU count and the CPUs this process may run on."""
    model = "unknown"
    ids = {}
    try:
        for ln in open("/proc/cpuinfo"):
            key = ln.split(":", 1)[0].strip()
            if key == "model name" and model == "unknown":
                model = ln.split(":", 1)[1].strip()
            elif key in ("cpu family", "model", "stepping") and key not in ids:
                ids[key] = ln.split(":", 1)[1].strip()
            elif not ln.strip() and model != "unknown":
                break
    except OSError:
        pass
    if ids:
        model += " (family " + ids.get("cpu family", "?") + ", model " + ids.get("model", "?") + \
            ", stepping " + ids.get("stepping", "?") + ")"
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def oracle_sample(p, w, Z, seed, run, budget_s, threads, mlp_theta=None):
    """The FP64 oracle on the same run from t = 0 for as many steps as fit in
    about budget_s seconds, with its per-group loops on `threads` threads."""
    import oracle as orc
    orc.set_threads(threads)
    o = orc.OracleFilter(p, w["cap"], seed, run, mlp_theta=mlp_theta)
    pairs = 0
    steps = 0
    t0 = time.perf_counter()
    for k in range(1, len(Z)):
        out = o.step(k, Z[k])
        pairs += int(out["n_pred"].sum()) * Z[k].shape[0]
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return pairs / el, steps / el, steps


def cpu_baseline(p, w, truth, Z, seed, run, budget_s, mlp_theta=None):
    """The FP64 oracle as it stands (plain C, one group per OpenMP thread) on
    the host: on every CPU this process may use (the reported value), and on
    one thread, each for about half of budget_s."""
    model, nproc, usable = host_cpu()
    v_all, s_all, n_all = oracle_sample(p, w, Z, seed, run, 0.5 * budget_s, usable, mlp_theta)
    v_one, s_one, n_one = oracle_sample(p, w, Z, seed, run, 0.5 * budget_s, 1, mlp_theta)
    return {"value": v_all, "unit": "pair-updates/s", "cores": usable, "kind": "oracle",
            "sample": f"first {n_all} steps of the same run (seed {seed}), FP64 C oracle, its groups on "
                      f"{usable} threads",
            "steps_per_s": s_all, "cpu": model, "nproc": nproc, "usable_cpus": usable,
            "single_thread": {"value": v_one, "steps_per_s": s_one, "steps": n_one, "cores": 1}}


if __name__ == "__main__":
    main()
