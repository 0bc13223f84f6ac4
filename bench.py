"""Benchmark: the simplification solver's hot path on one MI355X.

Workload: the 256^3 filament field (32 random tubes + N(0, 0.02^2) noise,
seed 0); non-signal pairs are the saddle-saddle pairs with persistence below
0.1 * range, every other pair is signal.

A step is one solver iteration (Alg. 1): gradient step, persistence map
(order, lower-star gradient, critical cells, the three pairings, diagram),
still-pair join and exact assignment.  The timed region runs `--steps`
iterations from the input field with the field already resident in HBM
(one ts_simplify call with j_max = steps; the initial diagram is inside
the timed region).  value = vertices * steps / time (Mverts/s).

Also reported: the persistence-map throughput (vertices / device time of
the persistence kernels per map), the per-stage device times (HIP events on
the library's stream), the roofline of the dominant kernel, and the CPU
oracle timed on a bounded crop of the same field.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--cancel] [--paper-stop] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "filament_256"

# Algorithmic HBM bytes per vertex of each persistence-map stage (per launch
# = per map): what the stage must read and write at minimum.
ALGO_BYTES_PER_VERTEX = {
    "K1 order keys": 4 + 8,      # read f, write (key, id)
    "K1 radix sort": 8 + 8,      # read (key, id), write sorted (key, id)
    "K2 rank": 4 + 8,            # read sorted id, write rank and order
    "K3 gradient": 4 + 16 + 4,   # read rank, write 16-byte code and descending neighbour
}


# HBM traffic of one k_gradient launch at 256^3, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (KiB per dispatch), each scaled by what the same counter
# reads for a plain 256 MiB device copy (fetch x2.0, write x1.0).  It belongs
# to the kernel source it was measured on: a changed kernel reports null.
K3_COUNTERS = {"source_sha1": "bc8c6567d936d94f39c2c5d8425661550676767c",
               "dims": (256, 256, 256), "fetch_kib": 98221.3, "write_kib": 404298.2,
               "fetch_scale": 2.0, "write_scale": 1.0}


# SQ_INSTS_VALU / SQ_WAVES of K3 from the instruction-mix pass recorded in
# profiles/k3_gradient_filament256_instruction_mix.md (same kernel source)
K3_VALU_PER_WAVE = {"source_sha1": "bc8c6567d936d94f39c2c5d8425661550676767c", "valu": 19138.0}
# untimed persistence maps before timing: the launch tuner tries 5 D1 block sizes
WARM_MAPS = 6
# one wave64 VALU instruction per CU per cycle (4 SIMDs x 16 lanes), 256 CUs at 2.4 GHz
VALU_ISSUE_PEAK_G = 256 * 2.4


def kernel_source_sha1(name="k_gradient"):
    """sha1 of a kernel's definition text in persistence.hip."""
    import hashlib
    path = os.path.join(ROOT, "paper_2407_12399_amd", "csrc", "persistence.hip")
    s = open(path).read()
    i = s.index("\n" + name + "(")
    i = s.rindex("\n", 0, i - 1) + 1
    j = s.index("\n}\n", i) + 3
    return hashlib.sha1(s[i:j].encode()).hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--dims", type=int, nargs=3, default=None)
    ap.add_argument("--cancel", action="store_true",
                    help="also run the solver to full cancellation (or j_max)")
    ap.add_argument("--paper-stop", action="store_true",
                    help="also time the solve to the paper's stop rule L <= 0.01 L0")
    ap.add_argument("--j-max", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-paper-auction", action="store_true",
                    help="skip the extra run with the paper's auction precision")
    ap.add_argument("--cpu-crop", type=int, default=48)
    ap.add_argument("--diag-reps", type=int, default=3)
    ap.add_argument("--diagram-only", action="store_true",
                    help="only run the persistence map --diag-reps times (for profilers)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch of 64 uneven fields")
    ap.add_argument("--batch-only", action="store_true",
                    help="only run the batched persistence map --diag-reps times (for profilers)")
    ap.add_argument("--warm-start", action="store_true",
                    help="also train the warm-start network (512 solver runs at 64^3) and "
                         "compare warm and cold solves on held-out 128^3 fields (minutes)")
    ap.add_argument("--warm-start-only", action="store_true",
                    help="only the warm-start measurement")
    ap.add_argument("--unet-only", action="store_true",
                    help="only time the warm-start network's forward pass and training step at 64^3")
    ap.add_argument("--ws-examples", type=int, default=512)
    ap.add_argument("--ws-steps", type=int, default=3000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 3 times (HBM counter calibration)")
    return ap.parse_args()


def cpu_baseline(f, crop, signal):
    """The oracle on a crop of the field: per-iteration time of its solver
    (two iterations minus the initial diagram), single-threaded."""
    import oracle
    oracle.build()
    c = np.ascontiguousarray(f[:crop, :crop, :crop])
    thr, mask, ties = signal
    dims = [d for d in range(3) if (mask >> d) & 1]
    t0 = time.perf_counter()
    oracle.simplify(c, threshold=thr, nonsignal_dims=dims, ties_signal=ties, j_max=0)
    t1 = time.perf_counter()
    _, rep = oracle.simplify(c, threshold=thr, nonsignal_dims=dims, ties_signal=ties, j_max=2)
    t2 = time.perf_counter()
    iters = max(rep.iterations, 1)
    per_iter = max((t2 - t1) - (t1 - t0), 1e-9) / iters
    return {"value": c.size / per_iter / 1e6, "unit": "Mverts/s", "cores": 1, "kind": "oracle",
            "sample": f"{crop}^3 crop of the same field, {iters} solver iterations "
                      f"(time of 2 iterations minus the initial diagram)",
            "persistence_map_mverts_s": c.size / (t1 - t0) / 1e6}


def batch_run(ts, fields, torch, args):
    """64 Gaussian-mixture fields with axes drawn from 24..96: the batched
    persistence map and solver steps against the same work field by field."""
    print("[bench] batch of 64 uneven fields", file=sys.stderr, flush=True)
    fb = [torch.from_numpy(x).cuda() for x in fields.uneven_batch(seed=args.seed)]
    nv = sum(int(x.numel()) for x in fb)

    def timed(fn, reps):
        ts_ = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts_.append(time.perf_counter() - t0)
        return float(np.median(ts_))

    for _ in range(WARM_MAPS):  # warm-up, including the launch tuner's trials
        ts.diagram_batch(fb)
    for x in fb:
        ts.diagram(x)
    stage = {}
    walls = []
    for _ in range(args.diag_reps):
        walls.append(timed(lambda: ts.diagram_batch(fb), 1))
        for k, v in ts.stage_times().items():
            stage.setdefault(k, []).append(v)
    dev_ms = sum(float(np.median(v)) for v in stage.values())
    seq = timed(lambda: [ts.diagram(x) for x in fb], 1)
    steps = args.steps
    tb = timed(lambda: ts.simplify_batch(fb, threshold=0.1, j_max=steps), 1)
    tsq = timed(lambda: [ts.simplify(x, threshold=0.1, j_max=steps) for x in fb], 1)
    return {"workload": "64 fields, 8 Gaussians + U[-0.05,0.05] noise, axes drawn from 24..96",
            "vertices": nv,
            "persistence_map_mverts_s": nv / (dev_ms * 1e-3) / 1e6,
            "persistence_map_ms": dev_ms,
            "diagram_batch_wall_s": float(np.median(walls)),
            "diagram_one_by_one_wall_s": seq,
            "solver_steps": steps,
            "simplify_batch_wall_s": tb, "simplify_one_by_one_wall_s": tsq,
            "solver_mverts_s": nv * steps / tb / 1e6}


def unet_run(ts, torch, reps=10):
    """Forward pass and training step (forward, backward, Adam) of the
    warm-start network on one 64^3 volume; achieved BF16 MFMA rate of the
    convolutions (2 * voxels * 27 * Cin * Cout per convolution, Cin as stored;
    a training step counts the forward, the weight gradient and the data
    gradient of every layer but the first)."""
    from paper_2407_12399_amd import warmstart
    D = 64
    rng = np.random.default_rng(0)
    inp = torch.from_numpy(np.stack([rng.random((D, D, D)), rng.random((D, D, D)) < 0.1], -1)
                           .astype(np.float32)).cuda()
    tgt = torch.from_numpy(rng.normal(0, 0.01, (D, D, D)).astype(np.float32)).cuda()
    p = warmstart.init_params(0)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    vox = [D ** 3, D ** 3, (D // 2) ** 3, (D // 2) ** 3, (D // 4) ** 3, (D // 4) ** 3,
           (D // 2) ** 3, (D // 2) ** 3, D ** 3, D ** 3]
    fl = [2.0 * n * 27 * ci * co for n, (ci, co) in zip(vox, warmstart.LAYERS)]
    fwd_flops = sum(fl)
    step_flops = fwd_flops + sum(fl) + sum(fl[1:])
    for k in range(3):
        ts.unet_forward(p, inp)
        _, g = ts.unet_grad(p, inp, tgt)
        ts.unet_adam(p, g, m, v, k + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ts.unet_forward(p, inp)
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for k in range(reps):
        _, g = ts.unet_grad(p, inp, tgt)
        ts.unet_adam(p, g, m, v, k + 4)
    torch.cuda.synchronize()
    tt = (time.perf_counter() - t0) / reps
    return {"volume": [D, D, D], "forward_ms": tf * 1e3, "train_step_ms": tt * 1e3,
            "forward_conv_gflop": fwd_flops / 1e9, "train_step_conv_gflop": step_flops / 1e9,
            "forward_tflop_s": fwd_flops / tf / 1e12, "train_step_tflop_s": step_flops / tt / 1e12,
            "peak_tflop_s": 2500.0, "forward_frac": fwd_flops / tf / 1e12 / 2500.0,
            "timing": "wall time around whole passes (host round trips included)"}


def warm_start_run(ts, torch, args):
    """Training of the warm-start network on plain-solver results (8 Gaussians
    + U[-0.05,0.05] noise at 64^3, seeds 0..), then cold and warm solves of
    held-out 128^3 fields (seeds 20000..) at the same stop rule."""
    from paper_2407_12399_amd import fields, warmstart

    def log(m):
        print(f"[bench] warm start: {m}", file=sys.stderr, flush=True)

    kw = dict(stop_mode=1, loss_ratio_s=1e-4, j_max=300)
    t0 = time.perf_counter()
    X, Y = warmstart.make_examples(args.ws_examples, dims=(64, 64, 64), seed0=0, log=log, **kw)
    data_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    p, hist = warmstart.train(X, Y, args.ws_steps, lr=1e-3, log=log, log_every=500)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    target_ms = float(Y.pow(2).mean())
    del X, Y
    evals = []
    for sd in (20000, 20001, 20002):
        f = torch.from_numpy(fields.gaussian_mixture((128, 128, 128), 8, 0.05, sd)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rc = ts.simplify(f, threshold=0.1, **kw)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, rw, tp = warmstart.warm_solve(p, f, **kw)
        torch.cuda.synchronize()
        tw = time.perf_counter() - t0
        evals.append({"seed": sd, "cold_iterations": rc.iterations, "cold_s": tc,
                      "warm_iterations": rw.iterations, "warm_s": tw, "proposal_s": tp,
                      "start_used": rw.init_used, "stopped": [rc.cancelled, rw.cancelled]})
        log(json.dumps(evals[-1]))
    return {"examples": args.ws_examples, "example_dims": [64, 64, 64], "train_steps": args.ws_steps,
            "stop_rule": "loss <= 1e-4 * loss at f0", "data_s": data_s, "train_s": train_s,
            "train_loss_first": hist[0][1], "train_loss_last": hist[-1][1],
            "target_mean_square": target_ms, "eval_128": evals}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    import torch

    import paper_2407_12399_amd as ts
    from paper_2407_12399_amd import fields

    torch.cuda.set_device(0)
    if args.copy_probe:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 3}))
        return
    if args.unet_only:
        print(json.dumps({"unet": unet_run(ts, torch)}))
        return
    if args.warm_start_only:
        print(json.dumps({"warm_start": warm_start_run(ts, torch, args)}))
        return
    if args.batch_only:
        fb = [torch.from_numpy(x).cuda() for x in fields.uneven_batch(seed=args.seed)]
        for _ in range(args.diag_reps + WARM_MAPS):
            ts.diagram_batch(fb)
        torch.cuda.synchronize()
        print(json.dumps({"batch_maps": args.diag_reps + WARM_MAPS}))
        return
    w = fields.WORKLOADS[WORKLOAD]
    dims = tuple(args.dims) if args.dims else w["dims"]
    print(f"[bench] generating {WORKLOAD} {dims} seed {args.seed}", file=sys.stderr, flush=True)
    f = fields.workload(WORKLOAD, args.seed, dims=dims)
    n = f.size
    ft = torch.from_numpy(f).cuda()
    thr, mask, ties = w["signal"]
    sig = dict(threshold=thr, nonsignal_dims=[d for d in range(3) if (mask >> d) & 1],
               ties_signal=ties)
    torch.cuda.synchronize()

    # persistence map alone (device time of the persistence stages per map)
    print("[bench] persistence map", file=sys.stderr, flush=True)
    # warm-up: workspace allocation, table upload, and the launch tuner's trial
    # maps (it tries each D1 block size once, then keeps the fastest)
    for _ in range(WARM_MAPS):
        ts.diagram(ft)
    diag_stage = {}
    wall = []
    for _ in range(args.diag_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        D = ts.diagram(ft)
        torch.cuda.synchronize()
        wall.append(time.perf_counter() - t0)
        for k, v in ts.stage_times().items():
            diag_stage.setdefault(k, []).append(v)
    stage_ms = {k: float(np.median(v)) for k, v in diag_stage.items()}
    if args.diagram_only:
        print(json.dumps({"persistence_map_ms": sum(stage_ms.values()), "stage_ms": stage_ms,
                          "wall_ms": float(np.median(wall)) * 1e3, "pairs": len(D)}))
        return
    pm_ms = sum(stage_ms.values())
    n_pairs = [int((D["dim"] == d).sum() - (D["essential"] if d == 0 else 0).sum())
               if d == 0 else int((D["dim"] == d).sum()) for d in range(3)]

    # solver steps
    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    if args.warmup > 0:
        ts.simplify(ft, j_max=args.warmup, **sig)
    torch.cuda.synchronize()
    print(f"[bench] timed {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    g, rep = ts.simplify(ft, j_max=args.steps, **sig)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps = rep.iterations
    solver_stage = ts.stage_times()
    value = n * steps / dt / 1e6 if steps > 0 else 0.0

    # dominant persistence kernel and its roofline
    dom = max((k for k in stage_ms if k in ALGO_BYTES_PER_VERTEX), key=lambda k: stage_ms[k])
    algo_bytes = ALGO_BYTES_PER_VERTEX[dom] * n
    achieved = algo_bytes / (stage_ms[dom] * 1e-3) / 1e9
    traffic = None
    c = K3_COUNTERS
    if dom == "K3 gradient" and tuple(dims) == c["dims"] and kernel_source_sha1() == c["source_sha1"]:
        traffic = (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "algo_bytes_per_launch": algo_bytes, "avg_launch_ms": stage_ms[dom]}
    # algorithmic HBM rate of every streaming stage (order and gradient)
    stage_hbm = {k: {"algo_bytes_per_vertex": ALGO_BYTES_PER_VERTEX[k], "ms": stage_ms[k],
                     "achieved_gbs": ALGO_BYTES_PER_VERTEX[k] * n / (stage_ms[k] * 1e-3) / 1e9,
                     "frac": ALGO_BYTES_PER_VERTEX[k] * n / (stage_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                 for k in ALGO_BYTES_PER_VERTEX if stage_ms.get(k)}
    order_keys = [k for k in ("K1 order keys", "K1 radix sort", "K2 rank") if stage_ms.get(k)]
    order_ms = sum(stage_ms[k] for k in order_keys)
    order_bytes = sum(ALGO_BYTES_PER_VERTEX[k] for k in order_keys) * n
    stage_hbm["vertex order (K1 + K2)"] = {
        "algo_bytes_per_vertex": order_bytes / n, "ms": order_ms,
        "achieved_gbs": order_bytes / (order_ms * 1e-3) / 1e9,
        "frac": order_bytes / (order_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    k3_issue = None
    if dom == "K3 gradient" and kernel_source_sha1() == K3_VALU_PER_WAVE["source_sha1"]:
        rate = n / 64 * K3_VALU_PER_WAVE["valu"] / (stage_ms[dom] * 1e-3) / 1e9
        k3_issue = {"bound": "alu", "kernel": dom, "achieved": rate, "peak": VALU_ISSUE_PEAK_G,
                    "unit": "G wave-level VALU instructions/s", "frac": rate / VALU_ISSUE_PEAK_G,
                    "valu_per_wave": K3_VALU_PER_WAVE["valu"]}
    out = {
        "metric": "time to full non-signal cancellation (s) + persistence-map Mverts/s at 256^3",
        "value": value, "unit": "Mverts/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": dt / max(steps, 1) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "dims": list(dims), "seed": args.seed,
                   "signal": "non-signal = saddle-saddle pairs with persistence < 0.1 range",
                   "step": "one solver iteration (update + persistence map + assignment)"},
        "persistence_map_mverts_s": n / (pm_ms * 1e-3) / 1e6,
        "persistence_map_ms": pm_ms,
        "persistence_map_wall_ms": float(np.median(wall)) * 1e3,
        "diagram_pairs": {"d0": n_pairs[0], "d1": n_pairs[1], "d2": n_pairs[2]},
        "stage_ms": stage_ms,
        "solver": {"iterations": steps, "loss0": rep.loss0, "loss": rep.loss,
                   "max_nonsignal_pers_rel": rep.max_nonsignal_pers / rep.range,
                   "persistence_s": rep.persistence_s, "assign_s": rep.assign_s,
                   "update_s": rep.update_s, "n_reduced_last": rep.n_reduced,
                   "regradient_frac": rep.n_regradient / (n * max(steps, 1)),
                   "n_still_last": rep.n_still, "n_targets": rep.n_targets,
                   "stage_ms_total": solver_stage},
        "roofline": roofline,
        "k3_issue": k3_issue,
        "stage_hbm": stage_hbm,
        # the map's largest stage by device time; it is latency-bound (rounds of
        # dependent column additions), so it has no byte or flop roofline
        "map_dominant_stage": {"stage": max(stage_ms, key=stage_ms.get),
                               "ms": max(stage_ms.values()),
                               "share": max(stage_ms.values()) / pm_ms},
    }
    # the paper's assignment setting (auction at relative precision 0.01)
    if not args.no_paper_auction:
        print(f"[bench] {args.steps} steps with the paper's auction precision", file=sys.stderr,
              flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rp = ts.simplify(ft, j_max=args.steps, assign_precision=0.01, **sig)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        out["paper_auction_precision_0_01"] = {
            "value": n * rp.iterations / dtp / 1e6 if rp.iterations else 0.0,
            "unit": "Mverts/s", "ms_per_step": dtp / max(rp.iterations, 1) * 1e3,
            "assign_s": rp.assign_s, "loss": rp.loss,
            "note": "assignment by an auction stopped at relative precision 0.01 (the paper's "
                    "setting); not parity with the exact oracle"}
    if args.paper_stop:
        print(f"[bench] solve to the paper's stop rule (j_max {args.j_max})", file=sys.stderr,
              flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rs = ts.simplify(ft, j_max=args.j_max, stop_mode=1, loss_ratio_s=0.01, **sig)
        torch.cuda.synchronize()
        out["paper_stop_run"] = {"wall_s": time.perf_counter() - t0, "iterations": rs.iterations,
                                 "stopped": rs.cancelled, "loss0": rs.loss0, "loss": rs.loss,
                                 "persistence_s": rs.persistence_s, "assign_s": rs.assign_s,
                                 "regradient_frac":
                                     rs.n_regradient / (n * max(rs.iterations, 1))}
    if args.cancel:
        print(f"[bench] full solve (j_max {args.j_max})", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g, rc = ts.simplify(ft, j_max=args.j_max, **sig)
        torch.cuda.synchronize()
        out["time_to_cancel_s"] = time.perf_counter() - t0 if rc.cancelled else None
        out["cancel_run"] = {"iterations": rc.iterations, "cancelled": rc.cancelled,
                             "wall_s": time.perf_counter() - t0,
                             "max_nonsignal_pers_rel": rc.max_nonsignal_pers / rc.range,
                             "linf": rc.linf, "max_signal_disp": rc.max_signal_disp}
    if not args.no_batch:
        out["batch"] = batch_run(ts, fields, torch, args)
    if args.warm_start:
        out["warm_start"] = warm_start_run(ts, torch, args)
    if not args.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(f, args.cpu_crop, w["signal"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
