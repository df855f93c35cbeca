"""Benchmark of the hot path: batched evaluation of an anchored cut-HDMR
expansion with adaptive sparse-grid components (the metric workload: d=100,
100 one-dimensional + 500 two-dimensional components, adaptive grids to level
8 with eps_gamma = 1e-4, m = 51 outputs, 4e6 next-state points).

One step = one hdmr_eval over all points, inputs resident in HBM.  Prints one
JSON line (see the keys below).  The model is built on the device with
asg_build_components from the seeded synthetic test function (untimed).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision plain|mixed]
                  [--no-cpu-baseline] [--points N]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK = 78.6e12     # MI355X FP64 vector FLOP/s (public spec)
HBM_PEAK = 8.0e12       # MI355X HBM3E bytes/s (public spec)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["plain", "mixed"], default="plain")
    ap.add_argument("--points", type=int, default=None)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the evaluation shards by points with no exchange, "
              "so --gpus N > 1 is not run in this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2202_06555_amd as hd
    import workloads.synth as ws

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    hd.hdmr_init(0)
    cfg = ws.config(args.config)
    n = cfg["n"] if args.points is None else args.points
    tf = ws.test_function_for(cfg)
    t0 = time.time()
    model = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"],
                                    max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    info = hd.hdmr_get_info(model)
    log("built model on device in %.1f s: %d components, %d rows, %.2f GB" %
        (time.time() - t0, info["n_components"], info["n_rows"], info["device_bytes"] / 1e9))
    X = torch.from_numpy(ws.points_for(cfg, n=n)).to(dev)
    m, d = cfg["m"], cfg["d"]
    Y = torch.empty((n, m), dtype=torch.float64, device=dev)
    prec = hd.PLAIN_FP64 if args.precision == "plain" else hd.MIXED
    hits, probes = hd.hdmr_eval_stats(model, X)
    log("nonzero basis products per point %.1f, lookups per point %.1f" % (hits / n, probes / n))
    for _ in range(args.warmup):
        hd.hdmr_eval(model, X, Y, precision=prec)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        hd.hdmr_eval(model, X, Y, precision=prec)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1) / args.steps
    t = ms / 1e3
    value = n * m / t
    flops = 2.0 * hits * m + n * m           # FMA per (nonzero, output) + anchor add
    achieved = flops / t
    out = {
        "metric": "HDMR-ASG point x output evals/sec at d=100, m=51 (%s)" %
                  ("plain FP64" if prec == hd.PLAIN_FP64 else "mixed"),
        "value": value,
        "unit": "point*outputs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == hd.PLAIN_FP64 else "f32/bf16x3/f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: d=%d, %d components (%d one-dim + %d two-dim), adaptive sparse grids max level %d "
                        "eps_gamma=%g, m=%d, %d next-state points" %
                        (args.config, d, info["n_components"], d, info["n_components"] - d, cfg["max_level"],
                         cfg["eps_gamma"], m, n),
            "grid_rows": info["n_rows"],
            "nonzeros_per_point": hits / n,
            "lookups_per_point": probes / n,
            "parallelism": "single GPU (points)",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": FP64_PEAK / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK,
            "traffic": None,
            "kernel": "k_pass_mfma (cell-sorted FP64 MFMA contraction, one launch per 32 outputs per pass)"
                      if prec == hd.PLAIN_FP64 else "mixed",
            "algorithmic_flops_per_launch": flops,
            "algorithmic_hbm_bytes_per_launch": float(n * d * 8 + n * m * 8 + info["device_bytes"]),
        },
        "wall_s_timed_region": wall,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample, ws)
        out["cpu_baseline"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


def cpu_baseline(cfg, sample, ws):
    """The FP64 oracle (C, OpenMP over points, level-wise mode) on its own build
    of the same workload, timed on this host's cores on a bounded sample."""
    import numpy as np

    import oracle
    tf = ws.test_function_for(cfg)
    t0 = time.time()
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user),
                                  max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    log("oracle build %.1f s" % (time.time() - t0))
    X = ws.points_for(cfg, n=sample)
    oracle.evaluate(model, X[:64])
    t0 = time.perf_counter()
    oracle.evaluate(model, X)
    t = time.perf_counter() - t0
    log("oracle eval of %d points: %.2f s" % (sample, t))
    return {"value": sample * cfg["m"] / t, "unit": "point*outputs/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d of the %d next-state points (seed %d), level-wise FP64 oracle with compensated sums"
                      % (sample, cfg["n"], cfg["seed"])}


if __name__ == "__main__":
    main()
