"""Benchmark of the hot path: batched evaluation of an anchored cut-HDMR
expansion with adaptive sparse-grid components.  Default workload: d=100,
100 one-dimensional + 500 two-dimensional components, adaptive grids to level
8 with eps_gamma = 1e-4, m = 51 outputs, 4e6 next-state points.

One step = one hdmr_eval over all points, inputs resident in HBM; the
default runs the plain FP64 leg (the headline value) and the mixed leg (the
"mixed" object).  Prints one JSON line.  The model is built on the device with asg_build_components from
the seeded synthetic test function (untimed).  The device time of every
evaluation stage is taken live with device events on the launch stream
(hdmr_timing_*); the roofline object prices the dominant kernel, the
matrix-core contraction (one launch per pass), by its algorithmic work:
2 flops per (point, stored row with a nonzero basis product, output), against
the matrix-core peak of its dtype (FP64 for plain, BF16 for mixed).  Also
reported: the problem-level bytes per launch (outputs, points and model once
per evaluation), the bytes this design moves (16 per point and output per
pass for the output read-modify-write), and the HBM traffic measured with
rocprofv3 FETCH_SIZE + WRITE_SIZE (profiles/, copy-calibrated).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision both|plain|mixed]
                  [--no-cpu-baseline] [--points N] [--calibrate-copy]
                  [--workload eval|grad|naive|irbc|batched|surrogate]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK = 78.6e12      # MI355X FP64 matrix FLOP/s
FP64_VECTOR_PEAK = 78.6e12  # 256 CUs x 128 FP64 flops per clock x 2.4 GHz
FP32_PEAK = 157.3e12     # MI355X FP32 vector FLOP/s
BF16_PEAK = 2.5e15       # MI355X dense BF16 matrix FLOP/s
HBM_PEAK = 8.0e12        # MI355X HBM3E bytes/s

KERNEL = {"plain": "k_tile_fp64", "mixed": "k_tile_mixed"}
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _source_hash():
    with open(os.path.join(ROOT, "paper_2202_06555_amd", "csrc", "eval_sorted.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _measured_traffic(kernel, workload):
    """HBM bytes per launch of the contraction kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when
    there is none or the kernel source changed since it was taken."""
    path = os.path.join(PROFILES, "%s_%s_traffic.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not h or not b or h.group(1) != _source_hash():
        return None
    return float(b.group(1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["both", "plain", "mixed"], default="both",
                    help="both: the plain FP64 line with the mixed leg beside it (default)")
    ap.add_argument("--points", type=int, default=None)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device copy first (scale reference for HBM counters)")
    ap.add_argument("--workload", choices=["eval", "batched", "surrogate", "grad", "naive", "irbc"], default="eval",
                    help="eval: the metric workload (default); batched: many models in one call; "
                         "surrogate: the learned part on the d=300 workload; grad: values and gradients "
                         "on the d=20 workload")
    ap.add_argument("--models", type=int, default=64, help="batched: number of models (of the 64-model workload)")
    ap.add_argument("--train-points", type=int, default=2_000_000, help="surrogate: interpolant training pairs")
    ap.add_argument("--epochs", type=int, default=3, help="surrogate: passes over the training pairs")
    ap.add_argument("--serve-points", type=int, default=2_000_000, help="surrogate: points served")
    ap.add_argument("--ti-steps", type=int, default=6, help="irbc: time-iteration steps after the residual timing")
    ap.add_argument("--train-seconds", type=float, default=0.0,
                    help="surrogate: train in one-epoch segments for this long (0: --epochs in one run)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the evaluation shards by points with no exchange, "
              "so --gpus N > 1 is not run here", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "grad":
        return bench_grad(args)
    if args.workload == "naive":
        return bench_naive(args)
    if args.workload == "irbc":
        return bench_irbc(args)

    import torch

    import paper_2202_06555_amd as hd
    import workloads.synth as ws

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    hd.hdmr_init(0)
    cfg = ws.config(args.config)
    n = cfg["n"] if args.points is None else args.points
    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 1 GiB read + 1 GiB written")
    tf = ws.test_function_for(cfg)
    t0 = time.time()
    model = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"],
                                    max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    info = hd.hdmr_get_info(model)
    build_s = time.time() - t0
    log("built model on device in %.1f s: %d components, %d rows, %d passes, %.2f GB" %
        (build_s, info["n_components"], info["n_rows"], info["n_passes"], info["device_bytes"] / 1e9))
    X = torch.from_numpy(ws.points_for(cfg, n=n)).to(dev)
    m, d = cfg["m"], cfg["d"]
    hits, probes = hd.hdmr_eval_stats(model, X)
    log("nonzero basis products per point %.1f, lookups per point %.1f" % (hits / n, probes / n))
    ceil = measured_ceilings()
    legs = {}
    outputs = {}
    precisions = [args.precision] if args.precision != "both" else ["plain", "mixed"]
    for name in precisions:
        prec = hd.PLAIN_FP64 if name == "plain" else hd.MIXED
        Y = torch.empty((n, m), dtype=torch.float64, device=dev)
        legs[name] = run_leg(hd, model, X, Y, prec, name, args, info, hits, n, m, d, ceil)
        outputs[name] = Y
    head = precisions[0]
    L = legs[head]
    out = {
        "metric": "HDMR-ASG point x output evaluations/sec at d=100, m=51",
        "value": L["value"],
        "unit": "point*outputs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": L["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "plain" else "f32 basis, bf16x3 mfma, f64 sum",
        "data": "synthetic",
        "config": {
            "workload": "%s: d=%d, %d components (%d one-dim + %d two-dim), adaptive sparse grids max level %d "
                        "eps_gamma=%g, m=%d, %d next-state points, %s precision" %
                        (args.config, d, info["n_components"], d, info["n_components"] - d, cfg["max_level"],
                         cfg["eps_gamma"], m, n, head),
            "grid_rows": info["n_rows"],
            "build_s_untimed": build_s,
            "nonzeros_per_point": hits / n,
            "lookups_per_point": probes / n,
            "parallelism": "single GPU (points)",
        },
        "roofline": L["roofline"],
        "wall_s_timed_region": L["wall_s"],
    }
    if "mixed" in legs and head != "mixed":
        M_ = legs["mixed"]
        out["mixed"] = {"value": M_["value"], "ms_per_step": M_["ms_per_step"],
                        "speedup_over_plain": L["ms_per_step"] / M_["ms_per_step"],
                        "dtype": "f32 basis, bf16x3 mfma (6 products), f32 partial sums folded into f64 every 16 "
                                 "passes, f64 c0",
                        "roofline": M_["roofline"], "wall_s_timed_region": M_["wall_s"]}
    if not args.no_cpu_baseline:
        cb, sample_idx, ref = cpu_baseline(cfg, args.cpu_sample, ws)
        cb["gpu_over_cpu"] = out["value"] / cb["value"]
        out["cpu_baseline"] = cb
        # error against the oracle on the baseline's sample (its outputs are the reference)
        errs = {}
        for name, Y in outputs.items():
            Ys = Y[torch.from_numpy(sample_idx).to(dev)].cpu().numpy()
            errs[name] = error_report(Ys, ref)
        out["error_vs_oracle"] = {"sample": cb["sample"], **errs}
        out["error_vs_oracle"]["bars"] = {"plain": "max-abs <= 1e-12",
                                          "mixed": "per output max|err|/max|F| <= 1e-6"}
    print(json.dumps(out), flush=True)


def error_report(Y, ref):
    """Max-abs error, worst per-output relative error max_p|err_o| / max_p|F_o|,
    and normwise error of Y against the oracle's values ref."""
    import numpy as np
    err = np.abs(Y - ref)
    per_out = err.max(axis=0) / np.maximum(np.abs(ref).max(axis=0), 1e-300)
    return {"max_abs": float(err.max()), "worst_output_rel": float(per_out.max()),
            "normwise": float(np.linalg.norm(Y - ref) / np.linalg.norm(ref))}


def measured_ceilings():
    """Run the device-ceiling microbenchmarks (paper_2202_06555_amd/bench_ceilings):
    HBM copy, random accumulator-row read-modify-write, FP64/BF16 MFMA, FP64
    VALU, LDS gather.  Returns the parsed lines, or {} if the program is absent."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2202_06555_amd", "bench_ceilings")
    if not os.path.exists(exe):
        return {}
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    res = {"rmw": []}
    for line in r.stdout.splitlines():
        try:
            o = json.loads(line)
        except ValueError:
            continue
        if o.get("probe") == "rmw":
            res["rmw"].append(o)
        else:
            res[o["probe"]] = o
    return res


def run_leg(hd, model, X, Y, prec, name, args, info, hits, n, m, d, ceil):
    """Warm-up, then args.steps timed evaluations; device-event stage timing
    and the roofline of the contraction kernel."""
    import torch
    for _ in range(args.warmup):
        hd.hdmr_eval(model, X, Y, precision=prec)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    hd.hdmr_timing_enable(True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        hd.hdmr_eval(model, X, Y, precision=prec, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    stages = {s: hd.hdmr_timing_read(s) for s in ("sort", "rows", "contract")}
    hd.hdmr_timing_enable(False)
    ms = ev0.elapsed_time(ev1) / args.steps
    value = n * m / (ms / 1e3)
    log("%s: step %.2f ms; per step: sort+rows (second stream, overlapped) %.1f ms, contract %.1f ms" %
        (name, ms, (stages["sort"][0] + stages["rows"][0]) / args.steps, stages["contract"][0] / args.steps))
    # roofline of the contraction kernel (one launch per pass and 64-output chunk)
    c_ms, c_launches = stages["contract"]
    launches_per_step = c_launches / args.steps
    per_launch_s = c_ms / 1e3 / c_launches
    P = info["n_passes"]
    AS = (m + 15) // 16 * 16
    flops_launch = 2.0 * hits * m / launches_per_step
    plain = prec == hd.PLAIN_FP64
    mfma_peak = FP64_PEAK if plain else BF16_PEAK
    # problem-level bytes of an evaluation: outputs once, points once, the model once
    alg_bytes_step = n * m * 8.0 + n * d * 8.0 + info["device_bytes"]
    # bytes this design must move per pass: the accumulator rows (AS values,
    # FP64 plain / FP32 mixed) read and written, the points' key coordinates
    acc_bytes = 8.0 if plain else 4.0
    design_bytes_step = (n * AS * 2 * acc_bytes * P + n * (8.0 * info["pass_key_dims"] + 4.0 * P))
    kern = KERNEL[name]
    traffic = _measured_traffic(kern, args.config)
    roof = {
        "bound": "mfma",
        "achieved": flops_launch / per_launch_s / 1e12,
        "peak": mfma_peak / 1e12,
        "unit": "TFLOP/s",
        "frac": flops_launch / per_launch_s / mfma_peak,
        "traffic": traffic,
        "kernel": kern,
        "launches_per_step": launches_per_step,
        "avg_launch_ms": per_launch_s * 1e3,
        "algorithmic_flops_per_launch": flops_launch,
        "algorithmic_bytes_per_launch": alg_bytes_step / launches_per_step,
        "design_bytes_per_launch": design_bytes_step / launches_per_step,
        "hbm_GBps_of_traffic": (traffic / per_launch_s / 1e9) if traffic else None,
        "hbm_frac_of_traffic": (traffic / per_launch_s / HBM_PEAK) if traffic else None,
        "stage_ms_per_step": {s: v[0] / args.steps for s, v in stages.items()},
        "stage_note": "sort and rows run on a second stream, overlapped with the contraction",
    }
    if not plain:
        # six BF16 products per useful FMA, and the FP32 vector peak for reference
        roof["mfma_issued_frac"] = 6.0 * roof["frac"]
        roof["frac_of_fp32_vector_peak"] = flops_launch / per_launch_s / FP32_PEAK
    if ceil:
        roof["measured_ceilings"] = ceiling_roofline(ceil, plain, flops_launch, per_launch_s, n, m, AS, P,
                                                     launches_per_step)
    return {"value": value, "ms_per_step": ms, "roofline": roof, "wall_s": wall}


def ceiling_roofline(ceil, plain, flops_launch, per_launch_s, n, m, AS, P, launches_per_step):
    """Multi-ceiling roofline of one contraction launch from the measured
    ceilings: matrix-core time of the products as issued (output columns padded
    to 16-wide tiles; six BF16 products per FMA in the mixed path) and the
    accumulator read-modify-write time at the measured random-row rate (the
    largest buffer of the ceiling run, 16-column line-aligned layout).  The
    bound is the larger; frac = bound / measured launch time."""
    pad = AS / m
    if plain:
        p_mfma = ceil["mfma_f64"]["TFLOPs"] * 1e12
        issued = flops_launch * pad
        acc_b = 8.0
    else:
        p_mfma = ceil["mfma_bf16"]["TFLOPs"] * 1e12
        issued = flops_launch * pad * 6.0
        acc_b = 4.0
    rows = [r for r in ceil["rmw"] if r["layout"] == "colblock16_m64"]
    big = max(rows, key=lambda r: r["rows"])
    rmw_Bps = big["useful_GBps"] * 1e9
    npass_launch = P / launches_per_step
    rmw_bytes = n * AS * 2 * acc_b * npass_launch
    if not plain:
        rmw_bytes += n * AS * (4 + 16 + 4) * npass_launch / 16.0   # folds every 16 passes
    t_mfma = issued / p_mfma
    t_rmw = rmw_bytes / rmw_Bps
    t_roof = max(t_mfma, t_rmw)
    return {"mfma_ceiling_TFLOPs": p_mfma / 1e12, "rmw_ceiling_GBps": rmw_Bps / 1e9,
            "hbm_copy_GBps": ceil.get("copy", {}).get("GBps"),
            "t_mfma_ms": t_mfma * 1e3, "t_rmw_ms": t_rmw * 1e3, "t_roof_ms": t_roof * 1e3,
            "t_measured_ms": per_launch_s * 1e3, "frac": t_roof / per_launch_s,
            "binding": "mfma" if t_mfma >= t_rmw else "accumulator read-modify-write"}


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps / 1e3


def _gen_c4(i):
    import workloads.synth as ws
    return ws.c4_model(i, seed=0)


def bench_batched(args):
    """The batched workload at its stated shape: 64 independent order-2 models,
    d ~ U{10..100}, m = d/2 + 1, all one- and two-dimensional components, each
    a random downward-closed grid of log-uniform size 50..20000, alpha ~
    N(0,1) 2^(-2|l|_1), n ~ logU(1e4, 1e6) uniform points per model
    (workloads.synth.c4_model).  Models are generated by a pool of host
    processes and uploaded one at a time (the host copy is dropped after the
    upload).  One hdmr_eval_batched call over all models: the gather-path
    models in one persistent launch replayed from a graph, the others on the
    cell-sorted path with the tile shape the autotuner measured best."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np

    count = args.models
    t0 = time.time()
    # the pool starts before any device use (spawned workers, no fork after HIP init)
    ex = ProcessPoolExecutor(max_workers=8, mp_context=mp.get_context("spawn"))
    futs = {}
    nxt = 0
    while nxt < min(count, 8):
        futs[nxt] = ex.submit(_gen_c4, nxt)
        nxt += 1

    import torch

    import paper_2202_06555_amd as hd

    hd.hdmr_init(0)
    gms, X, Y, meta = [], [], [], []
    for i in range(count):
        mo, P = futs.pop(i).result()
        log("model %d generated (d=%d) at %.1f s" % (i, mo["d"], time.time() - t0))
        if nxt < count:
            futs[nxt] = ex.submit(_gen_c4, nxt)
            nxt += 1
        gms.append(hd.hdmr_model_from_surpluses(mo))
        X.append(torch.from_numpy(P).to("cuda:0"))
        Y.append(torch.empty((P.shape[0], mo["m"]), dtype=torch.float64, device="cuda:0"))
        meta.append({"d": mo["d"], "m": mo["m"], "rows": int(sum(l.shape[0] for l in mo["levels"])),
                     "n": int(P.shape[0])})
        del mo, P
    ex.shutdown()
    setup_s = time.time() - t0
    rows = sum(mm["rows"] for mm in meta)
    npts = sum(mm["n"] for mm in meta)
    dev_gb = sum(hd.hdmr_get_info(g)["device_bytes"] for g in gms) / 1e9
    log("batched: %d models, %d rows, %d points, %.1f GB of models on the device, set up in %.1f s" %
        (len(gms), rows, npts, dev_gb, setup_s))
    hits = nz = probes = 0
    for i, (g, x, mm) in enumerate(zip(gms, X, meta)):
        h_, p_ = hd.hdmr_eval_stats(g, x)
        hits += h_ * mm["m"]
        nz += h_
        probes += p_
        log("work counted for %d models" % (i + 1))
    log("nonzero basis products per point %.1f, directory lookups per point %.1f" % (nz / npts, probes / npts))
    # path and tile-shape measurement, model by model (the choices persist
    # per model and size bucket; the batched calls below reuse them)
    t0 = time.time()
    for i in range(len(gms)):
        hd.hdmr_eval_batched([gms[i]], [X[i]], [Y[i]])
        torch.cuda.synchronize()
        log("tuned model %d (d=%d, %d rows, n=%d) at %.1f s" % (i, meta[i]["d"], meta[i]["rows"], meta[i]["n"],
                                                                time.time() - t0))
    _, paths = hd.hdmr_eval_batched(gms, X, Y)
    torch.cuda.synchronize()
    tune_s = time.time() - t0
    log("tuning %.1f s; paths %s" % (tune_s, paths.tolist()))
    t = _timed(lambda: hd.hdmr_eval_batched(gms, X, Y), args.steps, args.warmup)
    units = sum(mm["n"] * mm["m"] for mm in meta)
    flops = 2.0 * hits
    out = {
        "metric": "batched HDMR-ASG point x output evaluations/sec (%d models in one call)" % len(gms),
        "value": units / t, "unit": "point*outputs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%d order-2 models, d ~ U{10..100}, m = d/2+1, all one- and two-dim components, "
                               "random downward-closed grids of log-uniform size 50..20000, n ~ logU(1e4, 1e6) "
                               "uniform points" % len(gms),
                   "grid_rows": rows, "points": npts, "device_GB": dev_gb, "setup_s_untimed": setup_s,
                   "nonzeros_per_point": nz / npts, "lookups_per_point": probes / npts,
                   "surplus_row_GBps": 8.0 * hits / t / 1e9,
                   "tuning_call_s": tune_s,
                   "paths": {str(k): int((paths == k).sum()) for k in sorted(set(paths.tolist()))}},
        "roofline": {"bound": "alu", "achieved": flops / t / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": flops / t / FP64_VECTOR_PEAK, "traffic": None,
                     "kernel": "whole batched call (persistent gather launch + cell-sorted contractions)",
                     "note": "2 flops per nonzero basis product and output over all models, whole call timed"},
    }
    print(json.dumps(out), flush=True)


def bench_naive(args):
    """eq (3.16) evaluated term by term (hdmr_model_naive) against its
    regrouping a(x)^T b of eq (4.2) (the vectorised interpolation of Sec. 4.1),
    both built on the device from the same eq (4.2)-form build, at the d=20
    (all 190 pairs, 1e6 points) and d=100 (500 pairs, 4e6 points) workload
    shapes, plain FP64; the component form (w_S = 1) beside them.  Reports the
    naive / vectorised time ratio per shape and the error of both against the
    oracle's term-by-term sum on a sample."""
    import numpy as np
    import torch

    import paper_2202_06555_amd as hd
    import workloads.synth as ws

    hd.hdmr_init(0)
    shapes = {}
    for name in ("c2", "c3"):
        cfg = ws.config(name)
        tf = ws.test_function_for(cfg)
        kw = dict(comps=cfg["comps"], max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
        vec = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), form=1, **kw)
        comp = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), **kw)
        f_anchor = tf(cfg["anchor"][None, :])[0]
        naive = hd.hdmr_model_naive(vec, f_anchor)
        X = torch.from_numpy(ws.points_for(cfg)).to("cuda:0")
        n, m = X.shape[0], cfg["m"]
        Y = torch.empty((n, m), dtype=torch.float64, device="cuda:0")
        t = {}
        for label, mdl in (("vectorised", vec), ("naive", naive), ("component", comp)):
            t[label] = _timed(lambda: hd.hdmr_eval(mdl, X, Y), args.steps, args.warmup)
            log("%s %s: %.2f ms" % (name, label, t[label] * 1e3))
        rec = {"n": n, "m": m, "components": hd.hdmr_get_info(vec)["n_components"],
               "naive_terms": hd.hdmr_get_info(naive)["n_components"],
               "ms": {k: v * 1e3 for k, v in t.items()},
               "naive_over_vectorised": t["naive"] / t["vectorised"],
               "vectorised_evals_per_s": n * m / t["vectorised"]}
        if not args.no_cpu_baseline:
            import oracle
            model, info = oracle.build_model(cfg["comps"], cfg["d"], m, cfg["anchor"], (tf.c_fn, tf.c_user),
                                             max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"], form="paper")
            idx = np.arange(500)
            ref = oracle.evaluate_naive(model, X[:500].cpu().numpy(), info["f_anchor"])
            for label, mdl in (("vectorised", vec), ("naive", naive)):
                Ys = hd.hdmr_eval(mdl, X[:500].contiguous()).cpu().numpy()
                rec["max_abs_err_%s" % label] = float(np.abs(Ys[idx] - ref).max())
        shapes[name] = rec
    c3 = shapes["c3"]
    out = {
        "metric": "naive eq (3.16) / vectorised eq (4.2) evaluation time at d=100, m=51",
        "value": c3["naive_over_vectorised"], "unit": "ratio", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": c3["ms"]["vectorised"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "eq (4.2)-form builds of the d=20 (1e6 points) and d=100 (4e6 points) workloads "
                               "and their eq (3.16) term-by-term expansions", "shapes": shapes,
                   "paper_context": "the paper measures the vectorised form about 2.8x faster than the naive one "
                                    "on CPUs (smooth IRBC model, Sec. 5.1)"},
    }
    print(json.dumps(out), flush=True)


def bench_irbc(args):
    """The expectation operator of time iteration on the smooth IRBC model
    (Sec. 2.1): N = 50 countries (d = 100, m = 51), a synthetic previous policy
    built on the device (100 one-dim + 50 two-dim components, L = 7,
    eps_gamma = 1e-5), 40000 states with candidate choices; every state's 102
    monomial-rule next states go through hdmr_eval (4.08e6 evaluations per
    call), then the Euler and resource residuals are assembled."""
    import numpy as np
    import torch

    import paper_2202_06555_amd as hd
    from paper_2202_06555_amd import irbc
    import workloads.synth as ws

    hd.hdmr_init(0)
    N, n = 50, 40_000
    p = ws.irbc_params(N)
    g = ws.IrbcGuess(N)
    t0 = time.time()
    gm = hd.asg_build_components(g.d, g.m, g.anchor, g, comps=g.components(), max_level=7, eps_gamma=1e-5)
    build_s = time.time() - t0
    X, C = ws.irbc_states(n, N, seed=11)
    Xd, Cd = torch.from_numpy(X).to("cuda:0"), torch.from_numpy(C).to("cuda:0")
    R = torch.empty((n, N + 1), dtype=torch.float64, device="cuda:0")
    t = _timed(lambda: irbc.irbc_residuals(gm, p, Xd, Cd, residuals=R), args.steps, args.warmup)
    Q = 2 * (N + 1)
    Xn = torch.rand((n * Q, 2 * N), dtype=torch.float64, device="cuda:0")
    Yn = torch.empty((n * Q, N + 1), dtype=torch.float64, device="cuda:0")
    t_eval = _timed(lambda: hd.hdmr_eval(gm, Xn, Yn), args.steps, args.warmup)
    out = {
        "metric": "smooth-IRBC FOC residual evaluations (states/s) at N=50 (d=100, m=51)",
        "value": n / t, "unit": "states/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "N=50 countries, synthetic previous policy (150 components, L=7, eps_gamma=1e-5), "
                               "%d states, degree-3 monomial rule (%d nodes)" % (n, Q),
                   "policy_rows": hd.hdmr_get_info(gm)["n_rows"], "build_s_untimed": build_s,
                   "next_state_evals_per_s": n * Q * (N + 1) / t,
                   "hdmr_eval_ms_same_count_uniform_points": t_eval * 1e3},
    }
    out["config"]["time_iteration"] = time_iteration(hd, irbc, ws, args.ti_steps)
    if not args.no_cpu_baseline:
        import oracle
        from oracle import irbc as oirbc
        model, _ = oracle.build_model(g.components(), g.d, g.m, g.anchor, g, max_level=7, eps_gamma=1e-5)
        k = 40
        t0 = time.perf_counter()
        Ro, _ = oirbc.residuals(model, p, X[:k], C[:k])
        tc = time.perf_counter() - t0
        Rg = R[:k].cpu().numpy()
        out["error_vs_oracle"] = {"max_abs": float(np.abs(Rg - Ro).max()), "states": k}
        out["cpu_baseline"] = {"value": k / tc, "unit": "states/s", "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": "first %d states" % k}
    print(json.dumps(out), flush=True)


def time_iteration(hd, irbc, ws, steps, N=10):
    """Time iteration (Alg. 1) on the smooth IRBC model with N countries
    (d = 2N, m = N + 1) from the synthetic policy: each step is a build whose
    function is the device Newton solve of the first-order conditions at the
    build's nodes, with the previous policy inside the expectation (L = 5,
    eps_gamma = 1e-5, Newton tolerance 1e-11).  After every step: the Euler
    errors (Sec. 5) of the new policy on 10^4 uniform states, and the largest
    change of the policy there (the stopping test of Alg. 1)."""
    import numpy as np
    import torch
    p = ws.irbc_params(N)
    g = ws.IrbcGuess(N)
    comps = g.components()
    X, _ = ws.irbc_states(10_000, N, seed=41)
    Xd = torch.from_numpy(X).to("cuda:0")
    pol = hd.asg_build_components(g.d, g.m, g.anchor, g, comps=comps, max_level=5, eps_gamma=1e-5)

    def errs(model):
        e = irbc.irbc_euler_errors(model, p, Xd).cpu().numpy()
        return {"euler_log10_mean": float(np.log10(e[:, :N]).mean()),
                "euler_log10_max": float(np.log10(e[:, :N].max())),
                "resource_log10_max": float(np.log10(e[:, N].max()))}

    rec = [{"step": 0, **errs(pol)}]
    prev_vals = hd.hdmr_eval(pol, Xd).cpu().numpy()
    for s in range(1, steps + 1):
        t0 = time.perf_counter()
        new, iters, worst = irbc.irbc_time_step(pol, p, comps, max_level=5, eps_gamma=1e-5, max_iter=20, tol=1e-11)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        vals = hd.hdmr_eval(new, Xd).cpu().numpy()
        r = {"step": s, "seconds": dt, "newton_iterations_max": int(iters), "newton_residual_max": float(worst),
             "grid_rows": hd.hdmr_get_info(new)["n_rows"], "policy_change_max": float(np.abs(vals - prev_vals).max()),
             **errs(new)}
        rec.append(r)
        log("time-iteration step %d: %.2f s, %d rows, policy change %.2e, Euler errors log10 mean %.2f max %.2f" %
            (s, dt, r["grid_rows"], r["policy_change_max"], r["euler_log10_mean"], r["euler_log10_max"]))
        pol, prev_vals = new, vals
    return {"N": N, "d": 2 * N, "m": N + 1, "states_for_errors": X.shape[0], "steps": rec}


def bench_grad(args):
    """Values and gradients (hdmr_eval_grad) on the d=20 workload: 20 + 190
    components, adaptive L=7, m=11, 1e6 next-state points; the gradient is
    n x d x m FP64."""
    import torch

    import paper_2202_06555_amd as hd
    import workloads.synth as ws

    hd.hdmr_init(0)
    cfg = ws.config("c2")
    tf = ws.test_function_for(cfg)
    model = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"],
                                    max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    n, d, m = cfg["n"], cfg["d"], cfg["m"]
    X = torch.from_numpy(ws.points_for(cfg)).to("cuda:0")
    Y = torch.empty((n, m), dtype=torch.float64, device="cuda:0")
    G = torch.empty((n, d, m), dtype=torch.float64, device="cuda:0")
    hits, _ = hd.hdmr_eval_stats(model, X)
    # derivative products: in the zero-boundary basis every hat of a tuple
    # varies in its support, so each nonzero product of a k-dimensional
    # component carries k nonzero derivative products
    from paper_2202_06555_amd import surrogate as sg
    dhits = 0
    for k in sorted({len(S) for S in cfg["comps"]}):
        sub = sg.hdmr_model_select(model, comps=[s for s, S in enumerate(cfg["comps"]) if len(S) == k])
        dhits += k * hd.hdmr_eval_stats(sub, X)[0]
        hd.hdmr_free(sub)
    for _ in range(args.warmup):
        hd.hdmr_eval_grad(model, X, Y, G)
    torch.cuda.synchronize()
    hd.hdmr_timing_enable(True)
    t = _timed(lambda: hd.hdmr_eval_grad(model, X, Y, G), args.steps, 0)
    c_ms, c_launches = hd.hdmr_timing_read("contract")
    hd.hdmr_timing_enable(False)
    per_launch_s = c_ms / 1e3 / max(c_launches, 1)
    # value and derivative products, 2 flops per output each
    flops_launch = 2.0 * (hits + dhits) * m / max(c_launches / args.steps, 1)
    out = {
        "metric": "HDMR-ASG point x output value+gradient evaluations/sec at d=20, m=11",
        "value": n * m / t, "unit": "point*outputs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2: d=20, 210 components, adaptive L=7 eps_gamma=1e-4, m=11, 1e6 next-state "
                               "points; gradient n x d x m FP64", "grid_rows": hd.hdmr_get_info(model)["n_rows"]},
        "roofline": {"bound": "mfma", "achieved": flops_launch / per_launch_s / 1e12, "peak": FP64_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": flops_launch / per_launch_s / FP64_PEAK, "traffic": None,
                     "kernel": "k_tile_fp64<56, true, true> (cell-sorted contraction with derivative chains; "
                               "m <= 16, so the waves split each sub-tile's points)",
                     "launches_per_step": c_launches / args.steps, "avg_launch_ms": per_launch_s * 1e3,
                     "algorithmic_flops_per_launch": flops_launch,
                     "note": "2 m (value products + derivative products); k derivative products per nonzero "
                             "product of a k-dimensional component"},
    }
    print(json.dumps(out), flush=True)


def bench_surrogate(args):
    """The learned part on the d=300 workload: 300 one-dim + 300 two-dim
    components, L=7, m=151, order-2 terms scaled 1/100 (the paper's observed
    ratio).  Trains the BF16 network on interpolant pairs, validates each
    output on 1e5 fresh points, routes at max-abs 1e-4, and times network,
    interpolant and routed evaluation."""
    import numpy as np
    import torch

    import paper_2202_06555_amd as hd
    from paper_2202_06555_amd import surrogate as sg
    import workloads.synth as ws

    hd.hdmr_init(0)
    cfg = ws.config("c5")
    tf = ws.TestFunction(cfg["d"], cfg["m"], cfg["pairs"], cfg["seed"], ref=cfg["anchor"], pair_scale=0.01)
    full = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"],
                                   max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    c1 = [s for s, S in enumerate(cfg["comps"]) if len(S) == 1]
    o1 = sg.hdmr_model_select(full, comps=c1)
    d, m, w = cfg["d"], cfg["m"], 512
    ntr = args.train_points
    Xtr = torch.from_numpy(ws.points_for(cfg, n=ntr, seed=1)).to("cuda:0")
    Ytr = hd.hdmr_eval(full, Xtr) - hd.hdmr_eval(o1, Xtr)
    net = sg.mlp_create(d, w, m, ws.mlp_init_params(d, w, m, seed=0))
    sg.mlp_fit_standardization(net, Ytr)
    B = 4096
    steps = max(1, args.epochs * ntr // B)
    rng = np.random.default_rng(5)
    order = np.concatenate([rng.permutation(ntr) for _ in range(args.epochs + 1)])[:steps * B]
    order = torch.from_numpy(order.astype(np.int64)).to("cuda:0")
    Xv = torch.from_numpy(ws.points_for(cfg, n=100_000, seed=3)).to("cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    curve = []
    if args.train_seconds > 0:
        # training to a measured plateau: segments of one epoch, each a cosine
        # decay from a starting rate that falls log-linearly in wall time from
        # 1e-3 to 1e-6 over the training budget; after every segment the
        # per-output max-abs error on the validation points
        seg = max(1, ntr // B)
        lr, k, all_losses = 1e-3, 0, []
        gen = torch.Generator(device="cuda:0")
        gen.manual_seed(5)
        # the validation target of the network: full minus order-1 interpolant
        Rv = hd.hdmr_eval(full, Xv) - hd.hdmr_eval(o1, Xv)
        while time.perf_counter() - t0 < args.train_seconds:
            o = torch.randperm(ntr, device="cuda:0", generator=gen)[:seg * B]
            all_losses.append(sg.mlp_train(net, Xtr, Ytr, o, steps=seg, batch=B, lr0=lr))
            e = (sg.mlp_forward(net, Xv) - Rv).abs().amax(dim=0).cpu().numpy()
            kk = int((e <= 1e-4).sum())
            k += 1
            curve.append({"segment": k, "steps": k * seg, "seconds": time.perf_counter() - t0,
                          "loss": float(all_losses[-1][-min(200, seg):].mean()), "lr0": lr,
                          "val_max_err_max": float(e.max()), "val_max_err_median": float(np.median(e)),
                          "val_max_err_min": float(e.min()), "outputs_at_1e-4": int(kk)})
            log("segment %d: %d steps, %.1f s, loss %.4f, validated max-abs error min %.2e median %.2e max %.2e"
                % (k, k * seg, curve[-1]["seconds"], curve[-1]["loss"], e.min(), np.median(e), e.max()))
            lr = 1e-3 * 10.0 ** (-3.0 * min(1.0, (time.perf_counter() - t0) / args.train_seconds))
        del Rv
        losses = np.concatenate(all_losses)
        steps = k * seg
    else:
        losses = sg.mlp_train(net, Xtr, Ytr, order, steps=steps, batch=B, lr0=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del Xtr, Ytr, order
    route = sg.mlp_route_create(net, full, Xv, 1e-4)
    k, err, use = sg.mlp_route_info(route)
    Xs = torch.from_numpy(ws.points_for(cfg, n=args.serve_points, seed=2)).to("cuda:0")
    ns = Xs.shape[0]
    t_mlp = _timed(lambda: sg.mlp_forward(net, Xs), args.steps, 1)
    t_int = _timed(lambda: hd.hdmr_eval(full, Xs), args.steps, 1)
    t_rt = _timed(lambda: sg.mlp_eval_routed(route, Xs), args.steps, 1)
    flops_fwd = 2.0 * (d * w + 2 * w * w + w * m) * ns
    out = {
        "metric": "surrogate-routed point x output evaluations/sec at d=300, m=151 (fallback at max-abs 1e-4)",
        "value": ns * m / t_rt, "unit": "point*outputs/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": t_rt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 mfma / f32 accumulate (network); f64 (interpolant)", "data": "synthetic",
        "config": {"workload": "d=300, 300 one-dim + 300 two-dim components (order-2 terms x0.01), L=7, "
                               "eps_gamma=1e-4, m=151; width-512 4-layer GELU network trained on %d interpolant "
                               "pairs (%s, batch 4096); %d served points" %
                               (ntr, ("%d one-epoch segments in %.0f s" % (len(curve), t_train)) if curve
                                else "%d epochs" % args.epochs, ns),
                   "outputs_on_network": int(k), "validated_max_abs_err": {"min": float(err.min()),
                   "median": float(np.median(err)), "max": float(err.max())},
                   "train_s": t_train, "train_steps": int(steps), "training_curve": curve,
                   "loss_first": float(losses[:50].mean()), "loss_last": float(losses[-50:].mean()),
                   "network_only_evals_per_s": ns * m / t_mlp, "interpolant_evals_per_s": ns * m / t_int},
        "roofline": {"bound": "mfma", "achieved": flops_fwd / t_mlp / 1e12, "peak": BF16_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": flops_fwd / t_mlp / BF16_PEAK, "traffic": None,
                     "kernel": "k_gemm_wide<0, 1, EPI, 64> (network forward: 128 x 128 tiles)", "note": "whole forward timed (input conversion, four products, de-standardisation); flops of the four products"},
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(cfg, sample, ws):
    """The FP64 oracle (C, OpenMP over points, level-wise mode) on its own build
    of the same workload, timed on this host's cores on a bounded sample:
    median of 5 timed runs after one warm-up on all threads, and one run on a
    single thread over the first eighth of the sample.  Returns the baseline
    record, the sample's point indices and the oracle's values there."""
    import platform
    import statistics
    import numpy as np
    import oracle
    tf = ws.test_function_for(cfg)
    t0 = time.time()
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user),
                                  max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    log("oracle build %.1f s" % (time.time() - t0))
    X = ws.points_for(cfg, n=sample)
    threads = oracle.num_threads()
    ref = oracle.evaluate(model, X)          # warm-up; also the reference values
    times = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.evaluate(model, X)
        times.append(time.perf_counter() - t0)
    t = statistics.median(times)
    n1 = max(1, sample // 8)
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.evaluate(model, X[:n1])
    t1 = time.perf_counter() - t0
    oracle.set_num_threads(threads)
    log("oracle eval of %d points: median %.2f s on %d threads; %d points on 1 thread %.2f s" %
        (sample, t, threads, n1, t1))
    cpu = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    rec = {"value": sample * cfg["m"] / t, "unit": "point*outputs/s", "cores": threads, "kind": "oracle",
           "sample": "first %d of the %d next-state points (seed %d), level-wise FP64 oracle with compensated "
                     "sums; median of 5 runs after 1 warm-up" % (sample, cfg["n"], cfg["seed"]),
           "single_thread_value": n1 * cfg["m"] / t1, "single_thread_sample": n1,
           "nproc": os.cpu_count(), "cpu_model": cpu}
    return rec, np.arange(sample), ref


if __name__ == "__main__":
    main()
