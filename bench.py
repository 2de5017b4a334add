#!/usr/bin/env python3
"""Benchmark of the QoZ hot path on one MI355X.

Workload: a 512^3 float32 Gaussian random field with a k^-3 power spectrum
(synthetic stand-in for the paper's 512^3 cosmology field), bound
e = 1e-3 x value range.  One step = online tuning (Algorithm 1 + the
(alpha, beta) search, ratio target, 32^3 blocks at 1%, all dimension orders)
+ compression with the tuned parameters + decompression, all on the GPU
through the C ABI with the field resident in HBM.

Prints one JSON line.  `value` is field bytes / wall time per step (GB/s).
The warmup steps run with every kernel launch bracketed by HIP events on the
library's stream (per-kind table `kernels_warmup`, per step); the kind with
the largest summed time there is the roofline kernel, and in the timed
region only its launches carry events, so `roofline.achieved` is its
algorithmic bytes over its average launch duration measured live while the
rest of the step runs uninstrumented.  `roofline.cold_copy_TBps` is the
rate of a plain device copy of field-sized buffers that miss the last-level
cache (read + write bytes): the practical streaming ceiling next to the
8 TB/s peak.  cpu_baseline times the single-threaded CPU oracle on the same
field.
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_KINDS_EXCLUDED = ()


def cold_copy_tbps(numel, nbuf=6, reps=12):
    """Device-to-device copy rate (read + write bytes per second) of
    field-sized buffers, rotating over nbuf of them so that no copy finds
    its data in the 256 MB last-level cache: the practical HBM streaming
    ceiling the kernels are compared with."""
    import torch
    bufs = [torch.empty(numel, dtype=torch.float32, device="cuda")
            for _ in range(nbuf)]
    for i, b in enumerate(bufs):
        b.fill_(float(i))
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
        enable_timing=True)
    ms = 0.0
    for k in range(reps):
        src, dst = bufs[k % nbuf], bufs[(k + nbuf // 2) % nbuf]
        a.record()
        dst.copy_(src)
        z.record()
        z.synchronize()
        if k >= nbuf:  # the first pass touches every buffer once
            ms += a.elapsed_time(z)
    del bufs
    torch.cuda.empty_cache()
    return 2 * numel * 4 / (ms / (reps - nbuf) / 1e3) / 1e12


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=20)
    ap.add_argument("--log-normal", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-online tuner comparison")
    ap.add_argument("--no-autotune", action="store_true",
                    help="default sweep launch tiles")
    ap.add_argument("--cpu-reps", type=int, default=3,
                    help="oracle runs for the CPU baseline (median)")
    ap.add_argument("--cpu-crop", type=int, default=0,
                    help="edge of a central crop for the CPU baseline "
                         "(0 = whole field)")
    ap.add_argument("--traffic", type=str,
                    default=os.path.join(ROOT, "profiles",
                                         "traffic_512cube_grf.json"),
                    help="measured HBM bytes per launch (rocprofv3 FETCH_SIZE"
                         " + WRITE_SIZE, copy-calibrated); ignored for a "
                         "kernel whose source changed since")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times "
                         "(the reference for the traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; there is no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = 64 << 20
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "copies": 3}), flush=True)
        return

    import paper_2310_14133_amd as q
    from paper_2310_14133_amd import fields

    n = args.size
    dims = (n, n, n)
    print(f"bench: generating {dims} field (seed {args.seed})", file=sys.stderr,
          flush=True)
    x = fields.grf_torch(dims, args.seed, log_normal=args.log_normal,
                         device="cuda")
    torch.cuda.synchronize()
    vmin, vmax = float(x.min()), float(x.max())
    e = args.eps * (vmax - vmin)
    shape = q.make_shape(dims)
    codec = q.Codec(0)
    ctx = codec.ctx
    cfg = q.make_tune_config(block=32, sample_rate=0.01, all_orders=1)
    cap = q.qoz_compress_bound(shape)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    CR = q.TARGETS["cr"]

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step(record=None):
        if record is not None:
            ev[0].record(stream)
        p = q.Params()
        q.qoz_tune(ctx, x.data_ptr(), shape, e, CR, cfg, p, sh)
        if record is not None:
            ev[1].record(stream)
        nb = q.qoz_compress(ctx, x.data_ptr(), shape, e, p, CR, cfg,
                            out.data_ptr(), cap, sh)
        if record is not None:
            ev[2].record(stream)
        q.qoz_decompress(ctx, out.data_ptr(), nb, y.data_ptr(), y.numel(), sh)
        if record is not None:
            ev[3].record(stream)
            torch.cuda.synchronize()
            record["tune"].append(ev[0].elapsed_time(ev[1]))
            record["comp"].append(ev[1].elapsed_time(ev[2]))
            record["decomp"].append(ev[2].elapsed_time(ev[3]))
        return p, nb

    hbm_copy = cold_copy_tbps(x.numel())

    # one-time setup: launch tiles of the sweeps for this shape and the
    # parameters the tuner picks (the same in every step)
    p0 = q.Params()
    q.qoz_tune(ctx, x.data_ptr(), shape, e, CR, cfg, p0, sh)
    n_tuned, t_def, t_best = q.qoz_autotune_tiles(ctx, shape, p0, sh) \
        if not args.no_autotune else (0, 0.0, 0.0)
    print(f"bench: autotuned the launch tiles of {n_tuned} sweeps "
          f"({t_def:.4f} ms with the default tiles, {t_best:.4f} ms tuned)",
          file=sys.stderr, flush=True)

    # warmup with every kernel kind timed: the per-kind table and the
    # dominant kind (one extra untimed step when there is no warmup)
    print("bench: warmup", file=sys.stderr, flush=True)
    q.qoz_ctx_reset_timing(ctx)
    q.qoz_ctx_set_timing(ctx, True)
    nwarm = max(args.warmup, 1)
    for _ in range(nwarm):
        step()
    torch.cuda.synchronize()
    q.qoz_ctx_set_timing(ctx, False)
    kernels = q.timing_table(ctx)
    kinds = {k: v for k, v in kernels.items() if v[0] > 0}
    dom = max(kinds, key=lambda k: kinds[k][1])
    dom_kind = [q.qoz_prof_name(k) for k in range(q.qoz_prof_kinds())].index(
        dom)

    # timed region: K whole steps; only the dominant kind's launches are
    # bracketed with events, so the rest run uninstrumented
    q.qoz_ctx_reset_timing(ctx)
    q.qoz_ctx_set_timing_mask(ctx, 1 << dom_kind)
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    # the collector's full passes over torch's object graph take several ms
    # and would land on whichever step triggers them (as timeit does, the
    # collector is off while timing)
    gc.collect()
    gc.freeze()
    gc.disable()
    t0 = time.perf_counter()
    marks = []
    for _ in range(args.steps):
        p, nb = step()
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    step_ms = [(b - a) * 1e3 for a, b in zip([t0] + marks[:-1], marks)]
    print("bench: step ms " + " ".join(f"{v:.3f}" for v in step_ms),
          file=sys.stderr, flush=True)
    q.qoz_ctx_set_timing(ctx, False)
    timed = q.timing_table(ctx)[dom]
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # per-phase split (separate, untimed-for-value passes)
    rec = {"tune": [], "comp": [], "decomp": []}
    for _ in range(3):
        step(rec)
    med = {k: sorted(v)[len(v) // 2] for k, v in rec.items()}

    psnr, _, maxerr = codec.metrics(x, y, want_ssim=False)
    field_bytes = x.numel() * 4
    value = field_bytes / (ms_per_step / 1e3) / 1e9
    launches, tot_ms, algo_bytes = timed
    achieved = (algo_bytes / 1e9) / (tot_ms / 1e3)
    # the library counts every bin as a 4-byte code (the cost model's
    # width); the kernels store 2-byte bins, so per bin 2 bytes fewer move
    n_codes = x.numel() - ((n - 1) // 32 + 1) ** 3
    bins_per_launch = {"huffman_decode": n_codes, "huffman_encode": n_codes,
                       "huffman_count": n_codes, "histogram": n_codes}
    stored = None
    if dom in bins_per_launch:
        stored = (algo_bytes / launches - 2.0 * bins_per_launch[dom]) / 1e9 \
            / (tot_ms / launches / 1e3)
    from paper_2310_14133_amd import profiling
    traffic = profiling.load_traffic(args.traffic, dom)

    line = {
        "metric": "comp/decomp GB/s, 512^3 f32, eb 1e-3; tune time + CR vs "
                  "exhaustive @ fixed PSNR",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "step_ms": {"min": round(min(step_ms), 4),
                    "median": round(sorted(step_ms)[len(step_ms) // 2], 4),
                    "max": round(max(step_ms), 4)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"QoZ tune+compress+decompress, {n}^3 float32 "
                        "Gaussian random field P(k)~k^-3"
                        + (" exp-transformed" if args.log_normal else "")
                        + f", eb {args.eps:g} x value range, ratio target, "
                        "32^3 blocks at 1%, all dimension orders",
            "sweep_tiles": "autotuned" if n_tuned else "default",
            "field_bytes": field_bytes,
            "abs_eb": e,
        },
        "phases_ms": {k: round(v, 4) for k, v in med.items()},
        "compress_GBps": round(field_bytes / (med["comp"] / 1e3) / 1e9, 3),
        "decompress_GBps": round(field_bytes / (med["decomp"] / 1e3) / 1e9,
                                 3),
        "tune_ms": round(med["tune"], 4),
        "compression_ratio": round(field_bytes / nb, 4),
        "psnr_db": round(psnr, 4),
        "max_abs_err_over_eb": maxerr / e,
        "params": q.params_dict(p, 3),
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "code_bytes_counted": 4,
            "frac_at_stored_width": (round(stored / HBM_PEAK_GBS, 4)
                                     if stored is not None else None),
            "avg_launch_ms": round(tot_ms / launches, 5),
            "algo_bytes_per_launch": algo_bytes / launches,
            "cold_copy_TBps": round(hbm_copy, 3),
        },
        "kernels_warmup": {k: {"launches": v[0] / nwarm,
                               "ms": round(v[1] / nwarm, 4),
                               "algo_GBps": round((v[2] / 1e9) / (v[1] / 1e3),
                                                  1) if v[1] > 0 else None}
                           for k, v in kinds.items()},
    }

    # the learned tuner against the online tuner on the same field at the
    # PSNR targets 60 / 80 / 100 dB: tuning time at each target's nominal
    # bound, and the ratio of each tuner's parameters at equal PSNR (the
    # bound bisected until the final PSNR is within 0.05 dB above the
    # target, each step tuning at that bound)
    wpath = os.path.join(ROOT, "paper_2310_14133_amd", "tuner_mlp.bin")
    if os.path.exists(wpath) and not args.no_learned:
        from paper_2310_14133_amd import learned
        print("bench: learned tuner at equal PSNR", file=sys.stderr,
              flush=True)
        Pw = learned.load_weights(wpath)
        cfg_l = q.make_tune_config(block=32, sample_rate=learned.SAMPLE_RATE)
        rows = []
        for target in learned.PSNR_TARGETS:
            eb = learned.bound_for_psnr(vmax - vmin, target)
            (pl, fb), tl = learned._timed(lambda: codec.tune_learned(
                x, eb, Pw, 0.5, "psnr", cfg_l), reps=5)
            _, te = learned._timed(lambda: codec.tune(x, eb, "psnr", cfg_l),
                                   reps=5)
            cr_e, ps_e, _, _ = learned.equal_psnr(
                codec, x, target, lambda b: codec.tune(x, b, "psnr", cfg_l))
            cr_l, ps_l, _, _ = learned.equal_psnr(
                codec, x, target, lambda b: codec.tune_learned(
                    x, b, Pw, 0.5, "psnr", cfg_l)[0])
            rows.append({"psnr_target": target,
                         "online_tune_ms": round(te, 4),
                         "learned_tune_ms": round(tl, 4),
                         "tune_speedup": round(te / tl, 3),
                         "cr_online": round(cr_e, 4),
                         "cr_learned": round(cr_l, 4),
                         "cr_ratio_equal_psnr": round(cr_l / cr_e, 5),
                         "psnr_online": round(ps_e, 3),
                         "psnr_learned": round(ps_l, 3),
                         "fallback": bool(fb)})
        line["learned_tuner"] = {
            "rows": rows,
            "cr_ratio_min": min(r["cr_ratio_equal_psnr"] for r in rows),
            "tune_speedup_min": min(r["tune_speedup"] for r in rows),
            "fallback_rate": sum(r["fallback"] for r in rows) / len(rows)}

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(x, e, args)
    print(json.dumps(line), flush=True)
    codec.close()


def host_cpu():
    """CPU model and logical CPU count of this host, from lscpu."""
    import subprocess
    model, total = "unknown", os.cpu_count()
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True,
                             timeout=20).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() == "Model name":
                model = v.strip()
            elif k.strip() == "CPU(s)":
                total = int(v.strip())
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return model, total


def cpu_baseline(x, e, args):
    """The oracle (single-threaded C++) on the same workload, pinned to one
    host core (the process's affinity is narrowed to it for the duration,
    as taskset would), median of `args.cpu_reps` whole steps."""
    import numpy as np

    from oracle import ref
    xh = x.cpu().numpy()
    if args.cpu_crop:
        c = args.cpu_crop
        o = (xh.shape[0] - c) // 2
        xh = np.ascontiguousarray(xh[o:o + c, o:o + c, o:o + c])
    cfg = ref.tune_config(block=32, sample_rate=0.01, all_orders=1)
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    model, total = host_cpu()
    print(f"bench: cpu baseline on {xh.shape}, core {core}", file=sys.stderr,
          flush=True)
    runs = []
    os.sched_setaffinity(0, {core})
    try:
        for r in range(args.cpu_reps):
            t0 = time.perf_counter()
            p, _ = ref.tune(xh, e, "cr", cfg, want_trace=False)
            t1 = time.perf_counter()
            z = ref.compress(xh, e, p)
            t2 = time.perf_counter()
            ref.decompress(z)
            t3 = time.perf_counter()
            runs.append((t3 - t0, t1 - t0, t2 - t1, t3 - t2))
            print(f"bench: cpu baseline run {r + 1}: {t3 - t0:.3f} s",
                  file=sys.stderr, flush=True)
    finally:
        os.sched_setaffinity(0, allowed)
    runs.sort()
    tot, tt, tc, td = runs[len(runs) // 2]
    return {"value": round(xh.nbytes / tot / 1e9, 5), "unit": "GB/s",
            "cores": 1, "kind": "oracle",
            "sample": f"whole step (tune+compress+decompress) on "
                      f"{'x'.join(map(str, xh.shape))} of the same field, "
                      f"median of {len(runs)} runs",
            "pinned_core": core, "cpu_model": model, "host_cpus": total,
            "runs_s": [round(r[0], 3) for r in runs],
            "tune_s": round(tt, 3), "compress_s": round(tc, 3),
            "decompress_s": round(td, 3)}


if __name__ == "__main__":
    main()
