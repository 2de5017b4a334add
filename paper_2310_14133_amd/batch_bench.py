"""Batch workload: many fields of uneven shapes and bounds, compressed
(tuned per field) and decompressed one call at a time and as batches.

Workload (from one seed): 64 fields; one third 2D with sides U{256..2048},
the rest 3D between 64^3 and 384 x 384 x 256 (each side U{64..its cap}),
k^-3 random fields cut from the corner of one periodic field per shape
family (one FFT size), value-range-relative bounds log-uniform in
[1e-5, 1e-2].  Reports aggregate GB/s of input and p50 / p99 per-field
latency for the loop and for batches of 4 and 8 workers, the compression
(tuned in the call, and with parameters given) and decompression of the
whole batch through the device work queues (the batch calls write into
preallocated fields), and PSNR-mode tuning of the batch by the online
tuner and by the batched learned tuner.

    python -m paper_2310_14133_amd.batch_bench --fields 64
"""
import argparse
import json
import sys
import time

import numpy as np


def workload(n_fields, seed, device="cuda"):
    import torch
    from paper_2310_14133_amd import fields
    rng = np.random.default_rng(seed)
    big3 = fields.grf_torch((384, 384, 256), seed, device=device)
    big2 = fields.grf_torch((2048, 2048), seed + 1, device=device)
    xs, ebs = [], []
    for i in range(n_fields):
        if i % 3 == 2:
            sh = (int(rng.integers(256, 2049)), int(rng.integers(256, 2049)))
            src = big2
        else:
            sh = (int(rng.integers(64, 385)), int(rng.integers(64, 385)),
                  int(rng.integers(64, 257)))
            src = big3
        x = src[tuple(slice(0, v) for v in sh)].contiguous()
        x = (x - x.mean()) / x.std()
        xs.append(x.contiguous())
        vr = float((x.max() - x.min()).item())
        ebs.append(vr * 10.0 ** rng.uniform(-5.0, -2.0))
    del big3, big2
    torch.cuda.synchronize()
    return xs, ebs


def pct(v, p):
    return float(np.percentile(np.asarray(v), p))


def main(argv=None):
    import torch
    import paper_2310_14133_amd as q
    ap = argparse.ArgumentParser()
    ap.add_argument("--fields", type=int, default=64)
    ap.add_argument("--seed", type=int, default=400)
    ap.add_argument("--workers", type=int, nargs="+", default=[4, 8])
    ap.add_argument("--report", default="")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the batch bench runs on the GPU")
    codec = q.Codec(0)
    xs, ebs = workload(args.fields, args.seed)
    total = sum(x.numel() * 4 for x in xs)
    print(f"batch: {len(xs)} fields, {total / 1e9:.3f} GB", flush=True)
    res = {"fields": len(xs), "bytes": total, "seed": args.seed}

    def loop():
        lat_c, lat_d, zs, ys = [], [], [], []
        t0 = time.perf_counter()
        for x, e in zip(xs, ebs):
            t = time.perf_counter()
            z = codec.compress(x, e)
            torch.cuda.synchronize()
            lat_c.append((time.perf_counter() - t) * 1e3)
            zs.append(z)
        tc = time.perf_counter() - t0
        t0 = time.perf_counter()
        for z in zs:
            t = time.perf_counter()
            ys.append(codec.decompress(z))
            torch.cuda.synchronize()
            lat_d.append((time.perf_counter() - t) * 1e3)
        td = time.perf_counter() - t0
        return tc, td, lat_c, lat_d, zs, ys

    loop()  # warm-up: scratch allocations, code objects
    tc, td, lc, ld, zs_loop, ys_loop = loop()
    # the batch calls below write into preallocated fields
    outs = [torch.empty_like(y) for y in ys_loop]
    res["loop"] = {"compress_GBps": total / tc / 1e9,
                   "decompress_GBps": total / td / 1e9,
                   "compress_p50_ms": pct(lc, 50), "compress_p99_ms": pct(lc, 99),
                   "decompress_p50_ms": pct(ld, 50),
                   "decompress_p99_ms": pct(ld, 99)}
    print("batch: loop", json.dumps(res["loop"]), flush=True)
    for w in args.workers:
        codec.compress_batch(xs, ebs, workers=w)  # warm-up of the workers
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        zs, it = codec.compress_batch(xs, ebs, workers=w)
        tc = time.perf_counter() - t0
        t0 = time.perf_counter()
        ys, dit = codec.decompress_batch(zs, workers=w, out=outs)
        td = time.perf_counter() - t0
        same = all(torch.equal(a, b) for a, b in zip(zs, zs_loop)) and \
            all(torch.equal(a.view(torch.int32), b.view(torch.int32))
                for a, b in zip(ys, ys_loop))
        r = {"compress_GBps": total / tc / 1e9,
             "decompress_GBps": total / td / 1e9,
             "compress_p50_ms": pct([i.ms for i in it], 50),
             "compress_p99_ms": pct([i.ms for i in it], 99),
             "decompress_p50_ms": pct([i.ms for i in dit], 50),
             "decompress_p99_ms": pct([i.ms for i in dit], 99),
             "outputs_equal_loop": same}
        res[f"batch_w{w}"] = r
        print(f"batch: workers {w}", json.dumps(r), flush=True)
        del ys
    # compression through the device work queues (one stream): tuned
    # inside the call, then with the parameters given (the compression
    # engine alone, against the loop of single calls with those parameters)
    codec.compress_batch(xs, ebs, queue=True)  # warm-up: queue buffers
    torch.cuda.synchronize()
    tq = []
    for _ in range(3):
        t0 = time.perf_counter()
        zq, _ = codec.compress_batch(xs, ebs, queue=True)
        tq.append(time.perf_counter() - t0)
    same = all(torch.equal(a, b) for a, b in zip(zq, zs_loop))
    ps = [codec.tune(x, e) for x, e in zip(xs, ebs)]
    codec.compress_batch(xs, ebs, ps, queue=True)
    torch.cuda.synchronize()
    tp = []
    for _ in range(3):
        t0 = time.perf_counter()
        zp, _ = codec.compress_batch(xs, ebs, ps, queue=True)
        tp.append(time.perf_counter() - t0)
    same_p = all(torch.equal(a, b) for a, b in zip(zp, zs_loop))
    tl = []
    for _ in range(2):
        t0 = time.perf_counter()
        for x, e, p in zip(xs, ebs, ps):
            codec.compress(x, e, p)
        torch.cuda.synchronize()
        tl.append(time.perf_counter() - t0)
    r = {"compress_GBps": total / min(tq) / 1e9,
         "compress_ms": [round(v * 1e3, 3) for v in tq],
         "outputs_equal_loop": same,
         "given_params_compress_GBps": total / min(tp) / 1e9,
         "given_params_compress_ms": [round(v * 1e3, 3) for v in tp],
         "given_params_outputs_equal_loop": same_p,
         "given_params_loop_GBps": total / min(tl) / 1e9}
    res["queue_compress"] = r
    print("batch: queue compression", json.dumps(r), flush=True)
    del zq, zp
    # decompression through the device work queues (one stream)
    codec.decompress_queue(zs_loop, out=outs)  # warm-up: queue buffers
    torch.cuda.synchronize()
    tq = []
    for _ in range(3):
        t0 = time.perf_counter()
        ys, _ = codec.decompress_queue(zs_loop, out=outs)
        tq.append(time.perf_counter() - t0)
    same = all(torch.equal(a.view(torch.int32), b.view(torch.int32))
               for a, b in zip(ys, ys_loop))
    r = {"decompress_GBps": total / min(tq) / 1e9,
         "decompress_ms": [round(v * 1e3, 3) for v in tq],
         "outputs_equal_loop": same}
    res["queue"] = r
    print("batch: queue", json.dumps(r), flush=True)
    # the same with the device work replayed as a HIP graph
    codec.set_queue_graphs(True)
    for _ in range(2):  # first call direct, second captures
        codec.decompress_queue(zs_loop, out=outs)
    tq = []
    for _ in range(3):
        t0 = time.perf_counter()
        ys, _ = codec.decompress_queue(zs_loop, out=outs)
        tq.append(time.perf_counter() - t0)
    codec.set_queue_graphs(False)
    same = all(torch.equal(a.view(torch.int32), b.view(torch.int32))
               for a, b in zip(ys, ys_loop))
    r = {"decompress_GBps": total / min(tq) / 1e9,
         "decompress_ms": [round(v * 1e3, 3) for v in tq],
         "outputs_equal_loop": same}
    res["queue_graph"] = r
    print("batch: queue, graph replays", json.dumps(r), flush=True)
    res["tuning"] = tuning(codec, xs, ebs, total)
    print("batch: tuning", json.dumps(res["tuning"]), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(res, f, indent=1)
    codec.close()


def tuning(codec, xs, ebs, total):
    """PSNR-mode tuning of the whole batch: the online tuner one field at a
    time against the batched learned tuner (its 3D and 2D networks; fields
    below one feature block, or below the confidence margin, fall back to
    the online tuner), and the ratio each one's parameters give."""
    import torch
    import paper_2310_14133_amd as q
    from paper_2310_14133_amd import learned
    P = learned.load_weights(learned.WEIGHTS[3])
    P2 = learned.load_weights(learned.WEIGHTS[2])
    cfg = q.make_tune_config(block=32, sample_rate=learned.SAMPLE_RATE)

    def online():
        return [codec.tune(x, e, "psnr", cfg) for x, e in zip(xs, ebs)]

    def batch():
        its = codec.tune_learned_batch(xs, ebs, P, 0.5, "psnr", cfg,
                                       params_2d=P2)
        return [it.params for it in its], sum(it.used_fallback for it in its)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3

    po, to = timed(online)
    (pl, n_fb), tl = timed(batch)

    # tune + compress of the whole batch through the queues, PSNR target:
    # tuned inside the queue call by the online tuner, or by the batched
    # learned tuner first and then compressed with its parameters
    def e2e(fn, reps=3):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return min(ts)

    t_on = e2e(lambda: codec.compress_batch(xs, ebs, None, "psnr", cfg,
                                            queue=True))
    t_le = e2e(lambda: codec.compress_batch(xs, ebs, batch()[0], "psnr", cfg,
                                            queue=True))

    def stream_bytes(ps):
        return sum(int(codec.compress(x, e, p).numel())
                   for x, e, p in zip(xs, ebs, ps))

    return {"online_ms": to, "learned_batch_ms": tl,
            "learned_fallbacks": int(n_fb), "fields": len(xs),
            "cr_online": total / stream_bytes(po),
            "cr_learned": total / stream_bytes(pl),
            "queue_online_tune_compress_GBps": total / t_on / 1e9,
            "queue_learned_tune_compress_GBps": total / t_le / 1e9}


if __name__ == "__main__":
    main()
