"""Training and evaluation of the learned tuner's networks (one for 3D
fields, one for 2D fields).

Labels are the online tuner's own choices (qoz_tune, PSNR target, the
sampling of Sec. VI-A with b = 32 and r = 1 %) on synthetic fields; the
inputs are qoz_learned_features of the same fields at the same bounds; the
networks are trained with the library's forward / backward / Adam kernels
(qoz_mlp_train_step).  torch only holds device memory and index lists.

Training fields (fields.tuner_field): k^slope random fields with noise,
their skewed exponentials and multiscale fields, 3D shapes 64^3..256^3 and
2D shapes 256^2..2048^2; PSNR targets 40..100 dB.  Bounds follow PSNR
targets: a uniform error on [-e, e] has RMS e / sqrt(3), so
PSNR = 20 log10(range / RMS) gives e = sqrt(3) range 10^(-PSNR / 20).

Evaluation compares the network's parameters with the online tuner's at
equal PSNR: for each tuner, the bound is bisected (on the whole field,
each step tuning at that bound, compressing and decompressing) until the
final PSNR is at least the target and within 0.05 dB of it; the ratios at
those bounds are compared, with the tuning times and the fallback rate.

    python -m paper_2310_14133_amd.learned train --ndim 3 --fields 6000
    python -m paper_2310_14133_amd.learned eval --ndim 3 --n 512
"""
import argparse
import json
import math
import os
import struct
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "tuner_mlp.bin")
WEIGHTS = {3: DEFAULT_WEIGHTS, 2: os.path.join(HERE, "tuner_mlp_2d.bin")}
MAGIC = b"QMLP"
PSNR_TARGETS = (60.0, 80.0, 100.0)   # evaluation targets
TRAIN_PSNR = (40.0, 50.0, 60.0, 70.0, 80.0, 90.0, 100.0)
SAMPLE_RATE = 0.01
NPARAM, NFEAT = 22219, 32
OFF_W1 = 64
HIDDEN, NOUT = 128, 11


def bound_for_psnr(vrange, psnr):
    return math.sqrt(3.0) * vrange * 10.0 ** (-psnr / 20.0)


def save_weights(path, P):
    P = np.asarray(P, np.float32)
    assert P.size == NPARAM
    with open(path + ".tmp", "wb") as f:
        f.write(MAGIC + struct.pack("<III", 1, NPARAM, 0))
        f.write(P.tobytes())
    os.replace(path + ".tmp", path)


def load_weights(path=None, device="cuda"):
    """The parameter blob as a float32 tensor on `device`."""
    import torch
    path = path or DEFAULT_WEIGHTS
    with open(path, "rb") as f:
        head = f.read(16)
        if head[:4] != MAGIC:
            raise ValueError(f"{path}: not a tuner network file")
        ver, n, _ = struct.unpack("<III", head[4:])
        if ver != 1 or n != NPARAM:
            raise ValueError(f"{path}: version {ver}, {n} parameters")
        P = np.frombuffer(f.read(4 * n), np.float32).copy()
    return torch.from_numpy(P).to(device)


def init_params(seed, mu, sg):
    """He-style initial weights, zero biases; input shift and scale given."""
    rng = np.random.default_rng(seed)
    P = np.zeros(NPARAM, np.float32)
    P[0:32] = mu
    P[32:64] = sg
    o = OFF_W1
    P[o:o + HIDDEN * NFEAT] = rng.normal(0, math.sqrt(2 / NFEAT),
                                         HIDDEN * NFEAT)
    o += HIDDEN * NFEAT + HIDDEN
    P[o:o + HIDDEN * HIDDEN] = rng.normal(0, math.sqrt(2 / HIDDEN),
                                          HIDDEN * HIDDEN)
    o += HIDDEN * HIDDEN + HIDDEN
    P[o:o + NOUT * HIDDEN] = rng.normal(0, math.sqrt(1 / HIDDEN),
                                        NOUT * HIDDEN)
    return P


def label_of(q, p):
    return (int(p.interp[0]), q.ALPHAS.index(p.alpha), q.BETAS.index(p.beta))


def build_dataset(codec, seeds, ndim=3, targets=TRAIN_PSNR, log_every=250):
    """Features (N x 32) and labels (N x 3) on the device, one row per
    (field, PSNR target)."""
    import torch
    import paper_2310_14133_amd as q
    from paper_2310_14133_amd import fields
    cfg_f = q.make_tune_config(sample_rate=SAMPLE_RATE)
    cfg_t = q.make_tune_config(block=32, sample_rate=SAMPLE_RATE)
    feats, labels = [], []
    t0 = time.time()
    for i, seed in enumerate(seeds):
        x, _ = fields.tuner_field(seed, ndim)
        vr = float((x.max() - x.min()).item())
        for P in targets:
            e = bound_for_psnr(vr, P)
            feats.append(codec.learned_features(x, e, cfg_f))
            labels.append(label_of(q, codec.tune(x, e, "psnr", cfg_t)))
        del x
        if (i + 1) % log_every == 0 or i < 3:
            print(f"dataset: {i + 1}/{len(seeds)} fields, "
                  f"{time.time() - t0:.1f} s", flush=True)
    F = torch.stack(feats).contiguous()
    Y = torch.tensor(labels, dtype=torch.int32, device=F.device)
    return F, Y


def label_entropy(Y):
    """Entropy (bits) of each head's labels."""
    y = np.asarray(Y)
    out = []
    for h, k in enumerate((2, 5, 4)):
        c = np.bincount(y[:, h], minlength=k).astype(np.float64)
        p = c[c > 0] / c.sum()
        out.append(float(-(p * np.log2(p)).sum()))
    return out


def accuracy(codec, P, F, Y, rows):
    import torch
    idx = torch.as_tensor(rows, device=F.device, dtype=torch.long)
    z = codec.mlp_forward(P, F[idx].contiguous()).cpu().numpy()
    y = Y[idx].cpu().numpy()
    acc = []
    o = 0
    for h, k in enumerate((2, 5, 4)):
        acc.append(float(np.mean(np.argmax(z[:, o:o + k], 1) == y[:, h])))
        o += k
    return acc


def train(codec, F, Y, epochs=200, batch=256, lr0=2e-3, seed=0,
          val_frac=0.1, log_every=20):
    """Adam on the library's kernels; returns the blob with the lowest
    validation loss and a log."""
    import torch
    N = F.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(N)
    nval = max(1, int(N * val_frac))
    val, tr = perm[:nval], perm[nval:]
    Fh = F.cpu().numpy().astype(np.float64)
    mu = Fh[tr].mean(axis=0).astype(np.float32)
    sg = np.maximum(Fh[tr].std(axis=0), 1e-3).astype(np.float32)
    P = torch.from_numpy(init_params(seed, mu, sg)).to(F.device)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    val_idx = torch.from_numpy(val.astype(np.int32)).to(F.device)
    steps_per = max(1, len(tr) // batch)
    total = epochs * steps_per
    best = (float("inf"), P.clone(), -1)
    t = 0
    log = []
    t0 = time.time()
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(tr).astype(np.int32)).to(
            F.device)
        for k in range(steps_per):
            t += 1
            lr = lr0 * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * t / total)))
            codec.mlp_train_step(P, m, v, F, Y, order[k * batch:(k + 1) * batch],
                                 lr, t)
        _, vl = codec.mlp_grad(P, F, Y, val_idx)
        vl = float(vl.item())
        if vl < best[0]:
            best = (vl, P.clone(), ep)
        if (ep + 1) % log_every == 0 or ep == epochs - 1:
            _, tl = codec.mlp_grad(P, F, Y,
                                   torch.from_numpy(tr[:4096].astype(
                                       np.int32)).to(F.device))
            entry = {"epoch": ep + 1, "train_loss": float(tl.item()),
                     "val_loss": vl, "val_acc": accuracy(codec, P, F, Y, val),
                     "seconds": round(time.time() - t0, 2)}
            log.append(entry)
            print("train:", json.dumps(entry), flush=True)
    Pbest = best[1]
    return Pbest, {"best_epoch": best[2] + 1, "best_val_loss": best[0],
                   "val_acc": accuracy(codec, Pbest, F, Y, val),
                   "n_train": int(len(tr)), "n_val": int(nval),
                   "steps": t, "log": log}


def _timed(fn, reps=3):
    import torch
    fn()
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return out, best * 1e3


def equal_psnr(codec, x, target, tune, tol=0.05, max_steps=40):
    """Bisect the bound until the final PSNR of x under tune(e) is at least
    `target` and within `tol` dB of it (or the steps run out: then the last
    bound meeting the target).  Returns (ratio, psnr, bound, steps)."""
    vr = float((x.max() - x.min()).item())
    raw = x.numel() * 4
    memo = {}

    def run(e):
        if e not in memo:
            p = tune(e)
            z = codec.compress(x, e, p)
            y = codec.decompress(z)
            ps, _, me = codec.metrics(x, y, want_ssim=False)
            assert me <= e
            memo[e] = (raw / z.numel(), ps)
        return memo[e]

    e0 = bound_for_psnr(vr, target)
    lo, hi = e0, e0
    while run(lo)[1] < target:
        lo /= 2.0
    while run(hi)[1] >= target:
        hi *= 2.0
    steps = 0
    while run(lo)[1] - target > tol and steps < max_steps:
        mid = math.sqrt(lo * hi)
        if run(mid)[1] >= target:
            lo = mid
        else:
            hi = mid
        steps += 1
    cr, ps = run(lo)
    return cr, ps, lo, len(memo)


def evaluate(codec, P, seeds, shape=None, ndim=3, targets=PSNR_TARGETS,
             confidences=(0.0, 0.5), kind=None):
    """Per held-out field and PSNR target: tuning time of the online tuner
    and of the network at the target's nominal bound, and the ratio of each
    at equal PSNR (bisection of the bound)."""
    import paper_2310_14133_amd as q
    from paper_2310_14133_amd import fields
    cfg_t = q.make_tune_config(block=32, sample_rate=SAMPLE_RATE)
    rows = []
    for seed in seeds:
        x, rec = fields.tuner_field(seed, ndim, shape=shape, kind=kind)
        vr = float((x.max() - x.min()).item())
        for target in targets:
            e = bound_for_psnr(vr, target)
            pe, te = _timed(lambda: codec.tune(x, e, "psnr", cfg_t))
            cr_e, ps_e, e_e, n_e = equal_psnr(
                codec, x, target,
                lambda b: codec.tune(x, b, "psnr", cfg_t))
            row = {"seed": seed, "psnr_target": target, "recipe": rec,
                   "exhaustive_ms": te,
                   "exhaustive": [pe.interp[0], pe.alpha, pe.beta],
                   "cr_exhaustive": cr_e, "psnr_exhaustive": ps_e,
                   "bound_exhaustive": e_e, "steps_exhaustive": n_e}
            for c in confidences:
                (pl, fb), tl = _timed(lambda: codec.tune_learned(
                    x, e, P, c, "psnr", cfg_t))
                cr_l, ps_l, e_l, n_l = equal_psnr(
                    codec, x, target,
                    lambda b: codec.tune_learned(x, b, P, c, "psnr",
                                                 cfg_t)[0])
                row[f"c{c}"] = {"ms": tl, "fallback": fb,
                                "choice": [pl.interp[0], pl.alpha, pl.beta],
                                "cr": cr_l, "psnr": ps_l, "bound": e_l,
                                "steps": n_l}
            rows.append(row)
            print("eval:", json.dumps(row), flush=True)
        del x
    return rows, summarize(rows, confidences)


def summarize(rows, confidences=(0.0, 0.5)):
    summary = {}
    for c in confidences:
        k = f"c{c}"
        sp = [r["exhaustive_ms"] / r[k]["ms"] for r in rows]
        crr = [r[k]["cr"] / r["cr_exhaustive"] for r in rows]
        summary[k] = {
            "speedup_geomean": float(np.exp(np.mean(np.log(sp)))),
            "learned_ms_mean": float(np.mean([r[k]["ms"] for r in rows])),
            "exhaustive_ms_mean": float(np.mean([r["exhaustive_ms"]
                                                 for r in rows])),
            "fallback_rate": float(np.mean([r[k]["fallback"] for r in rows])),
            "cr_ratio_mean_equal_psnr": float(np.mean(crr)),
            "cr_ratio_min_equal_psnr": float(np.min(crr)),
            "choice_match": float(np.mean([r[k]["choice"] == r["exhaustive"]
                                           for r in rows])),
        }
    return summary


def main(argv=None):
    import torch
    import paper_2310_14133_amd as q
    from paper_2310_14133_amd import fields
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("train")
    a.add_argument("--ndim", type=int, default=3, choices=(2, 3))
    a.add_argument("--fields", type=int, default=6000)
    a.add_argument("--seed0", type=int, default=10000)
    a.add_argument("--epochs", type=int, default=200)
    a.add_argument("--out", default="")
    a.add_argument("--report", default="")
    b = sub.add_parser("eval")
    b.add_argument("--ndim", type=int, default=3, choices=(2, 3))
    b.add_argument("--weights", default="")
    b.add_argument("--fields", type=int, default=16)
    b.add_argument("--seed0", type=int, default=20000)
    b.add_argument("--n", type=int, default=0,
                   help="edge of the held-out fields (0: the training "
                        "workload's random shapes)")
    b.add_argument("--kind", default=None, choices=fields.TUNER_KINDS,
                   help="one field family (default: the training mix)")
    b.add_argument("--report", default="")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the learned tuner runs on the GPU")
    codec = q.Codec(0)
    if args.cmd == "train":
        out = args.out or WEIGHTS[args.ndim]
        seeds = list(range(args.seed0, args.seed0 + args.fields))
        t0 = time.time()
        F, Y = build_dataset(codec, seeds, args.ndim)
        t_data = time.time() - t0
        Yh = Y.cpu().numpy()
        ent = label_entropy(Yh)
        print(f"dataset: {F.shape[0]} rows in {t_data:.1f} s; label counts "
              f"interp {np.bincount(Yh[:, 0], minlength=2)} "
              f"alpha {np.bincount(Yh[:, 1], minlength=5)} "
              f"beta {np.bincount(Yh[:, 2], minlength=4)}; label entropy "
              f"(bits) {[round(v, 3) for v in ent]}", flush=True)
        t1 = time.time()
        P, rep = train(codec, F, Y, epochs=args.epochs)
        torch.cuda.synchronize()
        rep.update({"ndim": args.ndim, "fields": args.fields,
                    "rows": int(F.shape[0]), "dataset_seconds": t_data,
                    "train_seconds": time.time() - t1,
                    "label_counts": [np.bincount(Yh[:, h], minlength=k)
                                     .tolist()
                                     for h, k in enumerate((2, 5, 4))],
                    "label_entropy_bits": ent})
        save_weights(out, P.cpu().numpy())
        print("train done:", json.dumps({k: v for k, v in rep.items()
                                         if k != "log"}), flush=True)
        if args.report:
            with open(args.report, "w") as f:
                json.dump(rep, f, indent=1)
    else:
        P = load_weights(args.weights or WEIGHTS[args.ndim])
        seeds = list(range(args.seed0, args.seed0 + args.fields))
        shape = (args.n,) * args.ndim if args.n else None
        rows, summary = evaluate(codec, P, seeds, shape, args.ndim,
                                 kind=args.kind)
        print("eval summary:", json.dumps(summary), flush=True)
        if args.report:
            with open(args.report, "w") as f:
                json.dump({"ndim": args.ndim, "n": args.n, "kind": args.kind,
                           "rows": rows, "summary": summary}, f, indent=1)
    codec.close()


if __name__ == "__main__":
    main()
