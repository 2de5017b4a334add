"""Training and evaluation of the learned tuner's network.

Labels are the online tuner's own choices (qoz_tune, PSNR target, the
sampling of Sec. VI-A with b = 32 and r = 1 %) on synthetic fields; the
inputs are qoz_learned_features of the same fields at the same bounds; the
network is trained with the library's forward / backward / Adam kernels
(qoz_mlp_train_step).  torch only holds device memory and index lists.

Bounds follow PSNR targets: a uniform error on [-e, e] has RMS e / sqrt(3),
so PSNR = 20 log10(range / RMS) gives e = sqrt(3) range 10^(-PSNR / 20).

    python -m paper_2310_14133_amd.learned train --fields 10000 --out W.bin
    python -m paper_2310_14133_amd.learned eval --weights W.bin --n 512
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
MAGIC = b"QMLP"
PSNR_TARGETS = (60.0, 80.0, 100.0)
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


def build_dataset(codec, seeds, log_every=25):
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
        x, _ = fields.tuner_training_field(seed)
        vr = float((x.max() - x.min()).item())
        for P in PSNR_TARGETS:
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


def evaluate(codec, P, seeds, n, confidences=(0.0, 0.5)):
    """Per held-out field and PSNR target: tuning time, ratio and PSNR of
    the online tuner's and the network's parameters."""
    import paper_2310_14133_amd as q
    from paper_2310_14133_amd import fields
    cfg_t = q.make_tune_config(block=32, sample_rate=SAMPLE_RATE)
    rows = []
    for seed in seeds:
        x, rec = fields.tuner_training_field(seed, shape=(n, n, n))
        vr = float((x.max() - x.min()).item())
        raw = x.numel() * 4
        for target in PSNR_TARGETS:
            e = bound_for_psnr(vr, target)

            def quality(p):
                z = codec.compress(x, e, p)
                y = codec.decompress(z)
                ps, _, me = codec.metrics(x, y, want_ssim=False)
                assert me <= e
                return raw / z.numel(), ps

            pe, te = _timed(lambda: codec.tune(x, e, "psnr", cfg_t))
            cr_e, ps_e = quality(pe)
            row = {"seed": seed, "psnr_target": target, "slope": rec["slope"],
                   "noise": rec["noise"], "exhaustive_ms": te,
                   "exhaustive": [pe.interp[0], pe.alpha, pe.beta],
                   "cr_exhaustive": cr_e, "psnr_exhaustive": ps_e}
            for c in confidences:
                (pl, fb), tl = _timed(lambda: codec.tune_learned(
                    x, e, P, c, "psnr", cfg_t))
                cr_l, ps_l = quality(pl)
                # equal-PSNR ratio: 6.02 dB per bit per value
                bits_eq = 32.0 / cr_l + (ps_e - ps_l) / 6.02
                row[f"c{c}"] = {"ms": tl, "fallback": fb,
                                "choice": [pl.interp[0], pl.alpha, pl.beta],
                                "cr": cr_l, "psnr": ps_l,
                                "cr_equal_psnr": 32.0 / bits_eq}
            rows.append(row)
            print("eval:", json.dumps(row), flush=True)
        del x
    summary = {}
    for c in confidences:
        k = f"c{c}"
        sp = [r["exhaustive_ms"] / r[k]["ms"] for r in rows]
        summary[k] = {
            "speedup_geomean": float(np.exp(np.mean(np.log(sp)))),
            "learned_ms_mean": float(np.mean([r[k]["ms"] for r in rows])),
            "exhaustive_ms_mean": float(np.mean([r["exhaustive_ms"]
                                                 for r in rows])),
            "fallback_rate": float(np.mean([r[k]["fallback"] for r in rows])),
            "cr_ratio_mean": float(np.mean([r[k]["cr"] / r["cr_exhaustive"]
                                            for r in rows])),
            "cr_equal_psnr_ratio_mean": float(np.mean(
                [r[k]["cr_equal_psnr"] / r["cr_exhaustive"] for r in rows])),
            "psnr_diff_mean": float(np.mean([r[k]["psnr"] -
                                             r["psnr_exhaustive"]
                                             for r in rows])),
            "choice_match": float(np.mean([r[k]["choice"] == r["exhaustive"]
                                           for r in rows])),
        }
    return rows, summary


def main(argv=None):
    import torch
    import paper_2310_14133_amd as q
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("train")
    a.add_argument("--fields", type=int, default=10000)
    a.add_argument("--seed0", type=int, default=10000)
    a.add_argument("--epochs", type=int, default=200)
    a.add_argument("--out", default=DEFAULT_WEIGHTS)
    a.add_argument("--report", default="")
    b = sub.add_parser("eval")
    b.add_argument("--weights", default=DEFAULT_WEIGHTS)
    b.add_argument("--fields", type=int, default=16)
    b.add_argument("--seed0", type=int, default=20000)
    b.add_argument("--n", type=int, default=512)
    b.add_argument("--report", default="")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the learned tuner runs on the GPU")
    codec = q.Codec(0)
    if args.cmd == "train":
        seeds = list(range(args.seed0, args.seed0 + args.fields))
        t0 = time.time()
        F, Y = build_dataset(codec, seeds)
        t_data = time.time() - t0
        print(f"dataset: {F.shape[0]} rows in {t_data:.1f} s; label counts "
              f"interp {np.bincount(Y[:, 0].cpu().numpy(), minlength=2)} "
              f"alpha {np.bincount(Y[:, 1].cpu().numpy(), minlength=5)} "
              f"beta {np.bincount(Y[:, 2].cpu().numpy(), minlength=4)}",
              flush=True)
        t1 = time.time()
        P, rep = train(codec, F, Y, epochs=args.epochs)
        torch.cuda.synchronize()
        rep.update({"fields": args.fields, "rows": int(F.shape[0]),
                    "dataset_seconds": t_data,
                    "train_seconds": time.time() - t1})
        save_weights(args.out, P.cpu().numpy())
        print("train done:", json.dumps({k: v for k, v in rep.items()
                                         if k != "log"}), flush=True)
        if args.report:
            with open(args.report, "w") as f:
                json.dump(rep, f, indent=1)
    else:
        P = load_weights(args.weights)
        seeds = list(range(args.seed0, args.seed0 + args.fields))
        rows, summary = evaluate(codec, P, seeds, args.n)
        print("eval summary:", json.dumps(summary), flush=True)
        if args.report:
            with open(args.report, "w") as f:
                json.dump({"n": args.n, "rows": rows, "summary": summary}, f,
                          indent=1)
    codec.close()


if __name__ == "__main__":
    main()
