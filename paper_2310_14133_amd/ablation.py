"""Component study of the method (the ablation of Sec. VII) on a synthetic
field: each variant adds one part of the tuner back.

  levels      anchor-less level structure (only the origin is an anchor),
              one interpolator for every level, alpha = 1
  +anchors    anchor grid of stride 32 (Sec. V-B), otherwise as above
  +levelwise  Algorithm 1's per-level interpolators (Sec. VI-B), alpha = 1
  full        plus the (alpha, beta) search of Table I (Sec. VI-C)

Each variant is tuned in PSNR mode on 32^3 blocks sampled at 1 %, then the
field is compressed and decompressed with its parameters; the line gives
bits per value and PSNR, the two axes of a rate-distortion plot.

    python -m paper_2310_14133_amd.ablation --n 512 --eps 1e-2 1e-3 1e-4
"""
import argparse
import json
import sys

VARIANTS = [
    ("levels", True, 3),
    ("+anchors", False, 3),
    ("+levelwise", False, 1),
    ("full", False, 0),
]


def run(codec, x, eps_list, target="psnr", log_normal=False):
    import paper_2310_14133_amd as q
    vr = float((x.max() - x.min()).item())
    raw = x.numel() * 4
    rows = []
    for eps in eps_list:
        e = eps * vr
        for name, anchorless, abl in VARIANTS:
            s = q.sz3_anchor_stride(tuple(x.shape)) if anchorless else 32
            cfg = q.make_tune_config(block=32, sample_rate=0.01,
                                     all_orders=1, ablation=abl)
            p = codec.tune(x, e, target, cfg, anchor_stride=s)
            z = codec.compress(x, e, p)
            y = codec.decompress(z)
            ps, _, me = codec.metrics(x, y, want_ssim=False)
            assert me <= e
            row = {"eps": eps, "variant": name, "anchor_stride": s,
                   "ablation": abl, "cr": raw / z.numel(),
                   "bits_per_value": 8.0 * z.numel() / x.numel(),
                   "psnr": ps, "params": q.params_dict(p, x.dim())}
            rows.append(row)
            print("ablation:", json.dumps(row), flush=True)
    return rows


def main(argv=None):
    import torch
    import paper_2310_14133_amd as q
    from paper_2310_14133_amd import fields
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--seed", type=int, default=20)
    ap.add_argument("--eps", type=float, nargs="+", default=[1e-2, 1e-3, 1e-4])
    ap.add_argument("--log-normal", action="store_true")
    ap.add_argument("--report", default="")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the study runs on the GPU")
    codec = q.Codec(0)
    x = fields.grf_torch((args.n,) * 3, args.seed, log_normal=args.log_normal)
    rows = run(codec, x, args.eps)
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"n": args.n, "seed": args.seed,
                       "log_normal": args.log_normal, "rows": rows}, f,
                      indent=1)
    codec.close()


if __name__ == "__main__":
    main()
