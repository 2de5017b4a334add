"""Effect of the zero-word packing stage on the ratio, on synthetic fields
from rough to smooth, at value-range-relative bounds 1e-2 and 1e-3 (fixed
parameters: cubic, alpha = 1, the paper's default anchor stride).

The unpacked size is re-derived from the stream's own header counts (the
layout with the raw payload); packing applies only when it saves at least
3 %, so a rough field's two sizes agree.

    python -m paper_2310_14133_amd.packing_study --report packing.json
"""
import argparse
import json
import sys

import numpy as np


def unpacked_size(z):
    """Bytes of the same stream with a raw payload (format 4)."""
    h = z[:200].cpu().numpy().tobytes()
    u64 = lambda o: int(np.frombuffer(h[o:o + 8], np.uint64)[0])
    al8 = lambda v: (v + 7) // 8 * 8
    n_anchor, n_unpred, n_used = u64(136), u64(152), u64(160)
    n_chunks, n_words = u64(168), u64(176)
    off = al8(200 + 4 * n_anchor)
    off = al8(off + 2 * n_used)
    off = al8(off + n_used)
    off = al8(off + 8 * (n_chunks + 1))
    off = al8(off + 4 * (n_chunks + 1))
    off = al8(off + 14 * n_chunks)
    off = al8(off + 4 * n_unpred)
    return off + 4 * n_words


def cases():
    from paper_2310_14133_amd import fields
    return [
        ("grf k^-3 512^3", lambda: fields.grf_torch((512,) * 3, 20)),
        ("grf k^-3 512^3 log-normal",
         lambda: fields.grf_torch((512,) * 3, 20, log_normal=True)),
        ("grf k^-4 256^3", lambda: fields.grf_torch((256,) * 3, 21,
                                                     slope=-4.0)),
        ("bumps + waves 2048^2", lambda: __import__("torch").from_numpy(
            fields.bumps_and_waves(2048, 2)).cuda()),
        ("multiscale 192^3", lambda: __import__("torch").from_numpy(
            fields.multiscale((192, 192, 192), 3)).cuda()),
    ]


def main(argv=None):
    import torch
    import paper_2310_14133_amd as q
    ap = argparse.ArgumentParser()
    ap.add_argument("--eps", type=float, nargs="+", default=[1e-2, 1e-3])
    ap.add_argument("--report", default="")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the study runs on the GPU")
    codec = q.Codec(0)
    rows = []
    for name, make in cases():
        x = make().contiguous()
        vr = float((x.max() - x.min()).item())
        for eps in args.eps:
            e = eps * vr
            p = q.make_params(x.dim(), "cubic", None, 1.0, 1.5)
            z = codec.compress(x, e, p)
            y = codec.decompress(z)
            ps, _, me = codec.metrics(x, y, want_ssim=False)
            assert me <= e
            raw = x.numel() * 4
            ver = int(z[4].item())
            row = {"field": name, "eps": eps, "version": ver,
                   "cr": raw / z.numel(), "cr_unpacked": raw / unpacked_size(z),
                   "bits_per_value": 8.0 * z.numel() / x.numel(), "psnr": ps}
            rows.append(row)
            print("packing:", json.dumps(row), flush=True)
        del x
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rows, f, indent=1)
    codec.close()


if __name__ == "__main__":
    main()
