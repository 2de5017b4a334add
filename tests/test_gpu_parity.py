"""GPU parity: the gfx950 library against the CPU oracle, through the C ABI.

Streams and decompressed fields must be identical byte for byte; metrics
agree within 1e-9 relative; tuner decisions agree unless the oracle's own
margin is a near-tie (1e-9 relative)."""
import math

import numpy as np
import pytest

from paper_2310_14133_amd import fields
from parity_helpers import check_trace, near_tie, to_ref_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def codec():
    import torch
    import paper_2310_14133_amd as q
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = q.Codec(0)
    yield c
    c.close()


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def qparams(q, ref_p, ndim):
    """Same parameters in the library's struct."""
    p = q.Params()
    p.anchor_stride = ref_p.anchor_stride
    for l in range(16):
        p.interp[l] = ref_p.interp[l]
        for j in range(3):
            p.order[l][j] = ref_p.order[l][j]
    p.alpha, p.beta = ref_p.alpha, ref_p.beta
    return p


def roundtrip_check(codec, ref, x, e, rp):
    import paper_2310_14133_amd as q
    print(f"case shape={x.shape} e={e:.3g}", flush=True)
    xt = to_dev(x)
    z = codec.compress(xt, e, qparams(q, rp, x.ndim))
    y = codec.decompress(z)
    zr = ref.compress(x, e, rp)
    zg = z.cpu().numpy()
    assert zg.size == zr.size, (zg.size, zr.size)
    if not np.array_equal(zg, zr):
        diff = np.nonzero(zg != zr)[0]
        raise AssertionError(f"stream differs at {diff.size} bytes, first "
                             f"{diff[:8]}")
    yr = ref.decompress(zr)
    yg = y.cpu().numpy()
    assert np.array_equal(yg.view(np.uint32), yr.view(np.uint32))
    assert np.abs(x.astype(np.float64) - yr).max() <= e
    return zg


def test_cfg1_bumps_256_bitexact(codec, ref):
    """Plain method, 2D 256x256, cubic, alpha = beta = 1, order (0,1)."""
    x = fields.bumps_and_waves(256, seed=1)
    e = 1e-3 * (float(x.max()) - float(x.min()))
    rp = ref.make_params(2, "cubic", (0, 1), 1.0, 1.0)
    roundtrip_check(codec, ref, x, e, rp)


CASES = [
    ("2d_ragged", lambda: fields.grf((70, 45), 5), 1e-3, 16, "cubic",
     [(1, 0), (0, 1)] * 8, 1.5, 3.0),
    ("2d_linear", lambda: fields.bumps_and_waves(130, 2), 1e-4, 64,
     "linear", None, 1.25, 2.0),
    ("3d_ragged", lambda: fields.grf((19, 24, 33), 6), 1e-3, 8, "cubic",
     [(2, 0, 1), (1, 2, 0), (0, 1, 2)] * 6, 2.0, 4.0),
    ("3d_lognormal", lambda: fields.grf((40, 41, 42), 7, log_normal=True),
     1e-2, 32, "cubic", [(2, 1, 0)] * 16, 1.75, 3.0),
    ("3d_mixed", lambda: fields.multiscale((33, 65, 17), 8), 1e-5, 16,
     ["linear", "cubic"] * 8, [(0, 2, 1), (1, 0, 2)] * 8, 1.0, 1.5),
    ("spikes", lambda: fields.adversarial((60, 70), "spikes", 4), 1e-3, 16,
     "cubic", None, 1.5, 2.0),
    ("noise_tight", lambda: fields.adversarial((31, 33, 35), "noise", 5),
     1e-5, 8, "cubic", None, 1.0, 1.5),
    ("steps", lambda: fields.adversarial((17, 18, 19), "steps", 2), 1e-3, 4,
     "linear", None, 1.25, 1.5),
    ("alternating", lambda: fields.adversarial((25, 26), "alternating", 3),
     1e-2, 8, "cubic", None, 2.0, 2.0),
    ("zero", lambda: np.zeros((40, 41), np.float32), None, 16, "cubic",
     None, 1.0, 1.5),
    ("tiny2d", lambda: fields.grf((2, 3), 9), 1e-2, 2, "cubic", None, 1.0,
     1.5),
    ("tiny3d", lambda: fields.grf((2, 2, 5), 10), 1e-2, 4, "linear", None,
     1.0, 1.5),
    ("multi_chunk", lambda: fields.grf((3, 2500, 7), 11), 1e-4, 8, "cubic",
     None, 1.25, 3.0),
    # anchor-less level structure (only the origin is an anchor)
    ("anchorless_3d", lambda: fields.grf((40, 36, 44), 12), 1e-3, 64,
     "cubic", None, 1.0, 1.5),
    ("anchorless_2d", lambda: fields.grf((70, 45), 13), 1e-3, 128, "linear",
     None, 1.5, 2.0),
    # zero-word packed payloads (stream format 5)
    ("packed_2d", lambda: fields.bumps_and_waves(160, 2), 1e-2, 64, "cubic",
     None, 1.0, 1.5),
    ("packed_3d", lambda: fields.multiscale((48, 40, 56), 14), 1e-2, 16,
     "linear", None, 1.25, 2.0),
    # about 4700 used symbols: the second, larger device sort
    ("noise_big_sort", lambda: np.random.default_rng(5).normal(
        size=(48, 40, 44)).astype(np.float32), 1e-4, 8, "cubic", None, 1.0,
     1.5),
]


@pytest.mark.parametrize("name,make,rel,s,interp,order,alpha,beta", CASES)
def test_stream_bitexact(codec, ref, name, make, rel, s, interp, order,
                         alpha, beta):
    x = make()
    vr = float(x.max()) - float(x.min())
    e = rel * vr if rel else 0.5
    rp = ref.make_params(x.ndim, interp, order, alpha, beta, anchor_stride=s)
    roundtrip_check(codec, ref, x, e, rp)


# Every level-1 dimension order: with the contiguous dimension last the
# level-1 pass takes all three sweeps in one launch (tiles of rows along the
# middle sweep's dimension with recomputed neighbour rows, 512-point spans);
# the shapes give several tiles per row set, several spans per row and
# ragged ends of both.
L1_ORDERS = [(0, 1, 2), (1, 0, 2), (0, 2, 1), (1, 2, 0), (2, 0, 1),
             (2, 1, 0)]


@pytest.mark.parametrize("interp", ["cubic", "linear"])
@pytest.mark.parametrize("order", L1_ORDERS)
def test_level1_orders(codec, ref, order, interp):
    x = fields.grf((21, 38, 1100), 30 + L1_ORDERS.index(order))
    e = 1e-3 * (float(x.max()) - float(x.min()))
    rp = ref.make_params(3, interp, [order] + [(0, 1, 2)] * 15, 1.5, 2.0,
                         anchor_stride=8)
    roundtrip_check(codec, ref, x, e, rp)


@pytest.mark.parametrize("order", [(0, 1), (1, 0)])
def test_level1_orders_2d(codec, ref, order):
    x = fields.grf((67, 1300), 40)
    e = 1e-4 * (float(x.max()) - float(x.min()))
    rp = ref.make_params(2, "cubic", [order] + [(0, 1)] * 15, 1.25, 3.0,
                         anchor_stride=16)
    roundtrip_check(codec, ref, x, e, rp)


def test_gpu_decodes_oracle_stream(codec, ref):
    x = fields.grf((50, 60, 30), 12)
    e = 1e-4 * (float(x.max()) - float(x.min()))
    rp = ref.make_params(3, "cubic", None, 1.5, 3.0)
    zr = ref.compress(x, e, rp)
    import torch
    y = codec.decompress(torch.from_numpy(zr).cuda())
    assert np.array_equal(y.cpu().numpy(), ref.decompress(zr))


def test_deterministic(codec, ref):
    import paper_2310_14133_amd as q
    x = fields.grf((64, 64, 64), 13)
    e = 1e-3 * (float(x.max()) - float(x.min()))
    p = q.make_params(3, "cubic", None, 1.25, 2.0)
    xt = to_dev(x)
    a = codec.compress(xt, e, p).cpu().numpy()
    b = codec.compress(xt, e, p).cpu().numpy()
    assert np.array_equal(a, b)


def test_errors(codec, ref):
    import torch
    import paper_2310_14133_amd as q
    x = fields.grf((32, 32), 14)
    bad = x.copy()
    bad[5, 5] = np.nan
    p = q.make_params(2)
    with pytest.raises(q.QozError) as ei:
        codec.compress(to_dev(bad), 0.1, p)
    assert ei.value.status == q.QOZ_EINVAL
    with pytest.raises(q.QozError) as ei:
        codec.compress(to_dev(x), -1.0, p)
    assert ei.value.status == q.QOZ_EINVAL
    z = codec.compress(to_dev(x), 1e-3, p)
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(q.QozError) as ei:
        codec.compress_into(to_dev(x), 1e-3, p, small)
    assert ei.value.status == q.QOZ_ENOSPACE and ei.value.needed == z.numel()
    zc = z.clone()
    zc[0] ^= 0xFF
    with pytest.raises(q.QozError) as ei:
        codec.decompress(zc)
    assert ei.value.status == q.QOZ_EFORMAT
    # a corrupted payload word: the decoder either reports EFORMAT or
    # decodes exactly what the oracle decodes from the same bytes
    zn = z.cpu().numpy().copy()
    lay_n_words = int(np.frombuffer(zn[176:184].tobytes(), np.uint64)[0])
    assert lay_n_words > 0
    for flip_at in (-4, -8, -1):
        bad = zn.copy()
        bad[flip_at] ^= 0xA5
        print(f"corrupted payload byte {flip_at}", flush=True)
        out = torch.empty((32, 32), dtype=torch.float32, device="cuda")
        try:
            codec.decompress(torch.from_numpy(bad).cuda(), out=out)
        except q.QozError as err:
            assert err.status == q.QOZ_EFORMAT, err.status
            continue
        assert ref.decompress_status(bad) == ref.OK
        assert np.array_equal(out.cpu().numpy().view(np.uint32),
                              ref.decompress(bad).view(np.uint32))


def test_metrics_parity(codec, ref):
    for shape in [(200, 150), (40, 50, 60), (5, 30)]:
        x = fields.grf(shape, 15)
        y = (x + np.random.default_rng(0).normal(0, 1e-2, shape)).astype(
            np.float32)
        ps, ss, me = codec.metrics(to_dev(x), to_dev(y))
        pr, sr, mr = ref.metrics(x, y)
        assert abs(ps - pr) <= 1e-9 * abs(pr)
        assert abs(ss - sr) <= 1e-9 * abs(sr)
        assert me == mr


def test_error_ac_parity(codec, ref):
    # several rows per workgroup (3000 rows), rows of two points, errors
    # with and without lag-1 structure, and a real reconstruction
    rng = np.random.default_rng(4)
    cases = []
    for shape in [(200, 150), (40, 50, 60), (5, 30), (3000, 20), (64, 2),
                  (2, 333)]:
        x = fields.grf(shape, 16) if min(shape) > 2 else \
            rng.normal(size=shape).astype(np.float32)
        white = rng.normal(0, 1e-2, shape)
        smooth = np.cumsum(white, axis=-1) * 0.1
        cases.append((x, (x + white).astype(np.float32)))
        cases.append((x, (x + smooth).astype(np.float32)))
    x = fields.bumps_and_waves(128, 5)
    e = 1e-2 * (float(x.max()) - float(x.min()))
    p = ref.make_params(2, "cubic", (0, 1), 1.0, 1.0)
    cases.append((x, ref.decompress(ref.compress(x, e, p))))
    cases.append((x, x.copy()))  # no error at all: AC = 0
    for x, y in cases:
        print(f"error_ac shape={x.shape}", flush=True)
        g = codec.error_ac(to_dev(x), to_dev(np.ascontiguousarray(y)))
        r = ref.error_ac(x, y)
        assert abs(g - r) <= 1e-9, (x.shape, g, r)


TUNE_CASES = [
    ("2d_psnr_switch", lambda: fields.bumps_and_waves(128, 5), 32,
     dict(block=32, sample_rate=0.2), "psnr", 1e-2),
    ("2d_ssim", lambda: fields.bumps_and_waves(128, 5), 32,
     dict(block=32, sample_rate=0.2), "ssim", 1e-2),
    ("2d_cr", lambda: fields.bumps_and_waves(128, 5), 32,
     dict(block=32, sample_rate=0.2), "cr", 1e-3),
    ("3d_psnr_all", lambda: fields.grf((40, 36, 44), 32, log_normal=True),
     8, dict(block=8, sample_rate=0.2, all_orders=1), "psnr", 1e-3),
    ("3d_cr_all", lambda: fields.grf((36, 36, 36), 34), 8,
     dict(block=8, sample_rate=0.15, all_orders=1), "cr", 1e-4),
    ("3d_ssim", lambda: fields.multiscale((30, 34, 38), 33), 8,
     dict(block=8, sample_rate=0.2), "ssim", 1e-2),
    ("3d_default", lambda: fields.grf((96, 100, 90), 35), 0, {}, "psnr",
     1e-3),
    ("2d_ac", lambda: fields.bumps_and_waves(128, 5), 32,
     dict(block=32, sample_rate=0.2), "ac", 1e-2),
    ("3d_ac_all", lambda: fields.grf((36, 36, 36), 34), 8,
     dict(block=8, sample_rate=0.15, all_orders=1), "ac", 1e-3),
    # trials with thousands of used symbols (second device sort) and with
    # more than the device sorts hold (whole histograms)
    ("3d_noise_many_symbols", lambda: np.random.default_rng(7).normal(
        size=(48, 40, 44)).astype(np.float32), 16,
     dict(block=16, sample_rate=0.5), "psnr", 3e-5),
    ("3d_noise_huge_alphabet", lambda: np.random.default_rng(8).normal(
        size=(48, 40, 44)).astype(np.float32), 16,
     dict(block=16, sample_rate=0.5), "psnr", 4e-6),
]


@pytest.mark.parametrize("name,make,s,cfgkw,target,rel", TUNE_CASES)
def test_tune_parity(codec, ref, name, make, s, cfgkw, target, rel):
    """Tuner decisions and every intermediate value of the tuning (trace)
    against the oracle; the GPU's own parameters then give the oracle's
    stream."""
    import paper_2310_14133_amd as q
    x = make()
    e = rel * (float(x.max()) - float(x.min()))
    print(f"tune case {name} shape={x.shape}", flush=True)
    rp, tr = ref.tune(x, e, target, ref.tune_config(**cfgkw),
                      anchor_stride=s)
    gp, gt = codec.tune_traced(to_dev(x), e, target,
                               q.make_tune_config(**cfgkw), anchor_stride=s)
    d = x.ndim
    note = check_trace(gt, tr, target)
    if note is None:
        assert q.params_dict(gp, d) == ref.params_to_dict(rp, d)
    else:
        print(f"  {note}: the walks part there", flush=True)
    # the GPU's parameters through both encoders
    roundtrip_check(codec, ref, x, e, to_ref_params(ref, gp, d))


@pytest.mark.parametrize("shape,s,rel", [((40, 41, 42), 8, 1e-3),
                                         ((130, 129), 16, 1e-4),
                                         ((3, 200, 70), 32, 1e-2)])
def test_autotuned_tiles_keep_streams(codec, ref, shape, s, rel):
    # any launch tile gives the same bins: streams still equal the oracle's
    import paper_2310_14133_amd as q
    x = fields.grf(shape, 61)
    e = rel * (float(x.max()) - float(x.min()))
    rp = ref.make_params(x.ndim, "cubic", None, 1.25, 2.0, anchor_stride=s)
    n, t_def, t_best = codec.autotune_tiles(x.shape, qparams(q, rp, x.ndim))
    print(f"autotuned {n} sweeps for {shape}: {t_def:.4f} -> {t_best:.4f} ms",
          flush=True)
    assert n >= 1 and 0.0 < t_best <= t_def
    roundtrip_check(codec, ref, x, e, rp)


def test_packed_stream_corruption(codec, ref):
    import paper_2310_14133_amd as q
    x = fields.bumps_and_waves(160, 2)
    e = 1e-2 * (float(x.max()) - float(x.min()))
    rp = ref.make_params(2, "cubic", None, 1.0, 1.5, anchor_stride=64)
    z = ref.compress(x, e, rp)
    assert int(np.frombuffer(z[4:6].tobytes(), np.uint16)[0]) == 5
    y = codec.decompress(to_dev(z))
    assert np.array_equal(y.cpu().numpy().view(np.uint32),
                          ref.decompress(z).view(np.uint32))
    wp = int(np.frombuffer(z[196:200].tobytes(), np.uint32)[0])
    n_chunks = int(np.frombuffer(z[168:176].tobytes(), np.uint64)[0])
    pc_at = z.size - 8 * (n_chunks + 1)
    for name, at, val in [("offset past the payload", pc_at + 8, wp + 9),
                          ("first offset not zero", pc_at, 1)]:
        bad = z.copy()
        bad[at:at + 8] = np.frombuffer(np.array([val], np.uint64).tobytes(),
                                       np.uint8)
        print(f"packed corruption: {name}", flush=True)
        assert ref.decompress_status(bad) == ref.EFORMAT
        with pytest.raises(q.QozError) as err:
            codec.decompress(to_dev(bad))
        assert err.value.status == q.QOZ_EFORMAT


ABLATION_CASES = [
    ("2d_levelwise", lambda: fields.grf((80, 90), 31), 16,
     dict(block=16, sample_rate=0.1), "psnr", 1e-3, 2),
    ("3d_all_levelwise", lambda: fields.grf((40, 36, 44), 32,
                                           log_normal=True), 8,
     dict(block=8, sample_rate=0.2, all_orders=1), "psnr", 1e-3, 2),
    ("3d_no_ab", lambda: fields.grf((40, 36, 44), 32), 8,
     dict(block=8, sample_rate=0.2), "ssim", 1e-3, 1),
    # the anchor-less structure with neither switch's part: the baseline
    ("3d_sz3_like", lambda: fields.grf((40, 36, 44), 33), 64,
     dict(block=16, sample_rate=0.3), "cr", 1e-3, 3),
]


@pytest.mark.parametrize("name,make,s,cfgkw,target,rel,abl", ABLATION_CASES)
def test_tune_ablation_parity(codec, ref, name, make, s, cfgkw, target, rel,
                              abl):
    import paper_2310_14133_amd as q
    x = make()
    e = rel * (float(x.max()) - float(x.min()))
    print(f"ablation case {name} switches {abl}", flush=True)
    rp, tr = ref.tune(x, e, target, ref.tune_config(**cfgkw, ablation=abl),
                      anchor_stride=s)
    gp = codec.tune(to_dev(x), e, target,
                    q.make_tune_config(**cfgkw, ablation=abl),
                    anchor_stride=s)
    d = x.ndim
    if not abl & 2:
        for l in range(tr.Lt, 0, -1):
            errs = [tr.alg1_err[l - 1][c] for c in range(tr.ncand)]
            if near_tie(errs, tr.alg1_choice[l - 1]):
                pytest.skip(f"near tie in Algorithm 1 at level {l}")
    if not abl & 1:
        Ms = [tr.M[i] for i in range(20)]
        if near_tie(Ms, tr.best_pair, 1e-7):
            pytest.skip("near tie in the (alpha, beta) walk")
    assert q.params_dict(gp, d) == ref.params_to_dict(rp, d)
    if abl & 1:
        assert (gp.alpha, gp.beta) == (1.0, 1.5)
    if abl & 2:
        assert len({(gp.interp[l], tuple(gp.order[l][j] for j in range(d)))
                    for l in range(gp.levels)}) == 1
    roundtrip_check(codec, ref, x, e, rp)


def test_tune_ablation_rejects_unknown(codec):
    import paper_2310_14133_amd as q
    x = to_dev(fields.grf((40, 40), 3))
    with pytest.raises(q.QozError) as err:
        codec.tune(x, 1e-3, "cr", q.make_tune_config(ablation=4))
    assert err.value.status == q.QOZ_EINVAL


@pytest.mark.parametrize("n_syms", [12, 28])
def test_long_codes_bitexact(codec, ref, n_syms):
    """Fibonacci-distributed bins: codes longer than the decoder's tables
    (up to 26 bits) go through the canonical-limit path."""
    n0, n1 = 1025, 1025
    n_t = (n0 // 2) * (n1 // 2 + 1) + n0 * (n1 // 2)
    x = fields.bins_field(fields.fibonacci_bins(n_t, n_syms, seed=5), n0, n1)
    rp = ref.make_params(2, "linear", (0, 1), 1.0, 1.0, anchor_stride=2)
    roundtrip_check(codec, ref, x, 0.5, rp)
