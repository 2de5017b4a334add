"""Batched compression and decompression through the C ABI: every field's
stream equals the oracle's (given parameters) or the single-field call's
(tuned), whatever the number of workers; a failing field fails alone."""
import numpy as np
import pytest

from paper_2310_14133_amd import fields

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


def batch_fields():
    out = []
    shapes = [(70, 45), (19, 24, 33), (40, 41, 42), (130, 129), (3, 200, 7),
              (33, 65, 17), (2, 3), (64, 64, 64), (9, 300)]
    for i, sh in enumerate(shapes):
        x = fields.grf(sh, 100 + i, log_normal=(i % 3 == 1))
        rel = [1e-2, 1e-3, 1e-4, 1e-5][i % 4]
        out.append((x, rel * (float(x.max()) - float(x.min()))))
    return out


def qparams(q, ref_p):
    p = q.Params()
    p.anchor_stride = ref_p.anchor_stride
    for l in range(16):
        p.interp[l] = ref_p.interp[l]
        for j in range(3):
            p.order[l][j] = ref_p.order[l][j]
    p.alpha, p.beta = ref_p.alpha, ref_p.beta
    return p


@pytest.mark.parametrize("workers", [1, 3, 8])
def test_batch_streams_equal_oracle(codec, ref, workers):
    import paper_2310_14133_amd as q
    fs = batch_fields()
    rng = np.random.default_rng(workers)
    rps = []
    for x, _ in fs:
        s = [4, 8, 16, 32][rng.integers(0, 4)]
        rps.append(ref.make_params(x.ndim, ["linear", "cubic"][
            rng.integers(0, 2)], None, [1.0, 1.5, 2.0][rng.integers(0, 3)],
            [1.5, 3.0][rng.integers(0, 2)], anchor_stride=s))
    print(f"batch of {len(fs)} fields, {workers} workers", flush=True)
    zs, items = codec.compress_batch([to_dev(x) for x, _ in fs],
                                     [e for _, e in fs],
                                     [qparams(q, p) for p in rps],
                                     workers=workers)
    for i, ((x, e), rp) in enumerate(zip(fs, rps)):
        assert items[i].status == q.QOZ_OK
        zr = ref.compress(x, e, rp)
        assert np.array_equal(zs[i].cpu().numpy(), zr), i
    ys, ditems = codec.decompress_batch(zs, workers=workers)
    for i, (x, e) in enumerate(fs):
        yr = ref.decompress(ref.compress(x, e, rps[i]))
        assert ys[i].shape == x.shape
        assert np.array_equal(ys[i].cpu().numpy().view(np.uint32),
                              yr.view(np.uint32)), i
        assert ditems[i].status == q.QOZ_OK and ditems[i].ms > 0


def test_batch_tuned_equals_single_calls(codec):
    import paper_2310_14133_amd as q
    fs = [f for f in batch_fields() if min(f[0].shape) >= 9]
    cfg = q.make_tune_config(sample_rate=0.2)
    xs = [to_dev(x) for x, _ in fs]
    zs, items = codec.compress_batch(xs, [e for _, e in fs], None, "psnr",
                                     cfg, workers=4)
    for i, (x, e) in enumerate(fs):
        z1 = codec.compress(xs[i], e, None, "psnr", cfg)
        assert np.array_equal(zs[i].cpu().numpy(), z1.cpu().numpy()), i
        assert items[i].done_ms >= items[i].ms > 0


def test_batch_failing_field_fails_alone(codec, ref):
    import paper_2310_14133_amd as q
    fs = batch_fields()[:4]
    bad = fs[1][0].copy()
    bad.flat[17] = np.inf
    xs = [to_dev(x) for x, _ in fs]
    xs[1] = to_dev(bad)
    rps = [ref.make_params(x.ndim, "cubic", None, 1.0, 1.5) for x, _ in fs]
    with pytest.raises(q.QozError) as err:
        codec.compress_batch(xs, [e for _, e in fs],
                             [qparams(q, p) for p in rps], workers=2)
    assert err.value.status == q.QOZ_EINVAL
    # the others, alone and again in a batch without the bad field
    keep = [0, 2, 3]
    zs, items = codec.compress_batch([xs[i] for i in keep],
                                     [fs[i][1] for i in keep],
                                     [qparams(q, rps[i]) for i in keep],
                                     workers=2)
    for k, i in enumerate(keep):
        assert np.array_equal(zs[k].cpu().numpy(),
                              ref.compress(fs[i][0], fs[i][1], rps[i]))


def queue_cases(ref):
    """Streams of uneven shapes and parameters from the oracle: 2D and 3D,
    level-1 orders that end on the contiguous dimension (fused row kernels)
    and ones that do not, a packed payload, an anchor-free plan and a field
    too small for any sweep."""
    rng = np.random.default_rng(7)
    out = []
    for i, (x, e) in enumerate(batch_fields()):
        order = None
        if x.ndim == 3 and i % 2:
            order = [(2, 0, 1)] * 16  # level 1 ends off the contiguous axis
        rp = ref.make_params(x.ndim, ["linear", "cubic"][i % 2], order,
                             [1.0, 1.25, 2.0][i % 3], [1.5, 4.0][i % 2],
                             anchor_stride=[4, 8, 16, 32][rng.integers(0, 4)])
        out.append((f"grf{x.shape}", x, e, rp))
    x = fields.bumps_and_waves(160, 2)
    out.append(("packed 160^2", x, 1e-2 * float(x.max() - x.min()),
                ref.make_params(2, "cubic", None, 1.0, 1.5, anchor_stride=64)))
    x = fields.grf((96, 100, 90), 140)
    out.append(("grf 96x100x90", x, 1e-4 * float(x.max() - x.min()),
                ref.make_params(3, "cubic", None, 1.5, 2.0, anchor_stride=32)))
    x = fields.grf((1000, 700), 141, log_normal=True)
    out.append(("grf 1000x700", x, 1e-3 * float(x.max() - x.min()),
                ref.make_params(2, "linear", None, 1.0, 1.5,
                                anchor_stride=1024)))
    return out


def test_queue_outputs_equal_oracle(codec, ref):
    import paper_2310_14133_amd as q
    cases = queue_cases(ref)
    zs, yrs = [], []
    for name, x, e, rp in cases:
        z = ref.compress(x, e, rp)
        zs.append(to_dev(z))
        yrs.append(ref.decompress(z))
    assert any(int(np.frombuffer(z[4:6].cpu().numpy().tobytes(),
                                 np.uint16)[0]) == 5 for z in zs)
    print(f"queue of {len(zs)} streams", flush=True)
    import torch
    # with graphs on: call 1 runs the device work directly, call 2 (same
    # signature) captures it as a graph, calls 3 and 4 replay the graph;
    # eager work in between; call 5 with graphs off again
    codec.set_queue_graphs(True)
    for rep in range(5):
        if rep == 4:
            codec.set_queue_graphs(False)
        junk = torch.full((1 << 20,), float(rep), device="cuda")
        assert float(junk.mul_(3.0).sum().item()) == 3.0 * rep * (1 << 20)
        ys, items = codec.decompress_queue(zs)
        for i, (name, x, e, rp) in enumerate(cases):
            assert items[i].status == q.QOZ_OK, name
            assert tuple(items[i].shape.dims[:x.ndim]) == x.shape, name
            assert np.array_equal(ys[i].cpu().numpy().view(np.uint32),
                                  yrs[i].view(np.uint32)), (name, rep)
    # a batch of one, and an empty batch
    ys, items = codec.decompress_queue(zs[-2:-1])
    assert np.array_equal(ys[0].cpu().numpy().view(np.uint32),
                          yrs[-2].view(np.uint32))
    ys, items = codec.decompress_queue([])
    assert ys == [] and len(items) == 0


def test_queue_equals_single_calls_tuned(codec):
    # tuned streams of the library itself: queue output == qoz_decompress
    import paper_2310_14133_amd as q
    fs = [f for f in batch_fields() if min(f[0].shape) >= 9]
    cfg = q.make_tune_config(sample_rate=0.2)
    zs = [codec.compress(to_dev(x), e, None, "psnr", cfg) for x, e in fs]
    ys, items = codec.decompress_queue(zs)
    for i, z in enumerate(zs):
        y1 = codec.decompress(z)
        assert np.array_equal(ys[i].cpu().numpy().view(np.uint32),
                              y1.cpu().numpy().view(np.uint32)), i


def test_queue_bad_streams_fail_alone(codec, ref):
    import paper_2310_14133_amd as q
    cases = queue_cases(ref)
    zh = [ref.compress(x, e, rp) for _, x, e, rp in cases]
    packed = [i for i, z in enumerate(zh)
              if int(np.frombuffer(z[4:6].tobytes(), np.uint16)[0]) == 5][0]
    # a packed chunk offset past the payload: found by the device
    z = zh[packed].copy()
    wp = int(np.frombuffer(z[196:200].tobytes(), np.uint32)[0])
    n_chunks = int(np.frombuffer(z[168:176].tobytes(), np.uint64)[0])
    at = z.size - 8 * n_chunks
    z[at:at + 8] = np.frombuffer(np.array([wp + 9], np.uint64).tobytes(),
                                 np.uint8)
    assert ref.decompress_status(z) == ref.EFORMAT
    zs = [to_dev(v) for v in zh]
    zs[packed] = to_dev(z)
    # a stream cut short: found by the header check on the host
    cut = 2
    zs[cut] = zs[cut][:-8].clone()
    import torch
    outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda")
            for _, x, _, _ in cases]
    print(f"queue with bad streams {packed} and {cut}", flush=True)
    ys, items = codec.decompress_queue(zs, out=outs, check=False)
    for i, (name, x, e, rp) in enumerate(cases):
        if i in (packed, cut):
            assert items[i].status == q.QOZ_EFORMAT, name
            continue
        assert items[i].status == q.QOZ_OK, name
        assert np.array_equal(ys[i].cpu().numpy().view(np.uint32),
                              ref.decompress(zh[i]).view(np.uint32)), name
    with pytest.raises(q.QozError) as err:
        codec.decompress_queue(zs, out=outs)
    assert err.value.status == q.QOZ_EFORMAT


def test_queue_many_small_streams(codec, ref):
    # more streams than one 64-lane ballot covers: every queue's workgroup
    # lookup runs over several ballots
    import paper_2310_14133_amd as q
    rng = np.random.default_rng(11)
    zs, yrs, shapes = [], [], []
    for i in range(150):
        sh = ((int(rng.integers(5, 40)), int(rng.integers(5, 40)))
              if i % 2 else tuple(int(v) for v in rng.integers(3, 14, 3)))
        x = fields.grf(sh, 500 + i, log_normal=(i % 5 == 0))
        e = [1e-2, 1e-3, 1e-4][i % 3] * (float(x.max()) - float(x.min()))
        rp = ref.make_params(x.ndim, ["linear", "cubic"][i % 2], None,
                             1.25, 2.0, anchor_stride=[4, 8, 16][i % 3])
        z = ref.compress(x, e, rp)
        zs.append(to_dev(z))
        yrs.append(ref.decompress(z))
        shapes.append(sh)
    print(f"queue of {len(zs)} small streams", flush=True)
    ys, items = codec.decompress_queue(zs)
    for i in range(len(zs)):
        assert items[i].status == q.QOZ_OK, i
        assert ys[i].shape == shapes[i]
        assert np.array_equal(ys[i].cpu().numpy().view(np.uint32),
                              yrs[i].view(np.uint32)), i
