"""Batched compression through the device work queues (qoz_compress_queue)
through the C ABI: every field's stream equals the oracle's (given
parameters) or the single-field call's (tuned), byte for byte, for uneven
batches of 2D and 3D fields, packed and unpacked payloads, fields with more
used bins than the device sort holds, and fields that fail or do not fit
their buffer, which fail alone."""
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


def qparams(q, ref_p):
    p = q.Params()
    p.anchor_stride = ref_p.anchor_stride
    for l in range(16):
        p.interp[l] = ref_p.interp[l]
        for j in range(3):
            p.order[l][j] = ref_p.order[l][j]
    p.alpha, p.beta = ref_p.alpha, ref_p.beta
    return p


def version(z):
    return int(np.frombuffer(np.asarray(z[4:6]).tobytes(), np.uint16)[0])


def cases(ref):
    """Uneven shapes and parameters: 2D and 3D, level-1 orders that end on
    the contiguous dimension (fused row kernels) and ones that do not, a
    payload that zero-word packing shortens, a field with more used bins
    than the device sort holds, an anchor-free plan and a field too small
    for any sweep."""
    rng = np.random.default_rng(31)
    out = []
    shapes = [(70, 45), (19, 24, 33), (40, 41, 42), (130, 129), (3, 200, 7),
              (33, 65, 17), (2, 3), (64, 64, 64), (9, 300)]
    for i, sh in enumerate(shapes):
        x = fields.grf(sh, 300 + i, log_normal=(i % 3 == 1))
        e = [1e-2, 1e-3, 1e-4, 1e-5][i % 4] * float(x.max() - x.min())
        order = [(2, 0, 1)] * 16 if x.ndim == 3 and i % 2 else None
        rp = ref.make_params(x.ndim, ["linear", "cubic"][i % 2], order,
                             [1.0, 1.25, 2.0][i % 3], [1.5, 4.0][i % 2],
                             anchor_stride=[4, 8, 16, 32][rng.integers(0, 4)])
        out.append((f"grf{sh}", x, e, rp))
    x = fields.bumps_and_waves(160, 2)
    out.append(("packed 160^2", x, 1e-2 * float(x.max() - x.min()),
                ref.make_params(2, "cubic", None, 1.0, 1.5, anchor_stride=64)))
    x = np.random.default_rng(5).standard_normal((48, 50, 52)).astype(np.float32)
    out.append(("noise 48x50x52 (many bins)", x, 1e-5 * float(x.max() - x.min()),
                ref.make_params(3, "linear", None, 1.0, 1.5, anchor_stride=8)))
    x = fields.grf((1000, 700), 341, log_normal=True)
    out.append(("grf 1000x700", x, 1e-3 * float(x.max() - x.min()),
                ref.make_params(2, "linear", None, 1.0, 1.5,
                                anchor_stride=1024)))
    return out


def test_compress_queue_equals_oracle(codec, ref):
    import paper_2310_14133_amd as q
    cs = cases(ref)
    zr = [ref.compress(x, e, rp) for _, x, e, rp in cs]
    assert any(version(z) == 5 for z in zr)
    used = [int(np.frombuffer(z[160:168].tobytes(), np.uint64)[0])
            for z in zr]
    assert max(used) > 4096  # the noise field: more than the device sort
    print(f"queue compression of {len(cs)} fields", flush=True)
    for rep in range(2):  # the second call reuses the grown scratch
        zs, items = codec.compress_batch([to_dev(x) for _, x, _, _ in cs],
                                         [e for _, _, e, _ in cs],
                                         [qparams(q, rp) for *_, rp in cs],
                                         queue=True)
        for i, (name, x, e, rp) in enumerate(cs):
            assert items[i].status == q.QOZ_OK, name
            assert items[i].out_bytes == zr[i].size, name
            assert np.array_equal(zs[i].cpu().numpy(), zr[i]), (name, rep)
    ys, _ = codec.decompress_queue(zs)
    for i, (name, x, e, rp) in enumerate(cs):
        y = ys[i].cpu().numpy().astype(np.float64)
        assert np.abs(y - x).max() <= e, name
    print(f"  used bins per field: {used}", flush=True)


def test_compress_queue_tuned_equals_single_calls(codec):
    import paper_2310_14133_amd as q
    cfg = q.make_tune_config(sample_rate=0.2)
    xs, es = [], []
    for i, sh in enumerate([(40, 41, 42), (130, 129), (33, 65, 17),
                            (64, 64, 64), (300, 220)]):
        x = fields.grf(sh, 400 + i, log_normal=(i % 2 == 1))
        xs.append(to_dev(x))
        es.append([1e-2, 1e-3, 1e-4][i % 3] * float(x.max() - x.min()))
    for target in ("psnr", "cr"):
        zs, items = codec.compress_batch(xs, es, None, target, cfg, queue=True)
        for i in range(len(xs)):
            z1 = codec.compress(xs[i], es[i], None, target, cfg)
            assert np.array_equal(zs[i].cpu().numpy(), z1.cpu().numpy()), \
                (target, i)
            assert items[i].status == q.QOZ_OK and items[i].ms > 0


def test_compress_queue_mixed_params(codec, ref):
    # some fields with parameters, some tuned in the same call
    import paper_2310_14133_amd as q
    cfg = q.make_tune_config(sample_rate=0.2)
    cs = cases(ref)[:6]
    ps = [qparams(q, rp) if i % 2 == 0 else None
          for i, (*_, rp) in enumerate(cs)]
    xs = [to_dev(x) for _, x, _, _ in cs]
    zs, items = codec.compress_batch(xs, [e for _, _, e, _ in cs], ps, "cr",
                                     cfg, queue=True)
    for i, (name, x, e, rp) in enumerate(cs):
        if ps[i] is not None:
            assert np.array_equal(zs[i].cpu().numpy(),
                                  ref.compress(x, e, rp)), name
        else:
            z1 = codec.compress(xs[i], e, None, "cr", cfg)
            assert np.array_equal(zs[i].cpu().numpy(), z1.cpu().numpy()), name


def test_compress_queue_failures_alone(codec, ref):
    """A field with a non-finite value fails with EINVAL; a buffer that
    cannot hold the sections before the payload, and one that holds them
    but not the payload, fail with ENOSPACE and report the size the
    single-field call reports; the other fields' streams are unchanged."""
    import paper_2310_14133_amd as q
    cs = cases(ref)[:6]
    zr = [ref.compress(x, e, rp) for _, x, e, rp in cs]
    xs = [to_dev(x) for _, x, _, _ in cs]
    bad = cs[1][1].copy()
    bad.flat[17] = np.nan
    xs[1] = to_dev(bad)
    caps = [q.qoz_compress_bound(codec._field(x)) for x in xs]
    caps[2] = 300                 # not even the sections before the payload
    caps[3] = zr[3].size - 64     # the sections, not the whole payload
    ps = [qparams(q, rp) for *_, rp in cs]
    zs, items = codec.compress_batch(xs, [e for _, _, e, _ in cs], ps,
                                     queue=True, caps=caps, check=False)
    assert items[1].status == q.QOZ_EINVAL
    for i in (2, 3):  # unpacked streams: the size needed is the stream's
        assert version(zr[i]) != 5
        assert items[i].status == q.QOZ_ENOSPACE, i
        assert items[i].out_bytes == zr[i].size, i
    for i in (0, 4, 5):
        assert items[i].status == q.QOZ_OK
        assert np.array_equal(zs[i].cpu().numpy(), zr[i]), i
    with pytest.raises(q.QozError):
        codec.compress_batch(xs, [e for _, _, e, _ in cs], ps, queue=True,
                             caps=caps)


def test_compress_queue_many_fields(codec, ref):
    # more fields than one 64-lane ballot covers, and an empty batch
    import paper_2310_14133_amd as q
    rng = np.random.default_rng(12)
    xs, es, ps, zr = [], [], [], []
    for i in range(130):
        sh = ((int(rng.integers(5, 60)), int(rng.integers(5, 60)))
              if i % 2 else tuple(int(v) for v in rng.integers(3, 24, 3)))
        x = fields.grf(sh, 600 + i, log_normal=(i % 5 == 0))
        e = [1e-2, 1e-3, 1e-4][i % 3] * float(x.max() - x.min())
        rp = ref.make_params(x.ndim, ["linear", "cubic"][i % 2], None,
                             1.25, 2.0, anchor_stride=[4, 8, 16][i % 3])
        xs.append(to_dev(x))
        es.append(e)
        ps.append(qparams(q, rp))
        zr.append(ref.compress(x, e, rp))
    print(f"queue compression of {len(xs)} small fields", flush=True)
    zs, items = codec.compress_batch(xs, es, ps, queue=True)
    for i in range(len(xs)):
        assert items[i].status == q.QOZ_OK, i
        assert np.array_equal(zs[i].cpu().numpy(), zr[i]), i
    zs, items = codec.compress_batch([], [], None, queue=True)
    assert zs == [] and len(items) == 0


def test_compress_queue_tuned_groups_with_failures(codec, ref):
    """Twelve fields to tune (more than one round of the 8 tuning workers,
    so several compression groups) next to fields with parameters given:
    a field with a NaN fails its tuning with EINVAL, a too-small buffer
    fails with ENOSPACE, and every other stream equals the single-field
    call's; each field's group ends within the call."""
    import paper_2310_14133_amd as q
    cfg = q.make_tune_config(sample_rate=0.2)
    cs = cases(ref)[:4]
    xs, es, ps = [], [], []
    for i in range(12):
        sh = [(40, 41, 42), (130, 129), (33, 65, 17), (64, 64, 64)][i % 4]
        x = fields.grf(sh, 700 + i, log_normal=(i % 3 == 1))
        xs.append(to_dev(x))
        es.append([1e-2, 1e-3, 1e-4][i % 3] * float(x.max() - x.min()))
        ps.append(None)
    for _, x, e, rp in cs:
        xs.append(to_dev(x))
        es.append(e)
        ps.append(qparams(q, rp))
    bad = xs[5].cpu().numpy().copy()
    bad.flat[3] = np.nan
    xs[5] = to_dev(bad)
    caps = [q.qoz_compress_bound(codec._field(x)) for x in xs]
    caps[7] = 300
    zs, items = codec.compress_batch(xs, es, ps, "cr", cfg, queue=True,
                                     caps=caps, check=False)
    assert items[5].status == q.QOZ_EINVAL
    assert items[7].status == q.QOZ_ENOSPACE
    for i in range(len(xs)):
        if i in (5, 7):
            continue
        assert items[i].status == q.QOZ_OK, i
        z1 = codec.compress(xs[i], es[i], ps[i], "cr", cfg)
        assert np.array_equal(zs[i].cpu().numpy(), z1.cpu().numpy()), i
        assert 0 < items[i].done_ms <= items[i].ms, i
