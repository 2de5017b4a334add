"""The metrics entry point that allocates nothing (qoz_metrics_noalloc)
against qoz_metrics (PSNR of Eq. 1, SSIM of Eq. 2-3, maximum error), on
two calls in a row with the second input smaller, and against the oracle.
Its device scratch is one fixed array per device, so the second call must
not see anything the first call left there."""
import numpy as np
import pytest

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


def _pair(shape, seed, eps):
    """A smooth field and its reconstruction from a compression at eps."""
    import torch

    from paper_2310_14133_amd import fields
    x = fields.multiscale_torch(shape, seed)
    xh = x.cpu().numpy()
    noise = np.random.default_rng(seed + 1).uniform(-1.0, 1.0, xh.shape)
    e = eps * (float(xh.max()) - float(xh.min()))
    yh = (xh.astype(np.float64) + e * noise).astype(np.float32)
    return x, torch.from_numpy(yh).cuda(), xh, yh


def _close(a, b):
    return a == b or abs(a - b) <= 1e-9 * abs(b)


@pytest.mark.parametrize("window", [7, 5])
def test_noalloc_metrics_two_calls(codec, ref, window):
    import paper_2310_14133_amd as q
    stream = codec._stream()
    # first a larger 3D field, then a smaller 2D one, then a smaller 3D one
    for shape, seed in (((96, 100, 90), 501), ((130, 129), 502),
                        ((40, 41, 42), 503)):
        print(f"case noalloc metrics shape={shape} window={window}",
              flush=True)
        x, y, xh, yh = _pair(shape, seed, 1e-3)
        sh = q.make_shape(shape)
        got = q.qoz_metrics_noalloc(codec.ctx, x.data_ptr(), y.data_ptr(), sh,
                                    window, stream)
        want = q.qoz_metrics(codec.ctx, x.data_ptr(), y.data_ptr(), sh,
                             window, stream)
        for a, b in zip(got, want):
            assert _close(a, b), (shape, got, want)
        assert got[2] == want[2]
        pr, sr, mr = ref.metrics(xh, yh, window)
        assert _close(got[0], pr) and _close(got[1], sr), (got, pr, sr)
        assert got[2] == mr
        # without SSIM
        g2 = q.qoz_metrics_noalloc(codec.ctx, x.data_ptr(), y.data_ptr(), sh,
                                   window, stream, want_ssim=False)
        assert g2[1] is None and g2[0] == got[0] and g2[2] == got[2]


def test_noalloc_metrics_rejects_too_many_partials(codec):
    import torch

    import paper_2310_14133_amd as q
    # a 2D plane of 1024 x 131072: 255 x 2048 SSIM tiles exceed the fixed
    # scratch's 516096 partial sums; the call refuses before any launch
    shape = (1024, 131072)
    print(f"case noalloc metrics over the scratch limit shape={shape}",
          flush=True)
    x = torch.zeros(shape, dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(q.QozError) as ei:
        q.qoz_metrics_noalloc(codec.ctx, x.data_ptr(), y.data_ptr(),
                              q.make_shape(shape), 7, codec._stream())
    assert ei.value.status == q.QOZ_EINVAL
    # the same shape without SSIM needs no SSIM partials and runs
    ps, ss, me = q.qoz_metrics_noalloc(codec.ctx, x.data_ptr(), y.data_ptr(),
                                       q.make_shape(shape), 7,
                                       codec._stream(), want_ssim=False)
    assert ss is None and me == 0.0
