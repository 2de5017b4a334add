"""Oracle pins: PSNR (Eq. 1), windowed SSIM (Eq. 2-3) and the lag-1
autocorrelation of errors (Eq. 4).  CPU only."""
import math

import numpy as np
import pytest
from numpy.lib.stride_tricks import sliding_window_view

from paper_2310_14133_amd import fields


def test_psnr_constant_error_closed_form(ref):
    """A uniform error delta gives PSNR = 20 log10(vrange / delta)."""
    rng = np.random.default_rng(1)
    x = rng.integers(-1000, 1000, size=(50, 60)).astype(np.float32)
    delta = 2.0 ** -6
    y = (x + np.float32(delta)).astype(np.float32)
    assert np.all(y.astype(np.float64) - x == delta)   # exact in FP32
    psnr, _, maxerr = ref.metrics(x, y)
    vr = float(x.max()) - float(x.min())
    assert abs(psnr - 20 * math.log10(vr / delta)) < 1e-12
    assert maxerr == delta


def test_psnr_matches_numpy(ref):
    x = fields.grf((30, 40, 50), 3)
    y = (x + np.random.default_rng(2).normal(0, 1e-3, x.shape)).astype(
        np.float32)
    psnr, _, maxerr = ref.metrics(x, y)
    d = x.astype(np.float64) - y.astype(np.float64)
    vr = float(x.max()) - float(x.min())
    want = 20 * np.log10(vr / np.sqrt(np.mean(d * d)))
    assert abs(psnr - want) <= 1e-10 * abs(want)
    assert maxerr == np.abs(d).max()
    assert ref.metrics(x, x)[0] == math.inf


def ssim_numpy(x, y, w, vrange):
    """Independent route: numpy sliding windows, population moments."""
    x = x.astype(np.float64)
    y = y.astype(np.float64)
    win = tuple(min(w, n) for n in x.shape)
    axes = tuple(range(-x.ndim, 0))
    X = sliding_window_view(x, win)
    Y = sliding_window_view(y, win)
    mx, my = X.mean(axis=axes), Y.mean(axis=axes)
    vx, vy = X.var(axis=axes), Y.var(axis=axes)
    cxy = ((X - mx[(...,) + (None,) * x.ndim]) *
           (Y - my[(...,) + (None,) * x.ndim])).mean(axis=axes)
    c1, c2 = (0.01 * vrange) ** 2, (0.03 * vrange) ** 2
    s = ((2 * mx * my + c1) * (2 * cxy + c2)) / \
        ((mx ** 2 + my ** 2 + c1) * (vx + vy + c2))
    return float(s.mean()), s.size


@pytest.mark.parametrize("shape,w", [((40, 37), 7), ((12, 15, 18), 7),
                                     ((5, 30), 7), ((9, 9, 9), 3)])
def test_ssim_matches_independent_numpy(ref, shape, w):
    rng = np.random.default_rng(sum(shape))
    x = fields.grf(shape, 4)
    y = (x + rng.normal(0, 0.05, shape)).astype(np.float32)
    vr = float(x.max()) - float(x.min())
    want, nwin = ssim_numpy(x, y, w, vr)
    s_sep, n_sep = ref.ssim_sums(x, y, w, vr)
    s_dir, n_dir = ref.ssim_sums(x, y, w, vr, direct=True)
    assert n_sep == n_dir == nwin
    assert abs(s_sep / n_sep - want) < 1e-10
    assert abs(s_dir / n_dir - want) < 1e-10
    assert abs(s_sep - s_dir) <= 1e-12 * abs(s_dir)
    _, ssim, _ = ref.metrics(x, y, w)
    assert abs(ssim - s_sep / n_sep) < 1e-15


def test_ssim_identity_and_symmetry(ref):
    x = fields.grf((25, 26, 27), 5)
    y = (x * 0.9 + 0.1).astype(np.float32)
    assert ref.metrics(x, x)[1] == 1.0
    vr = float(x.max()) - float(x.min())
    assert ref.ssim_sums(x, y, 7, vr) == ref.ssim_sums(y, x, 7, vr)


def test_ssim_hand_example(ref):
    """One 2x2 window: x = (0,1,2,3), y = (0,1,2,5), vrange 3.
    mu_x = 1.5, mu_y = 2, var_x = 1.25, var_y = 3.5, cov = 2;
    c1 = 0.0009, c2 = 0.0081."""
    x = np.array([[0, 1], [2, 3]], np.float32)
    y = np.array([[0, 1], [2, 5]], np.float32)
    c1, c2 = 0.0009, 0.0081
    want = ((2 * 1.5 * 2 + c1) * (2 * 2 + c2)) / \
        ((1.5 ** 2 + 2 ** 2 + c1) * (1.25 + 3.5 + c2))
    s, n = ref.ssim_sums(x, y, 7, 3.0)
    assert n == 1 and abs(s - want) < 1e-15


def _with_errors(e):
    """x = 0, y = -e, so x - y = e exactly (e holds powers of two and small
    integers)."""
    e = np.asarray(e, np.float32)
    return np.zeros_like(e), -e


def test_ac_alternating_errors_is_minus_one(ref):
    """Errors +d, -d, +d, ... along every row: the lagged products are all
    -d^2 around a zero mean, so AC = -1 exactly."""
    e = np.tile(np.where(np.arange(10) % 2 == 0, 0.5, -0.5), (6, 7, 1))
    assert ref.error_ac(*_with_errors(e)) == -1.0


def test_ac_axis_is_the_fastest_dimension(ref):
    """Errors alternating along dimension 0 but constant along each row:
    neighbours in a row carry equal errors, so AC = +1 (it would be -1 along
    dimension 0)."""
    e = np.broadcast_to(np.where(np.arange(6) % 2 == 0, 0.25, -0.25)[:, None,
                                                                      None],
                        (6, 5, 8))
    assert ref.error_ac(*_with_errors(e)) == 1.0


def test_ac_constant_error_is_zero(ref):
    e = np.full((9, 11), 0.125, np.float32)
    assert ref.error_ac(*_with_errors(e)) == 0.0


@pytest.mark.parametrize("n", [5, 9, 33])
def test_ac_ramp_closed_form(ref, n):
    """Errors 0, 1, ..., n-1 in every row: mean (n-1)/2, variance
    (n^2-1)/12, lagged moment (n-3)(n+1)/12, so AC = (n-3)/(n-1)."""
    e = np.tile(np.arange(n, dtype=np.float32), (4, 1))
    got = ref.error_ac(*_with_errors(e))
    assert abs(got - (n - 3) / (n - 1)) <= 1e-15
