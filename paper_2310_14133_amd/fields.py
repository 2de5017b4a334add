"""Seeded synthetic input fields.

These generators only produce inputs; they hold none of the compressor's
arithmetic.  Both the GPU library's tests and the CPU oracle consume the same
bytes produced here.  The shapes and statistics stand in for the paper's
datasets (Table II), which are not available: smooth multiscale fields with a
k^-3 power spectrum (turbulence / climate / cosmology-like), optionally
exponentiated for a skewed, log-normal-like distribution (cosmology density),
plus localized Gaussian features.
"""
import numpy as np


def _freq_radius(shape):
    ks = [np.fft.fftfreq(n) for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    grids = np.meshgrid(*ks, indexing="ij", sparse=True)
    k2 = sum(g.astype(np.float64) ** 2 for g in grids)
    return np.sqrt(k2)


def grf(shape, seed, slope=-3.0, log_normal=False, dtype=np.float32):
    """Gaussian random field with power spectrum P(k) ~ k^slope.

    White N(0,1) noise from `seed` is filtered in Fourier space by
    |k|^(slope/2) (k in cycles per sample, the k=0 mode removed), then
    standardised to mean 0, std 1; `log_normal` applies exp().
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    spec = np.fft.rfftn(white)
    k = _freq_radius(shape)
    with np.errstate(divide="ignore"):
        amp = np.where(k > 0, k ** (slope / 2.0), 0.0)
    g = np.fft.irfftn(spec * amp, s=shape, axes=tuple(range(len(shape))))
    g = (g - g.mean()) / g.std()
    if log_normal:
        g = np.exp(g)
    return np.ascontiguousarray(g.astype(dtype))


def grf_torch(shape, seed, slope=-3.0, log_normal=False, device="cuda"):
    """Same recipe as grf() computed with torch on `device` (fast for 512^3).

    Deterministic for a given seed and device type; its bytes differ from
    grf()'s.  Whatever it returns is handed unchanged to every consumer.
    """
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    white = torch.randn(shape, generator=gen, device=device,
                        dtype=torch.float32)
    spec = torch.fft.rfftn(white)
    ks = [torch.fft.fftfreq(n, device=device) for n in shape[:-1]]
    ks.append(torch.fft.rfftfreq(shape[-1], device=device))
    k2 = None
    for i, kv in enumerate(ks):
        view = [1] * len(shape)
        view[i] = kv.numel()
        term = (kv.view(view)) ** 2
        k2 = term if k2 is None else k2 + term
    k = torch.sqrt(k2)
    amp = torch.where(k > 0, k.clamp_min(1e-30) ** (slope / 2.0),
                      torch.zeros_like(k))
    spec = spec * amp
    del k, k2, amp, white
    g = torch.fft.irfftn(spec, s=shape)
    del spec
    g = (g - g.mean()) / g.std()
    if log_normal:
        g = torch.exp(g)
    return g.contiguous()


def tuner_training_field(seed, device="cuda", shape=None):
    """One field of the learned tuner's workload: a k^slope random field
    (slope U[-4, -2]) plus white noise of relative std 10^U[-4, -2], shape
    U{64..256}^3 unless given, all drawn from `seed` (torch on `device`).
    Without a given shape the field is the corner of a periodic 256^3 field
    (one FFT size for every field), standardised again.
    Returns (field, recipe)."""
    import torch
    rng = np.random.default_rng(seed)
    crop = shape is None
    if crop:
        shape = tuple(int(v) for v in rng.integers(64, 257, 3))
    slope = float(rng.uniform(-4.0, -2.0))
    noise = float(10.0 ** rng.uniform(-4.0, -2.0))
    if crop:
        g = grf_torch((256, 256, 256), seed, slope=slope, device=device)
        g = g[:shape[0], :shape[1], :shape[2]]
        g = ((g - g.mean()) / g.std()).contiguous()
    else:
        g = grf_torch(shape, seed, slope=slope, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) + 104729)
    g += noise * torch.randn(shape, generator=gen, device=device,
                             dtype=torch.float32)
    return g.contiguous(), {"shape": shape, "slope": slope, "noise": noise}


TUNER_KINDS = ("grf", "lognormal", "multiscale")


def tuner_field(seed, ndim=3, device="cuda", shape=None, kind=None):
    """One field of the learned tuner's wider workload, drawn from `seed`
    (torch on `device`):

    * kind "grf": a k^slope random field (slope U[-4, -2]) plus white noise
      of relative std 10^U[-4, -2] (the tuner_training_field recipe);
    * kind "lognormal": exp(s g) of a k^slope field g (slope U[-4, -2]),
      s U[0.5, 1.5], standardised: a skewed, density-like field;
    * kind "multiscale": the k^-3 field plus 16 Gaussian bumps.

    Without a given shape: 3D U{64..256}^3, 2D U{256..2048}^2 (the corner
    of a periodic 256^3 / 2048^2 field, standardised again); kind uniform
    over TUNER_KINDS unless given.  Returns (field, recipe)."""
    import torch
    rng = np.random.default_rng(seed)
    if kind is None:
        kind = TUNER_KINDS[int(rng.integers(0, len(TUNER_KINDS)))]
    crop = shape is None
    full = (256,) * 3 if ndim == 3 else (2048, 2048)
    if crop:
        lo, hi = (64, 257) if ndim == 3 else (256, 2049)
        shape = tuple(int(v) for v in rng.integers(lo, hi, ndim))
    slope = float(rng.uniform(-4.0, -2.0))
    noise = float(10.0 ** rng.uniform(-4.0, -2.0))
    sigma = float(rng.uniform(0.5, 1.5))
    gshape = full if crop else shape
    if kind == "multiscale":
        g = multiscale_torch(gshape, seed, device=device)
    else:
        g = grf_torch(gshape, seed, slope=slope, device=device)
    if crop:
        g = g[tuple(slice(0, n) for n in shape)]
    if kind == "lognormal":
        g = torch.exp(sigma * ((g - g.mean()) / g.std()))
    g = ((g - g.mean()) / g.std()).contiguous()
    if kind == "grf":
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed) + 104729)
        g += noise * torch.randn(shape, generator=gen, device=device,
                                 dtype=torch.float32)
    rec = {"shape": shape, "kind": kind}
    if kind != "multiscale":
        rec["slope"] = slope
    if kind == "grf":
        rec["noise"] = noise
    if kind == "lognormal":
        rec["sigma"] = sigma
    return g.contiguous(), rec


def bumps_and_waves(n=256, seed=1, n_bumps=8, n_waves=3, noise=1e-3,
                    dtype=np.float32):
    """2D field: Gaussian bumps + plane waves + white noise.

    Bumps: centres U[0,n)^2, widths U[8,40], amplitudes N(0,1).  Waves:
    wavevector uniform in the disc |k| <= 0.1 rad/px, phase U[0,2pi),
    amplitude 1.  Noise: N(0, noise^2).
    """
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.arange(n, dtype=np.float64),
                         np.arange(n, dtype=np.float64), indexing="ij")
    f = np.zeros((n, n), np.float64)
    for _ in range(n_bumps):
        cy, cx = rng.uniform(0, n, 2)
        w = rng.uniform(8, 40)
        a = rng.normal()
        f += a * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * w * w))
    for _ in range(n_waves):
        r = 0.1 * np.sqrt(rng.uniform())
        th = rng.uniform(0, 2 * np.pi)
        ky, kx = r * np.sin(th), r * np.cos(th)
        ph = rng.uniform(0, 2 * np.pi)
        f += np.sin(ky * yy + kx * xx + ph)
    f += rng.normal(0.0, noise, size=(n, n))
    return np.ascontiguousarray(f.astype(dtype))


def multiscale(shape, seed, n_bumps=16, dtype=np.float32):
    """k^-3 random field (standardised) + Gaussian bumps.

    Bumps: centres uniform in the box, widths U[0.02, 0.1] * min(shape),
    amplitudes N(0,1).
    """
    base = grf(shape, seed, slope=-3.0, dtype=np.float64)
    rng = np.random.default_rng(seed + 7919)
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    m = min(shape)
    for _ in range(n_bumps):
        c = [rng.uniform(0, n) for n in shape]
        w = rng.uniform(0.02, 0.1) * m
        a = rng.normal()
        terms = [np.exp(-((ax - ci) ** 2) / (2 * w * w)) for ax, ci in
                 zip(axes, c)]
        g = terms[0]
        for t in terms[1:]:
            g = np.multiply.outer(g, t)
        base += a * g
    return np.ascontiguousarray(base.astype(dtype))


def multiscale_torch(shape, seed, n_bumps=16, device="cuda"):
    """Same recipe as multiscale() computed with torch on `device` (fast at
    the paper's shapes, e.g. 1008x1008x352): the k^-3 field of grf_torch
    (standardised) plus n_bumps Gaussian bumps, centres uniform in the box,
    widths U[0.02, 0.1] * min(shape), amplitudes N(0,1), drawn from
    `seed`.  Its bytes differ from multiscale()'s; whatever it returns is
    handed unchanged to every consumer."""
    import torch
    g = grf_torch(shape, seed, slope=-3.0, device=device)
    rng = np.random.default_rng(seed + 7919)
    m = min(shape)
    axes = [torch.arange(n, device=device, dtype=torch.float32)
            for n in shape]
    for _ in range(n_bumps):
        c = [rng.uniform(0, n) for n in shape]
        w = rng.uniform(0.02, 0.1) * m
        a = float(rng.normal())
        bump = None
        for i, (ax, ci) in enumerate(zip(axes, c)):
            t = torch.exp(-((ax - ci) ** 2) / (2.0 * w * w))
            view = [1] * len(shape)
            view[i] = shape[i]
            t = t.view(view)
            bump = t if bump is None else bump * t
        g += a * bump
    return g.contiguous()


def polynomial(shape, degree, seed=0, max_coef=3, dtype=np.float32):
    """Integer-coefficient polynomial of total degree <= `degree` in the
    grid coordinates; values are integers (exact in FP32 for small fields)."""
    rng = np.random.default_rng(seed)
    d = len(shape)
    coords = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape],
                         indexing="ij")
    f = np.zeros(shape, np.float64)
    import itertools
    for powers in itertools.product(range(degree + 1), repeat=d):
        if sum(powers) > degree:
            continue
        c = int(rng.integers(-max_coef, max_coef + 1))
        term = np.full(shape, float(c))
        for ax, pw in zip(coords, powers):
            term = term * ax ** pw
        f += term
    return np.ascontiguousarray(f.astype(dtype))


def adversarial(shape, kind, seed=0, dtype=np.float32):
    """Small fields that stress edge cases: 'steps', 'spikes' (+-1e30),
    'alternating', 'denormal', 'noise'."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    if kind == "steps":
        f = np.floor(grf(shape, seed, dtype=np.float64) * 2.0)
    elif kind == "spikes":
        f = grf(shape, seed, dtype=np.float64)
        idx = rng.choice(n, size=max(1, n // 50), replace=False)
        f.reshape(-1)[idx] = rng.choice([-1e30, 1e30], size=idx.size)
    elif kind == "alternating":
        f = np.ones(n)
        f[1::2] = -1.0
        f = f.reshape(shape) * rng.uniform(0.5, 2.0, size=shape)
    elif kind == "denormal":
        f = rng.uniform(-1, 1, size=shape) * 1e-39
    elif kind == "noise":
        f = rng.standard_normal(shape)
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(np.asarray(f).astype(dtype))


def bins_field(bins, n0, n1):
    """2D field whose quantization bins (anchor stride 2, linear
    interpolation, order (0, 1), bound 0.5 so the bin width is 1) are the
    given integers, in stream order.  Anchors are 0; the first sweep's
    targets (odd row, even column) take the bin value itself; the second
    sweep's targets (odd column) take the mean of their left and right
    neighbours plus the bin value.  n0 and n1 must be odd.  Used to force
    chosen histograms, e.g. very long Huffman codes."""
    assert n0 % 2 == 1 and n1 % 2 == 1
    f = np.zeros((n0, n1), np.float64)
    bins = np.asarray(bins, np.float64)
    n_s0 = (n0 // 2) * (n1 // 2 + 1)
    n_s1 = n0 * (n1 // 2)
    assert bins.size == n_s0 + n_s1
    f[1::2, 0::2] = bins[:n_s0].reshape(n0 // 2, n1 // 2 + 1)
    mean = 0.5 * (f[:, 0:-1:2] + f[:, 2::2])
    f[:, 1::2] = mean + bins[n_s0:].reshape(n0, n1 // 2)
    return np.ascontiguousarray(f.astype(np.float32))


def fibonacci_bins(total, n_syms, seed=0):
    """`total` bins whose counts follow a Fibonacci sequence over n_syms
    distinct values (the rest are 0), shuffled."""
    fib = [1, 1]
    while len(fib) < n_syms:
        fib.append(fib[-1] + fib[-2])
    vals = []
    for k, cnt in enumerate(fib[:n_syms]):
        vals += [k + 1] * cnt
    vals = vals[:total]
    vals += [0] * (total - len(vals))
    v = np.array(vals, np.int64)
    np.random.default_rng(seed).shuffle(v)
    return v
