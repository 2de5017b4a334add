"""Oracle of the learned tuner: block features and the small MLP that maps
them to the tuner's choices (interpolation type, alpha, beta of Eq. 5).

TEST INFRASTRUCTURE ONLY: the test suite uses it to check the GPU library;
the product never imports it.  Plain numpy, one block and one sample at a
time where it matters, FP64 except where the method fixes another
precision:

* the residuals and gradient magnitudes that decide a feature are formed in
  float32, in the operation order stated below, as the library forms them;
* the network multiplies bfloat16 operands (round to nearest even from
  float32) and sums in FP64 here (FP32 on the GPU); biases, activations,
  the softmax and Adam are FP64 here (FP32 on the GPU).

The paper tunes by trial compression only (Sec. VI); the learned part is a
stand-in for that search, so its features follow the quantities the search
looks at: the level-wise interpolation residuals of Sec. V-A / VI-B, the
value range and the error bound.

Features of one sampled block of 33 x 33 x 33 points (b = 32, Sec. VI-A),
e the absolute bound, all logs base 2:
  f[4(l-1) + 2t + 0] = log(1 + mean|r| / e)
  f[4(l-1) + 2t + 1] = log(1 + sqrt(mean r^2) / e)
      over the residuals r = x_p - pred_t(p) of level l = 1..5 (h =
      2^(l-1)): every point p on the h-grid of the block with coordinate
      p_k an odd multiple of h, for k = 0, 1, 2 in turn; t = 0 linear
      (b + c) * 0.5, t = 1 cubic ((b + c) * 9 - (a + d)) * 0.0625 where
      p_k - 3h >= 0 and p_k + 3h <= 32, else linear (a, b, c, d at p_k -
      3h, -h, +h, +3h), all in float32;
  f[20 + (q - 1)] = log(1 + sqrt(g2_(q)) / e), q = 1..10: the
      nearest-rank decile g2_(q) = sorted(g2)[ceil(q n / 10) - 1] of the
      n = 32^3 squared forward-difference gradients
      g2 = (dx*dx + dy*dy) + dz*dz (float32) at points with all
      coordinates in [0, 31];
  f[30] = log(1 + (max - min of the block) / e);
  f[31] = log(1 + (max - min over all sampled blocks together) / e), so
      that the features read the sampled blocks only, as the search of
      Sec. VI-A does.
A 2D field's sampled blocks are 33 x 33 points and the same 32 features
are formed over its two dimensions: the residuals along k = 0, 1 in turn,
and g2 = dx*dx + dy*dy at the n = 32^2 points with both coordinates in
[0, 31].
The field's features are the mean over its sampled blocks (FP64 sum in
block order, then float32).
"""
import numpy as np

NFEAT = 32
HIDDEN = 128
HEADS = (2, 5, 4)  # interpolation type, alpha index, beta index
NOUT = sum(HEADS)
BLOCK = 32
LT = 5

# parameter blob (float32): input shift and scale, then the three layers
OFF_MU = 0
OFF_SG = OFF_MU + NFEAT
OFF_W1 = OFF_SG + NFEAT
OFF_B1 = OFF_W1 + HIDDEN * NFEAT
OFF_W2 = OFF_B1 + HIDDEN
OFF_B2 = OFF_W2 + HIDDEN * HIDDEN
OFF_W3 = OFF_B2 + HIDDEN
OFF_B3 = OFF_W3 + NOUT * HIDDEN
NPARAM = OFF_B3 + NOUT


# ---------------------------------------------------------------- features
def _residual_sums(blk, l, cubic):
    """Sum |r| and sum r^2 (FP64) of level l's residuals over the three
    dimensions, and their count."""
    h = 1 << (l - 1)
    s1 = s2 = 0.0
    cnt = 0
    f32 = np.float32
    grid = blk[(slice(None, None, h),) * blk.ndim]  # coordinates 0, h, .., 32
    m = grid.shape[0]          # 32 / h + 1
    for k in range(blk.ndim):
        g = np.moveaxis(grid, k, 0)
        for j in range(1, m, 2):  # odd multiples of h along k
            b = g[j - 1]
            c = g[j + 1]
            lin = (b + c) * f32(0.5)
            if cubic and j - 3 >= 0 and j + 3 <= m - 1:
                a = g[j - 3]
                d = g[j + 3]
                pred = ((b + c) * f32(9.0) - (a + d)) * f32(0.0625)
            else:
                pred = lin
            r = (g[j] - pred).astype(np.float64)
            s1 += float(np.abs(r).sum())
            s2 += float((r * r).sum())
            cnt += r.size
    return s1, s2, cnt


def block_features(blk, e, vrange):
    """32 features (float32) of one 33^3 (or, for a 2D field, 33^2) float32
    block; formulas in the module docstring."""
    assert blk.ndim in (2, 3) and blk.dtype == np.float32
    assert blk.shape == (BLOCK + 1,) * blk.ndim
    f = np.zeros(NFEAT, np.float64)
    for l in range(1, LT + 1):
        for t in (0, 1):
            s1, s2, n = _residual_sums(blk, l, t)
            f[4 * (l - 1) + 2 * t] = np.log2(1.0 + (s1 / n) / e)
            f[4 * (l - 1) + 2 * t + 1] = np.log2(1.0 + np.sqrt(s2 / n) / e)
    x = blk
    if x.ndim == 3:
        dx = x[1:, :-1, :-1] - x[:-1, :-1, :-1]
        dy = x[:-1, 1:, :-1] - x[:-1, :-1, :-1]
        dz = x[:-1, :-1, 1:] - x[:-1, :-1, :-1]
        g2 = np.sort(((dx * dx + dy * dy) + dz * dz).ravel())
    else:
        dx = x[1:, :-1] - x[:-1, :-1]
        dy = x[:-1, 1:] - x[:-1, :-1]
        g2 = np.sort((dx * dx + dy * dy).ravel())
    n = g2.size
    for q in range(1, 11):
        v = float(g2[-(-q * n // 10) - 1])
        f[19 + q] = np.log2(1.0 + np.sqrt(v) / e)
    f[30] = np.log2(1.0 + (float(x.max()) - float(x.min())) / e)
    f[31] = np.log2(1.0 + vrange / e)
    return f.astype(np.float32)


def field_features(x, e, origins):
    """Per-block features and their mean (float32) for the blocks of a 2D
    or 3D float32 field at the given origins (Sec. VI-A sampling)."""
    blocks = []
    for o in origins:
        sl = tuple(slice(int(v), int(v) + BLOCK + 1) for v in o[:x.ndim])
        blocks.append(np.ascontiguousarray(x[sl]))
    vrange = (max(float(b.max()) for b in blocks) -
              min(float(b.min()) for b in blocks))
    rows = [block_features(b, e, vrange) for b in blocks]
    per = np.stack(rows)
    acc = np.zeros(NFEAT, np.float64)
    for r in per:
        acc += r.astype(np.float64)
    return per, (acc / len(per)).astype(np.float32)


# --------------------------------------------------------------- the MLP
def bf16(a):
    """Round float32 values to bfloat16 (nearest, ties to even), returned
    as float64.  Bit manipulation on the float32 pattern."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a), np.nan, out)


def unpack(P):
    P = np.asarray(P, np.float32)
    return dict(
        mu=P[OFF_MU:OFF_SG], sg=P[OFF_SG:OFF_W1],
        W1=P[OFF_W1:OFF_B1].reshape(HIDDEN, NFEAT), b1=P[OFF_B1:OFF_W2],
        W2=P[OFF_W2:OFF_B2].reshape(HIDDEN, HIDDEN), b2=P[OFF_B2:OFF_W3],
        W3=P[OFF_W3:OFF_B3].reshape(NOUT, HIDDEN), b3=P[OFF_B3:NPARAM])


def init_params(seed, mu=None, sg=None):
    """He-style random weights, zero biases (float32 blob)."""
    rng = np.random.default_rng(seed)
    P = np.zeros(NPARAM, np.float32)
    P[OFF_MU:OFF_SG] = 0.0 if mu is None else mu
    P[OFF_SG:OFF_W1] = 1.0 if sg is None else sg
    P[OFF_W1:OFF_B1] = rng.normal(0, np.sqrt(2.0 / NFEAT), HIDDEN * NFEAT)
    P[OFF_W2:OFF_B2] = rng.normal(0, np.sqrt(2.0 / HIDDEN), HIDDEN * HIDDEN)
    P[OFF_W3:OFF_B3] = rng.normal(0, np.sqrt(1.0 / HIDDEN), NOUT * HIDDEN)
    return P


def _q(a, use_bf16):
    return bf16(a) if use_bf16 else np.asarray(a, np.float64)


def normalise(feat, P):
    """(f - mu) / sg in float32, one sample per row."""
    p = unpack(P)
    return ((np.asarray(feat, np.float32) - p["mu"]) / p["sg"]).astype(
        np.float32)


def forward(P, feat, use_bf16=True):
    """Logits (FP64) of every sample; also the intermediate values."""
    p = unpack(P)
    xh = normalise(feat, P)
    X = _q(xh, use_bf16)
    a1 = X @ _q(p["W1"], use_bf16).T + p["b1"].astype(np.float64)
    h1 = np.maximum(a1, 0.0)
    H1 = _q(h1.astype(np.float32) if use_bf16 else h1, use_bf16)
    a2 = H1 @ _q(p["W2"], use_bf16).T + p["b2"].astype(np.float64)
    h2 = np.maximum(a2, 0.0)
    H2 = _q(h2.astype(np.float32) if use_bf16 else h2, use_bf16)
    z = H2 @ _q(p["W3"], use_bf16).T + p["b3"].astype(np.float64)
    return z, dict(X=X, H1=H1, H2=H2)


def _heads(z):
    o = 0
    for k in HEADS:
        yield o, k
        o += k


def loss_and_grad(P, feat, labels, use_bf16=True):
    """Mean over the batch of the summed softmax cross-entropies of the
    three heads, and its gradient with respect to the blob (zero for the
    input shift and scale).  labels: int array (B, 3)."""
    p = unpack(P)
    z, c = forward(P, feat, use_bf16)
    B = z.shape[0]
    labels = np.asarray(labels)
    loss = 0.0
    dz = np.zeros_like(z)
    for hi, (o, k) in enumerate(_heads(z)):
        zz = z[:, o:o + k]
        m = zz.max(axis=1, keepdims=True)
        ez = np.exp(zz - m)
        s = ez.sum(axis=1, keepdims=True)
        lse = m[:, 0] + np.log(s[:, 0])
        y = labels[:, hi]
        loss += float(np.sum(lse - zz[np.arange(B), y]))
        prob = ez / s
        prob[np.arange(B), y] -= 1.0
        dz[:, o:o + k] = prob / B
    loss /= B
    DZ = _q(dz.astype(np.float32) if use_bf16 else dz, use_bf16)
    W3 = _q(p["W3"], use_bf16)
    W2 = _q(p["W2"], use_bf16)
    g = np.zeros(NPARAM, np.float64)
    g[OFF_W3:OFF_B3] = (DZ.T @ c["H2"]).ravel()
    g[OFF_B3:NPARAM] = dz.sum(axis=0)
    dh2 = (DZ @ W3) * (c["H2"] > 0)
    DH2 = _q(dh2.astype(np.float32) if use_bf16 else dh2, use_bf16)
    g[OFF_W2:OFF_B2] = (DH2.T @ c["H1"]).ravel()
    g[OFF_B2:OFF_W3] = dh2.sum(axis=0)
    dh1 = (DH2 @ W2) * (c["H1"] > 0)
    DH1 = _q(dh1.astype(np.float32) if use_bf16 else dh1, use_bf16)
    g[OFF_W1:OFF_B1] = (DH1.T @ c["X"]).ravel()
    g[OFF_B1:OFF_W2] = dh1.sum(axis=0)
    return loss, g


ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam(P, m, v, g, lr, t):
    """One Adam step (bias-corrected, step t >= 1) on every trained entry
    (not the input shift and scale); returns new (P, m, v) in FP64."""
    P = np.asarray(P, np.float64).copy()
    m = np.asarray(m, np.float64).copy()
    v = np.asarray(v, np.float64).copy()
    s = slice(OFF_W1, NPARAM)
    m[s] = ADAM_B1 * m[s] + (1.0 - ADAM_B1) * g[s]
    v[s] = ADAM_B2 * v[s] + (1.0 - ADAM_B2) * g[s] * g[s]
    mh = m[s] / (1.0 - ADAM_B1 ** t)
    vh = v[s] / (1.0 - ADAM_B2 ** t)
    P[s] -= lr * mh / (np.sqrt(vh) + ADAM_EPS)
    return P, m, v


def predict(P, feat):
    """Chosen class and softmax probability of each head for one sample
    (bf16 forward)."""
    z, _ = forward(P, np.asarray(feat, np.float32).reshape(1, NFEAT))
    out = []
    for o, k in _heads(z):
        zz = z[0, o:o + k]
        i = int(np.argmax(zz))
        ez = np.exp(zz - zz.max())
        out.append((i, float(ez[i] / ez.sum())))
    return out
