"""Pins of the learned-tuner oracle (block features, bf16 MLP, Adam)
against closed forms, brute force and library routines."""
import numpy as np
import pytest
import torch

from oracle import ref, ref_learned as rl


# ------------------------------------------------------------- bf16 rounding
def test_bf16_matches_torch_rounding():
    rng = np.random.default_rng(0)
    vals = np.concatenate([
        rng.normal(0, 1, 4000), rng.normal(0, 1e-30, 100),
        rng.normal(0, 1e30, 100),
        # ties: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6, their negatives
        [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 0.0, -0.0,
         2.0 ** -130, 3.0e38]]).astype(np.float32)
    want = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64)
    assert np.array_equal(rl.bf16(vals), want.numpy())
    assert rl.bf16(np.float32(1 + 2.0 ** -8)) == 1.0
    assert rl.bf16(np.float32(1 + 3 * 2.0 ** -8)) == 1 + 2.0 ** -6


# ---------------------------------------------------------------- features
def counts(l, d=3):
    """Targets of level l per dimension, and how many of them along one
    dimension lack the cubic stencil's outer points (d-dimensional block)."""
    h = 1 << (l - 1)
    m = 32 // h + 1
    odd = list(range(1, m, 2))
    lin_only = [j for j in odd if not (j - 3 >= 0 and j + 3 <= m - 1)]
    return len(odd) * m ** (d - 1), len(lin_only) * m ** (d - 1)


def test_linear_field_features():
    # x = 2i + 3j - k: every residual 0, g2 = 4 + 9 + 1 everywhere
    i, j, k = np.meshgrid(*[np.arange(33, dtype=np.float32)] * 3,
                          indexing="ij")
    x = (2 * i + 3 * j - k).astype(np.float32)
    e = 0.25
    f = rl.block_features(x, e, vrange=200.0)
    assert np.all(f[:20] == 0.0)
    assert np.allclose(f[20:30], np.log2(1 + np.sqrt(14.0) / e), rtol=1e-7)
    assert f[30] == np.float32(np.log2(1 + (x.max() - x.min()) / e))
    assert f[31] == np.float32(np.log2(1 + 200.0 / e))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_quadratic_residuals_closed_form(axis):
    # x = t^2 along one axis (t from a block origin offset of 5): linear
    # residual -h^2 at every target along that axis, 0 along the others;
    # cubic exact where it has four points, -h^2 where it falls back.
    t = (np.arange(33, dtype=np.float32) + 5) ** 2
    shape = [1, 1, 1]
    shape[axis] = 33
    x = np.broadcast_to(t.reshape(shape), (33, 33, 33)).astype(np.float32)
    e = 0.5
    f = rl.block_features(np.ascontiguousarray(x), e, vrange=1.0)
    for l in range(1, 6):
        h = 1 << (l - 1)
        per_dim, lin_only = counts(l)
        n = 3 * per_dim
        lin_mean = per_dim * h * h / n
        cub_mean = lin_only * h * h / n
        lin_rms = np.sqrt(per_dim * h ** 4 / n)
        cub_rms = np.sqrt(lin_only * h ** 4 / n)
        exp = [np.log2(1 + lin_mean / e), np.log2(1 + lin_rms / e),
               np.log2(1 + cub_mean / e), np.log2(1 + cub_rms / e)]
        got = f[4 * (l - 1):4 * l].astype(np.float64)
        assert np.allclose(got, exp, rtol=2e-7), (l, got, exp)


def test_linear_field_features_2d():
    # x = 2i - 5j on a 33 x 33 block: every residual 0, g2 = 4 + 25
    i, j = np.meshgrid(*[np.arange(33, dtype=np.float32)] * 2, indexing="ij")
    x = (2 * i - 5 * j).astype(np.float32)
    e = 0.125
    f = rl.block_features(x, e, vrange=300.0)
    assert np.all(f[:20] == 0.0)
    assert np.allclose(f[20:30], np.log2(1 + np.sqrt(29.0) / e), rtol=1e-7)
    assert f[30] == np.float32(np.log2(1 + (x.max() - x.min()) / e))
    assert f[31] == np.float32(np.log2(1 + 300.0 / e))


@pytest.mark.parametrize("axis", [0, 1])
def test_quadratic_residuals_closed_form_2d(axis):
    # as the 3D case on a 33 x 33 block: targets along the two dimensions
    t = (np.arange(33, dtype=np.float32) + 2) ** 2
    shape = [1, 1]
    shape[axis] = 33
    x = np.ascontiguousarray(
        np.broadcast_to(t.reshape(shape), (33, 33)).astype(np.float32))
    e = 2.0
    f = rl.block_features(x, e, vrange=1.0)
    for l in range(1, 6):
        h = 1 << (l - 1)
        per_dim, lin_only = counts(l, 2)
        n = 2 * per_dim
        exp = [np.log2(1 + per_dim * h * h / n / e),
               np.log2(1 + np.sqrt(per_dim * h ** 4 / n) / e),
               np.log2(1 + lin_only * h * h / n / e),
               np.log2(1 + np.sqrt(lin_only * h ** 4 / n) / e)]
        got = f[4 * (l - 1):4 * l].astype(np.float64)
        assert np.allclose(got, exp, rtol=2e-7), (l, got, exp)
    # g2 = (2t + 1)^2 along the axis: nearest-rank deciles of 32 values
    # each taken 32 times
    d = np.diff(t.astype(np.float64))
    g2 = np.repeat(d * d, 32)
    for q in range(1, 11):
        v = np.percentile(g2, 10 * q, method="inverted_cdf")
        assert f[19 + q] == np.float32(np.log2(1 + np.sqrt(v) / e)), q


def test_gradient_deciles_nearest_rank():
    # x varies along axis 0 only: g2 = dx^2 with each of 32 values taken
    # 32*32 times; deciles by the inverted-CDF (nearest-rank) definition
    rng = np.random.default_rng(3)
    s = np.cumsum(rng.integers(0, 7, 33)).astype(np.float32)
    x = np.broadcast_to(s.reshape(33, 1, 1), (33, 33, 33)).astype(np.float32)
    e = 1.0
    f = rl.block_features(np.ascontiguousarray(x), e, vrange=1.0)
    g2 = np.repeat((np.diff(s).astype(np.float64)) ** 2, 32 * 32)
    for q in range(1, 11):
        v = np.percentile(g2, 10 * q, method="inverted_cdf")
        assert f[19 + q] == np.float32(np.log2(1 + np.sqrt(v) / e)), q


def test_field_features_mean_over_sampled_blocks():
    from paper_2310_14133_amd import fields
    x = fields.grf((70, 66, 80), 7)
    plan = ref.sample_plan(x.shape, cfg=ref.tune_config(block=32,
                                                        sample_rate=0.5))
    assert plan["block_dims"] == (33, 33, 33)
    per, mean = rl.field_features(x, 1e-3, plan["origins"])
    assert per.shape == (plan["nblocks"], 32)
    assert np.allclose(mean, per.astype(np.float64).mean(axis=0), rtol=1e-7)
    # each block on its own; the range feature spans all sampled blocks
    blks = [np.ascontiguousarray(x[o[0]:o[0] + 33, o[1]:o[1] + 33,
                                   o[2]:o[2] + 33]) for o in plan["origins"]]
    lo = min(float(b.min()) for b in blks)
    hi = max(float(b.max()) for b in blks)
    assert hi - lo < float(x.max()) - float(x.min())  # not the field's
    assert np.array_equal(per[-1], rl.block_features(blks[-1], 1e-3, hi - lo))
    assert np.all(per[:, 31] == per[0, 31])


def test_field_features_2d():
    from paper_2310_14133_amd import fields
    x = fields.grf((150, 170), 8)
    plan = ref.sample_plan(x.shape, cfg=ref.tune_config(block=32,
                                                        sample_rate=0.2))
    assert plan["block_dims"] == (33, 33)
    per, mean = rl.field_features(x, 1e-3, plan["origins"])
    assert per.shape == (plan["nblocks"], 32) and plan["nblocks"] > 1
    blks = [np.ascontiguousarray(x[o[0]:o[0] + 33, o[1]:o[1] + 33])
            for o in plan["origins"]]
    lo = min(float(b.min()) for b in blks)
    hi = max(float(b.max()) for b in blks)
    for r, b in zip(per, blks):
        assert np.array_equal(r, rl.block_features(b, 1e-3, hi - lo))
    acc = np.zeros(32)
    for r in per:
        acc += r.astype(np.float64)
    assert np.array_equal(mean, (acc / len(per)).astype(np.float32))


# --------------------------------------------------------------------- MLP
def random_problem(B, seed):
    rng = np.random.default_rng(seed)
    P = rl.init_params(seed, mu=rng.normal(0, 1, 32).astype(np.float32),
                       sg=rng.uniform(0.5, 2, 32).astype(np.float32))
    P[rl.OFF_B1:rl.OFF_W2] = rng.normal(0, 0.1, 128)
    P[rl.OFF_B2:rl.OFF_W3] = rng.normal(0, 0.1, 128)
    P[rl.OFF_B3:] = rng.normal(0, 0.1, 11)
    feat = rng.normal(0, 2, (B, 32)).astype(np.float32)
    lab = np.stack([rng.integers(0, k, B) for k in rl.HEADS], axis=1)
    return P, feat, lab


def test_gradient_matches_finite_differences():
    P, feat, lab = random_problem(5, 1)
    P64 = P.astype(np.float64)
    _, g = rl.loss_and_grad(P64, feat, lab, use_bf16=False)

    def loss_at(Q):
        # the float64 path: parameters used unrounded
        p = dict(
            W1=Q[rl.OFF_W1:rl.OFF_B1].reshape(128, 32), b1=Q[rl.OFF_B1:rl.OFF_W2],
            W2=Q[rl.OFF_W2:rl.OFF_B2].reshape(128, 128), b2=Q[rl.OFF_B2:rl.OFF_W3],
            W3=Q[rl.OFF_W3:rl.OFF_B3].reshape(11, 128), b3=Q[rl.OFF_B3:])
        X = rl.normalise(feat, P).astype(np.float64)
        h1 = np.maximum(X @ p["W1"].T + p["b1"], 0)
        h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0)
        z = h2 @ p["W3"].T + p["b3"]
        tot = 0.0
        o = 0
        for hi, k in enumerate(rl.HEADS):
            zz = z[:, o:o + k]
            lse = np.log(np.exp(zz).sum(axis=1))
            tot += np.sum(lse - zz[np.arange(len(z)), lab[:, hi]])
            o += k
        return tot / len(z)

    rng = np.random.default_rng(2)
    idx = np.concatenate([
        rng.integers(rl.OFF_W1, rl.OFF_B1, 12),
        rng.integers(rl.OFF_B1, rl.OFF_W2, 6),
        rng.integers(rl.OFF_W2, rl.OFF_B2, 12),
        rng.integers(rl.OFF_B2, rl.OFF_W3, 6),
        rng.integers(rl.OFF_W3, rl.OFF_B3, 12),
        np.arange(rl.OFF_B3, rl.NPARAM)])
    for i in idx:
        step = 1e-6
        Qp = P64.copy()
        Qp[i] += step
        Qm = P64.copy()
        Qm[i] -= step
        fd = (loss_at(Qp) - loss_at(Qm)) / (2 * step)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])
    assert np.all(g[:rl.OFF_W1] == 0.0)


def test_uniform_logits_loss():
    P, feat, lab = random_problem(7, 3)
    P[rl.OFF_W3:] = 0.0
    loss, g = rl.loss_and_grad(P, feat, lab)
    assert abs(loss - np.log(2 * 5 * 4)) < 1e-12
    # bias gradient: mean over samples of (uniform probability - one-hot)
    want = np.zeros(11)
    o = 0
    for hi, k in enumerate(rl.HEADS):
        for s in range(7):
            want[o:o + k] += 1.0 / k / 7
            want[o + lab[s, hi]] -= 1.0 / 7
        o += k
    assert np.allclose(g[rl.OFF_B3:], want, atol=1e-15)


def test_bf16_path_close_to_float64_path():
    P, feat, lab = random_problem(64, 4)
    z16, _ = rl.forward(P, feat, use_bf16=True)
    z64, _ = rl.forward(P, feat, use_bf16=False)
    assert np.linalg.norm(z16 - z64) <= 2e-2 * np.linalg.norm(z64)
    _, g16 = rl.loss_and_grad(P, feat, lab, use_bf16=True)
    _, g64 = rl.loss_and_grad(P, feat, lab, use_bf16=False)
    assert np.linalg.norm(g16 - g64) <= 3e-2 * np.linalg.norm(g64)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    P = rng.normal(size=rl.NPARAM)
    g = rng.normal(size=rl.NPARAM)
    z = np.zeros(rl.NPARAM)
    P1, m, v = rl.adam(P, z, z, g, 1e-3, 1)
    s = slice(rl.OFF_W1, None)
    assert np.allclose(P1[s], P[s] - 1e-3 * g[s] / (np.abs(g[s]) + 1e-8),
                       rtol=0, atol=1e-15)
    assert np.array_equal(P1[:rl.OFF_W1], P[:rl.OFF_W1])
    assert np.allclose(m[s], 0.1 * g[s]) and np.allclose(v[s], 0.001 * g[s] ** 2)


def test_training_fits_a_separable_toy():
    # labels decided by signs of three features: Adam on the float64 path
    # drives the loss far below its starting value
    rng = np.random.default_rng(6)
    feat = rng.normal(0, 1, (64, 32)).astype(np.float32)
    lab = np.stack([(feat[:, 0] > 0).astype(int),
                    (feat[:, 1] > 0).astype(int) * 4,
                    (feat[:, 2] > 0).astype(int) * 3], axis=1)
    P = rl.init_params(6).astype(np.float64)
    m = np.zeros(rl.NPARAM)
    v = np.zeros(rl.NPARAM)
    l0, _ = rl.loss_and_grad(P, feat, lab, use_bf16=False)
    for t in range(1, 151):
        _, g = rl.loss_and_grad(P, feat, lab, use_bf16=False)
        P, m, v = rl.adam(P, m, v, g, 3e-3, t)
    l1, _ = rl.loss_and_grad(P, feat, lab, use_bf16=False)
    assert l1 < 0.05 * l0
