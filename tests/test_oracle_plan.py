"""Oracle pins: level bounds (Eq. 5), level/sweep schedule (Sec. V), sampling
plan (Sec. VI-A).  CPU only."""
import itertools
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- Eq. 5 ---

def test_level_bound_policy(ref):
    """Sec. V-B policy: e_l <= e, e_1 = e, e_l non-increasing in l."""
    g = gold("paper_values.json")["alpha_beta_candidates"]
    e = 0.37
    for a, b in itertools.product(g["alpha"], g["beta"]):
        el, tw, iv = ref.level_bounds(e, a, b, 8)
        assert el[0] == e
        assert np.all(el <= e)
        assert np.all(np.diff(el) <= 0)
        # the cap beta: e_l never drops below e / beta
        assert np.all(el >= e / b * (1 - 1e-15))


def test_level_bound_fig5_example(ref):
    """Fig. 5 discussion: e = 0.1 on level 1 and 0.05 on level 2, i.e.
    min(alpha, beta) = 2; among the candidates exactly (2,2), (2,3), (2,4)."""
    g = gold("paper_values.json")
    ex = g["level_bound_example"]
    cand = g["alpha_beta_candidates"]
    hits = []
    for a, b in itertools.product(cand["alpha"], cand["beta"]):
        el, _, _ = ref.level_bounds(ex["e"], a, b, 6)
        assert el[0] == ex["e1"]
        if abs(el[1] - ex["e2"]) < 1e-15:
            hits.append((a, b))
    assert hits == [(2.0, 2.0), (2.0, 3.0), (2.0, 4.0)]


def test_level_bound_alpha_one_is_uniform(ref):
    for b in (1.5, 2.0, 3.0, 4.0):
        el, _, _ = ref.level_bounds(0.25, 1.0, b, 6)
        assert np.all(el == 0.25)


def test_level_bound_values_and_fp32_forms(ref):
    # alpha^(l-1) grows until it meets beta: alpha=1.5, beta=3, e=1
    el, tw, iv = ref.level_bounds(1.0, 1.5, 3.0, 5)
    expect = [1.0, 1 / 1.5, 1 / 2.25, 1 / 3.0, 1 / 3.0]
    assert np.allclose(el, expect, rtol=1e-15, atol=0)
    assert np.array_equal(tw, (2.0 * el).astype(np.float32))
    assert np.array_equal(iv, (1.0 / (2.0 * el)).astype(np.float32))


def test_distinct_bound_vectors(ref):
    """With Lt = 5 levels, 14 of the 20 (alpha, beta) pairs give distinct
    level-bound vectors (alpha = 1 collapses beta; beta = 1.5 caps early)."""
    cand = gold("paper_values.json")["alpha_beta_candidates"]
    vecs = set()
    for a, b in itertools.product(cand["alpha"], cand["beta"]):
        el, _, _ = ref.level_bounds(1.0, a, b, 5)
        vecs.add(tuple(el))
    assert len(vecs) == 14


# ------------------------------------------------------ sweep schedule ---

def v2(c):
    """2-adic valuation, with v2(0) = infinity."""
    if c == 0:
        return 10 ** 9
    return (c & -c).bit_length() - 1


def brute_stream_order(dims, s, orders):
    """Expected stream order of targets, derived point by point: a point's
    level is 1 + min valuation of its coordinates; its sweep is the last
    position (in the level's order) holding a coordinate of that valuation;
    codes run level L..1, sweep 0..d-1, row-major within a sweep."""
    L = int(math.log2(s))
    d = len(dims)
    keyed = []
    for p in itertools.product(*[range(n) for n in dims]):
        vs = [v2(c) for c in p]
        m = min(vs)
        if m >= L:
            continue
        l = m + 1
        order = orders[l - 1]
        j = max(pos for pos in range(d) if vs[order[pos]] == m)
        flat = int(np.ravel_multi_index(p, dims))
        keyed.append((-l, j, flat))
    keyed.sort()
    return np.array([k[2] for k in keyed], np.uint32), [k[0] for k in keyed]


@pytest.mark.parametrize("dims,s", [((9, 9), 4), ((6, 11), 4), ((17, 13), 8),
                                    ((5, 7, 9), 4), ((10, 13, 7), 4),
                                    ((9, 9, 9), 8)])
def test_stream_order_matches_pointwise_definition(ref, dims, s):
    rng = np.random.default_rng(len(dims) * 100 + s)
    d = len(dims)
    perms = list(itertools.permutations(range(d)))
    orders = [perms[rng.integers(len(perms))] for _ in range(16)]
    x = rng.standard_normal(dims).astype(np.float32)
    p = ref.make_params(d, "cubic", [list(o) for o in orders], 1.0, 1.0,
                        anchor_stride=s)
    idx, _, _ = ref.target_trace(x, 0.01, p)
    expect, _ = brute_stream_order(dims, s, orders)
    assert np.array_equal(idx, expect)
    # every non-anchor point is a target exactly once
    n_anchor = int(np.prod([(n - 1) // s + 1 for n in dims]))
    assert idx.size == x.size - n_anchor
    assert np.unique(idx).size == idx.size


@pytest.mark.parametrize("d", [2, 3])
def test_level_one_fraction(ref, d):
    """Sec. V-B: level 1 holds 75% (2D) / 87.5% (3D) of the points."""
    frac = gold("paper_values.json")["level1_fraction"][str(d)]
    n = 1025 if d == 2 else 129
    s = 64 if d == 2 else 32
    # closed form on an n = s*m + 1 grid: level-l targets are the points of
    # the stride-2^(l-1) grid that are not on the stride-2^l grid
    g = lambda l: (n - 1) // (1 << (l - 1)) + 1
    lvl1 = g(1) ** d - g(2) ** d
    assert abs(lvl1 / n ** d - frac) < 0.01
    # the oracle's schedule agrees on a small grid of the same form
    m = 33 if d == 2 else 17
    ss = 32 if d == 2 else 16
    x = np.zeros((m,) * d, np.float32)
    p = ref.make_params(d, "linear", None, 1.0, 1.0, anchor_stride=ss)
    idx, _, _ = ref.target_trace(x, 0.5, p)
    _, levels = brute_stream_order((m,) * d, ss, [tuple(range(d))] * 16)
    lv = -np.array(levels)
    for l in range(1, int(math.log2(ss)) + 1):
        gl = (m - 1) // (1 << (l - 1)) + 1
        gl1 = (m - 1) // (1 << l) + 1
        assert np.sum(lv == l) == gl ** d - gl1 ** d
    assert idx.size == m ** d - 2 ** d


def test_anchor_counts(ref):
    """Anchor grid: prod(floor((n_i - 1)/s) + 1) points, stored raw."""
    for dims, s, count in [((512, 512, 512), 32, 4096), ((256, 256), 64, 16),
                           ((6, 11), 4, 6), ((10, 13, 7), 4, 3 * 4 * 2)]:
        assert int(np.prod([(n - 1) // s + 1 for n in dims])) == count
    x = np.arange(10 * 13 * 7, dtype=np.float32).reshape(10, 13, 7)
    p = ref.make_params(3, "cubic", None, 1.0, 1.0, anchor_stride=4)
    _, _, _, anchors = ref.predict_quantize(x, 0.5, p)
    expect = x[::4, ::4, ::4].ravel()
    assert np.array_equal(anchors, expect)


# ----------------------------------------------------------- sampling ---

def test_sampling_rate_example(ref):
    """Sec. VI-A: 4x4 blocks at stride 10 sample 16% (2D)."""
    ex = gold("paper_values.json")["sampling_rate_example"]
    cfg = ref.tune_config(block=ex["block"], sample_rate=ex["rate"])
    plan = ref.sample_plan((400, 400), anchor_stride=64, cfg=cfg)
    assert plan["S"] == ex["stride"]
    assert abs((plan["b"] / plan["S"]) ** 2 - ex["rate"]) < 1e-12


def test_sampling_paper_defaults_and_512_cube(ref):
    dflt = gold("paper_values.json")["experiment_defaults"]
    p3 = ref.sample_plan((512, 512, 512))  # paper 3D defaults
    assert p3["b"] == dflt["3"]["block"]
    assert p3["S"] == round(16 * 0.005 ** (-1 / 3)) == 94
    assert p3["Lt"] == 4  # log2 min(16, 32)
    assert p3["nblocks"] == 6 ** 3
    p2 = ref.sample_plan((1800, 3600))
    assert p2["b"] == dflt["2"]["block"] and p2["Lt"] == 6
    assert p2["S"] == round(64 * 0.01 ** -0.5) == 640
    # 32^3 blocks at 1%: S = 149, 4 per dimension on 512 points
    cfg = ref.tune_config(block=32, sample_rate=0.01)
    p = ref.sample_plan((512, 512, 512), cfg=cfg)
    assert (p["S"], p["Lt"], p["nblocks"]) == (149, 5, 64)
    assert p["block_dims"] == (33, 33, 33)
    assert sorted(set(p["origins"][:, 0].tolist())) == [0, 149, 298, 447]
    # nominal rate (b/S)^3 close to r
    assert abs((32 / 149) ** 3 - 0.01) < 0.0001


def test_sampling_whole_field_fallback(ref):
    cfg = ref.tune_config(block=32, sample_rate=0.01)
    p = ref.sample_plan((20, 40, 40), cfg=cfg)
    assert p["nblocks"] == 1 and p["block_dims"] == (20, 40, 40)
