"""Oracle pins: interpolation stencils, polynomial reproduction, linear-scale
quantization and the error bound (Sec. III, Sec. V, Eq. 5).  CPU only."""
import itertools
import math

import numpy as np
import pytest

from paper_2310_14133_amd import fields

R = 32768
NODES = {"a": -3.0, "b": -1.0, "c": 1.0, "d": 3.0}


def lagrange_at_zero(nodes, vals):
    """Library route: numpy polynomial through the nodes, evaluated at 0."""
    coef = np.polyfit(np.array(nodes, np.float64), np.array(vals, np.float64),
                      len(nodes) - 1)
    return float(np.polyval(coef, 0.0))


@pytest.mark.parametrize("seed", range(20))
def test_stencils_match_polynomial_fits(ref, seed):
    rng = np.random.default_rng(seed)
    v = {k: float(np.float32(rng.uniform(-10, 10))) for k in "abcd"}
    cases = [
        # (cubic, has_a, has_c, has_d, nodes used)
        (1, 1, 1, 1, "abcd"), (1, 0, 1, 1, "bcd"), (1, 1, 1, 0, "abc"),
        (1, 0, 1, 0, "bc"), (0, 1, 1, 1, "bc"), (0, 0, 1, 0, "bc"),
        (1, 1, 0, 0, "ab"), (0, 1, 0, 0, "ab"), (1, 0, 0, 0, "b"),
        (0, 0, 0, 0, "b"),
    ]
    for cubic, ha, hc, hd, used in cases:
        got = ref.stencil(cubic, v["a"], v["b"], v["c"], v["d"], ha, hc, hd)
        if used == "b":
            want = v["b"]
        else:
            want = lagrange_at_zero([NODES[k] for k in used],
                                    [v[k] for k in used])
        assert abs(got - want) <= 1e-5 * max(1.0, abs(want)), (cubic, used)


def test_stencils_exact_on_integer_polynomials(ref):
    """4-point cubic reproduces degree 3; one-sided quadratics degree 2;
    the mean and the extrapolation degree 1 -- exactly, in FP32."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        c = rng.integers(-5, 6, size=4).astype(np.float64)
        h = int(rng.integers(1, 5))
        x0 = int(rng.integers(-20, 21))
        f = lambda t, deg: sum(c[i] * t ** i for i in range(deg + 1))
        pts = {k: x0 + NODES[k] * h for k in "abcd"}
        for deg, cubic, ha, hc, hd in [(3, 1, 1, 1, 1), (2, 1, 0, 1, 1),
                                       (2, 1, 1, 1, 0), (1, 1, 0, 1, 0),
                                       (1, 0, 1, 1, 1), (1, 1, 1, 0, 0),
                                       (1, 0, 1, 0, 0), (0, 1, 0, 0, 0)]:
            vals = {k: np.float32(f(pts[k], deg)) for k in "abcd"}
            got = ref.stencil(cubic, vals["a"], vals["b"], vals["c"],
                              vals["d"], ha, hc, hd)
            assert got == np.float32(f(x0, deg)), (deg, cubic, ha, hc, hd)
    # degree 4 is not reproduced: t^4 at (-3,-1,1,3) = (81,1,1,81) gives
    # (9*(1+1) - (81+81))/16 = -9 instead of 0
    vals = [np.float32(t ** 4) for t in (-3, -1, 1, 3)]
    assert ref.stencil(1, *vals, 1, 1, 1) == -9.0


def v2(c):
    c = int(c)
    return 10 ** 9 if c == 0 else (c & -c).bit_length() - 1


def level_and_dir(p, orders):
    vs = [v2(c) for c in p]
    m = min(vs)
    l = m + 1
    order = orders[l - 1]
    j = max(pos for pos in range(len(p)) if vs[order[pos]] == m)
    return l, order[j], 1 << m


@pytest.mark.parametrize("dims,s,deg,interp", [
    ((33, 33), 32, 1, "linear"), ((65, 65), 32, 2, "cubic"),
    ((17, 17, 17), 16, 1, "linear"), ((17, 17, 17), 8, 2, "cubic"),
    ((33, 17, 25), 8, 2, "cubic"), ((6, 11), 4, 0, "cubic"),
    ((10, 13, 7), 4, 0, "linear")])
def test_polynomial_reproduction(ref, dims, s, deg, interp):
    """Fields on n = s*m + 1 grids (no extrapolation needed): linear
    interpolation reproduces degree 1 everywhere; with m >= 2 every cubic
    target has at least three stencil points (one-sided quadratics at the
    edges), so cubic reproduces degree 2 everywhere.  Every bin is then the
    zero bin R and the reconstruction is exact.  Constants reproduce on any
    grid."""
    x = fields.polynomial(dims, deg, seed=deg + len(dims))
    rng = np.random.default_rng(3)
    perms = list(itertools.permutations(range(len(dims))))
    orders = [list(perms[rng.integers(len(perms))]) for _ in range(16)]
    p = ref.make_params(len(dims), interp, orders, 1.5, 3.0, anchor_stride=s)
    codes, recon, unpred, _ = ref.predict_quantize(x, 0.01, p)
    assert unpred.size == 0
    assert np.all(codes == R)
    assert np.array_equal(recon, x)


@pytest.mark.parametrize("dims,s", [((17, 17, 17), 16), ((33, 33), 32)])
def test_cubic_reproduces_degree_three_in_the_interior(ref, dims, s):
    """A target whose four stencil points exist and were reconstructed
    exactly is predicted exactly by the cubic rule on a degree-3 field."""
    x = fields.polynomial(dims, 3, seed=11, max_coef=1)
    d = len(dims)
    orders = [tuple(range(d))] * 16
    p = ref.make_params(d, "cubic", None, 1.0, 1.0, anchor_stride=s)
    idx, pred, codes = ref.target_trace(x, 0.25, p)
    _, recon, _, _ = ref.predict_quantize(x, 0.25, p)
    xf, rf = x.ravel(), recon.ravel()
    checked = 0
    for t in range(idx.size):
        pnt = np.unravel_index(int(idx[t]), dims)
        l, k, h = level_and_dir(pnt, orders)
        pk = pnt[k]
        if pk - 3 * h < 0 or pk + 3 * h > dims[k] - 1:
            continue
        st = int(np.prod(dims[k + 1:]))
        nb = [int(idx[t]) + o * h * st for o in (-3, -1, 1, 3)]
        if all(rf[i] == xf[i] for i in nb):
            assert pred[t] == xf[idx[t]]
            assert codes[t] == R
            checked += 1
    assert checked > 10


def test_quantizer_worked_example(ref):
    """Hand-worked 3x3 field, anchor stride 2, e = 0.25 (bin width 0.5):
    sweep along dim 0 then dim 1; later predictions use reconstructed values;
    halves round to even; an out-of-range residual is unpredictable."""
    x = np.array([[0.0, 0.75, 1.0],
                  [1.75, 2.975, 2.625],
                  [2.0, 1.0e6, 4.0]], np.float32)
    p = ref.make_params(2, "cubic", (0, 1), 1.0, 1.0, anchor_stride=2)
    codes, recon, unpred, anchors = ref.predict_quantize(x, 0.25, p)
    # stream order: (1,0) (1,2) | (0,1) (1,1) (2,1)
    # (1,0): pred 1, residual 0.75 -> 1.5 bins -> 2 (even), recon 2.0
    # (1,2): pred 2.5, residual 0.125 -> 0.25 -> 0, recon 2.5
    # (0,1): pred 0.5, residual 0.25 -> 0.5 -> 0 (even), recon 0.5
    # (1,1): pred (2.0 + 2.5)/2 = 2.25 from RECONSTRUCTED neighbours,
    #        residual 0.725 -> 1.45 -> 1, recon 2.75
    #        (original neighbours would give pred 2.1875 -> 1.575 -> 2)
    # (2,1): pred 3, residual ~1e6 -> beyond 32768 bins -> unpredictable
    assert codes.tolist() == [R + 2, R, R, R + 1, 0]
    assert unpred.tolist() == [1.0e6]
    assert anchors.tolist() == [0.0, 1.0, 2.0, 4.0]
    assert recon.tolist() == [[0.0, 0.5, 1.0], [2.0, 2.75, 2.5],
                              [2.0, 1.0e6, 4.0]]


FIELDS = [
    ("grf2", lambda: fields.grf((70, 45), 5)),
    ("bumps", lambda: fields.bumps_and_waves(64, 2)),
    ("grf3", lambda: fields.grf((19, 24, 33), 6)),
    ("lognormal3", lambda: fields.grf((20, 20, 20), 7, log_normal=True)),
    ("spikes", lambda: fields.adversarial((30, 31), "spikes", 1)),
    ("steps", lambda: fields.adversarial((17, 18, 19), "steps", 2)),
    ("alternating", lambda: fields.adversarial((25, 26), "alternating", 3)),
    ("noise", lambda: fields.adversarial((12, 13, 14), "noise", 4)),
]


@pytest.mark.parametrize("name,make", FIELDS)
@pytest.mark.parametrize("rel,alpha,beta,interp", [
    (1e-2, 1.0, 1.5, "cubic"), (1e-3, 1.75, 3.0, "linear"),
    (1e-4, 2.0, 4.0, "cubic")])
def test_error_bound_per_level(ref, name, make, rel, alpha, beta, interp):
    """|x - x'| <= e_l for every target of level l (hence <= e), and the
    decoder reproduces the encoder's reconstruction bit for bit."""
    x = make()
    d = x.ndim
    vr = float(x.max()) - float(x.min())
    e = rel * vr
    s = 16 if d == 2 else 8
    rng = np.random.default_rng(len(name))
    perms = list(itertools.permutations(range(d)))
    orders = [list(perms[rng.integers(len(perms))]) for _ in range(16)]
    p = ref.make_params(d, interp, orders, alpha, beta, anchor_stride=s)
    codes, recon, unpred, anchors = ref.predict_quantize(x, e, p)
    idx, _, _ = ref.target_trace(x, e, p)
    el, _, _ = ref.level_bounds(e, alpha, beta, int(math.log2(s)))
    err = np.abs(x.astype(np.float64).ravel() - recon.astype(np.float64).ravel())
    levels = np.array([level_and_dir(np.unravel_index(int(i), x.shape),
                                     orders)[0] for i in idx])
    for l in range(1, int(math.log2(s)) + 1):
        sel = idx[levels == l]
        if sel.size:
            assert err[sel].max() <= el[l - 1]
    assert err.max() <= e
    y = ref.reconstruct(codes, unpred, anchors, x.shape, e, p)
    assert np.array_equal(y, recon)
    if name == "spikes":
        assert unpred.size > 0


def test_zero_and_constant_fields(ref):
    for val in (0.0, 3.5):
        x = np.full((20, 21, 22), val, np.float32)
        p = ref.make_params(3, "cubic", None, 1.0, 1.0)
        codes, recon, unpred, _ = ref.predict_quantize(x, 1e-3, p)
        assert np.all(codes == R) and unpred.size == 0
        assert np.array_equal(recon, x)


def test_denormal_field_and_tiny_bound(ref):
    x = fields.adversarial((16, 17), "denormal", 5)
    p = ref.make_params(2, "cubic", None, 1.25, 2.0, anchor_stride=8)
    e = 1e-41
    codes, recon, unpred, anchors = ref.predict_quantize(x, e, p)
    assert np.abs(x.astype(np.float64) - recon).max() <= e
    y = ref.reconstruct(codes, unpred, anchors, x.shape, e, p)
    assert np.array_equal(y, recon)


def test_invalid_inputs_rejected(ref):
    x = fields.grf((16, 16), 1)
    p = ref.make_params(2)
    bad = x.copy()
    bad[3, 4] = np.nan
    for arr, e in [(bad, 0.1), (x, 0.0), (x, -1.0), (x, float("inf"))]:
        with pytest.raises(ref.OracleError) as ei:
            ref.predict_quantize(arr, e, p)
        assert ei.value.code == ref.EINVAL
    inf = x.copy()
    inf[0, 0] = np.inf
    with pytest.raises(ref.OracleError):
        ref.predict_quantize(inf, 0.1, p)
    q = ref.make_params(2, order=(0, 0))
    with pytest.raises(ref.OracleError):
        ref.predict_quantize(x, 0.1, q)
    q = ref.make_params(2, alpha=0.5)
    with pytest.raises(ref.OracleError):
        ref.predict_quantize(x, 0.1, q)
    q = ref.make_params(2, anchor_stride=12)
    with pytest.raises(ref.OracleError):
        ref.predict_quantize(x, 0.1, q)
