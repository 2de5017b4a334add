"""Shared checks of the GPU parity tests (imported by the test modules).

Tuner traces are compared element by element with the oracle's
(Algorithm 1, Sec. VI-B; the (alpha, beta) walk of Table I, Sec. VI-C):
per-level mean L1 errors within 1e-12 relative, bit rates exactly (both
sides divide the same integers), metrics within 1e-9 relative (PSNR, SSIM)
or absolute (-|AC|), the Table-I cases, e' factors and re-run results of
every challenge.  A decision may differ only where the oracle's own values
behind it are within the tie margin; the comparison stops there."""
import math

import numpy as np

TIE = 1e-9      # relative margin of a near-tie in a metric or L1 mean
TIE_SUMS = 1e-7  # SSIM and AC: sums over many windows or pairs


def near_tie(vals, chosen, rel=TIE):
    """Another candidate within `rel` of the chosen one but not equal to it.
    Exact ties (identical predictions, e.g. linear and cubic where only two
    stencil points exist) are resolved identically on both sides."""
    best = vals[chosen]
    return any(i != chosen and
               0 < abs(v - best) <= rel * max(abs(best), 1e-300)
               for i, v in enumerate(vals))


def _close(a, b, rel, absolute=False):
    if math.isinf(a) or math.isinf(b):
        return a == b
    if absolute:
        return abs(a - b) <= rel
    return abs(a - b) <= rel * max(abs(b), 1e-300)


def metric_close(a, b, target):
    if target == "cr":
        return a == b == 0.0
    if target == "ac":
        return _close(a, b, 1e-9, absolute=True)
    return _close(a, b, 1e-9)


def _tied(a, b, target):
    """Two of the oracle's values that a 1e-9 disagreement could reorder."""
    if target == "ac":
        return abs(a - b) <= 1e-7
    rel = TIE_SUMS if target == "ssim" else TIE
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


def check_trace(gt, rt, target):
    """Compare a GPU TuneTrace with the oracle's; returns None when every
    element was compared, else a note naming where a near-tie let the two
    walks part (everything before it was compared)."""
    assert (gt.Lt, gt.ncand, gt.nblocks, gt.block_points) == \
        (rt.Lt, rt.ncand, rt.nblocks, rt.block_points)
    nc = rt.ncand
    for l in range(rt.Lt, 0, -1):
        ge = [gt.alg1_err[l - 1][c] for c in range(nc)]
        re = [rt.alg1_err[l - 1][c] for c in range(nc)]
        for c in range(nc):
            assert _close(ge[c], re[c], 1e-12), (l, c, ge[c], re[c])
        gc, rc = gt.alg1_choice[l - 1], rt.alg1_choice[l - 1]
        if gc != rc:
            assert _tied(re[gc], re[rc], "psnr"), (l, gc, rc, re)
            return f"Algorithm 1 near-tie at level {l}"
    for i in range(20):
        assert gt.B[i] == rt.B[i], (i, gt.B[i], rt.B[i])
        assert metric_close(gt.M[i], rt.M[i], target), (i, gt.M[i], rt.M[i])
    inc = 0
    for i in range(1, 20):
        if gt.cmp_case[i] != rt.cmp_case[i]:
            # the case turns on B (exact) and M comparisons
            assert _tied(rt.M[inc], rt.M[i], target), \
                (i, gt.cmp_case[i], rt.cmp_case[i])
            return f"Table-I near-tie at pair {i}"
        assert gt.eprime[i] == rt.eprime[i], i
        if rt.eprime[i]:
            assert gt.Bp[i] == rt.Bp[i], (i, gt.Bp[i], rt.Bp[i])
            assert metric_close(gt.Mp[i], rt.Mp[i], target), \
                (i, gt.Mp[i], rt.Mp[i])
        else:
            assert math.isnan(gt.Bp[i]) and math.isnan(rt.Bp[i])
        # the oracle's incumbent after pair i
        cs = rt.cmp_case[i]
        if cs == 2:
            inc = i
        elif cs in (3, 4):
            B_I, M_I, B_II, M_II = rt.B[inc], rt.M[inc], rt.B[i], rt.M[i]
            if rt.Bp[i] != B_II:
                m_line = M_II + (rt.Mp[i] - M_II) * (B_I - B_II) / \
                    (rt.Bp[i] - B_II)
                if M_I < m_line:
                    inc = i
    assert inc == rt.best_pair
    if gt.best_pair != rt.best_pair:
        assert _tied(rt.M[gt.best_pair], rt.M[rt.best_pair], target)
        return "line test near-tie"
    return None


def to_ref_params(ref, qp, ndim):
    """The library's Params as the oracle's struct."""
    p = ref.Params()
    p.anchor_stride = qp.anchor_stride
    p.levels = qp.levels
    for l in range(16):
        p.interp[l] = qp.interp[l]
        for j in range(3):
            p.order[l][j] = qp.order[l][j]
    p.alpha, p.beta = qp.alpha, qp.beta
    return p


def to_lib_params(q, rp):
    """The oracle's Params as the library's struct."""
    p = q.Params()
    p.anchor_stride = rp.anchor_stride
    for l in range(16):
        p.interp[l] = rp.interp[l]
        for j in range(3):
            p.order[l][j] = rp.order[l][j]
    p.alpha, p.beta = rp.alpha, rp.beta
    return p


def streams_equal(zg, zr):
    assert zg.size == zr.size, (zg.size, zr.size)
    if not np.array_equal(zg, zr):
        diff = np.nonzero(zg != zr)[0]
        raise AssertionError(f"stream differs at {diff.size} bytes, first "
                             f"{diff[:8]}")
