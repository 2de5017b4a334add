"""Oracle pins: the online tuner -- Algorithm 1 (Sec. VI-B), the (alpha, beta)
candidates (Sec. VI-C-1) and the rate-quality comparison of Table I
(Sec. VI-C-2).  CPU only.

The brute-force checks drive the oracle's predictor (pinned on its own in
test_oracle_predict) block by block from Python, re-deriving every decision
with code written here, and compare with the oracle tuner's trace."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from paper_2310_14133_amd import fields

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PV = json.load(open(os.path.join(GOLD, "paper_values.json")))
ALPHAS = PV["alpha_beta_candidates"]["alpha"]
BETAS = PV["alpha_beta_candidates"]["beta"]


# ------------------------------------------------------------- Table I ---

def test_table1_cases(ref):
    # case 1: I has lower-or-equal rate and higher-or-equal metric
    assert ref.table1_case(1.0, 50.0, 2.0, 40.0) == 1
    assert ref.table1_case(1.0, 50.0, 1.0, 50.0) == 1   # identical -> I
    assert ref.table1_case(1.0, 50.0, 1.0, 40.0) == 1
    # case 2: II has lower-or-equal rate and higher-or-equal metric
    assert ref.table1_case(2.0, 40.0, 1.0, 50.0) == 2
    assert ref.table1_case(2.0, 50.0, 1.0, 50.0) == 2
    assert ref.table1_case(1.0, 40.0, 1.0, 50.0) == 2
    # case 3: I costs more and is better
    assert ref.table1_case(2.0, 50.0, 1.0, 40.0) == 3
    # case 4: I costs less and is worse
    assert ref.table1_case(1.0, 40.0, 2.0, 50.0) == 4


def test_table1_line(ref):
    # II at (1, 40) and (2, 50): the line through them has M = 30 + 10 B
    assert ref.table1_line(1.5, 44.0, 1.0, 40.0, 2.0, 50.0) == 1  # below
    assert ref.table1_line(1.5, 46.0, 1.0, 40.0, 2.0, 50.0) == 0  # above
    assert ref.table1_line(1.5, 45.0, 1.0, 40.0, 2.0, 50.0) == 0  # on: keep I
    assert ref.table1_line(3.0, 59.0, 1.0, 40.0, 2.0, 50.0) == 1  # extrapolated
    assert ref.table1_line(1.5, 10.0, 1.0, 40.0, 1.0, 50.0) == 0  # degenerate


def walk_table1(B, M, rerun, cr_mode):
    """Table I, written independently: incumbent I = pair 0, challenged by
    each later pair in order; cases 3/4 re-run II at 0.8e / 1.2e."""
    inc = 0
    log = []
    for i in range(1, len(B)):
        bi, mi, bii, mii = B[inc], M[inc], B[i], M[i]
        if cr_mode:
            if bii < bi:
                inc = i
            continue
        if bi <= bii and mi >= mii:
            continue
        if bi >= bii and mi <= mii:
            inc = i
            continue
        f = PV["eprime_factors"]["case3"] if (bi > bii and mi > mii) \
            else PV["eprime_factors"]["case4"]
        bp, mp = rerun(i, f)
        log.append((i, f))
        if bp == bii:
            continue
        mline = mii + (mp - mii) * (bi - bii) / (bp - bii)
        if mi < mline:
            inc = i
    return inc, log


# ----------------------------------------------------- block-wise driver ---

def extract_blocks(x, plan):
    bd = plan["block_dims"]
    out = []
    for o in plan["origins"]:
        sl = tuple(slice(int(a), int(a) + b) for a, b in zip(o, bd))
        out.append(np.ascontiguousarray(x[sl]))
    return out


def candidates(d, all_orders):
    if all_orders:
        orders = list(itertools.permutations(range(d)))
    else:
        orders = [tuple(range(d)), tuple(reversed(range(d)))]
    return [(t, o) for t in (0, 1) for o in orders]


def v2(c):
    c = int(c)
    return 10 ** 9 if c == 0 else (c & -c).bit_length() - 1


def target_levels(idx, dims):
    pts = np.array(np.unravel_index(idx.astype(np.int64), dims)).T
    out = np.empty(len(idx), np.int64)
    for i, p in enumerate(pts):
        out[i] = min(v2(c) for c in p) + 1
    return out


def params_for(ref, d, Lt, interp, order, alpha, beta):
    return ref.make_params(d, [interp[l] for l in range(16)],
                           [list(order[l]) for l in range(16)], alpha, beta,
                           anchor_stride=1 << Lt)


def alg1_bruteforce(ref, blocks, d, Lt, e, all_orders):
    cands = candidates(d, all_orders)
    interp = [0] * 16
    order = [tuple(range(d))] * 16
    errs, choice = {}, {}
    lv_cache = {}
    for l in range(Lt, 0, -1):
        best, ib = math.inf, None
        errs[l] = []
        for ci, (t, o) in enumerate(cands):
            it = list(interp)
            od = list(order)
            it[l - 1], od[l - 1] = t, o
            p = params_for(ref, d, Lt, it, od, 1.0, 1.0)
            s, n = 0.0, 0
            for b in blocks:
                idx, pred, _ = ref.target_trace(b, e, p)
                key = b.shape
                if key not in lv_cache:
                    lv_cache[key] = target_levels(idx, b.shape)
                sel = lv_cache[key] == l
                s += np.abs(b.ravel()[idx[sel]].astype(np.float64) -
                            pred[sel].astype(np.float64)).sum()
                n += int(sel.sum())
            cur = s / n if n else 0.0
            errs[l].append(cur)
            if cur < best:
                best, ib = cur, ci
        interp[l - 1], order[l - 1] = cands[ib]
        choice[l] = ib
    return errs, choice, interp, order


def trial_blockwise(ref, blocks, d, Lt, interp, order, alpha, beta, e,
                    vrange, target, w=7):
    """Bit rate and metric of one trial, aggregated over blocks."""
    p = params_for(ref, d, Lt, interp, order, alpha, beta)
    hist = np.zeros(2 * 32768, np.uint64)
    U = npts = 0
    sse = 0.0
    ssim_s, ssim_n = 0.0, 0
    errs = []
    for b in blocks:
        codes, recon, unpred, _ = ref.predict_quantize(b, e, p)
        hist += np.bincount(codes, minlength=hist.size).astype(np.uint64)
        U += unpred.size
        npts += b.size
        dd = b.astype(np.float64) - recon
        sse += float((dd * dd).sum())
        errs.append(dd.reshape(-1, b.shape[-1]))
        if target == "ssim":
            s, n = ref.ssim_sums(b, recon, w, vrange)
            ssim_s += s
            ssim_n += n
    bits = int((hist * ref.huffman_lengths(hist)).sum())
    B = (bits + 32.0 * U) / npts
    if target == "psnr":
        M = math.inf if sse == 0 else 20 * math.log10(vrange / math.sqrt(sse / npts))
    elif target == "ssim":
        M = ssim_s / ssim_n
    elif target == "ac":
        # lag 1 along rows; mean and variance over all block points
        r = np.concatenate(errs)
        mu = r.mean()
        var = ((r - mu) ** 2).mean()
        lag = ((r[:, :-1] - mu) * (r[:, 1:] - mu)).mean()
        M = -abs(lag / var) if var > 0 else 0.0
    else:
        M = 0.0
    return B, M, bits, U


CASES = [
    ("2d_psnr", lambda: fields.grf((80, 90), 31), (80, 90), 16,
     dict(block=16, sample_rate=0.1), "psnr", 1e-3),
    ("2d_cr", lambda: fields.bumps_and_waves(96, 3), (96, 96), 16,
     dict(block=16, sample_rate=0.1), "cr", 1e-2),
    ("3d_psnr_all", lambda: fields.grf((40, 36, 44), 32, log_normal=True),
     None, 8, dict(block=8, sample_rate=0.2, all_orders=1), "psnr", 1e-3),
    ("3d_ssim", lambda: fields.multiscale((30, 34, 38), 33), None, 8,
     dict(block=8, sample_rate=0.2), "ssim", 1e-2),
    ("3d_cr_all", lambda: fields.grf((36, 36, 36), 34), None, 8,
     dict(block=8, sample_rate=0.15, all_orders=1), "cr", 1e-4),
    # configurations whose walk switches incumbents and meets cases 2, 3, 4
    ("2d_psnr_switch", lambda: fields.bumps_and_waves(128, 5), None, 32,
     dict(block=32, sample_rate=0.2), "psnr", 1e-2),
    ("2d_ssim_switch", lambda: fields.bumps_and_waves(128, 5), None, 32,
     dict(block=32, sample_rate=0.2), "ssim", 1e-2),
    ("2d_cr_switch", lambda: fields.bumps_and_waves(128, 5), None, 32,
     dict(block=32, sample_rate=0.2), "cr", 1e-3),
    ("2d_psnr_case3", lambda: fields.bumps_and_waves(200, 6, noise=1e-4),
     None, 32, dict(block=32, sample_rate=0.2), "psnr", 1e-3),
    ("2d_ac", lambda: fields.grf((96, 100), 36), None, 16,
     dict(block=16, sample_rate=0.15), "ac", 1e-3),
    ("3d_ac_all", lambda: fields.multiscale((34, 36, 40), 37), None, 8,
     dict(block=8, sample_rate=0.2, all_orders=1), "ac", 1e-3),
]


@pytest.mark.parametrize("name,make,_,s,cfgkw,target,rel", CASES)
def test_tuner_bruteforce(ref, name, make, _, s, cfgkw, target, rel):
    x = make()
    d = x.ndim
    vr = float(x.max()) - float(x.min())
    e = rel * vr
    cfg = ref.tune_config(**cfgkw)
    p, tr = ref.tune(x, e, target, cfg, anchor_stride=s)
    plan = ref.sample_plan(x.shape, s, cfg)
    Lt = plan["Lt"]
    assert tr.Lt == Lt and tr.nblocks == plan["nblocks"]
    blocks = extract_blocks(x, plan)
    all_orders = bool(cfgkw.get("all_orders", 0))
    assert tr.ncand == (2 * math.factorial(d) if all_orders else 4)

    # Algorithm 1, re-derived
    errs, choice, interp, order = alg1_bruteforce(ref, blocks, d, Lt, e,
                                                  all_orders)
    for l in range(1, Lt + 1):
        assert choice[l] == tr.alg1_choice[l - 1], l
        got = [tr.alg1_err[l - 1][c] for c in range(tr.ncand)]
        assert np.allclose(got, errs[l], rtol=1e-12, atol=0)
    L = int(math.log2(s))
    for l in range(1, L + 1):
        src = min(l, Lt)
        assert p.interp[l - 1] == interp[src - 1]
        assert tuple(p.order[l - 1][j] for j in range(d)) == tuple(order[src - 1])

    # (alpha, beta) search, re-derived
    pairs = [(a, b) for a in ALPHAS for b in BETAS]
    B, M = [], []
    for i, (a, b) in enumerate(pairs):
        bi, mi, _, _ = trial_blockwise(ref, blocks, d, Lt, interp, order, a,
                                       b, e, vr, target)
        B.append(bi)
        M.append(mi)
        assert bi == tr.B[i]
        assert (mi == tr.M[i]) or abs(mi - tr.M[i]) <= 1e-11 * max(abs(mi), 1e-3)

    def rerun(i, f):
        a, b = pairs[i]
        bp, mp, _, _ = trial_blockwise(ref, blocks, d, Lt, interp, order, a,
                                       b, e * f, vr, target)
        assert bp == tr.Bp[i] and tr.eprime[i] == f
        return bp, mp

    inc, log = walk_table1(B, M, rerun, target == "cr")
    assert inc == tr.best_pair
    if name.endswith("switch") or name.endswith("case3"):
        assert inc != 0
    if name.endswith("case3"):
        assert 0.8 in [f for _, f in log] and 1.2 in [f for _, f in log]
    assert (p.alpha, p.beta) == pairs[inc]
    if target == "cr":
        assert not log
    # the tuned parameters compress within the bound
    y = ref.decompress(ref.compress(x, e, p))
    assert np.abs(x.astype(np.float64) - y).max() <= e


def test_single_block_trial_equals_real_compression(ref):
    """With the whole field as the only block (b = s = n - 1), a trial is
    the real compression: trial bits + 32 U equal the stream's Huffman cost
    plus 32 per unpredictable value, and trial PSNR is the real PSNR."""
    x = fields.grf((33, 33, 33), 40)
    vr = float(x.max()) - float(x.min())
    e = 1e-3 * vr
    cfg = ref.tune_config(block=32, sample_rate=1.0)
    p = ref.make_params(3, ["cubic", "linear"] * 8, [[2, 1, 0], [0, 2, 1]] * 8,
                        1.5, 3.0, anchor_stride=32)
    plan = ref.sample_plan(x.shape, 32, cfg)
    assert plan["nblocks"] == 1 and plan["block_dims"] == (33, 33, 33)
    r = ref.trial(x, e, p, cfg, vr)
    codes, recon, unpred, _ = ref.predict_quantize(x, e, p)
    hist = np.bincount(codes, minlength=65536).astype(np.uint64)
    bits = int((hist * ref.huffman_lengths(hist)).sum())
    assert r.payload_bits == bits and r.n_unpred == unpred.size
    assert r.n_points == x.size
    y = ref.decompress(ref.compress(x, e, p))
    psnr, _, _ = ref.metrics(x, y)
    trial_psnr = 20 * math.log10(vr / math.sqrt(r.sse / r.n_points))
    assert abs(trial_psnr - psnr) < 1e-9
    # ... and the trial's error autocorrelation is the real one
    ra = ref.trial(x, e, p, cfg, vr, want_ac=True)
    assert ra.ac == ref.error_ac(x, y)


def test_duplicate_bound_vectors_give_identical_trials(ref):
    x = fields.grf((48, 50), 41)
    vr = float(x.max()) - float(x.min())
    cfg = ref.tune_config(block=16, sample_rate=0.2)
    res = []
    for b in BETAS:
        p = ref.make_params(2, "cubic", None, 1.0, b, anchor_stride=16)
        r = ref.trial(x, 1e-3 * vr, p, cfg, vr, want_ssim=True)
        res.append((r.payload_bits, r.n_unpred, r.sse, r.ssim_sum))
    assert all(t == res[0] for t in res)


def test_candidate_counts_follow_paper():
    """Sec. V-B: 12 predictors per level in 3D; Sec. VI-B tests only 012/210."""
    g = PV["predictors_per_level_3d"]
    c = candidates(3, True)
    assert len(c) == g["count"]
    assert ["".join(map(str, o)) for _, o in c[:6]] == g["permutations"]
    assert ["".join(map(str, o)) for _, o in candidates(3, False)[:2]] == \
        PV["tested_orders"]["3"]


# ---- ablation switches (the component study of Sec. VII) ----
ABL_CASES = [
    ("2d", lambda: fields.grf((80, 90), 31), 16, dict(block=16,
                                                     sample_rate=0.1), 1e-3),
    ("3d_all", lambda: fields.grf((40, 36, 44), 32, log_normal=True), 8,
     dict(block=8, sample_rate=0.2, all_orders=1), 1e-3),
]


@pytest.mark.parametrize("name,make,s,cfgkw,rel", ABL_CASES)
def test_ablation_one_interpolator(ref, name, make, s, cfgkw, rel):
    # every candidate applied to all levels, trial-compressed block by
    # block at the uniform bound; the lowest bit rate (first on ties) wins
    x = make()
    d = x.ndim
    vr = float(x.max()) - float(x.min())
    e = rel * vr
    cfg = ref.tune_config(**cfgkw, ablation=ref.ABLATE_LEVELWISE)
    p, tr = ref.tune(x, e, "psnr", cfg, anchor_stride=s)
    plan = ref.sample_plan(x.shape, s, cfg)
    Lt = plan["Lt"]
    blocks = extract_blocks(x, plan)
    cands = candidates(d, bool(cfgkw.get("all_orders", 0)))
    Bs = []
    for t, o in cands:
        b, _, _, _ = trial_blockwise(ref, blocks, d, Lt, [t] * 16, [o] * 16,
                                     1.0, 1.5, e, vr, "cr")
        Bs.append(b)
    best = int(np.argmin(Bs))
    assert [tr.alg1_err[0][c] for c in range(len(cands))] == Bs
    L = int(math.log2(s))
    for l in range(L):
        assert p.interp[l] == cands[best][0]
        assert tuple(p.order[l][j] for j in range(d)) == tuple(cands[best][1])
    # the (alpha, beta) search still runs on top of the single choice
    full = ref.tune(x, e, "psnr", ref.tune_config(
        **cfgkw, ablation=ref.ABLATE_LEVELWISE | ref.ABLATE_AB),
        anchor_stride=s)[0]
    assert (full.alpha, full.beta) == (1.0, 1.5)
    assert [full.interp[l] for l in range(L)] == [p.interp[l]
                                                   for l in range(L)]


@pytest.mark.parametrize("name,make,s,cfgkw,rel", ABL_CASES)
def test_ablation_no_alpha_beta(ref, name, make, s, cfgkw, rel):
    # Algorithm 1 unchanged; alpha = 1 (uniform bounds), the first pair
    x = make()
    d = x.ndim
    e = rel * (float(x.max()) - float(x.min()))
    p_full, tr_full = ref.tune(x, e, "psnr", ref.tune_config(**cfgkw),
                               anchor_stride=s)
    p, tr = ref.tune(x, e, "psnr", ref.tune_config(
        **cfgkw, ablation=ref.ABLATE_AB), anchor_stride=s)
    assert (p.alpha, p.beta) == (1.0, 1.5)
    L = int(math.log2(s))
    for l in range(L):
        assert p.interp[l] == p_full.interp[l]
        assert all(p.order[l][j] == p_full.order[l][j] for j in range(d))
    assert tr.best_pair == 0
    el, _, _ = ref.level_bounds(e, 1.0, 1.5, L)
    assert np.all(el == e)


def test_ablation_rejects_unknown_switches(ref):
    x = fields.grf((40, 40), 3)
    with pytest.raises(ref.OracleError):
        ref.tune(x, 1e-3, "cr", ref.tune_config(ablation=4))


@pytest.mark.parametrize("shape", [(70, 45), (33, 65, 17)])
def test_anchorless_level_structure(ref, shape):
    # the SZ3-style structure: one anchor at the origin and
    # ceil(log2(max n)) levels; still within the bound
    import paper_2310_14133_amd as q
    x = fields.grf(shape, 4)
    s = q.sz3_anchor_stride(shape)
    assert s == 1 << math.ceil(math.log2(max(shape)))
    e = 1e-3 * (float(x.max()) - float(x.min()))
    p = ref.make_params(len(shape), "cubic", None, 1.0, 1.5, anchor_stride=s)
    codes, recon, unpred, anchors = ref.predict_quantize(x, e, p)
    assert anchors.size == 1 and anchors[0] == x.flat[0]
    assert codes.size + unpred.size * 0 == x.size - 1
    z = ref.compress(x, e, p)
    assert ref.inspect(z)[2].levels == int(math.log2(s))
    assert np.abs(x.astype(np.float64) - ref.decompress(z)).max() <= e
