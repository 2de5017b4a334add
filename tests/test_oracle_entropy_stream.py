"""Oracle pins: Huffman stage (Sec. VI-A names Huffman over the quantization
bins) and the compressed stream Z = C(X), X' = D(Z) (Sec. III).  CPU only."""
import heapq
import json
import os

import numpy as np
import pytest

from paper_2310_14133_amd import fields

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def optimal_cost(weights):
    """Independent optimum: sum of merged weights of a heap-driven Huffman
    (the cost of an optimal prefix code is unique)."""
    h = [int(w) for w in weights if w > 0]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a = heapq.heappop(h)
        b = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def test_textbook_example(ref):
    g = json.load(open(os.path.join(GOLD, "huffman_textbook.json")))
    w = np.array(g["weights"], np.uint64)
    ln = ref.huffman_lengths(w)
    assert int(np.sum(w * ln)) == g["optimal_cost"]
    assert ln.tolist() == g["lengths"]


@pytest.mark.parametrize("seed", range(12))
def test_lengths_optimal_and_complete(ref, seed):
    rng = np.random.default_rng(seed)
    nsym = int(rng.integers(2, 3000))
    kind = seed % 3
    if kind == 0:
        w = rng.integers(0, 1000, nsym)
    elif kind == 1:   # geometric, like quantization bins around R
        w = (1e6 * 0.6 ** np.abs(np.arange(nsym) - nsym // 2)).astype(np.int64)
    else:             # many ties
        w = rng.integers(0, 3, nsym) * 7
    w[rng.integers(nsym)] += 1
    w = w.astype(np.uint64)
    ln = ref.huffman_lengths(w)
    used = w > 0
    assert np.all((ln > 0) == used)
    if used.sum() > 1:
        # Kraft equality of a full binary tree
        assert sum(2.0 ** -int(l) for l in ln[used]) == 1.0
    assert int(np.sum(w * ln)) == optimal_cost(w)
    code = ref.huffman_codes(ln)
    # canonical codes are prefix-free and ordered by (length, symbol)
    syms = np.nonzero(used)[0]
    order = sorted(syms, key=lambda s: (ln[s], s))
    strings = [format(int(code[s]), "0%db" % ln[s]) for s in order]
    for a, b in zip(strings, strings[1:]):
        assert not b.startswith(a)
        assert int(b, 2) >= int(a, 2) << (len(b) - len(a))
    assert strings[0] == "0" * len(strings[0])


def test_single_symbol_length_one(ref):
    w = np.zeros(70, np.uint64)
    w[33] = 12
    ln = ref.huffman_lengths(w)
    assert ln[33] == 1 and ln.sum() == 1


def test_fibonacci_weights_depth(ref):
    """Fibonacci weights give the deepest Huffman tree: depth n-1 for n
    symbols (textbook worst case)."""
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    ln = ref.huffman_lengths(np.array(fib, np.uint64))
    assert int(ln.max()) == 39
    assert int(np.sum(np.array(fib, np.uint64) * ln)) == optimal_cost(fib)


CASES = [
    ("bumps256", lambda: fields.bumps_and_waves(256, 1), 1e-3, None),
    ("grf3", lambda: fields.grf((33, 40, 47), 2), 1e-3, None),
    ("grf3_tight", lambda: fields.grf((30, 30, 30), 3), 1e-5, None),
    ("spikes", lambda: fields.adversarial((60, 70), "spikes", 4), 1e-3, None),
    ("noise", lambda: fields.adversarial((31, 33, 35), "noise", 5), 1e-4, 8),
    ("zero", lambda: np.zeros((40, 41), np.float32), 1.0, None),
]


def chunk_sizes(shape, s, n_codes):
    """Bins per chunk.  Level l (levels L..1 in stream order, L = log2 s)
    holds the points on the stride-2^(l-1) grid that are not on the
    stride-2^l grid; its bins form chunks of max(4096 >> (l - 1), 1024),
    level boundaries rounded up to 64 bins, the last chunk of a level
    possibly shorter.  Returns (bins before level 1, sizes)."""
    L = int(s).bit_length() - 1
    on = lambda h: int(np.prod([(n - 1) // h + 1 for n in shape]))
    sizes, t, start = [], 0, 0
    for l in range(L, 0, -1):
        t += on(2 ** (l - 1)) - on(2 ** l)
        end = n_codes if l == 1 else min(-(-t // 64) * 64, n_codes)
        if l == 1:
            before_l1 = start
        c = max(4096 >> (l - 1), 1024)
        m = end - start
        sizes += [c] * (m // c) + ([m % c] if m % c else [])
        start = end
    return before_l1, sizes


@pytest.mark.parametrize("name,make,rel,s", CASES)
def test_stream_roundtrip(ref, name, make, rel, s):
    x = make()
    vr = float(x.max()) - float(x.min())
    e = rel * (vr if vr > 0 else 1.0)
    p = ref.make_params(x.ndim, "cubic", None, 1.25, 2.0,
                        anchor_stride=s or 0)
    z = ref.compress(x, e, p)
    assert z.size <= ref.compress_bound(x.shape)
    y = ref.decompress(z)
    codes, recon, unpred, _ = ref.predict_quantize(x, e, p)
    assert np.array_equal(y, recon)
    assert np.abs(x.astype(np.float64) - y).max() <= e
    dims, e2, p2 = ref.inspect(z)
    assert dims == x.shape and e2 == e
    assert p2.alpha == 1.25 and p2.beta == 2.0
    # payload bits = Huffman cost of the bins + word padding per chunk
    hist = np.bincount(codes, minlength=2 * 32768).astype(np.uint64)
    ln = ref.huffman_lengths(hist)
    bits = int(np.sum(hist * ln))
    stride = s or (64 if x.ndim == 2 else 32)
    _, sizes = chunk_sizes(x.shape, stride, codes.size)
    nchunks = len(sizes)
    assert int(np.frombuffer(z[168:176].tobytes(), np.uint64)[0]) == nchunks
    n_words = int(np.frombuffer(z[176:184].tobytes(), np.uint64)[0])
    assert bits <= 32 * n_words < bits + 32 * nchunks
    assert int(np.frombuffer(z[152:160].tobytes(), np.uint64)[0]) == unpred.size


def test_stream_header_fields(ref):
    x = fields.grf((20, 30), 9)
    p = ref.make_params(2, ["linear", "cubic"] * 8, [[1, 0], [0, 1]] * 8,
                        1.5, 3.0, anchor_stride=8)
    z = ref.compress(x, 0.01, p)
    assert bytes(z[:4]) == b"QOZ1"
    hdr = z[:200].tobytes()
    assert int(np.frombuffer(hdr[4:6], np.uint16)[0]) == 4  # version
    assert hdr[7] == 9                               # log2 segment size
    u64 = lambda o: int(np.frombuffer(hdr[o:o + 8], np.uint64)[0])
    u32 = lambda o: int(np.frombuffer(hdr[o:o + 4], np.uint32)[0])
    assert hdr[6] == 2
    assert (u64(8), u64(16), u64(24)) == (20, 30, 1)
    assert (u32(40), u32(44), u32(48), u32(52)) == (32768, 8, 3, 4096)
    assert list(hdr[72:75]) == [0, 1, 0]
    assert list(hdr[88:94]) == [1, 0, 0, 0, 1, 0]  # 3 bytes per level
    n_anchor = u64(136)
    assert n_anchor == 3 * 4 and u64(144) == 600 - 12
    # bins before level 1: level 3 (5 x 8 points of stride 4 minus the
    # 3 x 4 anchors = 28, rounded up to 64) and level 2 (10 x 15 - 5 x 8 =
    # 110; 64 + 110 = 174, rounded up to 192)
    assert u64(184) == 192 and u32(192) == 1024


def test_corrupt_streams_rejected(ref):
    x = fields.grf((40, 50), 1)
    z = ref.compress(x, 1e-3, ref.make_params(2))
    assert ref.decompress_status(z) == ref.OK
    bad = z.copy(); bad[0] ^= 0xFF
    assert ref.decompress_status(bad) == ref.EFORMAT
    bad = z.copy(); bad[4] = 9                       # version
    assert ref.decompress_status(bad) == ref.EFORMAT
    assert ref.decompress_status(z[:100]) == ref.EFORMAT
    assert ref.decompress_status(z[:-8]) == ref.EFORMAT
    for off in (136, 144, 160, 168, 176, 184, 192):  # counts, chunking
        bad = z.copy(); bad[off] ^= 0x01
        assert ref.decompress_status(bad) == ref.EFORMAT, off
    bad = z.copy(); bad[40] ^= 0x01                  # radius
    assert ref.decompress_status(bad) == ref.EFORMAT
    bad = z.copy(); bad[88] = 1; bad[89] = 1          # order not a permutation
    assert ref.decompress_status(bad) == ref.EFORMAT


def test_payload_bitflips_never_crash(ref):
    """Random payload corruption decodes to garbage or EFORMAT, never an
    out-of-bounds access (the oracle checks every read)."""
    x = fields.grf((48, 48), 2)
    z = ref.compress(x, 1e-3, ref.make_params(2))
    rng = np.random.default_rng(0)
    for _ in range(30):
        bad = z.copy()
        pos = int(rng.integers(200, z.size))
        bad[pos] ^= 1 << int(rng.integers(8))
        assert ref.decompress_status(bad) in (ref.OK, ref.EFORMAT)


def test_long_codes_roundtrip(ref):
    """Bins with Fibonacci counts force Huffman codes up to 26 bits; the
    field is built so its bins are exactly the chosen ones."""
    n0, n1 = 513, 1025
    n_t = (n0 // 2) * (n1 // 2 + 1) + n0 * (n1 // 2)
    b = fields.fibonacci_bins(n_t, 27, seed=3)
    x = fields.bins_field(b, n0, n1)
    p = ref.make_params(2, "linear", (0, 1), 1.0, 1.0, anchor_stride=2)
    codes, recon, unpred, _ = ref.predict_quantize(x, 0.5, p)
    assert np.array_equal(codes - 32768, b) and unpred.size == 0
    hist = np.bincount(codes, minlength=65536).astype(np.uint64)
    assert ref.huffman_lengths(hist).max() >= 24
    z = ref.compress(x, 0.5, p)
    assert np.array_equal(ref.decompress(z), recon)


def _segs_section(z):
    """Offset of the segment table: header, then 8-aligned anchors f32,
    symbols u16, lengths u8, chunk offsets u64[C+1], unpredictable
    prefix u32[C+1]."""
    u64 = lambda o: int(np.frombuffer(z[o:o + 8].tobytes(), np.uint64)[0])
    al8 = lambda v: (v + 7) // 8 * 8
    n_anchor, n_used, n_chunks = u64(136), u64(160), u64(168)
    off = al8(200 + 4 * n_anchor)
    off = al8(off + 2 * n_used)
    off = al8(off + n_used)
    off = al8(off + 8 * (n_chunks + 1))
    off = al8(off + 4 * (n_chunks + 1))
    return off, n_chunks


@pytest.mark.parametrize("shape,rel", [((70, 90, 40), 1e-3), ((33, 1500), 1e-4),
                                       ((2, 2065), 1e-3)])
def test_segment_table(ref, shape, rel):
    """Segment j of a chunk holds its bins j, j + 8, j + 16, ...; each stored
    segment length is the sum of the Huffman code lengths of those bins
    (0 for an empty segment), so a segment decodes on its own."""
    x = fields.grf(shape, 4)
    e = rel * (float(x.max()) - float(x.min()))
    p = ref.make_params(x.ndim, "cubic", None, 1.25, 2.0)
    z = ref.compress(x, e, p)
    codes, _, _, _ = ref.predict_quantize(x, e, p)
    hist = np.bincount(codes, minlength=65536).astype(np.uint64)
    ln = ref.huffman_lengths(hist).astype(np.int64)
    off, n_chunks = _segs_section(z)
    segs = np.frombuffer(z[off:off + 14 * n_chunks].tobytes(), np.uint16)
    segs = segs.reshape(n_chunks, 7).astype(np.int64)
    per_bin = ln[codes]
    _, sizes = chunk_sizes(x.shape, 64 if x.ndim == 2 else 32, codes.size)
    assert len(sizes) == n_chunks and sum(sizes) == codes.size
    want = np.zeros((n_chunks, 7), np.int64)
    lo = 0
    for c, m in enumerate(sizes):
        for j in range(7):
            want[c, j] = per_bin[lo + j:lo + m:8].sum()
        lo += m
    assert n_chunks >= 2 and codes.size % 4096 != 0
    assert np.array_equal(segs, want)
    # a wrong length is rejected
    bad = z.copy()
    bad[off + 2] ^= 0x01
    assert ref.decompress_status(bad) == ref.EFORMAT
    # so is a nonzero length for an empty segment
    tail = sizes[-1]
    if tail < 7:
        assert np.all(segs[-1, tail:] == 0)
        bad = z.copy()
        bad[off + 2 * (7 * (n_chunks - 1) + 6)] = 1
        assert ref.decompress_status(bad) == ref.EFORMAT


# ---- zero-word packing (format version 5) ----
def _sections(z):
    """Offsets of the payload and of the packed offsets, and the counts."""
    u64 = lambda o: int(np.frombuffer(z[o:o + 8].tobytes(), np.uint64)[0])
    u32 = lambda o: int(np.frombuffer(z[o:o + 4].tobytes(), np.uint32)[0])
    al8 = lambda v: (v + 7) // 8 * 8
    n_anchor, n_unpred = u64(136), u64(152)
    n_used, n_chunks, n_words = u64(160), u64(168), u64(176)
    off = al8(200 + 4 * n_anchor)
    off = al8(off + 2 * n_used)
    off = al8(off + n_used)
    coff_at = off
    off = al8(off + 8 * (n_chunks + 1))
    off = al8(off + 4 * (n_chunks + 1))
    off = al8(off + 14 * n_chunks)
    payload = al8(off + 4 * n_unpred)
    wp = u32(196)
    coff = np.frombuffer(z[coff_at:coff_at + 8 * (n_chunks + 1)].tobytes(),
                         np.uint64).astype(np.int64)
    return payload, wp, n_words, n_chunks, coff


def _raw_payload(ref, x, e, p, s):
    """The chunked MSB-first Huffman payload re-derived from the bins and
    the canonical code, chunk by chunk, segment by segment."""
    codes, _, _, _ = ref.predict_quantize(x, e, p)
    hist = np.bincount(codes, minlength=65536).astype(np.uint64)
    ln = ref.huffman_lengths(hist).astype(np.int64)
    cd = ref.huffman_codes(ln.astype(np.uint8)).astype(np.uint64)
    _, sizes = chunk_sizes(x.shape, s, codes.size)
    words, coff, lo = [], [0], 0
    for m in sizes:
        bits = []
        for j in range(8):
            for sym in codes[lo + j:lo + m:8]:
                L = int(ln[sym])
                v = int(cd[sym])
                bits.extend((v >> (L - 1 - b)) & 1 for b in range(L))
        bits += [0] * (-len(bits) % 32)
        for k in range(0, len(bits), 32):
            w = 0
            for b in bits[k:k + 32]:
                w = (w << 1) | b
            words.append(w)
        coff.append(len(words))
        lo += m
    return np.array(words, np.uint64), np.array(coff, np.int64)


def _pack(words, coff):
    """Bitmap + nonzero words per chunk when shorter than the raw chunk."""
    out, pcoff = [], [0]
    for c in range(len(coff) - 1):
        w = words[coff[c]:coff[c + 1]]
        n = len(w)
        nz = int(np.count_nonzero(w))
        nbm = -(-n // 32)
        if nbm + nz < n:
            bm = [0] * nbm
            for i in np.nonzero(w)[0]:
                bm[i // 32] |= 1 << (i % 32)
            out += bm + [int(v) for v in w if v]
        else:
            out += [int(v) for v in w]
        pcoff.append(len(out))
    return np.array(out, np.uint64), np.array(pcoff, np.int64)


def test_zero_word_packing_layout(ref):
    # a smooth field at a loose bound: mostly the zero bin, whose code is
    # all zero bits, so whole payload words vanish
    x = fields.bumps_and_waves(160, 2)
    e = 1e-2 * (float(x.max()) - float(x.min()))
    s = 64
    p = ref.make_params(2, "cubic", None, 1.0, 1.5, anchor_stride=s)
    z = ref.compress(x, e, p)
    assert int(np.frombuffer(z[4:6].tobytes(), np.uint16)[0]) == 5
    payload, wp, n_words, n_chunks, coff = _sections(z)
    raw, coff_r = _raw_payload(ref, x, e, p, s)
    assert raw.size == n_words and np.array_equal(coff, coff_r)
    packed, pcoff = _pack(raw, coff_r)
    assert packed.size == wp
    assert 100 * (wp + 2 * (n_chunks + 1)) <= 97 * n_words
    got = np.frombuffer(z[payload:payload + 4 * wp].tobytes(), np.uint32)
    assert np.array_equal(got.astype(np.uint64), packed)
    pc_at = (payload + 4 * wp + 7) // 8 * 8
    got_pc = np.frombuffer(z[pc_at:pc_at + 8 * (n_chunks + 1)].tobytes(),
                           np.uint64).astype(np.int64)
    assert np.array_equal(got_pc, pcoff) and z.size == pc_at + 8 * (n_chunks + 1)
    # and it decodes to the predictor's reconstruction
    _, recon, _, _ = ref.predict_quantize(x, e, p)
    assert np.array_equal(ref.decompress(z), recon)


def test_rough_field_stays_unpacked(ref):
    x = fields.grf((50, 60, 40), 3)
    e = 1e-3 * (float(x.max()) - float(x.min()))
    z = ref.compress(x, e, ref.make_params(3, "cubic", None, 1.0, 1.5))
    assert int(np.frombuffer(z[4:6].tobytes(), np.uint16)[0]) == 4
    assert int(np.frombuffer(z[196:200].tobytes(), np.uint32)[0]) == 0


def test_packing_lifts_the_one_bit_floor(ref):
    # without packing every bin costs at least one bit (ratio <= 32)
    x = fields.bumps_and_waves(256, 1)
    e = 1e-2 * (float(x.max()) - float(x.min()))
    z = ref.compress(x, e, ref.make_params(2, "cubic", None, 1.0, 1.5))
    assert x.nbytes / z.size > 32


def test_packed_stream_corruptions(ref):
    x = fields.bumps_and_waves(160, 2)
    e = 1e-2 * (float(x.max()) - float(x.min()))
    p = ref.make_params(2, "cubic", None, 1.0, 1.5, anchor_stride=64)
    z = ref.compress(x, e, p)
    payload, wp, n_words, n_chunks, coff = _sections(z)
    pc_at = (payload + 4 * wp + 7) // 8 * 8

    def status(b):
        return ref.decompress_status(b)

    bad = z.copy()
    bad[4] = 4  # version 4 with a packed count
    assert status(bad) == ref.EFORMAT
    bad = z.copy()
    bad[pc_at + 8:pc_at + 16] = np.frombuffer(
        np.array([wp + 5], np.uint64).tobytes(), np.uint8)
    assert status(bad) == ref.EFORMAT
    # a bitmap bit past the chunk's last word
    pcs = np.frombuffer(z[pc_at:pc_at + 8 * (n_chunks + 1)].tobytes(),
                        np.uint64).astype(np.int64)
    for c in range(n_chunks):
        n = coff[c + 1] - coff[c]
        if pcs[c + 1] - pcs[c] < n and n % 32:
            nbm = -(-n // 32)
            at = payload + 4 * (pcs[c] + nbm - 1)
            w = int(np.frombuffer(z[at:at + 4].tobytes(), np.uint32)[0])
            bad = z.copy()
            bad[at:at + 4] = np.frombuffer(
                np.array([w | (1 << 31)], np.uint32).tobytes(), np.uint8)
            assert status(bad) == ref.EFORMAT
            break
    else:
        pytest.fail("no packed chunk with a partial bitmap word")
