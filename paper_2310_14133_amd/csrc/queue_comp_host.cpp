/*
 * Batched compression through device work queues: C_theta of Sec. III for
 * many fields at once, in a number of launches that does not grow with the
 * batch:
 *
 *   1. (fields given without parameters are tuned by the online tuner of
 *      Sec. VI on up to 8 worker contexts with their own streams, largest
 *      field first, while this thread compresses the fields tuned so far,
 *      each group as one call of the steps below with its parameters
 *      given;)
 *   2. one upload of the queues, then one launch for every field's
 *      anchors, one launch per round of sweeps (the r-th sweep, or fused
 *      level-1 row pair, of every field), one launch for every field's
 *      histogram and one sorting the used bins of every histogram; one
 *      read-back of the sorted bins and status words (the first wait);
 *   3. the Huffman codes of Sec. VI-A on host threads (a field with more
 *      used bins than the device sort holds reads its whole histogram: one
 *      more wait when there is such a field);
 *   4. a second upload (code tables, the encoder's field records, the
 *      codebooks), one launch that zero-fills every field's sections before
 *      the payload and its encoder totals, one that copies codebooks and
 *      anchors into place, one counting the code bits and symbol-0 bins of
 *      every chunk of every field, one scan over all those chunks (two
 *      launches) and one encoding launch over them (runs of chunks in a
 *      grid stride, field after field); one read-back of the totals (the
 *      second wait);
 *   5. headers: one upload and one copy launch; a field whose zero-word
 *      packing pays is packed with its own few launches (the third wait).
 *
 * Every field's stream equals qoz_compress's byte for byte: the sweeps,
 * histogram and encoder run the single-field kernels' per-workgroup code.
 * A field whose output buffer cannot hold the sections before its payload
 * goes through qoz_compress instead (which reports the size it needs).
 */
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "qoz_internal.h"

namespace qoz {

/* worker contexts for the tunings of a batch's fields */
constexpr size_t kTuneWorkers = 8;
namespace {

constexpr size_t kAl = 256;
constexpr uint32_t kMaxCompQueue = 1u << 14;
constexpr size_t kHostThreads = 16;

inline size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

struct CField {
  uint32_t item = 0;
  Plan P;
  uint64_t N = 0, nch = 0;
  /* device scratch offsets (in c->cqueue) */
  size_t W = 0, codes = 0, anchors = 0, pbits = 0, status = 0;
  std::vector<CompJob> steps;
  /* the Huffman code and the stream's sections */
  std::vector<uint16_t> usym;
  std::vector<uint8_t> ulen;
  std::vector<uint64_t> keys, table;
  uint64_t n_unpred = 0, zero_entry = 0, n_words = 0, n_packed = 0;
  int32_t lo = 0;
  uint32_t tn = 0, max_len = 0, words_bound = 0;
  bool big = false; /* more used bins than the device sort holds */
  Layout lay0{}, lay{};
  size_t tab_up = 0, cb_up = 0, hdr_up = 0; /* in the second upload */
};

qoz_status sync_q(hipStream_t s) {
  QOZ_HIP(hipGetLastError());
  QOZ_HIP(hipStreamSynchronize(s));
  return QOZ_OK;
}

/* The Huffman code of a field from its (count << 16 | symbol) keys in
 * ascending order: lengths, canonical codes by ascending symbol, the code
 * table for the encoder.  False when a code would be longer than the
 * encoder's table allows. */
bool field_code(CField& f) {
  const std::vector<uint64_t>& keys = f.keys;
  std::vector<uint8_t> klen(keys.size());
  if (!huffman_lengths_sorted(keys.data(), (uint32_t)keys.size(),
                              klen.data()))
    return false;
  f.words_bound =
      chunk_words_bound(keys.data(), klen.data(), (uint32_t)keys.size(), kChunk);
  /* the used symbols in ascending order: each key's length placed at its
   * symbol (symbols are distinct), then one pass over the alphabet */
  const size_t n_used = keys.size();
  std::vector<uint8_t> len_of(kNSym, 0);
  f.n_unpred = 0;
  f.max_len = 0;
  for (size_t i = 0; i < n_used; ++i) {
    const uint32_t sym = (uint32_t)(keys[i] & 0xffffu);
    if (klen[i] == 0 || klen[i] > 56) return false;
    len_of[sym] = klen[i];
    if (sym == 0) f.n_unpred = keys[i] >> 16;
    f.max_len = std::max<uint32_t>(f.max_len, klen[i]);
  }
  f.usym.resize(n_used);
  f.ulen.resize(n_used);
  size_t m = 0;
  for (uint32_t sym = 0; sym < kNSym && m < n_used; ++sym)
    if (len_of[sym]) {
      f.usym[m] = (uint16_t)sym;
      f.ulen[m] = len_of[sym];
      ++m;
    }
  if (m != n_used) return false; /* a symbol twice */
  std::vector<uint64_t> ucode(n_used);
  canonical_codes_sparse(f.usym.data(), f.ulen.data(), (uint32_t)n_used,
                         ucode.data());
  int32_t lo = -1, hi = -1;
  f.zero_entry = 0;
  for (size_t i = 0; i < n_used; ++i) {
    if (f.usym[i] == 0) {
      f.zero_entry = (ucode[i] << 8) | f.ulen[i];
      continue;
    }
    if (lo < 0) lo = f.usym[i];
    hi = f.usym[i];
  }
  f.lo = lo;
  f.tn = lo < 0 ? 0 : (uint32_t)(hi - lo + 1);
  f.table.assign(f.tn, 0);
  for (size_t i = 0; i < n_used; ++i)
    if (f.usym[i]) f.table[f.usym[i] - lo] = (ucode[i] << 8) | f.ulen[i];
  f.lay0 = layout_of(f.P.n_anchor, n_used, f.nch, f.n_unpred, 0);
  return true;
}

template <class Fn>
void on_threads(size_t n, Fn fn) {
  std::atomic<size_t> next{0};
  auto work = [&]() {
    for (size_t k; (k = next.fetch_add(1)) < n;) fn(k);
  };
  const size_t nt = n < kHostThreads ? n : kHostThreads;
  std::vector<std::thread> th;
  for (size_t t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}

}  // namespace
}  // namespace qoz

using namespace qoz;

static qoz_status compress_queue(qoz_ctx* c, qoz_batch_item* items,
                                 uint32_t n, qoz_target target,
                                 const qoz_tune_config* cfg, hipStream_t s,
                                 bool* items_only);

/* Tuning overlapped with compression.  A thread hands the fields to tune
 * to the worker contexts (largest first); this thread waits for each
 * round of tunings (as many fields as workers, or the last ones), then
 * compresses everything ready and not yet compressed (the fields with
 * given parameters go with the first group) as one queue call with the
 * parameters given.  A field's stream is the single-field call's either
 * way. */
static qoz_status compress_tuning(qoz_ctx* c, qoz_batch_item* items,
                                  uint32_t n, std::vector<qoz_params>& pv,
                                  const std::vector<uint32_t>& to_tune,
                                  qoz_target target,
                                  const qoz_tune_config* cfg, hipStream_t s,
                                  std::chrono::steady_clock::time_point t0) {
  const size_t total = to_tune.size();
  const uint32_t nw = (uint32_t)std::min<size_t>(kTuneWorkers, total);
  QOZ_HIP(hipStreamSynchronize(s));
  QOZ_TRY(ensure_workers(c, nw));
  std::vector<uint64_t> pts(total, 1);
  for (size_t k = 0; k < total; ++k)
    for (uint32_t m = 0; m < items[to_tune[k]].shape.ndim && m < 3; ++m)
      pts[k] *= items[to_tune[k]].shape.dims[m];
  std::vector<uint32_t> order(total);
  for (uint32_t k = 0; k < order.size(); ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return pts[a] > pts[b]; });

  std::mutex mu;
  std::condition_variable cv;
  std::vector<uint32_t> ready; /* items with parameters, not compressed */
  size_t tuned = 0;            /* tunings ended (failed ones too) */
  std::string why;             /* the first failure's message */
  for (uint32_t i = 0; i < n; ++i)
    if (items[i].status == QOZ_OK && items[i].params) ready.push_back(i);
  std::thread tuner([&]() {
    run_on_workers(order, nw, [&](uint32_t w, uint32_t k) {
      const uint32_t i = to_tune[k];
      qoz_batch_item& it = items[i];
      qoz_params p = pv[i]; /* zeroed: the tuner reads its anchor stride */
      const qoz_status st = qoz_tune(c->workers[w], it.d_x, it.shape,
                                     it.abs_eb, target, cfg, &p,
                                     c->worker_streams[w]);
      std::lock_guard<std::mutex> g(mu);
      it.status = st;
      if (st == QOZ_OK) {
        pv[i] = p;
        ready.push_back(i);
      } else if (why.empty()) {
        why = std::string("tuning: ") + qoz_last_error();
      }
      ++tuned;
      cv.notify_one();
    });
  });
  size_t taken = 0; /* tunings ended at the last take */
  for (;;) {
    std::vector<uint32_t> grp;
    bool last;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&]() { return tuned == total || tuned - taken >= nw; });
      grp.swap(ready);
      taken = tuned;
      last = tuned == total;
    }
    if (!grp.empty()) {
      std::sort(grp.begin(), grp.end());
      std::vector<qoz_batch_item> sub(grp.size());
      for (size_t k = 0; k < grp.size(); ++k) {
        sub[k] = items[grp[k]];
        sub[k].params = &pv[grp[k]];
      }
      /* per-item statuses carry the outcome; a call that fails as a whole
       * fails every item it left marked OK */
      bool items_only = false;
      const qoz_status rc =
          compress_queue(c, sub.data(), (uint32_t)sub.size(), target, cfg,
                         s, &items_only);
      if (rc != QOZ_OK) {
        if (!items_only)
          for (qoz_batch_item& it : sub)
            if (it.status == QOZ_OK) it.status = rc;
        std::lock_guard<std::mutex> g(mu);
        if (why.empty()) why = qoz_last_error();
      }
      const double dm = std::chrono::duration<double, std::milli>(
                            std::chrono::steady_clock::now() - t0)
                            .count();
      for (size_t k = 0; k < grp.size(); ++k) {
        qoz_batch_item& it = items[grp[k]];
        it.status = sub[k].status;
        it.out_bytes = sub[k].out_bytes;
        it.done_ms = dm;
      }
    }
    if (last) break;
  }
  tuner.join();
  const double ms = std::chrono::duration<double, std::milli>(
                        std::chrono::steady_clock::now() - t0)
                        .count();
  for (uint32_t i = 0; i < n; ++i) items[i].ms = ms;
  clear_error();
  for (uint32_t i = 0; i < n; ++i)
    if (items[i].status != QOZ_OK)
      return fail(items[i].status,
                  why.empty() ? "a field of the batch failed" : why);
  return QOZ_OK;
}

extern "C" qoz_status qoz_compress_queue(qoz_ctx* c, qoz_batch_item* items,
                                         uint32_t n, qoz_target target,
                                         const qoz_tune_config* cfg,
                                         hipStream_t s) {
  return compress_queue(c, items, n, target, cfg, s, nullptr);
}

/* items_only (if given) is set when the returned error is an item's own
 * status (every other item's status is then its outcome) rather than a
 * failure of the call as a whole. */
static qoz_status compress_queue(qoz_ctx* c, qoz_batch_item* items,
                                 uint32_t n, qoz_target target,
                                 const qoz_tune_config* cfg, hipStream_t s,
                                 bool* items_only) {
  clear_error();
  if (!c || (n && !items)) return fail(QOZ_EINVAL, "NULL argument");
  if (n > kMaxCompQueue) return fail(QOZ_EINVAL, "batch too large");
  QOZ_TRY(set_device(c));
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t i = 0; i < n; ++i) {
    items[i].status = QOZ_OK;
    items[i].out_bytes = 0;
    items[i].ms = items[i].done_ms = 0.0;
  }
  if (!n) return QOZ_OK;

  /* 1. parameters and plans: the fields without parameters are tuned on
   * worker contexts, each on its own stream (largest first), after the
   * caller's stream has produced the inputs */
  std::vector<CField> F;
  F.reserve(n);
  std::vector<qoz_params> pv(n); /* given or tuned */
  std::vector<uint32_t> to_tune;
  std::vector<uint64_t> tsize;
  for (uint32_t i = 0; i < n; ++i) {
    qoz_batch_item& it = items[i];
    if (!it.d_x || ((uintptr_t)it.d_out & 7) != 0) {
      it.status = QOZ_EINVAL;
      continue;
    }
    if (it.params) {
      pv[i] = *it.params;
    } else {
      std::memset(&pv[i], 0, sizeof(pv[i]));
      to_tune.push_back(i);
    }
  }
  if (!to_tune.empty())
    return compress_tuning(c, items, n, pv, to_tune, target, cfg, s, t0);
  for (uint32_t i = 0; i < n; ++i) {
    qoz_batch_item& it = items[i];
    if (it.status != QOZ_OK) continue;
    const qoz_params& p = pv[i];
    CField f;
    f.item = i;
    it.status = make_plan(it.shape, it.abs_eb, p, &f.P);
    if (it.status != QOZ_OK) continue;
    f.N = (uint64_t)f.P.g.n[0] * f.P.g.n[1] * f.P.g.n[2];
    f.nch = f.P.n_chunks;
    F.push_back(std::move(f));
  }
  clear_error();
  const uint32_t nf = (uint32_t)F.size();
  if (!nf) {
    for (uint32_t i = 0; i < n; ++i)
      if (items[i].status != QOZ_OK) {
        if (items_only) *items_only = true;
        return fail(items[i].status, "a field of the batch failed");
      }
    return QOZ_OK;
  }

  /* 2. steps, rounds and the device layout: per-field scratch, the
   * histograms and sorted keys (contiguous, for the multi-histogram
   * sort), then the upload region of the first phase */
  size_t rounds = 0;
  for (CField& f : F) {
    size_t fz = SIZE_MAX, fa = SIZE_MAX, fb = SIZE_MAX;
    RowJob rj;
    const bool fuse = level1_rows(f.P, &fz, &fa, &fb, &rj);
    for (size_t i = 0; i < f.P.sweeps.size(); ++i) {
      CompJob j;
      std::memset(&j, 0, sizeof(j));
      j.g = f.P.g;
      if (fuse && (i == fz || i == fa || i == fb)) {
        if (i != fb) continue;
        j.rows = 1;
        j.rj = rj;
        j.write_w = fb + 1 < f.P.sweeps.size();
      } else {
        j.s = f.P.sweeps[i];
        j.write_w = i + 1 < f.P.sweeps.size();
      }
      f.steps.push_back(j);
    }
    rounds = std::max(rounds, f.steps.size());
  }
  size_t off = 0;
  const size_t hist_off = off;
  off += al(4ull * kNSym * nf);
  const size_t keys_off = off;
  off += al(8ull * (kSortCap + 1) * nf);
  for (CField& f : F) {
    f.W = off;
    off += al(4 * f.N);
    f.codes = off;
    off += al(2 * (f.P.n_codes + 16));
    f.anchors = off;
    off += al(4 * f.P.n_anchor);
    f.pbits = off;
    off += al(4 * f.nch);
    f.status = off; /* 8 status words, then the encoder's 3 totals */
    off += kAl;
  }
  /* per chunk of the batch (global chunk order of the encoded fields):
   * code bits and symbol-0 bins, their exclusive prefixes, scan scratch */
  uint64_t nt = 0;
  for (const CField& f : F) nt += f.nch;
  const size_t gbits_off = off;
  off += al(4 * nt + 4);
  const size_t gzeros_off = off;
  off += al(4 * nt + 4);
  const size_t gw_off = off;
  off += al(8 * (nt + 1));
  const size_t gz_off = off;
  off += al(8 * (nt + 1));
  const size_t gscan_off = off;
  off += al(chunk_scan_scratch(nt));
  const size_t geo_off = off;
  off += al(sizeof(ChunkGeo) * (nt ? nt : 1));
  const size_t gtot_off = off; /* the batch scan's totals */
  off += kAl;
  const size_t upA = off;
  const size_t anc_jobs = 0;
  size_t ua = al(sizeof(AnchorJob) * nf);
  const size_t anc_wg0 = ua;
  ua += al(4 * (nf + 1));
  const size_t hist_jobs = ua;
  ua += al(sizeof(HistJob) * nf);
  const size_t hist_wg0 = ua;
  ua += al(4 * (nf + 1));
  const size_t zero_list = ua;
  ua += al(sizeof(DevCopy) * 2 * nf);
  std::vector<size_t> rj_off(rounds), rw_off(rounds);
  for (size_t r = 0; r < rounds; ++r) {
    rj_off[r] = ua;
    ua += al(sizeof(CompJob) * nf);
    rw_off[r] = ua;
    ua += al(4 * (nf + 1));
  }
  const size_t upA_bytes = ua;
  off += upA_bytes;
  QOZ_TRY(ensure(c->cqueue, off));
  uint8_t* const D = (uint8_t*)c->cqueue.p;
  const size_t hdr = kPinSingleBytes;
  QOZ_TRY(ensure_pinned(c, hdr + upA_bytes));
  uint8_t* hu = (uint8_t*)c->pinned + hdr;
  std::memset(hu, 0, upA_bytes);

  AnchorJob* aj = (AnchorJob*)(hu + anc_jobs);
  uint32_t* aw = (uint32_t*)(hu + anc_wg0);
  HistJob* hj = (HistJob*)(hu + hist_jobs);
  uint32_t* hw = (uint32_t*)(hu + hist_wg0);
  DevCopy* zl = (DevCopy*)(hu + zero_list);
  uint32_t a_tot = 0, h_tot = 0;
  for (uint32_t k = 0; k < nf; ++k) {
    CField& f = F[k];
    const qoz_batch_item& it = items[f.item];
    uint32_t* st = (uint32_t*)(D + f.status);
    AnchorJob& a = aj[k];
    a.g = f.P.g;
    a.stride = f.P.s;
    for (int m = 0; m < 3; ++m) a.na[m] = f.P.na[m];
    a.x = it.d_x;
    a.W = (float*)(D + f.W);
    a.out = (float*)(D + f.anchors);
    a.status = st;
    aw[k] = a_tot;
    a_tot += anchor_job_workgroups(a);
    HistJob& h = hj[k];
    h.codes = (const uint16_t*)(D + f.codes);
    h.n = f.P.n_codes;
    h.hist = (uint32_t*)(D + hist_off) + (size_t)kNSym * k;
    hw[k] = h_tot;
    h_tot += hist_job_workgroups(h);
    zl[2 * k] = DevCopy{nullptr, h.hist, 4ull * kNSym};
    zl[2 * k + 1] = DevCopy{nullptr, st, kAl};
  }
  aw[nf] = a_tot;
  hw[nf] = h_tot;
  std::vector<uint32_t> r_total(rounds, 0), r_jobs(rounds, 0);
  std::vector<size_t> r_lds(rounds, 0);
  for (size_t r = 0; r < rounds; ++r) {
    CompJob* cj = (CompJob*)(hu + rj_off[r]);
    uint32_t* cw = (uint32_t*)(hu + rw_off[r]);
    uint32_t m = 0, tot = 0;
    for (CField& f : F) {
      if (r >= f.steps.size()) continue;
      CompJob j = f.steps[r];
      size_t lds = 0;
      const uint32_t wgs = comp_job_prepare(&j, &lds);
      if (!wgs) continue;
      j.x = items[f.item].d_x;
      j.W = (float*)(D + f.W);
      j.codes = (uint16_t*)(D + f.codes);
      j.status = (uint32_t*)(D + f.status);
      cj[m] = j;
      cw[m] = tot;
      tot += wgs;
      ++m;
      r_lds[r] = std::max(r_lds[r], lds);
    }
    cw[m] = tot;
    r_jobs[r] = m;
    r_total[r] = tot;
  }

  /* first phase on the device */
  uint8_t* const dA = D + upA;
  QOZ_TRY(to_device(c, dA, hu, upA_bytes, s));
  launch_copy_list((const DevCopy*)(dA + zero_list), 2 * nf, s);
  launch_anchor_q((const AnchorJob*)(dA + anc_jobs),
                  (const uint32_t*)(dA + anc_wg0), nf, a_tot, s);
  for (size_t r = 0; r < rounds; ++r)
    launch_sweep_round_comp_q((const CompJob*)(dA + rj_off[r]),
                              (const uint32_t*)(dA + rw_off[r]), r_jobs[r],
                              r_total[r], r_lds[r], s);
  launch_hist_q((const HistJob*)(dA + hist_jobs),
                (const uint32_t*)(dA + hist_wg0), nf, h_tot, s);
  launch_hist_sort((const uint32_t*)(D + hist_off), nf,
                   (uint64_t*)(D + keys_off), s);
  /* read back: sorted keys and status words of every field */
  const size_t kb = 8ull * (kSortCap + 1);
  const size_t back = al(kb * nf + (size_t)kAl * nf);
  QOZ_TRY(sync_q(s)); /* the first upload has been read */
  QOZ_TRY(ensure_pinned(c, hdr + back + al(sizeof(HostCopy) * 2 * nf)));
  uint8_t* hb = (uint8_t*)c->pinned + hdr;
  {
    HostCopy* hc = (HostCopy*)(hb + back);
    for (uint32_t k = 0; k < nf; ++k) {
      hc[2 * k] = HostCopy{D + keys_off + kb * k, hb + kb * k, kb};
      hc[2 * k + 1] = HostCopy{D + F[k].status, hb + kb * nf + kAl * k, 64};
    }
    QOZ_TRY(gather_to_host(c, hc, 2 * nf, s));
  }
  QOZ_TRY(sync_q(s));

  /* 3. Huffman codes */
  std::vector<uint32_t> bigs;
  for (uint32_t k = 0; k < nf; ++k) {
    CField& f = F[k];
    const uint32_t* st = (const uint32_t*)(hb + kb * nf + kAl * k);
    if (st[0] & kStNonFinite) {
      items[f.item].status = QOZ_EINVAL;
      continue;
    }
    const uint64_t* hk = (const uint64_t*)(hb + kb * k);
    if (hk[0] <= kSortCap) {
      f.keys.assign(hk + 1, hk + 1 + hk[0]);
    } else {
      f.big = true;
      bigs.push_back(k);
    }
  }
  /* whole histograms of the fields with more used bins than the device
   * sort holds: one read-back for all of them */
  std::vector<uint32_t> big_at(nf, 0);
  const size_t hbytes = 4ull * kNSym;
  if (!bigs.empty()) {
    QOZ_TRY(ensure_pinned(c, hdr + al(hbytes * bigs.size()) +
                                 al(sizeof(HostCopy) * bigs.size())));
    hb = (uint8_t*)c->pinned + hdr;
    HostCopy* hc = (HostCopy*)(hb + al(hbytes * bigs.size()));
    for (size_t b = 0; b < bigs.size(); ++b) {
      hc[b] = HostCopy{D + hist_off + hbytes * bigs[b], hb + hbytes * b,
                       hbytes};
      big_at[bigs[b]] = (uint32_t)b;
    }
    QOZ_TRY(gather_to_host(c, hc, (uint32_t)bigs.size(), s));
    QOZ_TRY(sync_q(s));
  }
  {
    /* per field on the host threads: the keys of a field with many used
     * bins from its histogram (radix passes), then its code */
    const uint8_t* hbig = hb;
    std::vector<char> ok(nf, 1);
    on_threads(nf, [&](size_t k) {
      CField& f = F[k];
      if (items[f.item].status != QOZ_OK) return;
      if (f.big)
        hist_keys_sorted(
            (const uint32_t*)(hbig + hbytes * big_at[k]), kNSym, &f.keys);
      ok[k] = field_code(f);
    });
    for (uint32_t k = 0; k < nf; ++k)
      if (!ok[k]) items[F[k].item].status = QOZ_EINVAL;
  }
  /* fields whose buffer cannot hold the sections before the payload go
   * through the single-field call, which reports the size needed */
  std::vector<uint32_t> single;
  std::vector<CField*> E;
  for (CField& f : F) {
    qoz_batch_item& it = items[f.item];
    if (it.status != QOZ_OK) continue;
    if (!it.d_out || it.cap < f.lay0.payload) {
      single.push_back(f.item);
      continue;
    }
    E.push_back(&f);
  }
  const uint32_t ne = (uint32_t)E.size();

  /* 4. the second upload: code tables, encoder records and chunk ranges,
   * codebooks, the zero and copy lists */
  size_t ub = 0;
  const size_t ef_off = ub;
  ub += al(sizeof(EncField) * (ne ? ne : 1));
  const size_t c0_off = ub;
  ub += al(8 * (ne + 1));
  const size_t cw0_off = ub; /* the count's workgroups per field */
  ub += al(4 * (ne + 1));
  for (CField* f : E) {
    f->tab_up = ub;
    ub += al(8 * (f->tn ? f->tn : 1));
    f->cb_up = ub;
    ub += al(f->lay0.coff - f->lay0.syms);
  }
  const size_t zl2 = ub;
  ub += al(sizeof(DevCopy) * 2 * (ne ? ne : 1));
  const size_t cl2 = ub;
  ub += al(sizeof(DevCopy) * 2 * (ne ? ne : 1));
  const size_t upB_bytes = ub;
  /* the second uploads have a buffer of their own (growing the first one
   * would move the fields' scratch) */
  const size_t hdr_bytes =
      al((size_t)kHeaderBytes * ne) + al(sizeof(DevCopy) * (ne ? ne : 1));
  QOZ_TRY(ensure(c->cqueue_up, std::max(upB_bytes, hdr_bytes)));
  QOZ_TRY(ensure_pinned(c, hdr + std::max(upB_bytes, hdr_bytes)));
  hu = (uint8_t*)c->pinned + hdr;
  std::memset(hu, 0, upB_bytes);
  uint8_t* const dB = (uint8_t*)c->cqueue_up.p;
  EncField* ef = (EncField*)(hu + ef_off);
  uint64_t* c0 = (uint64_t*)(hu + c0_off);
  uint32_t* cw0 = (uint32_t*)(hu + cw0_off);
  uint32_t count_wg = 0;
  DevCopy* z2 = (DevCopy*)(hu + zl2);
  DevCopy* cp2 = (DevCopy*)(hu + cl2);
  uint64_t n_chunks = 0;
  uint32_t max_words = 0, max_tn = 0;
  bool long_codes = false;
  for (uint32_t k = 0; k < ne; ++k) {
    CField& f = *E[k];
    const qoz_batch_item& it = items[f.item];
    uint8_t* out = (uint8_t*)it.d_out;
    if (f.tn)
      std::memcpy(hu + f.tab_up, f.table.data(), 8ull * f.tn);
    uint8_t* cb = hu + f.cb_up;
    std::memcpy(cb, f.usym.data(), 2 * f.usym.size());
    std::memcpy(cb + (f.lay0.lens - f.lay0.syms), f.ulen.data(),
                f.ulen.size());
    uint64_t* tot = (uint64_t*)(D + f.status + 32);
    EncField& e = ef[k];
    e.codes = (const uint16_t*)(D + f.codes);
    e.ch = f.P.chunks;
    e.nch = f.nch;
    e.tab = (const uint64_t*)(dB + f.tab_up);
    e.lo = f.lo;
    e.tn = f.tn;
    e.zero_entry = f.zero_entry;
    e.coff = (uint64_t*)(out + f.lay0.coff);
    e.upre = (uint32_t*)(out + f.lay0.upre);
    e.segs = (uint16_t*)(out + f.lay0.segs);
    e.payload = (uint32_t*)(out + f.lay0.payload);
    e.cap_words = (it.cap - f.lay0.payload) / 4;
    e.unpred = (float*)(out + f.lay0.unpred);
    e.x = it.d_x;
    e.g = f.P.g;
    e.totals = tot;
    e.status = (uint32_t*)(D + f.status);
    e.pack_bits = (uint32_t*)(D + f.pbits);
    fill_sweep_table(f.P, &e.st);
    c0[k] = n_chunks;
    n_chunks += f.nch;
    cw0[k] = count_wg;
    count_wg += count_workgroups(f.nch);
    max_words = std::max(max_words, std::min(encode_max_words(f.max_len),
                                             f.words_bound));
    long_codes |= f.max_len > 32;
    max_tn = std::max(max_tn, f.tn);
    /* zero fills: the sections before the payload and the totals; then
     * the codebook and the anchors into place */
    z2[2 * k] = DevCopy{nullptr, out, f.lay0.payload};
    z2[2 * k + 1] = DevCopy{nullptr, tot, 32};
    cp2[2 * k] = DevCopy{dB + f.cb_up, out + f.lay0.syms,
                         f.lay0.coff - f.lay0.syms};
    cp2[2 * k + 1] =
        DevCopy{D + f.anchors, out + f.lay0.anchors, 4 * f.P.n_anchor};
  }
  c0[ne] = n_chunks;
  cw0[ne] = count_wg;
  if (ne) {
    QOZ_TRY(to_device(c, dB, hu, upB_bytes, s));
    launch_copy_list((const DevCopy*)(dB + zl2), 2 * ne, s);
    launch_copy_list((const DevCopy*)(dB + cl2), 2 * ne, s);
    /* counts per chunk of every field, one scan over the batch's chunks,
     * then the encoding (a field's offsets are differences of the
     * batch-wide prefixes) */
    launch_huff_count((const EncField*)(dB + ef_off),
                      (const uint64_t*)(dB + c0_off),
                      (const uint32_t*)(dB + cw0_off), ne, count_wg,
                      (uint32_t*)(D + gbits_off), (uint32_t*)(D + gzeros_off),
                      (ChunkGeo*)(D + geo_off), s);
    launch_chunk_scan((const uint32_t*)(D + gbits_off),
                      (const uint32_t*)(D + gzeros_off), n_chunks,
                      (uint64_t*)(D + gw_off), (uint64_t*)(D + gz_off),
                      (uint64_t*)(D + gtot_off),
                      (uint64_t*)(D + gscan_off), s);
    launch_huff_encode((const EncField*)(dB + ef_off),
                       (const uint64_t*)(dB + c0_off),
                       (const ChunkGeo*)(D + geo_off),
                       (const uint64_t*)(D + gw_off),
                       (const uint64_t*)(D + gz_off), ne, n_chunks,
                       max_words, max_tn, long_codes, s);
    QOZ_TRY(sync_q(s)); /* the second upload has been read */
    QOZ_TRY(ensure_pinned(c, hdr + al((size_t)kAl * ne) +
                                 al(sizeof(HostCopy) * ne)));
    hb = (uint8_t*)c->pinned + hdr;
    HostCopy* hc = (HostCopy*)(hb + al((size_t)kAl * ne));
    for (uint32_t k = 0; k < ne; ++k)
      hc[k] = HostCopy{D + E[k]->status, hb + kAl * k, 64};
    QOZ_TRY(gather_to_host(c, hc, ne, s));
    QOZ_TRY(sync_q(s));
  }

  /* 5. headers (one upload, one copy launch); zero-word packing where it
   * pays, field by field */
  std::vector<CField*> H;
  for (uint32_t k = 0; k < ne; ++k) {
    CField& f = *E[k];
    qoz_batch_item& it = items[f.item];
    const uint32_t* st = (const uint32_t*)(hb + kAl * k);
    const uint64_t* tot = (const uint64_t*)(hb + kAl * k + 32);
    f.n_words = tot[0];
    f.n_packed = tot[2];
    if (tot[1] != f.n_unpred) {
      it.status = QOZ_EDEVICE;
      continue;
    }
    f.lay = layout_of(f.P.n_anchor, f.usym.size(), f.nch, f.n_unpred,
                      f.n_words);
    if (f.lay.total > it.cap || (st[0] & kStOverflow)) {
      it.status = QOZ_ENOSPACE;
      it.out_bytes = f.lay.total;
      continue;
    }
    it.out_bytes = f.lay.total;
    H.push_back(&f);
  }
  const uint32_t nh = (uint32_t)H.size();
  if (nh) {
    const size_t hl = al((size_t)kHeaderBytes * nh);
    const size_t ub3 = hl + al(sizeof(DevCopy) * nh);
    hu = (uint8_t*)c->pinned + hdr; /* ub3 <= the region sized above */
    DevCopy* hcpy = (DevCopy*)(hu + hl);
    for (uint32_t k = 0; k < nh; ++k) {
      CField& f = *H[k];
      write_header(hu + (size_t)kHeaderBytes * k, f.P, f.n_unpred,
                   f.usym.size(), f.n_words);
      hcpy[k] = DevCopy{dB + (size_t)kHeaderBytes * k, items[f.item].d_out,
                        kHeaderBytes};
    }
    QOZ_TRY(to_device(c, dB, hu, ub3, s));
    launch_copy_list((const DevCopy*)(dB + hl), nh, s);
    QOZ_TRY(sync_q(s));
  }
  for (CField* fp : H) {
    CField& f = *fp;
    const uint64_t nch = f.nch;
    if (!f.n_words ||
        100 * (f.n_packed + 2 * (nch + 1)) > (uint64_t)kPackPercent * f.n_words)
      continue;
    qoz_batch_item& it = items[f.item];
    uint8_t* out = (uint8_t*)it.d_out;
    const Layout lp = layout_of(f.P.n_anchor, f.usym.size(), nch, f.n_unpred,
                                f.n_words, f.n_packed);
    QOZ_TRY(ensure(c->pcoff, 8 * (nch + 1)));
    QOZ_TRY(ensure(c->chunk_zeros, 4 * nch));
    QOZ_TRY(ensure(c->upre, 8 * (nch + 1)));
    QOZ_TRY(ensure(c->scan, chunk_scan_scratch(nch)));
    QOZ_TRY(ensure(c->status, 256));
    QOZ_TRY(ensure(c->ptmp, 4 * f.n_packed + 4));
    uint64_t* pcoff = (uint64_t*)c->pcoff.p;
    uint64_t* totals = (uint64_t*)((uint8_t*)c->status.p + 64);
    launch_chunk_scan((const uint32_t*)(D + f.pbits),
                      (const uint32_t*)c->chunk_zeros.p, nch, pcoff,
                      (uint64_t*)c->upre.p, totals, (uint64_t*)c->scan.p, s);
    uint32_t* raw = (uint32_t*)(out + f.lay.payload);
    launch_pack_write(raw, (const uint64_t*)(out + f.lay.coff), pcoff, nch,
                      (uint32_t*)c->ptmp.p, s);
    {
      void* dst[2] = {raw, out + lp.pcoff};
      const void* src[2] = {c->ptmp.p, pcoff};
      const uint64_t bytes[2] = {4 * f.n_packed, 8 * (nch + 1)};
      launch_copy_regions(dst, src, bytes, 2, s);
    }
    if (lp.pcoff > f.lay.payload + 4 * f.n_packed)
      launch_zero_u32((uint32_t*)(out + f.lay.payload + 4 * f.n_packed),
                      (lp.pcoff - f.lay.payload - 4 * f.n_packed) / 4, s);
    uint8_t* hs = (uint8_t*)c->pinned + hdr;
    write_header(hs, f.P, f.n_unpred, f.usym.size(), f.n_words);
    const uint16_t ver = kStreamVersionPacked;
    const uint32_t npk = (uint32_t)f.n_packed;
    std::memcpy(hs + 4, &ver, 2);
    std::memcpy(hs + 196, &npk, 4);
    QOZ_TRY(to_device(c, out, hs, kHeaderBytes, s));
    QOZ_TRY(sync_q(s));
    it.out_bytes = lp.total;
  }
  /* fields the queue could not take */
  for (uint32_t i : single) {
    qoz_batch_item& it = items[i];
    size_t ob = 0;
    it.status = qoz_compress(c, it.d_x, it.shape, it.abs_eb, &pv[i], target,
                             cfg, it.d_out, it.cap, &ob, s);
    it.out_bytes = ob;
  }
  const double ms = std::chrono::duration<double, std::milli>(
                        std::chrono::steady_clock::now() - t0)
                        .count();
  for (uint32_t i = 0; i < n; ++i) items[i].ms = items[i].done_ms = ms;
  for (uint32_t i = 0; i < n; ++i)
    if (items[i].status != QOZ_OK) {
      if (items_only) *items_only = true;
      return fail(items[i].status, "a field of the batch failed");
    }
  return QOZ_OK;
}
