/*
 * Batched decompression through device work queues.  The inverse of
 * Sec. III's D_theta for many streams at once, in a fixed number of
 * launches whatever the batch size:
 *
 *   1. the headers of all streams are read back together (one wait), then
 *      all Huffman codebooks (a second wait); host threads build the
 *      decoding tables, and the tables and queues go up in one copy;
 *   2. one launch decodes every stream's chunks: the queue gives each
 *      stream a range of workgroups;
 *   3. one launch puts every stream's exact values (anchors and
 *      unpredictable bins) at their points (a packed payload is expanded
 *      before step 2, one small launch per packed stream);
 *   4. the interpolation sweeps run in rounds: round r is one launch over
 *      the r-th sweep (or fused level-1 row pair) of every stream, whose
 *      earlier sweeps all ran in earlier rounds;
 *   5. one read-back of the per-stream status words (a third wait).
 *
 * Every target is computed by the single-stream kernels' code, so each
 * output equals qoz_decompress's bit for bit.  The sweeps use the default
 * launch tiles (4 rows of 64 targets per workgroup).
 *
 * Steps 2-5 read everything that changes from call to call (streams,
 * outputs, tables) from the uploaded queues, so with graphs enabled a batch
 * with the same launch signature (grids, queue layout, scratch addresses,
 * packed payloads) as the call before replays them as one HIP graph.
 */
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "qoz_internal.h"

namespace qoz {
namespace {

constexpr size_t kAl = 256;
/* the host keeps each stream's decoding tables (about 18 KB) for the call */
constexpr uint32_t kMaxQueueFields = 1u << 14;
constexpr size_t kTableThreads = 16;

inline size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

struct QField {
  uint32_t item = 0;
  Plan P;
  uint64_t nu = 0, nused = 0, nw = 0, npk = 0;
  Layout lay{};
  size_t cb_pin = 0;               /* codebook in the pinned staging */
  DecTables tabs{};
  std::vector<uint32_t> sorted;
  size_t tab_off = 0, syms_off = 0; /* in the device upload region */
  size_t codes_off = 0, upos_off = 0, ptmp_off = 0; /* scratch region */
  std::vector<SweepJob> steps;
};

qoz_status sync_stream(hipStream_t s) {
  QOZ_HIP(hipGetLastError());
  QOZ_HIP(hipStreamSynchronize(s));
  return QOZ_OK;
}

void write_shape(const Plan& P, qoz_shape* out) {
  std::memset(out, 0, sizeof(*out));
  out->ndim = (uint32_t)P.d;
  if (P.d == 2) {
    out->dims[0] = P.g.n[1];
    out->dims[1] = P.g.n[2];
    out->dims[2] = 1;
  } else {
    for (int i = 0; i < 3; ++i) out->dims[i] = P.g.n[i];
  }
}

/* The device work of a call as a HIP graph (when enabled): a call whose
 * signature equals
 * the previous call's captures its sequence once (on the context's capture
 * stream, where nothing runs) and launches the graph on s; later calls with
 * the same signature launch it again.  Other calls issue the sequence on s
 * directly and remember their signature. */
template <class Issue>
qoz_status run_queue_graph(qoz_ctx* c, const std::vector<uint64_t>& sig,
                           Issue issue, hipStream_t s) {
  if (!c->queue_graphs) return issue(s);
  if (c->qgraph_exec && sig == c->qgraph_sig) {
    QOZ_HIP(hipGraphLaunch(c->qgraph_exec, s));
    return QOZ_OK;
  }
  if (sig != c->qgraph_last) {
    c->qgraph_last = sig;
    return issue(s);
  }
  if (!c->capture_stream)
    QOZ_HIP(hipStreamCreateWithFlags(&c->capture_stream,
                                     hipStreamNonBlocking));
  QOZ_HIP(hipStreamBeginCapture(c->capture_stream,
                                hipStreamCaptureModeThreadLocal));
  const qoz_status st = issue(c->capture_stream);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(c->capture_stream, &g);
  if (st != QOZ_OK || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    c->qgraph_last.clear();
    return st != QOZ_OK ? st : hip_fail(ee, "hipStreamEndCapture");
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
  if (c->qgraph_exec) (void)hipGraphExecDestroy(c->qgraph_exec);
  c->qgraph_exec = ex;
  c->qgraph_sig = sig;
  QOZ_HIP(hipGraphLaunch(c->qgraph_exec, s));
  return QOZ_OK;
}

}  // namespace
}  // namespace qoz

using namespace qoz;

extern "C" qoz_status qoz_ctx_set_queue_graphs(qoz_ctx* c, int enable) {
  clear_error();
  if (!c) return fail(QOZ_EINVAL, "NULL argument");
  QOZ_TRY(set_device(c));
  c->queue_graphs = enable != 0;
  if (!c->queue_graphs && c->qgraph_exec) {
    QOZ_HIP(hipGraphExecDestroy(c->qgraph_exec));
    c->qgraph_exec = nullptr;
  }
  c->qgraph_sig.clear();
  c->qgraph_last.clear();
  return QOZ_OK;
}

extern "C" qoz_status qoz_decompress_queue(qoz_ctx* c,
                                           qoz_batch_dec_item* items,
                                           uint32_t n, hipStream_t s) {
  clear_error();
  if (!c || (n && !items)) return fail(QOZ_EINVAL, "NULL argument");
  if (n > kMaxQueueFields) return fail(QOZ_EINVAL, "batch too large");
  QOZ_TRY(set_device(c));
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t i = 0; i < n; ++i) {
    items[i].status = QOZ_OK;
    items[i].ms = items[i].done_ms = 0.0;
  }
  if (!n) return QOZ_OK;

  /* 1a. headers */
  const size_t hdr = kPinSingleBytes;
  QOZ_TRY(ensure_pinned(c, hdr + (size_t)n * kAl + al(sizeof(HostCopy) * n)));
  uint8_t* pin = (uint8_t*)c->pinned;
  {
    HostCopy* hc = (HostCopy*)(pin + hdr + (size_t)n * kAl);
    uint32_t m = 0;
    for (uint32_t i = 0; i < n; ++i) {
      qoz_batch_dec_item& it = items[i];
      if (!it.d_in || ((uintptr_t)it.d_in & 7) != 0)
        it.status = QOZ_EINVAL;
      else if (it.in_bytes < kHeaderBytes)
        it.status = QOZ_EFORMAT;
      else
        hc[m++] = HostCopy{it.d_in, pin + hdr + (size_t)i * kAl, kHeaderBytes};
    }
    QOZ_TRY(gather_to_host(c, hc, m, s));
  }
  QOZ_TRY(sync_stream(s));
  std::vector<QField> F;
  F.reserve(n);
  size_t cb_bytes = 0;
  for (uint32_t i = 0; i < n; ++i) {
    qoz_batch_dec_item& it = items[i];
    if (it.status != QOZ_OK) continue;
    QField f;
    f.item = i;
    const qoz_status st =
        parse_header(pin + hdr + (size_t)i * kAl, it.in_bytes, true, &f.P,
                     &f.nu, &f.nused, &f.nw, &f.npk);
    if (st != QOZ_OK) {
      it.status = st;
      continue;
    }
    const uint64_t N = (uint64_t)f.P.g.n[0] * f.P.g.n[1] * f.P.g.n[2];
    if (!it.d_y || it.y_cap_elems < N) {
      it.status = QOZ_ENOSPACE;
      continue;
    }
    f.lay = layout_of(f.P.n_anchor, f.nused, f.P.n_chunks, f.nu, f.nw, f.npk);
    f.cb_pin = hdr + cb_bytes;
    cb_bytes += al(f.lay.coff - f.lay.syms);
    F.push_back(std::move(f));
  }

  /* 1b. codebooks, then the decoding tables on the host */
  QOZ_TRY(ensure_pinned(c, hdr + cb_bytes + al(sizeof(HostCopy) * F.size())));
  pin = (uint8_t*)c->pinned;
  {
    HostCopy* hc = (HostCopy*)(pin + hdr + cb_bytes);
    for (size_t k = 0; k < F.size(); ++k)
      hc[k] = HostCopy{(const uint8_t*)items[F[k].item].d_in + F[k].lay.syms,
                       pin + F[k].cb_pin, F[k].lay.coff - F[k].lay.syms};
    QOZ_TRY(gather_to_host(c, hc, (uint32_t)F.size(), s));
  }
  QOZ_TRY(sync_stream(s));
  {
    /* tables on up to kTableThreads host threads */
    std::vector<char> ok(F.size(), 0);
    std::atomic<size_t> next{0};
    auto work = [&]() {
      for (size_t k; (k = next.fetch_add(1)) < F.size();) {
        QField& f = F[k];
        const uint8_t* cb = pin + f.cb_pin;
        ok[k] = build_dec_tables((const uint16_t*)cb,
                                 cb + (f.lay.lens - f.lay.syms),
                                 (uint32_t)f.nused, &f.tabs, &f.sorted);
      }
    };
    size_t nt = F.size() < kTableThreads ? F.size() : kTableThreads;
    std::vector<std::thread> th;
    for (size_t t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
    for (size_t k = 0; k < F.size(); ++k)
      if (!ok[k]) items[F[k].item].status = QOZ_EFORMAT;
  }
  std::vector<QField> G;
  G.reserve(F.size());
  for (QField& f : F)
    if (items[f.item].status == QOZ_OK) G.push_back(std::move(f));
  const uint32_t nf = (uint32_t)G.size();

  /* 2. queues: per-field steps, rounds */
  size_t rounds = 0;
  for (QField& f : G) {
    size_t fz = SIZE_MAX, fa = SIZE_MAX, fb = SIZE_MAX;
    RowJob rj;
    const bool fuse = level1_rows(f.P, &fz, &fa, &fb, &rj);
    for (size_t i = 0; i < f.P.sweeps.size(); ++i) {
      SweepJob j;
      std::memset(&j, 0, sizeof(j));
      j.g = f.P.g;
      if (fuse && (i == fz || i == fa || i == fb)) {
        if (i != fb) continue;
        j.rows = 1;
        j.rj = rj;
      } else {
        j.s = f.P.sweeps[i];
      }
      f.steps.push_back(j);
    }
    if (f.steps.size() > rounds) rounds = f.steps.size();
  }

  /* device layout: upload region (tables, queues, status words), then
   * per-field scratch */
  size_t up = 0;
  for (QField& f : G) {
    f.tab_off = up;
    up += al(sizeof(DecTables));
    f.syms_off = up;
    up += al(4 * (f.sorted.size() ? f.sorted.size() : 1));
  }
  std::vector<size_t> st_tab(nf);
  for (uint32_t k = 0; k < nf; ++k) {
    st_tab[k] = up;
    up += al(sizeof(SweepTable));
  }
  const size_t ex_jobs = up;
  up += al(sizeof(ExactJob) * (nf ? nf : 1));
  const size_t ex_wg0 = up;
  up += al(4 * (nf + 1));
  const size_t dec_jobs = up;
  up += al(sizeof(DecJob) * (nf ? nf : 1));
  const size_t dec_wg0 = up;
  up += al(4 * (nf + 1));
  std::vector<size_t> rj_off(rounds), rw_off(rounds);
  for (size_t r = 0; r < rounds; ++r) {
    rj_off[r] = up;
    up += al(sizeof(SweepJob) * (nf ? nf : 1));
    rw_off[r] = up;
    up += al(4 * (nf + 1));
  }
  const size_t st_off = up;
  up += al(4 * (nf ? nf : 1));
  const size_t upload = up;
  for (QField& f : G) {
    f.codes_off = up;
    up += al(2 * (f.P.n_codes + 16));
    f.upos_off = up;
    up += al(4 * (f.nu + 1));
    f.ptmp_off = up;
    if (f.npk) up += al(4 * f.nw + 4);
  }
  QOZ_TRY(ensure(c->queue, up));
  QOZ_TRY(ensure_pinned(c, hdr + upload + al(4 * (nf ? nf : 1))));
  pin = (uint8_t*)c->pinned;
  uint8_t* const hu = pin + hdr;         /* host image of the upload */
  uint8_t* const dq = (uint8_t*)c->queue.p; /* its device address */
  std::memset(hu, 0, upload);

  DecJob* dj = (DecJob*)(hu + dec_jobs);
  uint32_t* dw = (uint32_t*)(hu + dec_wg0);
  uint32_t dec_total = 0;
  for (uint32_t k = 0; k < nf; ++k) {
    QField& f = G[k];
    const uint8_t* in = (const uint8_t*)items[f.item].d_in;
    std::memcpy(hu + f.tab_off, &f.tabs, sizeof(DecTables));
    if (!f.sorted.empty())
      std::memcpy(hu + f.syms_off, f.sorted.data(), 4 * f.sorted.size());
    DecJob& j = dj[k];
    j.payload = f.npk ? (const uint32_t*)(dq + f.ptmp_off)
                      : (const uint32_t*)(in + f.lay.payload);
    j.n_words = f.nw;
    j.coff = (const uint64_t*)(in + f.lay.coff);
    j.upre = (const uint32_t*)(in + f.lay.upre);
    j.segs = (const uint16_t*)(in + f.lay.segs);
    j.ch = f.P.chunks;
    j.n_unpred = f.nu;
    j.tabs = (const DecTables*)(dq + f.tab_off);
    j.syms = (const uint32_t*)(dq + f.syms_off);
    j.codes = (uint16_t*)(dq + f.codes_off);
    j.upos = (uint32_t*)(dq + f.upos_off);
    j.status = (uint32_t*)(dq + st_off) + k;
    dw[k] = dec_total;
    dec_total += decode_workgroups(f.P.chunks.count());
  }
  dw[nf] = dec_total;
  ExactJob* ej = (ExactJob*)(hu + ex_jobs);
  uint32_t* ew = (uint32_t*)(hu + ex_wg0);
  uint32_t ex_total = 0;
  for (uint32_t k = 0; k < nf; ++k) {
    const QField& f = G[k];
    const uint8_t* in = (const uint8_t*)items[f.item].d_in;
    fill_sweep_table(f.P, (SweepTable*)(hu + st_tab[k]));
    ExactJob& e = ej[k];
    e.g = f.P.g;
    e.stride = f.P.s;
    for (int d = 0; d < 3; ++d) e.na[d] = f.P.na[d];
    e.anchors = (const float*)(in + f.lay.anchors);
    e.st = (const SweepTable*)(dq + st_tab[k]);
    e.upos = (const uint32_t*)(dq + f.upos_off);
    e.vals = (const float*)(in + f.lay.unpred);
    e.n_unpred = f.nu;
    e.n_codes = f.P.n_codes;
    e.W = items[f.item].d_y;
    e.status = (uint32_t*)(dq + st_off) + k;
    ew[k] = ex_total;
    ex_total += exact_job_workgroups(&e);
  }
  ew[nf] = ex_total;
  std::vector<uint32_t> r_total(rounds, 0), r_jobs(rounds, 0);
  std::vector<size_t> r_lds(rounds, 0);
  for (size_t r = 0; r < rounds; ++r) {
    SweepJob* sj = (SweepJob*)(hu + rj_off[r]);
    uint32_t* sw = (uint32_t*)(hu + rw_off[r]);
    uint32_t m = 0, tot = 0;
    for (QField& f : G) {
      if (r >= f.steps.size()) continue;
      SweepJob j = f.steps[r];
      size_t lds = 0;
      const uint32_t wgs = sweep_job_prepare(&j, &lds);
      if (!wgs) continue;
      j.W = items[f.item].d_y;
      j.codes = (const uint16_t*)(dq + f.codes_off);
      sj[m] = j;
      sw[m] = tot;
      tot += wgs;
      ++m;
      if (lds > r_lds[r]) r_lds[r] = lds;
    }
    sw[m] = tot;
    r_jobs[r] = m;
    r_total[r] = tot;
  }

  /* 3. device work: upload, launches, status read-back.  Everything a
   * launch reads from the call (streams, outputs, tables) goes through the
   * uploaded queues, except the expansion of packed payloads, so the same
   * sequence serves any batch with the same signature below. */
  uint32_t* hs = (uint32_t*)(pin + hdr + upload);
  auto issue = [&](hipStream_t q) -> qoz_status {
    QOZ_TRY(to_device(c, dq, hu, upload, q));
    for (uint32_t k = 0; k < nf; ++k) {
      const QField& f = G[k];
      if (!f.npk) continue;
      const uint8_t* in = (const uint8_t*)items[f.item].d_in;
      launch_unpack((const uint32_t*)(in + f.lay.payload), f.npk,
                    (const uint64_t*)(in + f.lay.coff),
                    (const uint64_t*)(in + f.lay.pcoff), f.P.n_chunks, f.nw,
                    (uint32_t*)(dq + f.ptmp_off),
                    (uint32_t*)(dq + st_off) + k, q);
    }
    launch_huff_decode_q((const DecJob*)(dq + dec_jobs),
                         (const uint32_t*)(dq + dec_wg0), nf, dec_total, q);
    launch_exact_q((const ExactJob*)(dq + ex_jobs),
                   (const uint32_t*)(dq + ex_wg0), nf, ex_total, q);
    for (size_t r = 0; r < rounds; ++r)
      launch_sweep_round_q((const SweepJob*)(dq + rj_off[r]),
                           (const uint32_t*)(dq + rw_off[r]), r_jobs[r],
                           r_total[r], r_lds[r], q);
    QOZ_TRY(to_host(c, hs, dq + st_off, 4 * (nf ? nf : 1), q));
    return QOZ_OK;
  };
  /* the signature: every value the sequence passes to the device */
  std::vector<uint64_t> sig = {(uintptr_t)dq, (uintptr_t)c->pinned, hdr,
                               upload, st_off, nf, dec_jobs, dec_wg0,
                               dec_total, ex_jobs, ex_wg0, ex_total, rounds};
  for (size_t r = 0; r < rounds; ++r) {
    sig.push_back(rj_off[r]);
    sig.push_back(rw_off[r]);
    sig.push_back(r_jobs[r]);
    sig.push_back(r_total[r]);
    sig.push_back(r_lds[r]);
  }
  for (uint32_t k = 0; k < nf; ++k) {
    const QField& f = G[k];
    if (!f.npk) continue;
    sig.insert(sig.end(), {k, (uintptr_t)items[f.item].d_in, f.lay.payload,
                           f.lay.coff, f.lay.pcoff, f.npk, f.P.n_chunks, f.nw,
                           f.ptmp_off});
  }
  QOZ_TRY(run_queue_graph(c, sig, issue, s));
  QOZ_TRY(sync_stream(s));
  const double ms = std::chrono::duration<double, std::milli>(
                        std::chrono::steady_clock::now() - t0)
                        .count();
  for (uint32_t k = 0; k < nf; ++k) {
    qoz_batch_dec_item& it = items[G[k].item];
    if (hs[k] & kStBadStream)
      it.status = QOZ_EFORMAT;
    else
      write_shape(G[k].P, &it.shape);
  }
  for (uint32_t i = 0; i < n; ++i) items[i].ms = items[i].done_ms = ms;
  for (uint32_t i = 0; i < n; ++i)
    if (items[i].status != QOZ_OK)
      return fail(items[i].status, "a stream of the batch failed");
  return QOZ_OK;
}
