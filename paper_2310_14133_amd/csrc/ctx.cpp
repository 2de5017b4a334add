/*
 * Context, scratch memory, error reporting and kernel timing of the QoZ GPU
 * library.
 */
#include <cstdio>
#include <cstring>
#include <string>

#include "qoz_internal.h"

namespace qoz {

static thread_local std::string g_last_error;

qoz_status fail(qoz_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

qoz_status hip_fail(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  g_last_error = m;
  return e == hipErrorOutOfMemory ? QOZ_ENOMEM : QOZ_EDEVICE;
}

void clear_error() { g_last_error.clear(); }

qoz_status set_device(qoz_ctx* c) {
  QOZ_HIP(hipSetDevice(c->device));
  return QOZ_OK;
}

qoz_status ensure(DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes && b.p) return QOZ_OK;
  if (b.p) {
    QOZ_HIP(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes < 256 ? 256 : bytes;
  QOZ_HIP(hipMalloc(&b.p, want));
  b.bytes = want;
  return QOZ_OK;
}

/* The host staging buffer is coherent pinned memory that the device reads
 * and writes directly: transfers to and from it are small kernels on the
 * library's stream (no copy engine, whose first uses in a process can stall
 * the stream for milliseconds). */
qoz_status ensure_pinned(qoz_ctx* c, size_t bytes) {
  if (bytes <= c->pinned_bytes && c->pinned) return QOZ_OK;
  if (c->pinned) {
    QOZ_HIP(hipHostFree(c->pinned));
    c->pinned = nullptr;
    c->pinned_dev = nullptr;
    c->pinned_bytes = 0;
  }
  QOZ_HIP(hipHostMalloc(&c->pinned, bytes,
                        hipHostMallocMapped | hipHostMallocCoherent));
  c->pinned_bytes = bytes;
  QOZ_HIP(hipHostGetDevicePointer(&c->pinned_dev, c->pinned, 0));
  return QOZ_OK;
}

static qoz_status pinned_dev(qoz_ctx* c, const void* h, size_t bytes,
                             void** d) {
  const uint8_t* base = (const uint8_t*)c->pinned;
  const uint8_t* p = (const uint8_t*)h;
  if (!base || p < base || p + bytes > base + c->pinned_bytes)
    return fail(QOZ_EDEVICE, "host transfer outside the staging buffer");
  *d = (uint8_t*)c->pinned_dev + (p - base);
  return QOZ_OK;
}

qoz_status to_host(qoz_ctx* c, void* h_dst, const void* d_src, size_t bytes,
                   hipStream_t s) {
  void* d = nullptr;
  QOZ_TRY(pinned_dev(c, h_dst, bytes, &d));
  launch_copy_host(d, d_src, bytes, true, s);
  QOZ_HIP(hipGetLastError());
  return QOZ_OK;
}

qoz_status gather_to_host(qoz_ctx* c, HostCopy* copies, uint32_t n,
                          hipStream_t s) {
  if (!n) return QOZ_OK;
  for (uint32_t i = 0; i < n; ++i)
    QOZ_TRY(pinned_dev(c, copies[i].dst, copies[i].bytes, &copies[i].dst));
  void* list = nullptr;
  QOZ_TRY(pinned_dev(c, copies, sizeof(HostCopy) * n, &list));
  launch_gather_host((const HostCopy*)list, n, s);
  QOZ_HIP(hipGetLastError());
  return QOZ_OK;
}

qoz_status to_device(qoz_ctx* c, void* d_dst, const void* h_src,
                     size_t bytes, hipStream_t s) {
  void* d = nullptr;
  QOZ_TRY(pinned_dev(c, h_src, bytes, &d));
  launch_copy_host(d_dst, d, bytes, false, s);
  QOZ_HIP(hipGetLastError());
  return QOZ_OK;
}

ProfSlot& prof_slot() {
  static thread_local ProfSlot slot;
  return slot;
}

static hipEvent_t pool_event(qoz_ctx* c) {
  hipEvent_t e = nullptr;
  if (!c->event_pool.empty()) {
    e = c->event_pool.back();
    c->event_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

hipEvent_t prof_begin(qoz_ctx* c, hipStream_t s, int kind) {
  (void)s;
  if (!((c->timing_mask >> kind) & 1u)) return nullptr;
  hipEvent_t a = pool_event(c);
  if (!a) return nullptr;
  hipEvent_t b = pool_event(c);
  if (!b) {
    c->event_pool.push_back(a);
    return nullptr;
  }
  prof_slot() = ProfSlot{a, b};
  return a;
}

void prof_end(qoz_ctx* c, hipStream_t s, hipEvent_t a, int kind,
              double bytes) {
  (void)s;
  if (!a) return;
  ProfSlot& slot = prof_slot();
  const hipEvent_t b = slot.stop;
  /* no launch took the start event: nothing ran, nothing is timed */
  const bool launched = slot.start == nullptr;
  slot = ProfSlot{};
  if (!launched) {
    c->event_pool.push_back(a);
    c->event_pool.push_back(b);
    return;
  }
  c->pending.push_back({kind, a, b, bytes});
}

void prof_collect(qoz_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess &&
        hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof_launches[p.kind] += 1;
      c->prof_ms[p.kind] += ms;
      c->prof_bytes[p.kind] += p.bytes;
    }
    c->event_pool.push_back(p.a);
    c->event_pool.push_back(p.b);
  }
  c->pending.clear();
}

static const char* kProfNames[PK_COUNT] = {
    "check_range",     "anchors",         "sweep_comp_level1",
    "sweep_comp",      "histogram",       "huffman_count",
    "huffman_encode",  "huffman_decode",  "sweep_decomp_level1",
    "sweep_decomp",    "tune_gather",     "tune_alg1",
    "tune_trial",      "ssim",            "reduce",
    "row_comp_level1", "row_decomp_level1", "learned_features",
    "mlp",             "zero_word_pack"};

}  // namespace qoz

using namespace qoz;

extern "C" {

qoz_status qoz_ctx_create(int hip_device, qoz_ctx** out) {
  clear_error();
  if (!out) return fail(QOZ_EINVAL, "out is NULL");
  int n = 0;
  QOZ_HIP(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n)
    return fail(QOZ_EINVAL, "no such HIP device");
  qoz_ctx* c = new (std::nothrow) qoz_ctx();
  if (!c) return fail(QOZ_ENOMEM, "context allocation failed");
  c->device = hip_device;
  qoz_status st = set_device(c);
  if (st == QOZ_OK) {
    const hipError_t e = fixed_scratch_addr(hip_device, &c->fixed_scratch);
    if (e != hipSuccess) st = hip_fail(e, "hipGetSymbolAddress(scratch)");
  }
  if (st == QOZ_OK) st = ensure_pinned(c, 2u << 20);
  if (st != QOZ_OK) {
    qoz_ctx_destroy(c);
    return st;
  }
  *out = c;
  return QOZ_OK;
}

void qoz_ctx_destroy(qoz_ctx* c) {
  if (!c) return;
  for (qoz_ctx* w : c->workers) qoz_ctx_destroy(w);
  (void)hipSetDevice(c->device);
  for (hipStream_t st : c->worker_streams) (void)hipStreamDestroy(st);
  if (c->qgraph_exec) (void)hipGraphExecDestroy(c->qgraph_exec);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  DevBuf* bufs[] = {&c->W,          &c->codes,      &c->hist,
                    &c->chunk_bits, &c->chunk_zeros, &c->coff,
                    &c->upre,       &c->status,     &c->enc_table,
                    &c->dec_tables, &c->dec_syms,   &c->anchors,
                    &c->partial,    &c->tune_x,     &c->tune_wc,
                    &c->tune_wt,    &c->tune_desc,  &c->tune_hist,
                    &c->tune_stats, &c->tune_l1,    &c->ssim_part,
                    &c->upos,       &c->hsort,      &c->scan,
                    &c->feat,       &c->mlp_io,     &c->mlp_part,
                    &c->mlp_loss,   &c->hsort_ids,  &c->pcoff,
                    &c->chunk_geo,
                    &c->ptmp,       &c->queue,      &c->lbatch,
                    &c->cqueue,     &c->cqueue_up};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (c->pinned) (void)hipHostFree(c->pinned);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  delete c;
}

const char* qoz_last_error(void) { return g_last_error.c_str(); }

qoz_status qoz_ctx_set_timing(qoz_ctx* c, int on) {
  if (!c) return fail(QOZ_EINVAL, "ctx is NULL");
  c->timing_mask = on ? ~0ull : 0ull;
  return QOZ_OK;
}

qoz_status qoz_ctx_set_timing_mask(qoz_ctx* c, uint64_t mask) {
  if (!c) return fail(QOZ_EINVAL, "ctx is NULL");
  c->timing_mask = mask;
  return QOZ_OK;
}

qoz_status qoz_ctx_reset_timing(qoz_ctx* c) {
  if (!c) return fail(QOZ_EINVAL, "ctx is NULL");
  for (int k = 0; k < PK_COUNT; ++k) {
    c->prof_launches[k] = 0;
    c->prof_ms[k] = 0;
    c->prof_bytes[k] = 0;
  }
  return QOZ_OK;
}

int qoz_prof_kinds(void) { return PK_COUNT; }

const char* qoz_prof_name(int kind) {
  return kind >= 0 && kind < PK_COUNT ? kProfNames[kind] : "";
}

qoz_status qoz_ctx_get_timing(qoz_ctx* c, int kind, uint64_t* launches,
                              double* total_ms, double* algo_bytes) {
  if (!c || kind < 0 || kind >= PK_COUNT)
    return fail(QOZ_EINVAL, "bad context or kind");
  if (launches) *launches = c->prof_launches[kind];
  if (total_ms) *total_ms = c->prof_ms[kind];
  if (algo_bytes) *algo_bytes = c->prof_bytes[kind];
  return QOZ_OK;
}

}  // extern "C"
