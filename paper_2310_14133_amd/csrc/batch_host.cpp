/*
 * Batches of fields: worker threads, each with its own context (scratch
 * and pinned staging) and its own stream, take fields from a shared
 * queue, largest first.  A field's host steps (the Huffman code built from
 * its histogram, the tuner's decisions, the read-back of sizes) then
 * overlap the kernels of fields on other streams, and small fields no
 * longer leave the GPU idle between launches.  Each field runs the
 * single-field path unchanged, so its bytes are the same.
 */
#include <algorithm>
#include <atomic>
#include <chrono>
#include <functional>
#include <numeric>
#include <thread>
#include <vector>

#include "qoz_internal.h"

namespace qoz {

constexpr uint32_t kMaxWorkers = 64;
constexpr uint32_t kDefaultWorkers = 4;

qoz_status ensure_workers(qoz_ctx* c, uint32_t n) {
  while (c->workers.size() < n) {
    qoz_ctx* w = nullptr;
    QOZ_TRY(qoz_ctx_create(c->device, &w));
    hipStream_t st = nullptr;
    const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      qoz_ctx_destroy(w);
      return hip_fail(e, "hipStreamCreateWithFlags");
    }
    c->workers.push_back(w);
    c->worker_streams.push_back(st);
  }
  return QOZ_OK;
}

/* Runs fn(worker, index) over items in the given order on `workers`
 * threads (the caller's thread is worker 0). */
template <class Fn>
static void run_queue(const std::vector<uint32_t>& order, uint32_t workers,
                      const Fn& fn) {
  std::atomic<uint32_t> next{0};
  auto body = [&](uint32_t w) {
    for (;;) {
      const uint32_t k = next.fetch_add(1);
      if (k >= order.size()) break;
      fn(w, order[k]);
    }
  };
  std::vector<std::thread> th;
  for (uint32_t w = 1; w < workers; ++w) th.emplace_back(body, w);
  body(0);
  for (auto& t : th) t.join();
}

void run_on_workers(const std::vector<uint32_t>& order, uint32_t workers,
                    const std::function<void(uint32_t, uint32_t)>& fn) {
  run_queue(order, workers, fn);
}

static double ms_since(std::chrono::steady_clock::time_point t) {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now() - t)
      .count();
}

static uint64_t points_of(const qoz_shape& sh) {
  uint64_t n = 1;
  for (uint32_t i = 0; i < sh.ndim && i < 3; ++i) n *= sh.dims[i];
  return n;
}

/* Largest first, ties in index order. */
static std::vector<uint32_t> by_size(uint32_t n,
                                     const std::vector<uint64_t>& size) {
  std::vector<uint32_t> order(n);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    return size[a] > size[b];
  });
  return order;
}

static qoz_status prepare(qoz_ctx* c, uint32_t& workers, uint32_t n,
                          hipStream_t s) {
  if (workers == 0) workers = kDefaultWorkers;
  if (workers > kMaxWorkers) return fail(QOZ_EINVAL, "too many workers");
  if (workers > n) workers = n ? n : 1;
  QOZ_TRY(set_device(c));
  QOZ_HIP(hipStreamSynchronize(s));
  return ensure_workers(c, workers);
}

}  // namespace qoz

using namespace qoz;

extern "C" qoz_status qoz_compress_batch(qoz_ctx* c, qoz_batch_item* items,
                                         uint32_t n, qoz_target target,
                                         const qoz_tune_config* cfg,
                                         uint32_t workers, hipStream_t s) {
  clear_error();
  if (!c || (n && !items)) return fail(QOZ_EINVAL, "NULL argument");
  QOZ_TRY(prepare(c, workers, n, s));
  std::vector<uint64_t> size(n);
  for (uint32_t i = 0; i < n; ++i) size[i] = points_of(items[i].shape);
  const auto t0 = std::chrono::steady_clock::now();
  run_queue(by_size(n, size), workers, [&](uint32_t w, uint32_t i) {
    qoz_batch_item& it = items[i];
    const auto ti = std::chrono::steady_clock::now();
    it.out_bytes = 0;
    it.status = qoz_compress(c->workers[w], it.d_x, it.shape, it.abs_eb,
                             it.params, target, cfg, it.d_out, it.cap,
                             &it.out_bytes, c->worker_streams[w]);
    it.ms = ms_since(ti);
    it.done_ms = ms_since(t0);
  });
  for (uint32_t w = 0; w < workers; ++w)
    QOZ_HIP(hipStreamSynchronize(c->worker_streams[w]));
  for (uint32_t i = 0; i < n; ++i)
    if (items[i].status != QOZ_OK)
      return fail(items[i].status, "a field of the batch failed");
  return QOZ_OK;
}

extern "C" qoz_status qoz_decompress_batch(qoz_ctx* c,
                                           qoz_batch_dec_item* items,
                                           uint32_t n, uint32_t workers,
                                           hipStream_t s) {
  clear_error();
  if (!c || (n && !items)) return fail(QOZ_EINVAL, "NULL argument");
  QOZ_TRY(prepare(c, workers, n, s));
  std::vector<uint64_t> size(n);
  for (uint32_t i = 0; i < n; ++i) size[i] = items[i].y_cap_elems;
  const auto t0 = std::chrono::steady_clock::now();
  run_queue(by_size(n, size), workers, [&](uint32_t w, uint32_t i) {
    qoz_batch_dec_item& it = items[i];
    const auto ti = std::chrono::steady_clock::now();
    it.status = qoz_decompress(c->workers[w], it.d_in, it.in_bytes, it.d_y,
                               it.y_cap_elems, &it.shape,
                               c->worker_streams[w]);
    it.ms = ms_since(ti);
    it.done_ms = ms_since(t0);
  });
  for (uint32_t w = 0; w < workers; ++w)
    QOZ_HIP(hipStreamSynchronize(c->worker_streams[w]));
  for (uint32_t i = 0; i < n; ++i)
    if (items[i].status != QOZ_OK)
      return fail(items[i].status, "a field of the batch failed");
  return QOZ_OK;
}
