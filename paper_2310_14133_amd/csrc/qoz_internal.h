/*
 * Internal declarations of the QoZ GPU library (gfx950).  Not part of the
 * public ABI.
 *
 * Geometry convention: every field is handled as a 3D grid (n0, n1, n2)
 * with n2 contiguous; a 2D field (a, b) becomes (1, a, b) and its dimension
 * order is shifted by one (real dimension m -> grid dimension m + 1).
 */
#ifndef QOZ_INTERNAL_H
#define QOZ_INTERNAL_H
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <functional>
#include <vector>

#include "../../include/qoz.h"

namespace qoz {

constexpr int32_t kRadius = 32768;         /* bins on each side of zero */
constexpr uint32_t kNSym = 2 * kRadius;    /* Huffman alphabet */
constexpr uint32_t kChunk = 4096;          /* bins per level-1 chunk */
constexpr uint32_t kSegLog2 = 9;           /* a chunk holds 8 segments of */
constexpr uint32_t kSeg = 1u << kSegLog2;  /* 512 bins, each decodable alone */
constexpr uint32_t kSegPerChunk = kChunk / kSeg;
constexpr size_t kHeaderBytes = 200;
/* pinned staging bytes of the single-field calls; the batched
 * decompression stages past them */
constexpr size_t kPinSingleBytes = 2u << 20;
/* Fixed device scratch of the calls that allocate nothing: a file-scope
 * device array of this many bytes per device (status words, the range and
 * SSE partial sums, then the SSIM partial sums). */
constexpr size_t kFixedScratchBytes = 4u << 20;
constexpr size_t kFixedStatusOff = 0;
constexpr size_t kFixedPartialOff = 256;
constexpr size_t kFixedSsimOff = 64u << 10;
constexpr uint16_t kStreamVersion = 4;       /* unpacked payload */
constexpr uint16_t kStreamVersionPacked = 5; /* zero-word packed payload */
constexpr uint32_t kPackPercent = 97; /* pack when packed <= 97 % of raw */

/* Chunks of the bin stream, by level: level l (levels L..1 in stream
 * order) is cut into chunks of max(kChunk >> (l - 1), kMinChunk) bins, level
 * boundaries rounded up to a multiple of 64 bins (at most all bins), a
 * level's last chunk possibly shorter.  Coarser levels carry more long
 * codes per bin, so their segments are shorter, to decode in about the
 * time of a level-1 segment; the rounding keeps chunk starts 128-byte
 * aligned in the bin array. */
constexpr uint32_t kMinChunk = 1024;
struct Chunks {
  uint32_t n = 0;                          /* regions: one per level */
  uint32_t size[QOZ_MAX_LEVELS];           /* chunk size of region r */
  uint64_t start[QOZ_MAX_LEVELS + 1];      /* first bin; start[n] = bins */
  uint64_t first[QOZ_MAX_LEVELS + 1];      /* first chunk; first[n] = all */
  /* the regions whose first chunk is at or before c, less one (first[] is
   * non-decreasing); unrolled, so that on the device the reads of a
   * uniform c stay scalar loads outside any loop */
  __host__ __device__ uint32_t region(uint64_t c) const {
    uint32_t r = 0;
#pragma unroll
    for (uint32_t i = 1; i < QOZ_MAX_LEVELS; ++i)
      r += (i < n && c >= first[i]) ? 1u : 0u;
    return r;
  }
  __host__ __device__ uint64_t begin(uint64_t c) const {
    const uint32_t r = region(c);
    return start[r] + (c - first[r]) * size[r];
  }
  __host__ __device__ uint64_t end(uint64_t c) const {
    const uint32_t r = region(c);
    const uint64_t e = start[r] + (c - first[r] + 1) * size[r];
    return e < start[r + 1] ? e : start[r + 1];
  }
  __host__ __device__ uint64_t count() const { return n ? first[n] : 0; }
};
constexpr int kSymBits = 12;               /* decoder table width */
constexpr int kMaxCodeLen = 63;

/* status word bits reported by kernels */
constexpr uint32_t kStNonFinite = 1u;
constexpr uint32_t kStBadStream = 2u;
constexpr uint32_t kStOverflow = 4u;

struct Geo {
  uint32_t n[3];  /* grid extents */
  uint32_t st[3]; /* element strides: st[2] = 1 */
};

/* One (level, dimension) sweep: its target sub-grid and quantizer. */
struct Sweep {
  uint32_t start[3], step[3], cnt[3];
  uint32_t k;      /* grid dimension interpolated along */
  uint32_t h;      /* 2^(l-1) */
  uint32_t cubic;  /* 0 linear, 1 cubic */
  uint32_t level;
  uint64_t code_off; /* position of the first target's bin in the stream */
  uint64_t count;    /* targets */
  float twoeb, inv;  /* FP32 bin width 2 e_l and its reciprocal */
  double eb;         /* e_l */
};

/* Level-1 fusion of sweep A (along dimension a, or none: a = -1) with the
 * following sweep B along the contiguous dimension, over the rows (p0, p1)
 * = (i0 * rstep[0], i1 * rstep[1]); when the level's order is (f, a, 2),
 * also of the first sweep F (f = -1: not fused). */
constexpr uint32_t kRowMaxEven = 8192; /* rows of up to 16384 points */
struct RowJob {
  int32_t a, f;
  uint32_t rstep[2], rcnt[2];
  /* set by the launcher: tiles of T rows (along a) by S points */
  uint32_t T, S, tilesT, tiles2;
  /* the sweep's bins of a row start on a multiple of 4 (8-byte access) */
  uint32_t vecA, vecB, vecF;
  Sweep A, B, F;
};

/* Complete plan of one compression / decompression. */
struct Plan {
  Geo g;
  int d = 0;           /* real dimensionality */
  uint32_t s = 0, L = 0;
  double e = 0, alpha = 1, beta = 1;
  uint8_t interp[QOZ_MAX_LEVELS];
  uint8_t order[QOZ_MAX_LEVELS][3]; /* real dimensions */
  uint32_t na[3];      /* anchors per grid dimension */
  uint64_t n_anchor = 0, n_codes = 0, n_chunks = 0;
  Chunks chunks;
  std::vector<Sweep> sweeps;
};

/* Byte offsets of the stream sections (see the stream layout notes). */
struct Layout {
  uint64_t anchors, syms, lens, coff, upre, segs, unpred, payload, pcoff,
      total;
};

/* Sweep table used by kernels that map a stream position back to a point. */
struct SweepTable {
  uint32_t n;
  uint64_t off[3 * QOZ_MAX_LEVELS + 1];
  uint32_t start[3 * QOZ_MAX_LEVELS][3];
  uint32_t step[3 * QOZ_MAX_LEVELS][3];
  uint32_t cnt[3 * QOZ_MAX_LEVELS][3];
};

/* Canonical-Huffman decoding tables (device copy). */
/* second-level decoder entries (codes of kSymBits + 1 .. kSymBits + 8 bits) */
constexpr uint32_t kEnt2 = 1024;
constexpr uint32_t kEnt2Depth = 8;
struct DecTables {
  /* indexed by the next kSymBits bits: for a code of at most kSymBits bits
   * its length (bits 0-5), 0x40 if it is symbol 0's code, and its symbol
   * (bits 16-31); for a prefix of longer codes that has a second-level
   * table, 0x80 | (d << 8) | (offset << 12): the next d bits index
   * ent2[offset ..]; 0 otherwise (a longer code without one, or invalid) */
  uint32_t ent[1u << kSymBits];
  /* second level: entries as in ent for the codes of a prefix whose length
   * exceeds kSymBits by at most the prefix's d; 0 for longer or invalid */
  uint32_t ent2[kEnt2];
  uint64_t first[kMaxCodeLen + 1];
  uint32_t cnt[kMaxCodeLen + 1];
  uint32_t off[kMaxCodeLen + 1];
  uint32_t maxlen;
  uint32_t n_used;
  uint32_t zlen;  /* length of symbol 0's code (0 if unused) */
  uint64_t zcode; /* symbol 0's code */
  /* (first code of length L + count of length L) << (63 - L): a 64-bit
   * left-justified window V starts with a codeword longer than L iff
   * (V >> 1) >= lim_half[L] */
  uint64_t lim_half[kMaxCodeLen + 1];
};

/* Tuner: one level of a candidate parameter set on the sampled blocks. */
struct TrialLevel {
  float twoeb, inv;
  double eb;
  uint32_t cubic;
  uint32_t order[3]; /* grid dimensions */
};
struct TrialDesc {
  TrialLevel lv[QOZ_MAX_LEVELS];
};

/* Profiling kinds */
enum ProfKind {
  PK_CHECK = 0,
  PK_ANCHOR,
  PK_SWEEP_COMP_L1,
  PK_SWEEP_COMP,
  PK_HIST,
  PK_HUFF_COUNT,
  PK_HUFF_ENC,
  PK_HUFF_DEC,
  PK_SWEEP_DEC_L1,
  PK_SWEEP_DEC,
  PK_TUNE_GATHER,
  PK_TUNE_ALG1,
  PK_TUNE_TRIAL,
  PK_SSIM,
  PK_REDUCE,
  PK_ROW_COMP_L1,
  PK_ROW_DEC_L1,
  PK_LEARN_FEAT,
  PK_MLP,
  PK_PACK,
  PK_COUNT
};

/* Sweep launch tile: ty rows of 64 targets per workgroup (a power of two
 * up to 16), rpt rows per lane; the default is (4, 1). */
struct SweepTile {
  uint8_t ty = 4, rpt = 1;
};

/* Growable device buffer. */
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct PendingEvent {
  int kind;
  hipEvent_t a, b;
  double bytes;
};

}  // namespace qoz

struct qoz_ctx {
  int device = 0;
  /* scratch */
  qoz::DevBuf W, codes, hist, chunk_bits, chunk_zeros, coff, upre, status,
      enc_table, dec_tables, dec_syms, anchors, partial, tune_x, tune_wc,
      tune_wt, tune_desc, tune_hist, tune_stats, tune_l1, ssim_part, upos,
      hsort, scan, feat, mlp_io, mlp_part, mlp_loss, hsort_ids, pcoff, ptmp,
      queue, lbatch, cqueue, cqueue_up, chunk_geo;
  /* sweep launch tiles chosen by qoz_autotune_tiles, per plan signature */
  std::map<std::vector<uint32_t>, std::vector<qoz::SweepTile>> tiles_comp,
      tiles_decomp;
  /* work-queue decompression replayed as a graph (queue_host.cpp) */
  bool queue_graphs = false;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t qgraph_exec = nullptr;
  std::vector<uint64_t> qgraph_sig, qgraph_last;
  /* batch workers: their contexts and streams */
  std::vector<qoz_ctx*> workers;
  std::vector<hipStream_t> worker_streams;
  /* this device's copy of the fixed scratch array (its device address) */
  void* fixed_scratch = nullptr;
  /* pinned host staging */
  void* pinned = nullptr;
  void* pinned_dev = nullptr; /* its device address */
  size_t pinned_bytes = 0;
  /* instrumentation */
  uint64_t timing_mask = 0; /* bit k: time launches of kind k */
  std::vector<qoz::PendingEvent> pending;
  std::vector<hipEvent_t> event_pool;
  uint64_t prof_launches[qoz::PK_COUNT] = {0};
  double prof_ms[qoz::PK_COUNT] = {0};
  double prof_bytes[qoz::PK_COUNT] = {0};
};

namespace qoz {

/* ---- errors --------------------------------------------------------- */
qoz_status fail(qoz_status st, const std::string& msg);
qoz_status hip_fail(hipError_t e, const char* what);
void clear_error();
#define QOZ_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return qoz::hip_fail(e_, #call); \
  } while (0)
#define QOZ_TRY(expr)                     \
  do {                                    \
    qoz_status s_ = (expr);               \
    if (s_ != QOZ_OK) return s_;          \
  } while (0)

/* ---- context helpers ------------------------------------------------- */
qoz_status ensure(DevBuf& b, size_t bytes);
qoz_status ensure_pinned(qoz_ctx* c, size_t bytes);
/* stream-ordered transfers between device memory and the pinned staging
 * buffer (the host pointer must lie inside it) */
qoz_status to_host(qoz_ctx* c, void* h_dst, const void* d_src, size_t bytes,
                   hipStream_t s);
qoz_status to_device(qoz_ctx* c, void* d_dst, const void* h_src,
                     size_t bytes, hipStream_t s);
/* Instrumented launch bracket: call prof_begin before and prof_end after
 * the launches of one kind; resolved by prof_collect after the stream is
 * synchronised.  The bracket's two events travel with the kernel launches
 * themselves (QOZ_LAUNCH): the first launch inside takes the start event,
 * every launch the stop event, so the time measured is from the first
 * kernel's start to the last one's end, whatever the stream did before. */
hipEvent_t prof_begin(qoz_ctx* c, hipStream_t s, int kind);
void prof_end(qoz_ctx* c, hipStream_t s, hipEvent_t a, int kind,
              double bytes);
void prof_collect(qoz_ctx* c);
/* the calling thread's open bracket (null events outside one) */
struct ProfSlot {
  hipEvent_t start = nullptr, stop = nullptr;
};
ProfSlot& prof_slot();
/* Every kernel launch of the library: hipLaunchKernelGGL's arguments. */
#define QOZ_LAUNCH(kernel, grid, block, lds, stream, ...)                  \
  do {                                                                     \
    ::qoz::ProfSlot& slot_ = ::qoz::prof_slot();                          \
    hipEvent_t start_ = slot_.start;                                       \
    slot_.start = nullptr;                                                 \
    hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, start_,        \
                          slot_.stop, 0, __VA_ARGS__);                     \
  } while (0)
qoz_status set_device(qoz_ctx* c);

/* ---- host planning (plan.cpp) --------------------------------------- */
bool shape_ok(const qoz_shape& sh, int* d, uint64_t n[3]);
Geo make_geo(int d, const uint64_t* n);
bool params_ok(const qoz_params& p, int d, uint32_t* L);
void level_bounds(double e, double alpha, double beta, uint32_t L,
                  double* eb, float* twoeb, float* inv);
qoz_status make_plan(const qoz_shape& sh, double e, const qoz_params& p,
                     Plan* plan);
/* key of a plan's sweep geometry for the tile tables */
std::vector<uint32_t> tile_key(const Plan& p);
/* target sub-grid of sweep j of level l over geometry g (grid dims) */
void sweep_grid(const Geo& g, const uint32_t* order_grid, int d, int j,
                uint32_t h, uint32_t* start, uint32_t* step, uint32_t* cnt);
/* n_packed: packed payload words of a format-5 stream, 0 for format 4 */
Layout layout_of(uint64_t n_anchor, uint64_t n_used, uint64_t n_chunks,
                 uint64_t n_unpred, uint64_t n_words, uint64_t n_packed = 0);
void write_header(uint8_t* h, const Plan& p, uint64_t n_unpred,
                  uint64_t n_used, uint64_t n_words);
qoz_status parse_header(const uint8_t* h, size_t in_bytes, bool need_all, Plan* plan,
                        uint64_t* n_unpred, uint64_t* n_used,
                        uint64_t* n_words, uint64_t* n_packed);
void fill_sweep_table(const Plan& p, SweepTable* t);
/* Level-1 row fusion: indices of sweeps A (SIZE_MAX if none) and B and the
 * job; false when the level has no sweep along the contiguous dimension or
 * its rows are too long for the row kernels. */
/* The fused level-1 sweeps of a plan: indices of F (SIZE_MAX when not
 * fused), A (SIZE_MAX when none) and B; false when there is no fusion. */
bool level1_rows(const Plan& P, size_t* iz, size_t* ia, size_t* ib,
                 RowJob* rj);

/* ---- batch workers (batch_host.cpp) ---------------------------------- */
/* at least n worker contexts (each with its own stream) on c's device */
qoz_status ensure_workers(qoz_ctx* c, uint32_t n);
/* fn(worker, item) over items in the given order on `workers` threads */
void run_on_workers(const std::vector<uint32_t>& order, uint32_t workers,
                    const std::function<void(uint32_t, uint32_t)>& fn);

/* ---- Huffman (host side, huffman_host.cpp) ---------------------------- */
bool huffman_lengths(const uint32_t* hist, uint32_t nsym, uint8_t* len);
/* Used symbols sorted on the device: keys (count << 16) | symbol in
 * ascending order; lengths per key, or the total code bits. */
constexpr uint32_t kSortCap = 4096;
constexpr uint32_t kSortCapBig = 16384; /* second pass, 128 KB of LDS */
bool huffman_lengths_sorted(const uint64_t* keys, uint32_t n, uint8_t* len);
uint64_t huffman_cost_sorted(const uint64_t* keys, uint32_t n);
/* The used symbols of a whole histogram as keys (count << 16) | symbol in
 * ascending order (radix passes over the count). */
void hist_keys_sorted(const uint32_t* hist, uint32_t nsym,
                      std::vector<uint64_t>* keys);
/* An upper bound on the payload words of any chunk of at most `chunk`
 * bins: the `chunk` longest code occurrences of the field (keys as above,
 * lens[i] the length of keys[i]'s symbol). */
uint32_t chunk_words_bound(const uint64_t* keys, const uint8_t* lens,
                           uint32_t n, uint32_t chunk);
/* Canonical codes for ascending symbols syms[0..n) with lengths lens. */
void canonical_codes_sparse(const uint16_t* syms, const uint8_t* lens,
                            uint32_t n, uint64_t* codes);
/* histograms ids[0..n) sorted with up to kSortCapBig used symbols each
 * (output stride kSortCapBig + 1); hist_sort_big_fits() first */
bool hist_sort_big_fits();
void launch_hist_sort_big(const uint32_t* hist, const uint32_t* ids,
                          uint32_t n, uint64_t* out, hipStream_t s);
void launch_hist_sort(const uint32_t* hist, uint32_t n_hist, uint64_t* out,
                      hipStream_t s);
void canonical_codes(const uint8_t* len, uint32_t nsym, uint64_t* code);
bool build_dec_tables(const uint16_t* syms, const uint8_t* lens,
                      uint32_t n_used, DecTables* t,
                      std::vector<uint32_t>* sorted_syms);
uint64_t huffman_cost(const uint32_t* hist, uint32_t nsym);
uint64_t huffman_cost_hist(const uint32_t* hist, uint32_t nsym);

/* ---- launchers (kernels_*.hip) -------------------------------------- */
void launch_init_status(uint32_t* status, hipStream_t s);
void launch_anchor_copy(const Geo& g, uint32_t stride, const uint32_t na[3],
                        const float* x, float* W, float* out, uint32_t* status,
                        hipStream_t s);
void launch_anchor_scatter(const Geo& g, uint32_t stride, const uint32_t na[3],
                           const float* in, float* W, hipStream_t s);
bool sweep_tile_ok(SweepTile t);
void launch_sweep_comp(const Geo& g, const Sweep& sw, const float* x,
                       float* W, uint16_t* codes, bool write_w,
                       uint32_t* status, hipStream_t s,
                       SweepTile t = SweepTile());
void launch_sweep_decomp(const Geo& g, const Sweep& sw, float* W,
                         const uint16_t* codes, hipStream_t s,
                         SweepTile t = SweepTile());
void launch_row_comp(const Geo& g, const RowJob& rj, const float* x, float* W,
                     uint16_t* codes, bool write_w, uint32_t* status,
                     hipStream_t s);
void launch_row_decomp(const Geo& g, const RowJob& rj, float* W,
                       const uint16_t* codes, hipStream_t s);
void launch_unpred_scatter(const Geo& g, const SweepTable& st,
                           const uint32_t* upos, const float* vals,
                           uint64_t n_unpred, uint64_t n_codes, float* W,
                           uint32_t* status, hipStream_t s);
void launch_hist(const uint16_t* codes, uint64_t n, uint32_t* hist,
                 hipStream_t s);
void launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s);
/* device-to-device copies of up to four regions (n <= 4) in one launch */
void launch_copy_regions(void* const* dst, const void* const* src,
                         const uint64_t* bytes, uint32_t n, hipStream_t s);
/* bytes from device memory to coherent host memory (to_host) or back */
void launch_copy_host(void* dst, const void* src, size_t bytes, bool to_host,
                      hipStream_t s);
/* scratch bytes launch_chunk_scan needs */
uint64_t chunk_scan_scratch(uint64_t n_chunks);
void launch_chunk_scan(const uint32_t* chunk_bits,
                       const uint32_t* chunk_zeros, uint64_t n_chunks,
                       uint64_t* coff, uint64_t* upre, uint64_t* totals,
                       uint64_t* scratch, hipStream_t s);
/* One field of an encoding (see kernels_huff.hip): its bins, chunks and
 * code table, the stream sections the encoder fills, its totals (payload
 * words, symbol-0 bins, packed words: zero on entry) and status word. */
struct EncField {
  const uint16_t* codes;
  Chunks ch;
  uint64_t nch;
  const uint64_t* tab; /* (code << 8) | length for symbols [lo, lo + tn) */
  int32_t lo;
  uint32_t tn;
  uint64_t zero_entry; /* symbol 0's entry */
  uint64_t* coff;
  uint32_t* upre;
  uint16_t* segs;
  uint32_t* payload;
  uint64_t cap_words;
  float* unpred;
  const float* x;
  Geo g;
  uint64_t* totals;
  uint32_t* status;
  uint32_t* pack_bits;
  SweepTable st;
};
/* A chunk's first bin and bin count, written by the count and read by the
 * encoder (one 16-byte scalar load instead of the level table's search). */
struct ChunkGeo {
  uint64_t begin;
  uint32_t n;
  uint32_t pad;
};
/* Code bits and symbol-0 bins of every chunk of fields[0..nf) (chunk0[f]:
 * the first chunk of field f in the global chunk order, chunk0[nf] the
 * total) into bits[] and zeros[] at global chunk indices; field f's
 * workgroups start at wg0[f] (count_workgroups(its chunks) of them),
 * wg0[nf] = total_wg. */
uint32_t count_workgroups(uint64_t n_chunks);
void launch_huff_count(const EncField* fields, const uint64_t* chunk0,
                       const uint32_t* wg0, uint32_t nf, uint32_t total_wg,
                       uint32_t* bits, uint32_t* zeros, ChunkGeo* geo,
                       hipStream_t s);
/* Chunks of every field, one workgroup per chunk at a time, as many
 * workgroups as the device holds at once taking chunks in a grid stride
 * over the global chunk order; gw and gz are the chunk scan's exclusive
 * prefixes of the counted words and symbol-0 bins (n_chunks + 1 each),
 * geo the count's chunk geometry; max_words bounds a chunk's payload
 * words, max_tn the fields' code table sizes (the LDS window), long_codes
 * selects the variant for codes longer than 32 bits. */
void launch_huff_encode(const EncField* fields, const uint64_t* chunk0,
                        const ChunkGeo* geo, const uint64_t* gw,
                        const uint64_t* gz, uint32_t nf, uint64_t n_chunks,
                        uint32_t max_words, uint32_t max_tn, bool long_codes,
                        hipStream_t s);
/* payload words a chunk can need with codes of at most max_len bits */
uint32_t encode_max_words(uint32_t max_len);
/* zero-word packing of the payload (stream format 5): pack_bits[c] from
 * the encoder is 32 x the chunk's packed word count, scanned into pcoff */
void launch_pack_write(const uint32_t* raw, const uint64_t* coff,
                       const uint64_t* pcoff, uint64_t n_chunks,
                       uint32_t* dst, hipStream_t s);
void launch_unpack(const uint32_t* src, uint64_t n_packed,
                   const uint64_t* coff, const uint64_t* pcoff,
                   uint64_t n_chunks, uint64_t n_words, uint32_t* raw,
                   uint32_t* status, hipStream_t s);
/* Work queues of the batched decompression: one entry per field (decode)
 * or per field and round (sweeps); entry j owns the launch's workgroups
 * [wg0[j], wg0[j + 1]). */
struct DecJob {
  const uint32_t* payload;
  uint64_t n_words;
  const uint64_t* coff;
  const uint32_t* upre;
  const uint16_t* segs;
  Chunks ch;
  uint64_t n_unpred;
  const DecTables* tabs;
  const uint32_t* syms;
  uint16_t* codes;
  uint32_t* upos;
  uint32_t* status;
};
struct SweepJob {
  Geo g;
  uint32_t rows;   /* 0: sweep s; 1: fused level-1 rows rj */
  uint32_t gx, gy; /* sweep grid (set by sweep_job_prepare) */
  Sweep s;
  RowJob rj;
  float* W;
  const uint16_t* codes;
};
/* one compression sweep (or fused level-1 row pair) of one field */
struct CompJob {
  Geo g;
  uint32_t rows;    /* 0: sweep s; 1: fused level-1 rows rj */
  uint32_t gx, gy;  /* sweep grid (set by comp_job_prepare) */
  uint32_t write_w; /* the reconstruction is read by later sweeps */
  Sweep s;
  RowJob rj;
  const float* x;
  float* W;
  uint16_t* codes;
  uint32_t* status;
};
/* the anchors of one field: into W and the anchor list out */
struct AnchorJob {
  Geo g;
  uint32_t stride, na[3];
  const float* x;
  float* W;
  float* out;
  uint32_t* status;
};
/* one histogram: bins codes[0..n) into hist[65536] (zero on entry) */
struct HistJob {
  const uint16_t* codes;
  uint64_t n;
  uint32_t* hist;
};
/* a device-to-device copy, or a zero fill when src is NULL */
struct DevCopy {
  const void* src;
  void* dst;
  uint64_t bytes;
};
/* anchors and unpredictable values of one stream */
struct ExactJob {
  Geo g;
  uint32_t stride, na[3];
  uint32_t wg_anchor; /* set by exact_job_workgroups */
  const float* anchors;
  const SweepTable* st; /* device copy */
  const uint32_t* upos;
  const float* vals;
  uint64_t n_unpred, n_codes;
  float* W;
  uint32_t* status;
};
/* a device-to-host copy; dst is the device address of pinned staging */
struct HostCopy {
  const void* src;
  void* dst;
  uint64_t bytes;
};
void launch_gather_host(const HostCopy* list, uint32_t n, hipStream_t s);
/* work queues of batched compression: each job owns the launch's
 * workgroups [wg0[j], wg0[j + 1]) */
uint32_t comp_job_prepare(CompJob* j, size_t* lds);
void launch_sweep_round_comp_q(const CompJob* jobs, const uint32_t* wg0,
                               uint32_t n_jobs, uint32_t total_wg, size_t lds,
                               hipStream_t s);
uint32_t anchor_job_workgroups(const AnchorJob& j);
void launch_anchor_q(const AnchorJob* jobs, const uint32_t* wg0,
                     uint32_t n_jobs, uint32_t total_wg, hipStream_t s);
uint32_t hist_job_workgroups(const HistJob& j);
void launch_hist_q(const HistJob* jobs, const uint32_t* wg0, uint32_t n_jobs,
                   uint32_t total_wg, hipStream_t s);
/* copies / zero fills list[0..n) (device memory), one workgroup each */
void launch_copy_list(const DevCopy* list, uint32_t n, hipStream_t s);
/* copies[0..n), an array inside the pinned staging whose dst fields hold
 * host addresses inside it, in one launch */
qoz_status gather_to_host(qoz_ctx* c, HostCopy* copies, uint32_t n,
                          hipStream_t s);
uint32_t exact_job_workgroups(ExactJob* j);
void launch_exact_q(const ExactJob* jobs, const uint32_t* wg0,
                    uint32_t n_jobs, uint32_t total_wg, hipStream_t s);
uint32_t decode_workgroups(uint64_t n_chunks);
void launch_huff_decode_q(const DecJob* jobs, const uint32_t* wg0,
                          uint32_t n_jobs, uint32_t total_wg, hipStream_t s);
/* workgroups of the job and its LDS bytes; sets its grid or rows per
 * workgroup */
uint32_t sweep_job_prepare(SweepJob* j, size_t* lds);
void launch_sweep_round_q(const SweepJob* jobs, const uint32_t* wg0,
                          uint32_t n_jobs, uint32_t total_wg, size_t lds,
                          hipStream_t s);
void launch_huff_decode(const uint32_t* payload, uint64_t n_words,
                        const uint64_t* coff, const uint32_t* upre,
                        const uint16_t* segs, const Chunks& chunks,
                        uint64_t n_unpred, const DecTables* tabs,
                        const uint32_t* syms, uint16_t* codes,
                        uint32_t* upos, uint32_t* status, hipStream_t s);
void launch_range(const float* x, uint64_t n, float* part_min,
                  float* part_max, uint32_t* status, uint32_t nparts,
                  hipStream_t s);
uint32_t range_parts(uint64_t n);
void launch_sse_max(const float* x, const float* y, uint64_t n,
                    double* part_sse, double* part_max, uint32_t nparts,
                    hipStream_t s);
uint32_t sse_parts(uint64_t n);
/* learned tuner: network shape and parameter blob offsets */
constexpr uint32_t kMlpFeat = QOZ_MLP_NFEAT;
constexpr uint32_t kMlpHidden = QOZ_MLP_HIDDEN;
constexpr uint32_t kMlpOut = QOZ_MLP_NOUT;
constexpr uint32_t kHeadInterp = 2, kHeadAlpha = 5, kHeadBeta = 4;
constexpr uint32_t kOffMu = 0;
constexpr uint32_t kOffSg = kOffMu + kMlpFeat;
constexpr uint32_t kOffW1 = kOffSg + kMlpFeat;
constexpr uint32_t kOffB1 = kOffW1 + kMlpHidden * kMlpFeat;
constexpr uint32_t kOffW2 = kOffB1 + kMlpHidden;
constexpr uint32_t kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr uint32_t kOffW3 = kOffB2 + kMlpHidden;
constexpr uint32_t kOffB3 = kOffW3 + kMlpOut * kMlpHidden;
constexpr uint32_t kMlpParams = kOffB3 + kMlpOut;
static_assert(kMlpParams == QOZ_MLP_NPARAM, "parameter blob size");
static_assert(kHeadInterp + kHeadAlpha + kHeadBeta == kMlpOut, "heads");
constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;
bool block_features_fit();
/* features of nb sampled 33^3 blocks into feat[nb][32] (aux: 3 floats per
 * block), their mean into mean[32], kStNonFinite into status[0] when a
 * sampled value is NaN or Inf */
/* One field of a batched feature extraction: its blocks' origins, the
 * per-block features and (min, max, flag) triples, the pooled features
 * and status word. */
struct FeatJob {
  const float* x;
  Geo g;
  const uint32_t* origins;
  uint32_t nb;
  double e;
  float* feat;
  float* aux;
  float* mean;
  uint32_t* status;
};
/* the 3D jobs' blocks (total3 workgroups, wg3 their prefix), the 2D jobs'
 * blocks, then the pooling of all n jobs (all: jobs3 then jobs2) */
void launch_block_features_q(const FeatJob* jobs3, const uint32_t* wg3,
                             uint32_t n3, uint32_t total3,
                             const FeatJob* jobs2, const uint32_t* wg2,
                             uint32_t n2, uint32_t total2,
                             const FeatJob* all, uint32_t n, hipStream_t s);
void launch_block_features(const float* x, const Geo& g,
                           const uint32_t* origins, uint32_t nb, double e,
                           float* feat, float* aux, float* mean,
                           uint32_t* status, hipStream_t s);
uint32_t mlp_tiles(uint32_t B);
bool mlp_fit();
void launch_mlp_forward(const float* P, const float* X, uint32_t B,
                        float* logits, hipStream_t s);
void launch_mlp_grad(const float* P, const float* X, const int32_t* labels,
                     const uint32_t* index, uint32_t n_rows, uint32_t B,
                     float* part, double* loss_part, hipStream_t s);
void launch_mlp_reduce(const float* part, uint32_t nw, float* grad, float* P,
                       float* m, float* v, float lr, float bc1, float bc2,
                       bool adam, const double* loss_part, uint32_t B,
                       double* loss, hipStream_t s);

/* lag-1 error autocorrelation (Eq. 4): pass-0 partials p0 hold sum e (one
 * double per part), pass-1 partials p1 the centred sum of squares and the
 * centred lagged sum (two per part) */
uint32_t ac_parts(uint64_t nrows, uint32_t len, uint64_t* rows_per_wg);
void launch_ac_field(const float* x, const float* y, uint64_t nrows,
                     uint32_t len, double* p0, double* p1, hipStream_t s);
void launch_ac_items(const float* xs, const float* wt, uint32_t ntrial,
                     uint32_t nb, uint32_t size, uint32_t len, double* p0,
                     double* p1, hipStream_t s);
/* AC from the summed centred moments: n points, p neighbour pairs */
inline double ac_from_sums(double ss, double lag, double n, double p) {
  const double var = ss / n;
  if (!(var > 0.0) || !(p > 0.0)) return 0.0;
  return (lag / p) / var;
}
/* SSIM sums over a batch of equally shaped fields */
struct SsimJob {
  uint32_t P, Rn, Cn;  /* field extents (2D: P = 1) */
  uint32_t wp, wr, wc; /* window extents */
  uint64_t field_stride; /* elements between batch items */
  uint32_t batch;        /* items; y item i is compared with x item i % x_mod */
  uint32_t x_mod;
  double c1, c2;
};
uint64_t ssim_parts(const SsimJob& j);
/* Device address of the fixed scratch array (kFixedScratchBytes) on device
 * `dev`, which must be the current device; looked up once per device. */
hipError_t fixed_scratch_addr(int dev, void** out);
/* false when the device cannot give the window ring its LDS */
bool launch_ssim(const SsimJob& j, const float* x, const float* y,
                 double* parts, hipStream_t s);

/* tuner kernels (kernels_tune.hip) */
struct BlockGeo {
  Geo g;             /* block grid */
  uint32_t size;     /* points per block */
  uint32_t nb;       /* blocks */
  uint32_t Lt;
  uint32_t d;
};
/* the sampled blocks into xs and a second copy into wc; kStNonFinite into
 * status[0] when a sampled value is NaN or Inf */
void launch_gather_blocks(const float* x, const Geo& g, const BlockGeo& bg,
                          const uint32_t* origins_dev, float* xs, float* wc,
                          uint32_t* status, hipStream_t s);
/* whether Algorithm 1's level-l working copies fit in LDS on the current
 * device (then no per-candidate copies in wt are made) */
bool alg1_in_lds(const BlockGeo& bg, uint32_t l);
/* the trials' per-level interpolation types and orders (desc[0..ntrial),
 * levels 1..Lt) from Algorithm 1's choices pick[l - 1] among the level's
 * candidates cand[(l - 1) * ncand ..] */
void launch_trial_fill(TrialDesc* desc, uint32_t ntrial, uint32_t Lt,
                       const TrialDesc* cand, uint32_t ncand,
                       const uint32_t* pick, hipStream_t s);
/* keep: a finer level follows and reads the chosen reconstruction (else
 * the in-LDS path keeps none of them) */
void launch_alg1_level(const BlockGeo& bg, uint32_t l, const float* xs,
                       const float* wc, float* wt, uint32_t ncand,
                       const TrialDesc* cand_desc, double* l1_part,
                       bool in_lds, bool keep, hipStream_t s);
/* the level's choice (first strict minimum) to *pick and, with keep, its
 * reconstruction committed to wc */
void launch_alg1_pick(const BlockGeo& bg, uint32_t l, const float* xs,
                      const TrialDesc* cand_desc, const double* l1_part,
                      uint32_t ncand, double count, uint32_t* pick,
                      const float* wt, float* wc, bool in_lds, bool keep,
                      hipStream_t s);
/* keep_wt: leave each trial's reconstruction of each block in wt */
void launch_trial(const BlockGeo& bg, const float* xs, float* wt,
                  uint32_t ntrial, const TrialDesc* desc, uint32_t* hist,
                  double* sse_part, uint32_t* unpred_part, bool keep_wt,
                  hipStream_t s);

}  // namespace qoz
#endif
