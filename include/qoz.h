/*
 * qoz.h -- C ABI of the MI355X (gfx950) QoZ library.
 *
 * QoZ (Liu, Di, Zhao, Liang, Chen, Cappello, "Dynamic Quality Metric Oriented
 * Error-bounded Lossy Compression for Scientific Datasets", SC22) compresses
 * a float32 field X under an absolute bound e: every decompressed value x'
 * satisfies |x - x'| <= e (Sec. III).  Prediction is a multi-level
 * interpolation over an anchor grid, with a per-level interpolator (linear or
 * cubic, and a dimension order) and per-level bounds
 * e_l = e / min(alpha^(l-1), beta) (Sec. V, Eq. 5); the bins are Huffman
 * coded (Sec. VI-A).  An online tuner picks the interpolators and
 * (alpha, beta) for a target metric by trial compression of sampled blocks
 * (Sec. VI, Algorithm 1, Table I).
 *
 * Conventions for every entry point:
 *  - Device pointers (d_*) are HIP device memory on the context's device;
 *    host pointers (h_*) are host memory.  The caller owns all of them; the
 *    library never frees or retains them beyond the call.
 *  - Work is enqueued on `stream` (0 = the null stream) and the call is
 *    synchronous: it returns after the stream has drained the work.
 *  - Return value is a qoz_status; nothing is thrown across the ABI.
 *    Out-parameters are written only on QOZ_OK, except *out_bytes on
 *    QOZ_ENOSPACE (the size needed).  On any error the contents of output
 *    buffers are unspecified.  qoz_last_error() gives a message for the
 *    calling thread's last failure.
 *  - A qoz_ctx owns the device scratch of one device and is not thread-safe;
 *    use one context per thread (or serialise calls).
 *  - Fields are float32, row-major with dims[0] slowest, ndim 2 or 3, every
 *    used dimension >= 2, fewer than 2^32 points; unused dims are ignored.
 */
#ifndef QOZ_H
#define QOZ_H
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QOZ_OK = 0,
  QOZ_EINVAL = 1,   /* bad argument: shape, e <= 0 or non-finite, alpha or
                       beta < 1, bad order, NaN/Inf in the input */
  QOZ_ENOSPACE = 2, /* output capacity too small (*out_bytes = needed) */
  QOZ_EFORMAT = 3,  /* malformed or truncated compressed stream */
  QOZ_EDEVICE = 4,  /* a HIP runtime error */
  QOZ_ENOMEM = 5    /* device or host allocation failed */
} qoz_status;

/* Quality target of the tuner (Sec. III): the ratio at the fixed bound,
 * PSNR (Eq. 1), SSIM (Eq. 2-3), or the lag-1 autocorrelation of the errors
 * (Eq. 4; the AC-preferred mode of Sec. VII), where the tuner prefers the
 * smallest |AC|. */
typedef enum {
  QOZ_TARGET_CR = 0,
  QOZ_TARGET_PSNR = 1,
  QOZ_TARGET_SSIM = 2,
  QOZ_TARGET_AC = 3
} qoz_target;

typedef struct {
  uint32_t ndim;    /* 2 or 3 */
  uint64_t dims[3]; /* dims[0] slowest */
} qoz_shape;

#define QOZ_MAX_LEVELS 16

/* Parameter set theta (Sec. III, Sec. V-B, Eq. 5). */
typedef struct {
  uint32_t anchor_stride; /* s: power of two >= 2; 0 -> 64 (2D), 32 (3D)
                             (the paper's settings, Sec. VII-A) */
  uint32_t levels;        /* log2(s); written by the library */
  uint8_t interp[QOZ_MAX_LEVELS];   /* [l-1]: 0 linear, 1 cubic */
  uint8_t order[QOZ_MAX_LEVELS][3]; /* [l-1]: permutation of 0..ndim-1,
                                       the dimension swept first first */
  double alpha, beta;               /* >= 1 */
} qoz_params;

/* Tuner configuration (Sec. VI-A, VI-B); zero fields take the defaults. */
typedef struct {
  uint32_t block;         /* b: power of two; 0 -> 64 (2D), 16 (3D) */
  uint32_t sample_stride; /* S; 0 -> round(b * r^(-1/ndim)) */
  double sample_rate;     /* r in (0,1]; 0 -> 0.01 (2D), 0.005 (3D) */
  uint32_t all_orders;    /* 0: increasing and decreasing dimension orders
                             (Sec. VI-B); 1: all ndim! orders */
  uint32_t ssim_window;   /* 0 -> 7 */
  uint32_t ablation;      /* QOZ_ABLATE_* switches; 0 = the whole method */
} qoz_tune_config;

/* Ablation switches (the component study of Sec. VII), each leaving one
 * part of the tuner out.  QOZ_ABLATE_AB: no (alpha, beta) search, alpha = 1
 * (every level at the bound).  QOZ_ABLATE_LEVELWISE: instead of Algorithm 1,
 * one interpolator (type and dimension order) for every level, the
 * candidate whose trial compression of the sampled blocks at the uniform
 * bound has the lowest bit rate.  The anchor-less level structure is an
 * anchor stride of the next power of two >= the largest dimension. */
#define QOZ_ABLATE_AB 1u
#define QOZ_ABLATE_LEVELWISE 2u

typedef struct qoz_ctx qoz_ctx;

/* Context of the compressor C, decompressor D and tuner of Sec. III: the
 * device scratch that their steps (the level sweeps of Sec. V-B, the
 * Huffman stage of Sec. VI-A, the sampled-block trials of Sec. VI) reuse
 * from call to call, grown on first use and freed by qoz_ctx_destroy.  The
 * paper's single-core compressor has no counterpart; the context only
 * holds memory and never changes a result.  Create one on HIP device
 * `hip_device`; *out receives it.  Errors: EINVAL (NULL out, bad device),
 * EDEVICE, ENOMEM.  qoz_ctx_destroy(NULL) does nothing; destroying frees
 * every allocation of the context (and its batch workers). */
qoz_status qoz_ctx_create(int hip_device, qoz_ctx** out);
void qoz_ctx_destroy(qoz_ctx* ctx);

/* Worst-case size in bytes of a compressed stream Z (Sec. III) of this
 * shape, for any parameters and bound: the fixed header, the anchor grid
 * of Sec. V-B stored raw, the largest codebook of the bins, the per-chunk
 * tables, a Huffman payload (Sec. VI-A) of at most 16 bits per bin (an
 * optimal prefix code is never longer in total than the fixed 16-bit
 * code of the 65536 bins) plus one word of padding per chunk, and every
 * non-anchor value unpredictable (raw float32).  *bytes receives it.
 * Errors: EINVAL (bad shape, NULL bytes). */
qoz_status qoz_compress_bound(qoz_shape shape, size_t* bytes);

/* Online tuning (Sec. VI): sample blocks of d_x, choose per-level
 * interpolators by mean L1 prediction error (Algorithm 1), then (alpha,
 * beta) by the rate-quality comparison of Table I for `target` at bound
 * abs_eb.  On input out->anchor_stride selects s (0 = default); on QOZ_OK
 * *out holds the tuned parameters.  cfg may be NULL (defaults).
 * Errors: EINVAL (shape, bound, target, cfg, non-finite input), EDEVICE,
 * ENOMEM. */
qoz_status qoz_tune(qoz_ctx* ctx, const float* d_x, qoz_shape shape,
                    double abs_eb, qoz_target target,
                    const qoz_tune_config* cfg, qoz_params* out,
                    hipStream_t stream);

/* Record of one tuning, for checking the tuner's intermediate values
 * (Algorithm 1 of Sec. VI-B; the (alpha, beta) walk of Sec. VI-C, Table I).
 * alg1_err[l-1][c]: mean absolute prediction error of interpolator
 * candidate c (interpolation type outer, dimension order inner) on level l
 * of the sampled blocks at the uniform bound; alg1_choice[l-1]: the first
 * strict minimum.  Under QOZ_ABLATE_LEVELWISE, alg1_err[0][c] is candidate
 * c's trial bit rate over every level and every alg1_choice[l-1] (l <= Lt)
 * the one chosen.  Pair i is (alpha, beta) = ({1, 1.25, 1.5, 1.75, 2}[i/4],
 * {1.5, 2, 3, 4}[i%4]); B[i] its trial bit rate (Huffman bits of the bins
 * aggregated over the blocks plus 32 per unpredictable value, per block
 * point) and M[i] its metric (PSNR, SSIM, -|AC|; 0 for the ratio target)
 * at bound e; where the walk re-ran pair i at e' = eprime[i] * e (Table I
 * cases 3 and 4), Bp[i] and Mp[i] (else NaN, eprime 0); cmp_case[i] the
 * Table-I case when pair i (i >= 1) challenged the incumbent; best_pair
 * the pair chosen.  Under QOZ_ABLATE_AB no pair is tried and the pair
 * fields stay 0. */
#define QOZ_MAX_CAND 12
#define QOZ_NPAIRS 20
typedef struct {
  uint32_t Lt;           /* levels covered by the sampled blocks */
  uint32_t ncand;        /* interpolator candidates per level */
  uint64_t nblocks;      /* sampled blocks */
  uint64_t block_points; /* points in all sampled blocks */
  double alg1_err[QOZ_MAX_LEVELS][QOZ_MAX_CAND];
  uint32_t alg1_choice[QOZ_MAX_LEVELS];
  double B[QOZ_NPAIRS], M[QOZ_NPAIRS];
  double Bp[QOZ_NPAIRS], Mp[QOZ_NPAIRS];
  double eprime[QOZ_NPAIRS];
  int32_t cmp_case[QOZ_NPAIRS];
  uint32_t best_pair;
} qoz_tune_trace;

/* qoz_tune that also fills *trace (not NULL).  Same decisions and errors
 * as qoz_tune; the per-level error sums of Algorithm 1 are read back, one
 * small copy per level. */
qoz_status qoz_tune_traced(qoz_ctx* ctx, const float* d_x, qoz_shape shape,
                           double abs_eb, qoz_target target,
                           const qoz_tune_config* cfg, qoz_params* out,
                           qoz_tune_trace* trace, hipStream_t stream);

/* Compression Z = C_theta(X) (Sec. III) into d_out[0..cap).  params == NULL
 * runs qoz_tune(target, cfg) first.  On QOZ_OK *out_bytes is the stream
 * size; on QOZ_ENOSPACE it is the size needed.  The stream is
 * self-describing (shape, bound and parameters are in its header).
 * Errors: EINVAL, ENOSPACE, EDEVICE, ENOMEM. */
qoz_status qoz_compress(qoz_ctx* ctx, const float* d_x, qoz_shape shape,
                        double abs_eb, const qoz_params* params,
                        qoz_target target, const qoz_tune_config* cfg,
                        void* d_out, size_t cap, size_t* out_bytes,
                        hipStream_t stream);

/* Decompression X' = D_theta(Z) (Sec. III) of d_in[0..in_bytes) into
 * d_y (capacity y_cap_elems floats).  *out_shape (may be NULL) receives the
 * shape.  Errors: EFORMAT (bad stream), ENOSPACE (y too small), EDEVICE,
 * ENOMEM. */
qoz_status qoz_decompress(qoz_ctx* ctx, const void* d_in, size_t in_bytes,
                          float* d_y, size_t y_cap_elems,
                          qoz_shape* out_shape, hipStream_t stream);

/* Read the self-describing header of a stream Z held in host memory: the
 * field's shape, the absolute bound e and the parameter set theta of
 * Sec. III (anchor stride and levels, per-level interpolation type and
 * dimension order of Sec. V-B, alpha and beta of Eq. 5).  h_in[0..in_bytes)
 * is only read.  Any output may be NULL.  Errors: EFORMAT (too short, bad
 * magic or version, inconsistent counts). */
qoz_status qoz_inspect(const void* h_in, size_t in_bytes, qoz_shape* shape,
                       double* abs_eb, qoz_params* params);

/* Quality of d_y against d_x (Sec. III): PSNR (Eq. 1) with
 * vrange = max(X) - min(X); mean SSIM (Eq. 2-3) over all ssim_window^ndim
 * windows inside the field (0 -> 7; a dimension shorter than the window
 * uses its length); maximum absolute error.  Sums in FP64.  Any output may
 * be NULL.  Errors: EINVAL, EDEVICE, ENOMEM. */
qoz_status qoz_metrics(qoz_ctx* ctx, const float* d_x, const float* d_y,
                       qoz_shape shape, uint32_t ssim_window, double* psnr,
                       double* ssim, double* max_abs_err, hipStream_t stream);

/* qoz_metrics for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments and results, bit for bit, but no device or host allocation.
 * Its device scratch is one fixed array of 4 MiB per device, held from
 * the library's load until the process ends, whose address qoz_ctx_create
 * looks up; the host side uses the context's pinned staging buffer, which
 * qoz_ctx_create allocated.  The SSIM pass needs one partial sum per 64 x 4
 * window origins of a row plane per slab of 32 planes; a shape needing
 * more than (4 MiB - 64 KiB) / 8 = 516096 of them (3D fields up to about
 * 4e9 points fit, e.g. 1600^3; 2D fields up to about 1.3e8 points) is
 * rejected with EINVAL before any launch.  Every call on one device shares
 * the array and it keeps the last call's contents (each call initialises
 * what it reads): calls that overlap on one device (on any stream, from
 * any context) race, so callers serialise them.
 * Errors: EINVAL, EDEVICE. */
qoz_status qoz_metrics_noalloc(qoz_ctx* ctx, const float* d_x,
                               const float* d_y, qoz_shape shape,
                               uint32_t ssim_window, double* psnr,
                               double* ssim, double* max_abs_err,
                               hipStream_t stream);

/* Lag-1 autocorrelation of the errors e = d_x - d_y (Eq. 4) along the
 * fastest (last) dimension: the mean and population variance of e over all
 * points, the lagged moment over every pair of neighbours in a row; 0 when
 * the errors are constant.  Sums in FP64.  Errors: EINVAL, EDEVICE,
 * ENOMEM. */
qoz_status qoz_error_ac(qoz_ctx* ctx, const float* d_x, const float* d_y,
                        qoz_shape shape, double* ac, hipStream_t stream);

/* Tile autotuning of the interpolation sweeps: for the plan of `shape`
 * and `params` (anchor stride, levels, orders), times every sweep of
 * compression and decompression on scratch data with each candidate
 * launch tile (rows per workgroup 1..16, rows per lane 1..4) and keeps the
 * fastest per sweep in ctx; later qoz_compress / qoz_decompress calls with
 * the same sweep geometry use them (results are the same for any tile).
 * *n_sweeps (may be NULL) receives the number of sweeps tuned;
 * *ms_default and *ms_tuned (may be NULL) the summed time of those sweeps,
 * compression and decompression, with the default tile (4 rows per
 * workgroup, 1 per lane) and with the chosen ones (each the fastest of its
 * repetitions).  Synchronous.  Errors: EINVAL, EDEVICE, ENOMEM. */
qoz_status qoz_autotune_tiles(qoz_ctx* ctx, qoz_shape shape,
                              const qoz_params* params, uint32_t* n_sweeps,
                              float* ms_default, float* ms_tuned,
                              hipStream_t stream);

/* ---- Batches -------------------------------------------------------------
 * Many fields of uneven shapes and bounds in one call.  Worker threads,
 * each with a context and stream of its own (created on first use, kept
 * with ctx), take fields from a shared queue, largest first, so one
 * field's host steps (Huffman code, tuner decisions) overlap other fields'
 * kernels.  Every field's result is the single-field call's, byte for
 * byte.  The call first waits for `stream` (inputs written there are
 * ready) and returns when every output is complete.  Different items must
 * not share outputs. */
typedef struct {
  const float* d_x;          /* in: field (device) */
  qoz_shape shape;           /* in */
  double abs_eb;             /* in */
  const qoz_params* params;  /* in: NULL = tune with the batch's target */
  void* d_out;               /* in: stream buffer (device) */
  size_t cap;                /* in: its capacity in bytes */
  size_t out_bytes;          /* out: stream size (or size needed) */
  qoz_status status;         /* out: the field's own status */
  double ms;                 /* out: wall time of the field's call */
  double done_ms;            /* out: completion time after the batch start */
} qoz_batch_item;

/* Compression of items[0..n): as qoz_compress for each (target and cfg
 * apply to items without params).  workers: threads (0 = 4; at most 64).
 * Returns QOZ_OK when every item succeeded, else the status of the first
 * failing item in index order (each item keeps its own status).
 * Errors: EINVAL (arguments), EDEVICE, ENOMEM, or an item's status. */
qoz_status qoz_compress_batch(qoz_ctx* ctx, qoz_batch_item* items, uint32_t n,
                              qoz_target target, const qoz_tune_config* cfg,
                              uint32_t workers, hipStream_t stream);

typedef struct {
  const void* d_in;   /* in: stream (device) */
  size_t in_bytes;    /* in */
  float* d_y;         /* in: output field (device) */
  size_t y_cap_elems; /* in */
  qoz_shape shape;    /* out */
  qoz_status status;  /* out */
  double ms;          /* out */
  double done_ms;     /* out */
} qoz_batch_dec_item;

/* Decompression of items[0..n): as qoz_decompress for each; workers and
 * status as qoz_compress_batch. */
qoz_status qoz_decompress_batch(qoz_ctx* ctx, qoz_batch_dec_item* items,
                                uint32_t n, uint32_t workers,
                                hipStream_t stream);

/* Decompression of items[0..n) (at most 16384) on `stream` through device
 * work queues, in a number of launches that does not grow with n: the
 * headers and codebooks of all streams are read back together, one launch
 * decodes every stream's Huffman chunks, and each round of inverse sweeps
 * (the r-th sweep, or fused level-1 row pair, of every stream) is one
 * launch, as is the placing of every stream's exact values (anchors,
 * unpredictable bins); a workgroup finds its stream from the queue's
 * running count of workgroups.  A packed payload takes one more launch of
 * its own.  Outputs equal qoz_decompress's bit for
 * bit; sweeps use the default launch tiles.  Items must not share
 * outputs.  ms and done_ms of every item are the call's duration.  Returns
 * as qoz_compress_batch; a stream that fails its checks leaves the others
 * decoded.  Scratch: the field's codes, unpredictable positions and (when
 * packed) the expanded payload of every stream at once, kept in ctx.
 * Errors: EINVAL, EDEVICE, ENOMEM, or an item's status. */
qoz_status qoz_decompress_queue(qoz_ctx* ctx, qoz_batch_dec_item* items,
                                uint32_t n, hipStream_t stream);

/* Compression of items[0..n) (at most 16384) on `stream` through device
 * work queues, in a number of launches that does not grow with n: one
 * launch places every field's anchors, each round of sweeps (the r-th
 * sweep, or fused level-1 row pair, of every field; Sec. V-B) is one
 * launch, one launch counts every field's bins and one sorts the used
 * bins of every histogram; the Huffman codes (Sec. VI-A) are built on host
 * threads; one launch fills every field's sections before its payload,
 * one counts the code bits of every chunk of every field, one scan (two
 * launches) turns the counts into chunk offsets and one encoding launch
 * codes the chunks of every field.  Three waits per call (four when a
 * field uses more than 4096 distinct bins), plus the few launches of each
 * field whose zero-word packing pays.  Items without params are
 * tuned with the online tuner (target, cfg) on up to 8 worker contexts of
 * ctx, each with its own stream (the call first waits for `stream`, whose
 * work may produce the inputs), largest first; meanwhile the calling
 * thread compresses, as the steps above, the fields tuned so far each time
 * a round of tunings (as many as workers) has ended.  Every
 * stream equals qoz_compress's byte for byte; sweeps use the default
 * launch tiles.  A field whose output cannot hold the sections before its
 * payload is compressed by qoz_compress after the queue (and reports the
 * size needed).  ms of every item is the call's duration; done_ms is when
 * its group ended (the call's duration when nothing is tuned).
 * Returns as qoz_compress_batch.  Scratch: every field's reconstruction,
 * bins and histogram at once, kept in ctx.
 * Errors: EINVAL, EDEVICE, ENOMEM, or an item's status. */
qoz_status qoz_compress_queue(qoz_ctx* ctx, qoz_batch_item* items, uint32_t n,
                              qoz_target target, const qoz_tune_config* cfg,
                              hipStream_t stream);

/* With enable != 0, qoz_decompress_queue keeps its device work (upload,
 * launches, status read-back) as a HIP graph: a call whose launch
 * signature (grids, queue layout, scratch addresses, packed payloads)
 * equals the previous call's captures it once on an internal stream, and
 * later calls with that signature launch the graph on their stream.  In
 * practice that is the same batch layout again (equal shapes, codebook
 * sizes and packing).  Off by default; turning it off frees the graph.
 * Errors: EINVAL, EDEVICE. */
qoz_status qoz_ctx_set_queue_graphs(qoz_ctx* ctx, int enable);

/* ---- Learned tuner ------------------------------------------------------
 * A stand-in for the trial search of Sec. VI: a small network maps
 * features of the sampled blocks to the search's choices (one interpolation
 * type for every level, alpha and beta of Eq. 5), with the search itself as
 * the fallback when the network is unsure.
 *
 * Parameters are one float32 blob of QOZ_MLP_NPARAM entries: input shift
 * mu[32] and scale sg[32] (x = (f - mu) / sg, not trained), then W1[128][32],
 * b1[128], W2[128][128], b2[128], W3[11][128], b3[11] (row-major, output
 * index first).  Outputs 0-1 score linear / cubic, 2-6 alpha in {1, 1.25,
 * 1.5, 1.75, 2}, 7-10 beta in {1.5, 2, 3, 4}.  Products take bfloat16
 * operands (round to nearest even) with FP32 accumulation; the loss is the
 * batch mean of the three heads' summed softmax cross-entropies.  Every
 * d_params passed below must be 16-byte aligned (EINVAL otherwise). */
#define QOZ_MLP_NFEAT 32
#define QOZ_MLP_HIDDEN 128
#define QOZ_MLP_NOUT 11
#define QOZ_MLP_NPARAM 22219

/* Features of a 2D or 3D field for the learned tuner: the blocks of
 * b = 32 (33^d points) sampled as in Sec. VI-A at cfg's rate and stride
 * (rate 0 -> 0.01; stride 0 -> round(32 rate^(-1/d)); cfg->block is
 * ignored), 32 float32 features each (level-wise linear / cubic residual
 * statistics of the original values along each dimension, deciles of the
 * squared forward-difference gradient, the block's value range and the
 * range over all sampled blocks, all relative to abs_eb), and their mean
 * over the blocks into d_mean[32].  Only the sampled blocks are read.
 * d_block (may be NULL) receives the per-block rows, *nblocks (may be
 * NULL) their count; with d_block non-NULL, block_cap is its capacity in
 * rows.  Every dimension must be >= 33.  Errors: EINVAL (shape, bound,
 * cfg, NaN or Inf in a sampled block, block_cap too small), EDEVICE,
 * ENOMEM. */
qoz_status qoz_learned_features(qoz_ctx* ctx, const float* d_x,
                                qoz_shape shape, double abs_eb,
                                const qoz_tune_config* cfg, float* d_mean,
                                float* d_block, uint64_t block_cap,
                                uint64_t* nblocks, hipStream_t stream);

/* Logits d_logits[batch][11] of feature rows d_feat[batch][32].
 * Asynchronous on `stream`.  Errors: EINVAL, EDEVICE, ENOMEM. */
qoz_status qoz_mlp_forward(qoz_ctx* ctx, const float* d_params,
                           const float* d_feat, uint32_t batch,
                           float* d_logits, hipStream_t stream);

/* Gradient of the batch loss with respect to every blob entry (0 for mu
 * and sg) into d_grad[QOZ_MLP_NPARAM] and the loss into *d_loss (device
 * double).  The batch is rows d_index[0..batch) of d_feat[n_rows][32] and
 * d_labels[n_rows][3] (interpolation, alpha index, beta index), or rows
 * 0..batch-1 when d_index is NULL; rows >= n_rows contribute nothing (the
 * mean still divides by batch) and labels outside their head's range are
 * clamped into it.  d_index must hold batch entries.  Asynchronous.
 * Errors: EINVAL, EDEVICE, ENOMEM. */
qoz_status qoz_mlp_grad(qoz_ctx* ctx, const float* d_params,
                        const float* d_feat, const int32_t* d_labels,
                        const uint32_t* d_index, uint32_t n_rows,
                        uint32_t batch, float* d_grad, double* d_loss,
                        hipStream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected at step
 * t >= 1) of learning rate lr on the trained entries of d_params, with the
 * moment blobs d_m and d_v (same layout; start at zero), on the batch as in
 * qoz_mlp_grad.  d_loss (device double, may be NULL) receives the loss
 * before the step.  Asynchronous.  Errors: EINVAL, EDEVICE, ENOMEM. */
qoz_status qoz_mlp_train_step(qoz_ctx* ctx, float* d_params, float* d_m,
                              float* d_v, const float* d_feat,
                              const int32_t* d_labels, const uint32_t* d_index,
                              uint32_t n_rows, uint32_t batch, float lr,
                              uint32_t t, double* d_loss, hipStream_t stream);

/* Learned tuning: features of d_x, one forward pass of the network
 * d_params (trained on fields of d_x's dimensionality), and per head the
 * class of highest score.  When the smallest of the three heads' softmax
 * probabilities is below min_confidence, or a dimension is below 33, the
 * online tuner (qoz_tune with `fallback_target` and cfg) decides instead
 * and *used_fallback (may be NULL) is set to 1, else 0.  The network's
 * parameters use every level's interpolation type from its first head and
 * the identity dimension order.  On input out->anchor_stride selects s.
 * The network path reads only the sampled blocks (NaN or Inf elsewhere is
 * left to qoz_compress to reject).  Errors: as qoz_tune. */
qoz_status qoz_tune_learned(qoz_ctx* ctx, const float* d_x, qoz_shape shape,
                            double abs_eb, const float* d_params,
                            double min_confidence, qoz_target fallback_target,
                            const qoz_tune_config* cfg, qoz_params* out,
                            int* used_fallback, hipStream_t stream);

/* Learned tuning of many fields: the features of every supported field
 * (every dimension >= 33; a 2D field only when d_params_2d, the network
 * for 2D fields, is not NULL), one forward pass per network (d_params for
 * the 3D fields) over all of them, then the online tuner, one field at a
 * time in item order, for the fields that are unsupported or below
 * min_confidence.  Each item's params and used_fallback equal what
 * qoz_tune_learned gives for it alone with its network.
 * params.anchor_stride is read on input (0 = default).  Synchronous.
 * Returns QOZ_OK when every item succeeded, else the status of the first
 * failing item in index order (each item keeps its own).
 * Errors: EINVAL, EDEVICE, ENOMEM, or an item's status. */
typedef struct {
  const float* d_x;   /* in: field (device) */
  qoz_shape shape;    /* in */
  double abs_eb;      /* in */
  qoz_params params;  /* in: anchor_stride; out: parameters */
  int used_fallback;  /* out */
  qoz_status status;  /* out */
} qoz_learned_item;

qoz_status qoz_tune_learned_batch(qoz_ctx* ctx, qoz_learned_item* items,
                                  uint32_t n, const float* d_params,
                                  const float* d_params_2d,
                                  double min_confidence,
                                  qoz_target fallback_target,
                                  const qoz_tune_config* cfg,
                                  hipStream_t stream);

/* Message describing the calling thread's last failed call ("" if none);
 * the text is owned by the library and stays valid until the thread's next
 * call into it.  It states which check of the entry point failed (a bound
 * of Sec. III, a shape rule, a stream check, a HIP error). */
const char* qoz_last_error(void);

/* ---- instrumentation ----------------------------------------------------
 * With timing on, the library brackets its kernel launches with HIP events
 * on the call's stream and accumulates, per kernel kind, the launch count,
 * the summed duration and the algorithmic bytes those launches must move
 * (inputs read once plus outputs written once).  Kinds are numbered
 * 0..qoz_prof_kinds()-1 and named by qoz_prof_name().  Errors: EINVAL. */
qoz_status qoz_ctx_set_timing(qoz_ctx* ctx, int on);
/* Time only the kinds whose bit is set (bit k = kind k); timing every
 * launch adds a pair of event records per kernel to the caller's host
 * time, so a benchmark can time just the kinds it reports. */
qoz_status qoz_ctx_set_timing_mask(qoz_ctx* ctx, uint64_t mask);
qoz_status qoz_ctx_reset_timing(qoz_ctx* ctx);
int qoz_prof_kinds(void);
const char* qoz_prof_name(int kind);
qoz_status qoz_ctx_get_timing(qoz_ctx* ctx, int kind, uint64_t* launches,
                              double* total_ms, double* algo_bytes);

#ifdef __cplusplus
}
#endif
#endif
