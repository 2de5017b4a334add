/*
 * qoz_ref.h -- C ABI of the CPU oracle for the QoZ hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded CPU
 * implementation of what the QoZ predictor, quantizer, entropy stage and
 * online tuner compute (Liu et al., "Dynamic Quality Metric Oriented
 * Error-bounded Lossy Compression for Scientific Datasets", SC22).  It exists
 * to check the GPU library.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product never does.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * All functions take host pointers and return one of the QREF_* codes.
 * Out-parameters are written only on QREF_OK (and *needed on QREF_ENOSPACE).
 */
#ifndef QOZ_REF_H
#define QOZ_REF_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  QREF_OK = 0,
  QREF_EINVAL = 1,   /* bad argument, non-finite input */
  QREF_ENOSPACE = 2, /* output capacity too small */
  QREF_EFORMAT = 3   /* malformed compressed stream */
};

enum {
  QREF_TARGET_CR = 0,
  QREF_TARGET_PSNR = 1,
  QREF_TARGET_SSIM = 2,
  QREF_TARGET_AC = 3 /* lag-1 error autocorrelation (Eq. 4) */
};

#define QREF_MAX_LEVELS 16
#define QREF_RADIUS 32768
#define QREF_CHUNK 4096 /* level-1 chunk; coarser levels halve it */
#define QREF_SEG 512 /* bins per segment: a chunk holds 8 */
#define QREF_MAX_CAND 12
#define QREF_NPAIRS 20

/* float32 field, row-major, dims[0] slowest; ndim 2 or 3; unused dims = 1 */
typedef struct {
  uint32_t ndim;
  uint64_t dims[3];
} qref_shape;

/* Parameter set theta (Sec. III): per-level interpolator (type and dimension
 * order, Sec. V-B) and the level-bound factors alpha, beta (Eq. 5). */
typedef struct {
  uint32_t anchor_stride; /* s, power of two; 0 -> 64 (2D) / 32 (3D) */
  uint32_t levels;        /* log2(s); written by the oracle */
  uint8_t interp[QREF_MAX_LEVELS];   /* [l-1]: 0 linear, 1 cubic */
  uint8_t order[QREF_MAX_LEVELS][3]; /* [l-1]: permutation of 0..ndim-1 */
  double alpha, beta;                /* >= 1 */
} qref_params;

/* Sampling and candidate configuration of the online tuner (Sec. VI). */
typedef struct {
  uint32_t block;         /* b, power of two; 0 -> 64 (2D) / 16 (3D) */
  uint32_t sample_stride; /* S; 0 -> round(b * r^(-1/d)) */
  double sample_rate;     /* r; 0 -> 0.01 (2D) / 0.005 (3D) */
  uint32_t all_orders;    /* 0: increasing + decreasing orders; 1: all d! */
  uint32_t ssim_window;   /* 0 -> 7 */
  uint32_t ablation;      /* QREF_ABLATE_* switches (ablation of Sec. VII) */
} qref_tune_config;

/* Ablation switches: components of the method left out one at a time. */
#define QREF_ABLATE_AB 1u        /* no (alpha, beta) search: alpha = 1 */
#define QREF_ABLATE_LEVELWISE 2u /* one interpolator for every level */

/* Record of one tuner run, for tests. */
typedef struct {
  uint32_t Lt;            /* highest level covered by the sampled blocks */
  uint32_t ncand;         /* interpolator candidates per level */
  uint64_t nblocks;       /* sampled blocks */
  uint64_t block_points;  /* points in all sampled blocks */
  double alg1_err[QREF_MAX_LEVELS][QREF_MAX_CAND]; /* [l-1][cand] mean L1 */
  uint32_t alg1_choice[QREF_MAX_LEVELS];           /* [l-1] winning cand */
  double B[QREF_NPAIRS], M[QREF_NPAIRS];   /* (bit rate, metric) at e */
  double Bp[QREF_NPAIRS], Mp[QREF_NPAIRS]; /* at e' (NaN if not run) */
  double eprime[QREF_NPAIRS];              /* factor of e' (0 if none) */
  int32_t cmp_case[QREF_NPAIRS]; /* Table-I case when pair i challenged */
  uint32_t best_pair;            /* index alpha_i*4 + beta_j */
} qref_tune_trace;

/* Result of one trial compression over the sampled blocks. */
typedef struct {
  uint64_t payload_bits; /* Huffman bits of the aggregated bins */
  uint64_t n_unpred;
  uint64_t n_points; /* points in all blocks (corners included) */
  uint64_t n_codes;
  double sse;        /* sum of squared errors over all block points */
  double ssim_sum;   /* sum of window SSIMs over windows inside blocks */
  uint64_t n_windows;
  double B;          /* (payload_bits + 32 * n_unpred) / n_points */
  double ac;         /* lag-1 error autocorrelation over the blocks' rows */
} qref_trial_result;

/* ---- level plan (Eq. 5) ------------------------------------------------ */
int qref_level_bounds(double e, double alpha, double beta, uint32_t L,
                      double* e_l, float* twoeb, float* inv);

/* ---- prediction + quantization stage only (Sec. V) --------------------- */
/* codes[n_codes] in stream order; recon[N] the reconstructed field;
 * unpred[n_unpred] in stream order; anchors[n_anchor] row-major.
 * Capacities: codes, unpred >= N; anchors >= N. */
int qref_predict_quantize(const float* x, qref_shape shape, double e,
                          const qref_params* params, int32_t* codes,
                          float* recon, float* unpred, float* anchors,
                          uint64_t* n_codes, uint64_t* n_unpred,
                          uint64_t* n_anchor);
/* Inverse of the stage above. */
int qref_reconstruct(const int32_t* codes, uint64_t n_codes,
                     const float* unpred, uint64_t n_unpred,
                     const float* anchors, uint64_t n_anchor,
                     qref_shape shape, double e, const qref_params* params,
                     float* y);
/* Stream-order trace: flat index, prediction (before quantization) and bin
 * of every target; arrays of capacity N. */
int qref_target_trace(const float* x, qref_shape shape, double e,
                      const qref_params* params, uint32_t* idx, float* pred,
                      int32_t* codes, uint64_t* n_codes);
/* Single stencil evaluation along one line (for isolated tests).
 * a,b,c,d = values at -3h,-h,+h,+3h; has_a/has_c/has_d flags. */
float qref_stencil(int cubic, float a, float b, float c, float d, int has_a,
                   int has_c, int has_d);

/* ---- entropy stage (canonical Huffman) --------------------------------- */
int qref_huffman_lengths(const uint64_t* hist, uint32_t nsym, uint8_t* len);
int qref_huffman_codes(const uint8_t* len, uint32_t nsym, uint64_t* code);

/* ---- full stream -------------------------------------------------------- */
int qref_compress_bound(qref_shape shape, uint32_t anchor_stride,
                        size_t* bytes);
/* params == NULL -> qref_tune(target, cfg) first. */
int qref_compress(const float* x, qref_shape shape, double e,
                  const qref_params* params, int target,
                  const qref_tune_config* cfg, void* out, size_t cap,
                  size_t* out_bytes);
int qref_decompress(const void* in, size_t in_bytes, float* y,
                    size_t y_cap_elems, qref_shape* out_shape);
int qref_inspect(const void* in, size_t in_bytes, qref_shape* shape,
                 double* e, qref_params* params);

/* ---- quality metrics (Eq. 1-3) ----------------------------------------- */
int qref_metrics(const float* x, const float* y, qref_shape shape,
                 uint32_t ssim_window, double* psnr, double* ssim,
                 double* max_abs_err);
/* Lag-1 autocorrelation of the errors x - y along the fastest dimension
 * (Eq. 4): mean and population variance over all points, lagged products
 * over all adjacent pairs of a row; 0 when the errors are constant. */
int qref_error_ac(const float* x, const float* y, qref_shape shape,
                  double* ac);
/* Window sums of SSIM over all windows fully inside the field, with c1, c2
 * from vrange; direct (O(N w^d)) and separable (O(N w d)) variants. */
int qref_ssim_direct(const float* x, const float* y, qref_shape shape,
                     uint32_t w, double vrange, double* sum,
                     uint64_t* nwin);
int qref_ssim_separable(const float* x, const float* y, qref_shape shape,
                        uint32_t w, double vrange, double* sum,
                        uint64_t* nwin);

/* ---- online tuner (Sec. VI) --------------------------------------------- */
/* Sampling plan: block size b, stride S, Lt, block count, origins
 * (row-major, ndim entries per block; cap = entries). */
int qref_sample_plan(qref_shape shape, uint32_t anchor_stride,
                     const qref_tune_config* cfg, uint32_t* b, uint32_t* S,
                     uint32_t* Lt, uint64_t* nblocks, uint64_t* block_dims,
                     uint64_t* origins, uint64_t origins_cap);
/* One trial: theta at bound e_trial over the sampled blocks; want: bit 0
 * the SSIM sums, bit 1 the error autocorrelation. */
int qref_trial(const float* x, qref_shape shape, double e_trial,
               const qref_params* theta, const qref_tune_config* cfg,
               double vrange, uint32_t want, qref_trial_result* res);
/* Table-I case of (B_I, M_I) vs (B_II, M_II): 1..4. */
int qref_table1_case(double BI, double MI, double BII, double MII);
/* Line test of Table I cases 3/4: 1 if II is better, 0 if I stays. */
int qref_table1_line(double BI, double MI, double BII, double MII,
                     double BIIp, double MIIp);
int qref_tune(const float* x, qref_shape shape, double e, int target,
              const qref_tune_config* cfg, qref_params* out,
              qref_tune_trace* trace);

#ifdef __cplusplus
}
#endif
#endif
