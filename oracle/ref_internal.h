/*
 * Internal declarations of the CPU oracle (test infrastructure only; see
 * qoz_ref.h).  Everything here is plain, sequential C++17.
 */
#ifndef QOZ_REF_INTERNAL_H
#define QOZ_REF_INTERNAL_H
#include <cstdint>
#include <cstring>
#include <vector>

#include "qoz_ref.h"

namespace qref {

/* memcpy that accepts an empty range (an empty vector's data() may be
 * null, which memcpy does not allow even for zero bytes) */
inline void copy_bytes(void* dst, const void* src, size_t n) {
  if (n) std::memcpy(dst, src, n);
}

/* A d-dimensional row-major grid (dims[0] slowest). */
struct Grid {
  int d = 0;
  int64_t n[3] = {1, 1, 1};
  int64_t stride[3] = {0, 0, 0};
  int64_t N = 0;
};
/* Lag-1 autocorrelation of e over nrows rows of len values (Eq. 4). */
double ac_of_rows(const double* e, int64_t nrows, int64_t len);
Grid make_grid(int d, const int64_t* n);
bool shape_to_grid(const qref_shape& s, Grid* g); /* validates dims */

/* Per-level interpolator choice: type and dimension order (Sec. V-B). */
struct LevelPlan {
  int interp[QREF_MAX_LEVELS];
  int order[QREF_MAX_LEVELS][3];
};

/* Per-level bounds (Eq. 5) and their FP32 forms used by the quantizer. */
struct LevelBounds {
  double eb[QREF_MAX_LEVELS];
  float twoeb[QREF_MAX_LEVELS];
  float inv[QREF_MAX_LEVELS];
};
void bounds_uniform(double e, int L, LevelBounds* b);
void bounds_eq5(double e, double alpha, double beta, int L, LevelBounds* b);

/* What a run of sweeps reports. */
struct SweepSink {
  std::vector<int32_t>* codes = nullptr; /* quantization bins, stream order */
  std::vector<float>* unpred = nullptr;  /* unpredictable values */
  uint64_t* hist = nullptr;              /* 2R-bin histogram (optional) */
  uint64_t n_unpred = 0;
  uint64_t n_codes = 0;
  std::vector<uint32_t>* targets = nullptr; /* flat index per code */
  std::vector<float>* preds = nullptr;      /* prediction per code */
  int l1_level = 0;        /* level whose |x - pred| is summed (0: none) */
  double l1_sum = 0.0;
  uint64_t l1_count = 0;
};

float stencil(int cubic, float a, float b, float c, float d, bool has_a,
              bool has_c, bool has_d);

/* Store the anchor grid (every coordinate a multiple of s) into W, and
 * optionally append the values (row-major) to `anchors`. */
void place_anchors(const float* x, const Grid& g, int64_t s, float* W,
                   std::vector<float>* anchors);

/* Compression sweeps for levels l_hi..l_lo (inclusive, descending). */
void compress_levels(const float* x, const Grid& g, int l_hi, int l_lo,
                     const LevelPlan& plan, const LevelBounds& lb, float* W,
                     SweepSink* sink);
/* Decompression sweeps for all levels L..1; returns false on stream error. */
bool decompress_levels(const Grid& g, int L, const LevelPlan& plan,
                       const LevelBounds& lb, const int32_t* codes,
                       uint64_t n_codes, const float* unpred,
                       uint64_t n_unpred, float* W);

int64_t count_anchors(const Grid& g, int64_t s);

/* Huffman */
bool huffman_lengths(const uint64_t* hist, uint32_t nsym, uint8_t* len);
void canonical_codes(const uint8_t* len, uint32_t nsym, uint64_t* code);
uint64_t huffman_bits(const uint64_t* hist, const uint8_t* len,
                      uint32_t nsym);

/* SSIM sums (separable, plane-streamed) */
void ssim_separable_sums(const float* x, const float* y, const Grid& g,
                         int w, double vrange, double* sum, uint64_t* nwin);

bool validate_params(const qref_params& p, int d, int* L);
bool all_finite(const float* x, int64_t N);
void value_range(const float* x, int64_t N, double* vmin, double* vmax);

}  // namespace qref
#endif
