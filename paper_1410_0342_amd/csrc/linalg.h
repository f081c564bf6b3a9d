// Linear algebra around the fit: a matrix defined entry by entry on the
// observed set (the loss derivatives G of Section 7.6, or the standardized
// table of Section 7.5) materialized in the table's own layout, its products
// with blocks of vectors, tall-skinny products with the factors, and the
// small symmetric eigenproblems the host solves in double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glrm_device.h"

namespace glrm {

// Entry-wise matrices on the observed set (0 elsewhere).
struct EntryArgs {
    int64_t m, n, mp, ldp;   // dense: the padded table (NaN = unobserved)
    int32_t k;
    const float *Ap;
    const uint8_t *codes;    // per column (ldp)
    LossTab lt;
    const float *colw;       // per-column loss weight (n) or null
    const float *X, *Y;      // factors (m x k, n x k), for the derivative matrix
    const float *mu, *cs;    // per-column offset and scale (n), for the standardized table
};

// Dense: V (mp x ldp) = the loss derivative dL_j(x_i . y_j, A_ij) (times the
// column's weight) on the observed set, 0 elsewhere.
hipError_t launch_dense_grad_matrix(const EntryArgs &a, float *V, hipStream_t st);
// Dense: V = cs_j (A_ij - mu_j) on the observed set, 0 elsewhere.
hipError_t launch_dense_scaled_matrix(const EntryArgs &a, float *V, hipStream_t st);
// COO: the same per listed entry (row, col, A in row-major order).
hipError_t launch_coo_grad_values(const EntryArgs &a, const int32_t *row, const int32_t *col, const float *A,
                                  int64_t nnz, float *out, hipStream_t st);
hipError_t launch_coo_scaled_values(const EntryArgs &a, const int32_t *col, const float *A, int64_t nnz,
                                    float *out, hipStream_t st);
// out[p] = in[perm[p]] (the column-grouped order of per-entry values).
hipError_t launch_permute(const int32_t *perm, const float *in, int64_t nnz, float *out, hipStream_t st);

constexpr int LA_MAXB = 96;        // widest vector block
constexpr int LA_TCHUNKS = 64;     // row chunks of the transposed dense product, at most

// out (m x b) = alpha * V (m x n, leading dimension ldp) . B (n x b)
hipError_t launch_dense_apply(const float *V, int64_t m, int64_t n, int64_t ldp, const double *B, int32_t b,
                              double alpha, double *out, hipStream_t st);
// out (n x b) = alpha * V^T . Q (m x b); part holds chunks x n x b partial sums
int dense_apply_t_chunks(int64_t m, int64_t n);
hipError_t launch_dense_apply_t(const float *V, int64_t m, int64_t n, int64_t ldp, const double *Q, int32_t b,
                                double alpha, double *part, double *out, hipStream_t st);
// out (rows x b) = alpha * sum over each segment's entries of val[e] B[idx[e], :]
hipError_t launch_seg_apply(const int32_t *ptr, const int32_t *idx, const float *val, int64_t rows, const double *B,
                            int32_t b, double alpha, double *out, hipStream_t st);

// Tall-skinny products.  U is rows x k with leading dimension ldu.
//   out (k x b) = U^T B             (part: blocks x k x b)
int tall_tmul_blocks(int64_t rows);
hipError_t launch_tall_tmul_f(const float *U, int64_t rows, int32_t k, int64_t ldu, const double *B, int32_t b,
                              double *part, double *out, hipStream_t st);
hipError_t launch_tall_tmul_d(const double *U, int64_t rows, int32_t k, int64_t ldu, const double *B, int32_t b,
                              double *part, double *out, hipStream_t st);
//   out (rows x b) = beta * out + alpha * U S       (S: k x b)
hipError_t launch_tall_mul_f(const float *U, int64_t rows, int32_t k, int64_t ldu, const double *S, int32_t b,
                             double alpha, double beta, double *out, hipStream_t st);
hipError_t launch_tall_mul_d(const double *U, int64_t rows, int32_t k, int64_t ldu, const double *S, int32_t b,
                             double alpha, double beta, double *out, hipStream_t st);
// The Gram matrix U^T U (k x k) of a float factor.
hipError_t launch_gram_f(const float *U, int64_t rows, int32_t k, double *part, double *out, hipStream_t st);

// Vectors: *nrm2 = sum of squares (fixed order); v /= sqrt(*nrm2); est[slot] = sqrt(*nrm2).
hipError_t launch_sumsq(const double *v, int64_t len, double *part, double *nrm2, hipStream_t st);
hipError_t launch_normalize(double *v, int64_t len, const double *nrm2, double *est, int32_t slot, hipStream_t st);
// A deterministic start vector: v_j = 1 + u_j, u_j uniform in [0, 1) from a
// counter-based hash of j (SplitMix64).
hipError_t launch_start_vector(double *v, int64_t len, uint64_t seed, hipStream_t st);
// Float copy of a double block (rows x b), into a destination of leading dimension ldd.
hipError_t launch_to_float(const double *src, int64_t rows, int32_t b, int32_t cols, float *dst, int64_t ldd,
                           int32_t col0, hipStream_t st);

// ---- per-column sums for the loss scaling of Section 4.3 ----------------------
// MODE 0: min and max of the observed entries; 1: sum of dL_j(mid_j, a);
// 2: sum of L_j(mid_j, a).  Dense: partials over row chunks (part: R x 2 x n
// doubles) then a fixed-order reduction into out (2 x n); COO: one wavefront
// per column of the column-grouped copy, straight into out.
// The per-column passes of the loss scaling (Section 4.3): mode 0 the least
// and largest value, mode 1 the derivative sums at COL_PTS points of each
// column's bracket [lo, hi], mode 2 the loss sum at mid.  out holds the
// results as slot-major arrays of n (slot p of column j at p n + j).
// Each search pass keeps one of 2^COL_BITS sub-intervals of every bracket, at
// COL_PTS = 2^COL_BITS - 1 points; COL_PASSES passes take it past 64 halvings.
#ifndef GLRM_COL_BITS
#define GLRM_COL_BITS 4
#endif
constexpr int COL_BITS = GLRM_COL_BITS;
constexpr int COL_PTS = (1 << COL_BITS) - 1;
constexpr int COL_PASSES = (64 + COL_BITS - 1) / COL_BITS;
constexpr int COL_SLOTS = 16;                  // partial slots per row chunk and column
static_assert(COL_BITS >= 1 && COL_PTS < COL_SLOTS, "a pass's points fit the slots");
constexpr int COL_CHUNKS_MAX = 1024;
constexpr int64_t COL_PART_BUDGET = int64_t(1) << 22;   // doubles of partials, at most (or one chunk)
struct ColArgs {
    int64_t m, n, mp, ldp;
    const float *Ap;            // dense table (NaN = unobserved)
    const int32_t *col_ptr;     // COO column view
    const float *csc_val;
    const uint8_t *codes;
    LossTab lt;
    const double *lo, *hi;      // n: the bracket (mode 1)
    const double *mid;          // n: the point of mode 2
};
int col_pass_chunks(int64_t m, int64_t n);
int64_t col_part_doubles(int64_t m, int64_t n);     // partials of the dense passes
hipError_t launch_col_pass(const ColArgs &a, int mode, bool coo, double *part, double *out, hipStream_t st);
// lo, hi (n): the bracket; mid = (lo + hi) / 2.  init: lo = min - 1, hi = max + 1
// from out (mode 0); step: the sub-interval, between two of mode 1's points,
// that keeps the derivative's sign change.
hipError_t launch_bracket(double *lo, double *hi, double *mid, const double *out, const int32_t *count, int64_t n,
                          bool init, hipStream_t st);
// mu_j = mid_j (0 for an empty column); sigma2_j = S_j / (n_j - 1), or 1 when
// n_j < 2 or S_j <= 0 (S_j = out[j], mode 2).
hipError_t launch_scaling_finish(const double *mid, const double *out, const int32_t *count, int64_t n, float *mu,
                                 float *sigma2, hipStream_t st);
// cs_j = m / (sigma_j m_j) (0 for an empty column), mu0_j = mu_j or 0 (Section 7.5).
hipError_t launch_svd_scales(const float *mu, const float *sigma2, const int32_t *count, int64_t m, int64_t n,
                             float *cs, float *mu0, hipStream_t st);
// dst[i ldd + col0 + c] = src[i b + c] * (rowscale ? sqrt(rowscale[i]) : 1), c < cols
hipError_t launch_to_float_scaled(const double *src, int64_t rows, int32_t b, int32_t cols, const float *rowscale,
                                  float *dst, int64_t ldd, int32_t col0, hipStream_t st);
// dst[i ldd + col] = value (value_vec ? value_vec[i] : value)
hipError_t launch_fill_column(float *dst, int64_t rows, int64_t ldd, int32_t col, float value,
                              const float *value_vec, hipStream_t st);
// double copy of a float block: dst (rows x b) = src (rows x b)
hipError_t launch_to_double(const float *src, int64_t len, double *dst, hipStream_t st);

}  // namespace glrm

