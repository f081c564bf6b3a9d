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

}  // namespace glrm

