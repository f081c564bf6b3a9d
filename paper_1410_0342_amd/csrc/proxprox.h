// The prox-prox update for quadratic losses (Sections 7.2 and 7.3) on the
// dense layout: per row of the table (a column of A for the Y half-step, on
// the transposed copy), the Gram data G_i = sum_j w v_j v_j^T, b_i =
// sum_j w A_ij v_j over the row's observed entries, a Cholesky factorization
// of G_i + I / (2 alpha_i) in double, `inner` updates
//     x <- prox_{alpha r}((G_i + I / (2 alpha))^-1 (b_i + x / (2 alpha))),
// and the row objective's check of the step rule.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glrm_device.h"

namespace glrm {

// Floats of one row's Gram data: the upper 4 x 4 tiles of G (kp / 4 tiles a
// side) in slots padded to a multiple of four tiles, then b in 64 floats.
// The Gram pass writes whole 16-row panels: gram holds the rows padded to 16,
// and gpart splits x (rows padded to 16) rows.
int pp_gram_floats(int kp);
// Column splits of a row (partials summed in a fixed order afterwards).
constexpr int PP_SPLITS_MAX = 32;

struct PPArgs {
    int64_t rows, cols, ldt;      // the table (rows x cols, leading dimension ldt; NaN = unobserved)
    int32_t k, kp;
    const float *T;
    const float *wcol;            // per-column weight (cols, padded) or null
    const float *wrow;            // per-row weight (rows) or null
    float *U;                     // updated factor, rows x k (in/out)
    const float *V;               // fixed factor, cols x k
    float *alpha;                 // rows (in/out)
    Reg reg;
    int32_t inner;
    float step_up, step_down;
    float *gram;                  // rows (padded to 16) x gsz (final Gram data)
    float *gpart;                 // splits x rows (padded to 16) x gsz (partials)
    int32_t splits;
    float *trial;                 // rows x k
    float *fpart;                 // splits x rows x 2 (old and trial loss sums)
    double *rowobj;               // per row: the decided objective (loss + r), or r alone
    int32_t obj_with_loss;        // 1: rowobj = decided loss + r; 0: r of the decided row only
    int32_t *rej;                 // per row: 1 if rejected
};

hipError_t launch_pp_gram(const PPArgs &a, hipStream_t st);
hipError_t launch_pp_solve(const PPArgs &a, hipStream_t st);
hipError_t launch_pp_check(const PPArgs &a, hipStream_t st);
// Padded transposed copy: dst (ldp x mp) from src (mp x ldp); NaN stays NaN.
hipError_t launch_transpose(const float *src, int64_t rows, int64_t cols, float *dst, hipStream_t st);
// The sweep's F (the rows' and columns' decided values) and rejection counts,
// summed in a fixed order through `part` (pp_finalize_part_doubles() doubles).
int pp_finalize_part_doubles();
hipError_t launch_pp_finalize(const double *rowobj_x, const int32_t *rej_x, int64_t m, const double *rowobj_y,
                              const int32_t *rej_y, int64_t n, double *part, double *stats, long long *istats,
                              double *history, int32_t sweep, hipStream_t st);

}  // namespace glrm
