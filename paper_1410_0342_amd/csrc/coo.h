// Sparse (row-sorted COO) path: layout of its workspace region and its entry
// points, used by the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>

#include "../../include/glrm.h"
#include "glrm_device.h"

namespace glrm {

// Sets the thread's last-error message and returns `code` (host driver).
int set_error(int code, const char *fmt, ...);

struct CooLayout {
    int64_t m = 0, n = 0, nnz = 0;
    int kp = 0;
    size_t total = 0;
    size_t row_ptr = 0;    // int32 [m + 1]
    size_t col_ptr = 0;    // int32 [n + 1]
    size_t csc_row = 0;    // int32 [nnz]   row of each entry, column-grouped
    size_t csc_val = 0;    // float [nnz]
    size_t perm_in = 0, perm_out = 0, keys_out = 0;  // sort scratch (int32 [nnz] each)
    size_t sort_tmp = 0, sort_tmp_bytes = 0;
    size_t flags = 0;      // int32 [4] validation result
    size_t part = 0, part_bytes = 0;  // double partials of the objective
    size_t xs = 0;         // padded copy of X (m x kp, fp32), updated in place by the row walk
    size_t ys = 0;         // padded copy of Y (n x kp, fp32), updated in place by the column walk
    size_t xsb = 0, ysb = 0;   // bfloat16 copies of xs and ys (the BF16 fit's trial passes)
    size_t zc = 0;         // per entry (row-blocked order): z kept between the BF16 column passes
    // Row-blocked column-grouped copy for the column step: entries ordered by
    // (row block, column, row), rows in blocks of 2^rb_shift, with segment
    // pointers per (row block, column).  blk = false: not built (too many
    // segments or columns for it); the column step then walks whole columns.
    bool blk = false;
    int rb_shift = 0;
    int64_t nb = 0;        // row blocks
    size_t bkey = 0, bperm = 0, brow = 0, bval = 0, seg = 0;
    size_t bpart0 = 0, bpart1 = 0;     // per-XCD partials of the two column passes
    size_t yplus = 0, hold = 0, rplus = 0;
};

// The parts of the COO region other passes read: the row pointers, the
// column-grouped copy and the permutation that made it.
struct CooView {
    const int32_t *row_ptr, *col_ptr, *csc_row;
    const float *csc_val;
};
CooView coo_view(const CooLayout &cl, char *base);
const int32_t *coo_perm(const CooLayout &cl, char *base);

void coo_layout(const glrm_data *d, int kp, CooLayout &cl);
int coo_prepare(const glrm_data *d, int kp, const CooLayout &cl, char *base, int32_t *row_count, int32_t *col_count,
                hipStream_t st);
int coo_check_result(const CooLayout &cl, char *base, hipStream_t st);
int coo_objective(const glrm_data *d, const CooLayout &cl, char *base, const uint8_t *codes, const LossTab &lt,
                  const float *X, const float *Y, int prec, double **parts, int *nparts, hipStream_t st);
int coo_grad(const glrm_data *d, int kp, const CooLayout &cl, char *base, const uint8_t *codes, const LossTab &lt,
             const float *X, const float *Y, int prec, float *dX, float *dY, double **parts, int *nparts,
             hipStream_t st);
int coo_fit_supported(const glrm_data *d, int kp, const CooLayout &cl, int prec);
int coo_fit(const glrm_data *d, int kp, const CooLayout &cl, char *base, const uint8_t *codes, const LossTab &lt,
            float *X, float *Y, float *alpha_x, float *alpha_y, const glrm_fit_opts *o, double *history,
            double *stats, long long *istats, int *sweeps, hipStream_t st,
            const std::function<hipError_t(int)> &tstart, const std::function<hipError_t()> &tstop);

}  // namespace glrm
