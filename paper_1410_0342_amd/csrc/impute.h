// Argument block and launchers of the imputation pass (impute.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glrm_device.h"

namespace glrm {

// X, Y, the table and the output are separate kernel arguments, so the kernel
// can take them as non-aliasing.
struct ImputeArgs {
    int64_t m, n, ldh, lda;
    int32_t k;
    int32_t rows_per_block;
    int32_t keep_observed;  // dense with a mask: entries with mask != 0 keep A
    const uint8_t *codes;   // per-column loss codes (n, device)
    LossTab lt;
};

// A table with multi-dimensional losses (Section 6): feature j's block is
// rows fcol[j] .. of Y; fkind / flev are its loss kind and levels (device).
struct ImputeMDArgs {
    int64_t m, nf, ldh, lda;
    int32_t k;
    int32_t keep_observed;
    const int32_t *fcol, *fkind, *flev;
};

// Workgroups of one imputation launch (about eight per CU).
constexpr int64_t IMPUTE_TARGET_BLOCKS = 2048;
constexpr int IMPUTE_MAX_K = 64;

int impute_rows_per_block(int64_t m, int64_t n);
hipError_t launch_impute(const ImputeArgs &a, const float *X, const float *Y, const float *A, const uint8_t *mask,
                         float *out, hipStream_t st);
hipError_t launch_impute_md(const ImputeMDArgs &a, const float *X, const float *Y, const float *A, const uint8_t *mask,
                            float *out, hipStream_t st);
hipError_t launch_scatter_observed(int64_t nnz, int64_t m, int64_t n, int64_t ldh, const int32_t *row,
                                   const int32_t *col, const float *val, float *out, hipStream_t st);

}  // namespace glrm
