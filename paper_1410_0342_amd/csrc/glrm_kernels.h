// Kernel argument blocks and launchers shared by the host driver and the
// kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glrm_device.h"

#define GLRM_MAXK_DEV 64

namespace glrm {

// Padded shadows of Y (or of the trial Y+) in the layouts the matrix-core
// operands want.  Rows are padded to ldp (a multiple of 16), k to kp.
struct YShadow {
    float *f32;      // ldp x kp   (FP32 operand rows)
    float *t32;      // kp x ldp   (FP32, transposed: S3 operand)
    __bf16 *hi;      // ldp x kp   (bf16 high part)
    __bf16 *lo;      // ldp x kp   (bf16 low part, split precision)
    __bf16 *tb;      // kp x ldp   (bf16 high part, transposed: S3 operand)
};

// A loss shared by every column, as scalars (kind < 0: per-column table).
struct LossU {
    int32_t kind, levels;
    float param;
};

// Wavefronts per workgroup of the two passes over the table (fit), by pass
// and padded rank kp.  The fused row pass keeps four Y operands and the
// Y-gradient accumulators per tile resident, so it runs one wavefront per SIMD
// (up to 512 registers); the trial-column pass holds less and runs two per
// SIMD while kp <= 32.
constexpr int xstep_waves(int kp) { return 4; }
constexpr int ycheck_waves(int kp) { return kp >= 64 ? 4 : 8; }
// The objective-and-gradient pass: at kp = 64 eight wavefronts of two tiles,
// whose resident operands leave room for two wavefronts per SIMD; four
// elsewhere.
constexpr int grad_waves(int kp) { return kp >= 64 ? 8 : 4; }

struct XStepArgs {
    int64_t m, mp, ldp;
    int32_t k;
    const float *Ap;        // mp x ldp, NaN = unobserved
    const uint8_t *codes;   // ldp
    LossTab lt;
    LossU lu;
    Reg rx;
    float *X;               // m x k (in/out)
    float *alpha;           // m (in/out)
    float step_up, step_down;
    YShadow ycur;
    float *part_dy;         // P x ldp x kp
    float *part_h;          // P x ldp
    float *part_rowreg;     // P
    int32_t *part_rej;      // P
};

struct YProxArgs {
    int64_t n, ldp;
    int32_t k, P;
    const float *part_dy;
    const float *part_h;
    Reg ry;
    const float *Y;         // n x k
    const float *alpha;     // n
    float *Yplus;           // n x k
    YShadow yplus;
    float *h_old, *ry_plus, *ry_old;  // n
};

struct YCheckArgs {
    int64_t m, mp, ldp;
    int32_t k;
    const float *Ap;
    const uint8_t *codes;
    LossTab lt;
    LossU lu;
    const float *X;
    YShadow yplus;
    float *part_hp;         // P x ldp
    int32_t ncb;            // column blocks per panel (workgroups b with b % ncb == c take block c)
};

// Block decisions (multi-dimensional losses, Section 6): the columns
// blk0[j] .. blk1[j]-1 of a block share one decision on the sums of their
// objectives.  They take two launches: phase 1 stores every column's trial
// objective in hpc, phase 2 decides; phase 0 decides per column in one.
struct YAcceptArgs {
    int64_t n, ldp;
    int32_t k, P;
    int32_t phase;
    float *hpc;
    const int32_t *blk0, *blk1;
    const float *part_hp;
    const float *ry_plus, *h_old;
    float *alpha;
    float step_up, step_down;
    const float *Yplus;
    float *Y;
    YShadow yplus, ycur;
    double *part_F;
    int32_t *part_rejc;
};

struct FinalizeArgs {
    const double *part_F;
    const int32_t *part_rejc;
    int32_t n_colparts;
    const float *part_rowreg;
    const int32_t *part_rej;
    int32_t n_rowparts;
    double *stats;          // [0] = F tracked by the sweep
    long long *istats;      // [0] rows rejected, [1] columns rejected
    double *history;        // may be null
    int32_t sweep;
};

struct YShadowArgs {
    int64_t n, ldp;
    int32_t k;
    const float *Y;
    YShadow ys;
    YShadow yp;             // trial shadows to clear (pointers may be null)
};

struct LossGradArgs {
    int64_t m, mp, ldp;
    int32_t k;
    const float *Ap;
    const uint8_t *codes;
    LossTab lt;
    LossU lu;
    const float *X;
    YShadow ycur;
    float *dX;              // m x k, written when part_dx is null
    float *part_dx;         // CB x m x k or null
    float *part_dy;         // P x ldp x kp
    double *part_obj;       // P * CB
};

// The row half-step in column blocks (tables wider than the fused row pass
// takes): the passes over the table ...
struct XWideArgs {
    int64_t m, mp, ldp;
    int32_t k;
    const float *Ap;
    const uint8_t *codes;
    LossTab lt;
    LossU lu;
    const float *X;         // the rows the pass evaluates, m x k
    YShadow ycur;
    float *part_f;          // CB x mp: row loss sums per column block (modes 0, 1)
    float *part_dx;         // CB x m x k: row gradients per column block (mode 0)
    float *part_dy;         // P x ldp x kp: Y-gradient partials per row chunk (mode 2)
    float *part_h;          // P x ldp: column loss sums per row chunk (mode 2)
};

// ... and the per-row steps and decisions between them.
struct XWideRowArgs {
    int64_t m, mp;
    int32_t k, ncb;
    Reg rx;
    float *X;               // m x k (decisions write the accepted rows)
    float *alpha;           // m
    const float *part_f;    // CB x mp (loss sums at X)
    const float *part_fp;   // CB x mp (loss sums at X+)
    const float *part_dx;   // CB x m x k
    float *Xp;              // m x k trial rows
    float *rsum;            // 3 x mp: loss sum at X, r(x), r(x+)
    float step_up, step_down;
    float *part_rowreg;     // grid: regularizers of the decided rows
    int32_t *part_rej;      // grid: rejected rows
};

struct ReduceArgs {
    int64_t m, n, ldp;
    int32_t k, P, CB;
    const float *part_dy;
    const float *part_dx;
    float *dY, *dX;
};

struct Obj64Args {
    int64_t m, n, mp, ldp;
    int32_t k;
    const float *Ap;
    const uint8_t *codes;
    LossTab lt;
    const float *X, *Y;
    double *part_obj;
};

// Columns of a table embedded for multi-dimensional losses (Section 6): packed
// column j reads column emb_src[j] of A and, by emb_kind[j], copies the value
// (EMB_COPY) or encodes +1 / -1 for value == emb_thr[j] (EMB_EQ, the
// categorical one-vs-all columns) or value > emb_thr[j] (EMB_GT, the
// multi-dimensional ordinal thresholds).
enum { EMB_COPY = 0, EMB_EQ = 1, EMB_GT = 2 };
struct EmbedMap {
    const int32_t *src, *thr;   // null: no embedding (column j is column j of A)
    const uint8_t *kind;
};

struct PackArgs {
    int64_t m, n, lda, mp, ldp;
    const float *A;
    const uint8_t *mask;
    float *Ap;
    int32_t *row_count;     // m (zeroed by the kernel itself)
    int32_t *col_count;     // n (zeroed beforehand)
    EmbedMap emb;
};

// ---- launchers (dense.hip) ----
hipError_t launch_xstep(const XStepArgs &a, int kp, int tpw, int prec, int grid, hipStream_t st);
hipError_t launch_ycheck(const YCheckArgs &a, int kp, int tpw, int prec, int grid, hipStream_t st);
// Workgroups of the instance the launchers above pick that fit on one CU.
int xstep_blocks(int kp, int tpw, int prec, bool quad);
int ycheck_blocks(int kp, int tpw, int prec, bool quad);
hipError_t launch_yprox(const YProxArgs &a, int kp, int prec, hipStream_t st);
hipError_t launch_yaccept(const YAcceptArgs &a, int kp, int prec, int blocks, hipStream_t st);
int yaccept_blocks(int64_t n, int kp);
hipError_t launch_finalize(const FinalizeArgs &a, hipStream_t st);
hipError_t launch_yshadow(const YShadowArgs &a, int kp, int prec, hipStream_t st);
hipError_t launch_lossgrad(const LossGradArgs &a, int kp, int tpw, int prec, bool want_grad, int gx, int gy,
                           hipStream_t st);
// mode: 0, 1 or 2 (XWideArgs); tpw 16 for kp <= 32, 4 for kp = 64; grid gx x gy.
hipError_t launch_xwide(const XWideArgs &a, int mode, int kp, int tpw, int prec, int gx, int gy, hipStream_t st);
int xwide_blocks(int kp, int tpw, int prec, bool quad);   // column-pass workgroups per CU
hipError_t launch_xwide_step(const XWideRowArgs &a, hipStream_t st);
// grid: workgroups of 64 rows at a time, one row partial each (part_rowreg, part_rej)
hipError_t launch_xwide_decide(const XWideRowArgs &a, int grid, hipStream_t st);
hipError_t launch_reduce_dy(const ReduceArgs &a, int kp, hipStream_t st);
hipError_t launch_reduce_dx(const ReduceArgs &a, hipStream_t st);
hipError_t launch_objective64(const Obj64Args &a, int grid, hipStream_t st);

// ---- launchers (common.hip) ----
hipError_t launch_pack_dense(const PackArgs &a, hipStream_t st);
hipError_t launch_init_alpha(const int32_t *count, int64_t len, float scale, float *alpha, hipStream_t st);
hipError_t launch_prox(Reg r, float *V, int64_t rows, int32_t k, int64_t ldv, const float *alpha, hipStream_t st);
hipError_t launch_regsum(Reg r, const float *V, int64_t rows, int32_t k, double *part, int blocks, hipStream_t st);
hipError_t launch_reg_grad(Reg r, const float *V, int64_t rows, int32_t k, float *dV, hipStream_t st);
hipError_t launch_sum_doubles(const double *a, int32_t na, const double *b, int32_t nb, double *out, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t len, int32_t v, hipStream_t st);
hipError_t launch_pad_weights(const float *src, const int32_t *map, int64_t n, int64_t ldp, float *dst, hipStream_t st);

}  // namespace glrm
