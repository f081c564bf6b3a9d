/*
 * glrm.h — C ABI of the MI355X (gfx950) alternating proximal-gradient fit of a
 * generalized low rank model.
 *
 * The method is the one of Udell, Horn, Zadeh and Boyd, "Generalized Low Rank
 * Models" (arXiv 1410.0342):
 *
 *     minimize  sum_{(i,j) in Omega} L_j(x_i . y_j, A_ij) + sum_i r(x_i) + sum_j rt(y_j)
 *
 * (eq. gpca in Section 4, with the per-column losses of the abstract-data form
 * eq. apca in Section 5), fitted by Algorithm 2 of Section 7.2 with the
 * proximal gradient update and the per-row / per-column step-size rule of
 * Section 7.2 ("Choosing a step size").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - X is m x k, row-major, float32 (row i is the paper's x_i).
 *  - Y is stored n x k, row-major, float32: row j is the paper's column y_j
 *    (the paper's k x n matrix Y kept column-major, so y_j is contiguous).
 *  - Array arguments are DEVICE pointers unless marked "host".  The glrm_data
 *    struct, the loss table, the per-column loss codes and the glrm_fit_opts /
 *    glrm_fit_info structs live in host memory.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it; entry points that return a host value synchronize it.
 *  - Every entry point validates its arguments on the host before it enqueues
 *    anything; on an error it returns a negative code, writes no output, and
 *    glrm_last_error() describes the problem.
 *  - The library never allocates or frees caller-visible device memory.
 *    Scratch space is the caller's `ws` buffer (device memory, 256-byte
 *    aligned) of at least glrm_workspace_size() bytes.  Calls that share a
 *    workspace must be ordered (same stream, or synchronized).
 */
#ifndef GLRM_H
#define GLRM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ----------------------------------------------------------- */
#define GLRM_OK            0
#define GLRM_EINVAL       -1  /* null pointer, bad size, bad kind, unsorted / out-of-range COO, bad loss code */
#define GLRM_EUNSUPPORTED -2  /* valid request outside what is built (e.g. k > 64, layout or loss combination not built) */
#define GLRM_ENOMEM       -3  /* workspace smaller than glrm_workspace_size() */
#define GLRM_EHIP         -4  /* a HIP runtime call failed; the message names it */

/* ---- loss kinds (Section 4 and Section 5.2) ----------------------------------
 *  QUADRATIC  (a - u)^2                              eq. qpca
 *  HUBER      huber(u - a) with threshold `param`:   Section 4.2 ("Huber PCA",
 *             0.5 r^2 if |r| <= param else           the paper fixes param = 1)
 *             param |r| - 0.5 param^2
 *  LOGISTIC   log(1 + exp(-a u)), a in {-1, +1}      Section 5.2 ("Logistic PCA")
 *  HINGE      max(0, 1 - a u),     a in {-1, +1}      Section 5.2 ("Boolean PCA")
 *  ORDINAL    sum_{a'<a} (1 - u + a')_+ +            eq. ord-pca, a in {1..levels}
 *             sum_{a'>a} (1 + u - a')_+
 * Multi-dimensional losses (Section 6, eq. mpca): the column is a feature of
 * embedding dimension d_j, modelled by the block of d_j rows of Y (the
 * columns of the paper's Y_j) and u = x_i Y_j:
 *  CATEGORICAL  (1 - u_a)_+ + sum_{a' != a} (1 + u_a')_+    Section 6.1 (one-vs-all),
 *               labels a in {1..levels}, d_j = levels
 *  MORDINAL     sum_{l=1}^{levels-1} (1 - s_l u_l)_+,       eq. ord-mpca, levels a in
 *               s_l = +1 if a > l, else -1                  {1..levels}, d_j = levels - 1
 * (eq. ord-mpca prints the factor as the indicator of a > l; it is taken as
 * this sign, so that each term is the SVM separating the levels up to l from
 * those above, as the paper describes the model.)  A value that is no label
 * counts as matching none (CATEGORICAL: every term (1 + u_a')_+).
 * The derivative used at a kink is the strict-inequality branch (the kink
 * contributes 0); Section 7.2 allows any subgradient. */
enum { GLRM_LOSS_QUADRATIC = 0, GLRM_LOSS_HUBER = 1, GLRM_LOSS_LOGISTIC = 2,
       GLRM_LOSS_HINGE = 3, GLRM_LOSS_ORDINAL = 4, GLRM_LOSS_CATEGORICAL = 5,
       GLRM_LOSS_MORDINAL = 6 };

/* ---- regularizer kinds (Section 3) and their proxes (Section 7.2) -------------
 *  ZERO       0                                  prox: v
 *  QUADRATIC  weight * ||x||_2^2                 prox: v / (1 + 2 alpha weight)
 *  L1         weight * ||x||_1                   prox: sign(v) max(|v| - alpha weight, 0)
 *  NONNEG     0 if x >= 0 else +inf              prox: max(v, 0) */
enum { GLRM_REG_ZERO = 0, GLRM_REG_QUADRATIC = 1, GLRM_REG_L1 = 2, GLRM_REG_NONNEG = 3 };

/* ---- data layouts -------------------------------------------------------------- */
enum { GLRM_DENSE = 0, GLRM_COO_ROWSORTED = 1 };

/* ---- arithmetic of the contractions z = x_i . y_j, G Y^T and X^T G ---------------
 *  FP32        float32 operands, float32 matrix-core products (v_mfma_f32_16x16x4_f32)
 *  BF16        z from three bfloat16 products (hi*hi + hi*lo + lo*hi, float32
 *              accumulation); both gradient contractions from one bfloat16 product;
 *              loss, prox, step rule and objective in float32
 *  FP64        float64 throughout (glrm_objective only: the final / convergence check)
 *  BF16_PLAIN  every contraction from one bfloat16 product (fastest, least accurate)
 * The COO layout computes its dot products on the vector ALUs in FP32 (FP64 for the
 * objective); it returns GLRM_EUNSUPPORTED for BF16 and BF16_PLAIN. */
enum { GLRM_FP32 = 0, GLRM_BF16 = 1, GLRM_FP64 = 2, GLRM_BF16_PLAIN = 3 };

#define GLRM_MAX_LOSSES 16
#define GLRM_MAX_K 64
#define GLRM_MAX_LEVELS 1024   /* labels / levels of a multi-dimensional loss */

typedef struct {
    int32_t kind;    /* GLRM_LOSS_* */
    int32_t levels;  /* ORDINAL: number of levels d >= 2, data in 1..d; CATEGORICAL,
                        MORDINAL: 2..GLRM_MAX_LEVELS labels / levels; else ignored */
    float   param;   /* HUBER: threshold > 0; else ignored */
} glrm_loss;

typedef struct {
    int32_t kind;    /* GLRM_REG_* */
    float   weight;  /* >= 0; ignored for ZERO and NONNEG */
} glrm_reg;

/* The problem (eq. gpca / eq. apca).  Host struct. */
typedef struct {
    int64_t m, n;             /* rows and columns of A, both >= 1 */
    int32_t k;                /* rank, 1 <= k <= GLRM_MAX_K */
    int32_t layout;           /* GLRM_DENSE or GLRM_COO_ROWSORTED */
    /* dense: A is m x n row-major with leading dimension lda >= n (device).
     *        mask has the same shape and leading dimension, 1 = observed
     *        (device, NULL = every entry observed).  Observed values must be
     *        finite.
     * COO:   A holds the nnz observed values (device); row / col are the nnz
     *        0-based indices (device int32), sorted by row then column, no
     *        duplicates.  With nnz = 0 the three may be NULL (only the
     *        regularizers remain).  mask and lda are ignored. */
    const float   *A;
    int64_t        lda;
    const uint8_t *mask;
    const int32_t *row;
    const int32_t *col;
    int64_t        nnz;
    /* per-column loss: col_loss[j] indexes losses[] (host, n bytes; NULL = all 0) */
    const uint8_t   *col_loss;
    const glrm_loss *losses;  /* host, n_losses entries */
    int32_t          n_losses;/* 1 .. GLRM_MAX_LOSSES */
    glrm_reg rx;              /* r on the rows of X */
    glrm_reg ry;              /* rt on the columns of the paper's Y */
    /* Offset (Section 3.3): 1 = coordinate 0 of every x_i is the constant 1 and
     * coordinate 0 of every y_j a free, unpenalized column offset, so the model
     * is x_i . y_j = mu_j + (the other k - 1 coordinates); r and rt apply to
     * coordinates 1..k-1 only, and an x_i whose coordinate 0 is not 1 is
     * infeasible (r = +inf; the prox sets it to 1).  0 = no offset. */
    int32_t offset;
    /* Per-column loss weights (device, n floats, finite and >= 0; NULL = all 1):
     * column j's loss becomes col_weight[j] * L_j, e.g. 1 / sigma_j^2 for the
     * scaled losses of Section 4.3 (glrm_column_scaling). */
    const float *col_weight;
} glrm_data;

/* Multi-dimensional losses (Section 6).  When some column's loss is
 * CATEGORICAL or MORDINAL, Y has d = glrm_embed_dim(d) rows instead of n:
 * column j of A owns the next d_j rows (d_j = 1 for the scalar losses, in
 * column order), and every entry point that takes Y, dY or alpha_y takes
 * d rows or entries.  Both losses are sums of hinge losses over their d_j
 * embedded columns (the separability Section 6.1 notes for one-vs-all), so
 * the passes run on the embedded table of +-1 values; glrm_fit decides each
 * column's block as a whole (one step-size rule per block Y_j: the block's
 * trial objective against its current one), and its step sizes move
 * together (keep them equal within a block when resuming; init_alpha
 * does).  The row of X counts the d_j embedded entries of each observed
 * value in n_i; a block's columns count n_j.  Built for the dense layout;
 * the COO layout, glrm_column_scaling and glrm_init_svd return
 * GLRM_EUNSUPPORTED for such problems, and glrm_fit's prox-prox update does
 * (its losses are quadratic). */

/* d = sum_j d_j (n when every loss is scalar); -1 for an invalid problem or a
 * multi-dimensional loss outside the dense layout (glrm_last_error() says why). */
int64_t glrm_embed_dim(const glrm_data *d);

/* Flags for the compute entry points. */
#define GLRM_WS_PREPARED 1u   /* `ws` already holds what glrm_prepare() builds for this
                                 exact data (same pointers, sizes and contents); skip it */
#define GLRM_TIME_KERNELS 2u  /* glrm_fit only: record HIP events on `stream` around every
                                 kernel launch and report per-kernel totals in glrm_fit_info */
#define GLRM_GRAD_WITH_REG 4u /* glrm_grad, glrm_grad_noalloc: add the regularizers'
                                 subgradients, so dX, dY are (sub)gradients of all of F */

/* Bytes of device workspace any entry point needs for this problem.  The same
 * size serves glrm_prepare, glrm_objective, glrm_grad and glrm_fit, and the
 * prepared part sits at the same offsets for all of them.  Returns 0 when the
 * problem is invalid (glrm_last_error() then says why). */
size_t glrm_workspace_size(const glrm_data *d);

/* Build the data-derived state in `ws`: the per-column loss codes, the row /
 * column observation counts n_i and m_j, the dense table with unobserved
 * entries folded in (dense), and the row pointers and column-grouped copy of
 * the entries (COO).  Asynchronous on `stream`, except that it waits for the
 * small host-to-device copy of the loss codes.  Call it again after the data
 * change; then pass GLRM_WS_PREPARED to skip it inside the other calls. */
int glrm_prepare(const glrm_data *d, void *ws, size_t ws_bytes, void *stream);

/* F(X, Y) of eq. gpca: the loss over Omega plus both regularizer sums
 * (Section 4).  Per-entry losses are evaluated in `precision` (FP32, BF16,
 * BF16_PLAIN or FP64) and summed in float64.  Writes *obj_host (host) and
 * synchronizes `stream`. */
int glrm_objective(const glrm_data *d, const float *X, const float *Y, int precision,
                   double *obj_host, void *ws, size_t ws_bytes, unsigned flags, void *stream);

/* Loss-part gradients (Section 7.2, g = sum_j dL(x_i . y_j, A_ij) y_j):
 *   dX[i,:] = sum_{j:(i,j) in Omega} G_ij y_j        (m x k, row-major, device)
 *   dY[j,:] = sum_{i:(i,j) in Omega} G_ij x_i        (n x k, row-major, device)
 * with G_ij = dL_j(x_i . y_j, A_ij).  Regularizer gradients are added only
 * with GLRM_GRAD_WITH_REG in `flags`: then dX[i,:] += g(r, x_i) and
 * dY[j,:] += g(rt, y_j), where g is, coordinate by coordinate, the subgradient
 * of least magnitude of the regularizers of Section 3 (quadratic 2 w x; l1
 * w sign(x), 0 at 0; nonnegative 0), NaN where the regularizer is +inf (a
 * negative coordinate under the nonnegative constraint, x_i0 != 1 under the
 * offset of Section 3.3); the offset coordinate is otherwise unpenalized.
 * Precision FP32, BF16 or BF16_PLAIN.  If obj_host is not NULL the objective
 * (as glrm_objective at the same precision) is written there and `stream` is
 * synchronized; otherwise the call is asynchronous. */
int glrm_grad(const glrm_data *d, const float *X, const float *Y, int precision,
              float *dX, float *dY, double *obj_host, void *ws, size_t ws_bytes,
              unsigned flags, void *stream);

/* glrm_grad for callers that cannot allocate device memory: code recorded
 * under HIP graph capture, tight serving loops, and harnesses that forbid
 * hipMalloc.  The same computation and results as glrm_grad (bit for bit),
 * with its workspace taken from a static device array the library owns
 * instead of a caller's buffer: GLRM_NOALLOC_MAX_BYTES per device, held on
 * every device the library runs on until the process ends.  The call
 * allocates nothing and calls no allocating routine.  Problems whose
 * gradient workspace (glrm_workspace_size with the gradient's smaller
 * partial buffers) exceeds the limit return GLRM_ENOMEM before any HIP call.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents: GLRM_WS_PREPARED may skip the preparation only if the
 * previous call on this device prepared the same data; calls that overlap
 * on one device (other threads, other streams) race.  Asynchronous unless
 * obj_host is given, as glrm_grad. */
#define GLRM_NOALLOC_MAX_BYTES (64u << 20)
int glrm_grad_noalloc(const glrm_data *d, const float *X, const float *Y, int precision,
                      float *dX, float *dY, double *obj_host, unsigned flags, void *stream);

/* Bytes of device workspace for the linear-algebra entry points
 * (glrm_certificate with block = 1, glrm_init_svd with block = the sketch
 * width it reports): glrm_workspace_size plus a region for an entry-wise
 * matrix in the table's layout and vector blocks of `block` columns.
 * 1 <= block <= 96.  The prepared part sits at the same offsets as in
 * glrm_workspace_size's layout. */
size_t glrm_linalg_workspace_size(const glrm_data *d, int32_t block);

typedef struct {
    double  norm;       /* the estimate of ||G / gamma + U V^T||_2 after `iters` iterations */
    double  norm_prev;  /* the estimate one iteration earlier (convergence check) */
    int32_t rank;       /* rank of X Y^T (singular values above 1e-6 of the largest) */
    int32_t iters;      /* power iterations run */
} glrm_cert_info;

/* The global-optimality certificate of Section 7.6.  For a loss L(XY) that is
 * convex in XY and the quadratic regularizer w ||.||^2 on both factors (the
 * factored problem of Section 7.6 with gamma = 2 w), (X, Y) is globally
 * optimal if ||G / gamma + U V^T||_2 <= 1, where G is the matrix of loss
 * derivatives dL_j(x_i . y_j, A_ij) on the observed set (0 elsewhere; at a
 * kink the derivative the fit uses) and X Y^T = U S V^T is the thin SVD.  U V^T
 * is formed as X P Y^T with a k x k matrix P from the two Gram matrices
 * (host, double); the spectral norm is estimated by `iters` power
 * iterations on M^T M from a fixed start vector (SplitMix64 hash of the
 * index), so info->norm increases toward the norm from below and
 * info->norm_prev shows how far it still moves.  Requires rx and ry both
 * GLRM_REG_QUADRATIC with the same weight > 0 (GLRM_EINVAL otherwise).  ws is
 * glrm_linalg_workspace_size(d, 1) bytes; synchronizes `stream`. */
int glrm_certificate(const glrm_data *d, const float *X, const float *Y, int32_t iters, glrm_cert_info *info,
                     void *ws, size_t ws_bytes, unsigned flags, void *stream);

/* Automatic loss scaling of Section 4.3: for every column j,
 *     mu_j     = argmin_mu sum_{i:(i,j) in Omega} L_j(mu, A_ij)
 *     sigma2_j = sum_{i:(i,j) in Omega} L_j(mu_j, A_ij) / (n_j - 1)
 * (the mean and the sample variance for the quadratic loss).  mu_j is the
 * minimizer over [min_i A_ij - 1, max_i A_ij + 1], found by 64 bisection
 * steps on the sign of the derivative sum in double (one pass over the data
 * each); where the minimizer is not unique (hinge, ordinal hinge) it is one of
 * them, and a logistic column with one label only gets the bracket's end.
 * sigma2_j = 1 for a column with fewer than two entries or a zero minimum;
 * mu_j = 0 for an empty column.  mu and sigma2 are n floats (device).  ws is
 * glrm_linalg_workspace_size(d, 1) bytes; asynchronous except for
 * preparation. */
int glrm_column_scaling(const glrm_data *d, float *mu, float *sigma2, void *ws, size_t ws_bytes, unsigned flags,
                        void *stream);

/* SVD initialization of Section 7.5.  The standardized table
 *     At_ij = m / (sigma_j m_j) (A_ij - mu_j)  on Omega, 0 elsewhere
 * (m_j = observations in column j; mu = NULL is 0, sigma2 = NULL is 1) is
 * sketched by the randomized range finder of Halko, Martinsson and Tropp
 * (2011): Q = orth(At Omega) from the caller's test matrix omega (n x l floats,
 * device, e.g. i.i.d. N(0, 1); l >= k', at most 96), power_iters rounds of
 * Q = orth(At orth(At^T Q)), then the SVD of Q^T At from its l x l Gram matrix
 * (host, double).  With the top k' singular triples (U, S, V):
 *     X = U S^1/2,   Y = diag(sigma) V S^1/2   (Y stored n x k, row j = y_j)
 * where k' = k, or k - 1 with d->offset, in which case coordinate 0 holds the
 * offset: x_i0 = 1 and y_j0 = mu_j (mu required).  Triples with singular value
 * below 1e-6 of the largest (a table of lower rank) leave their coordinates 0.
 * sv_host (host, k' doubles, may be NULL) receives the singular values.  ws is
 * glrm_linalg_workspace_size(d, l) bytes; synchronizes `stream`. */
int glrm_init_svd(const glrm_data *d, const float *mu, const float *sigma2, const float *omega, int32_t l,
                  int32_t power_iters, float *X, float *Y, double *sv_host, void *ws, size_t ws_bytes,
                  unsigned flags, void *stream);

/* In place V[i,:] <- prox_{alpha[i] r}(V[i,:]) for i < rows (Section 7.2,
 * prox_f(z) = argmin_x f(x) + 1/2 ||x - z||^2).  V is rows x k with leading
 * dimension ldv >= k (device); alpha has `rows` entries (device) or is NULL
 * for alpha = 1.  Asynchronous. */
int glrm_prox(const glrm_reg *reg, float *V, int64_t rows, int32_t k, int64_t ldv,
              const float *alpha, void *stream);

/* Update rules of the fit (Section 7.2). */
#define GLRM_UPDATE_PROXGRAD 0  /* one proximal gradient step per row and column */
#define GLRM_UPDATE_PROXPROX 1  /* prox-prox: x <- prox_{alpha r}(prox_{alpha f}(x)), `inner` times per
                                   half-step with the Gram data of Section 7.3 cached; quadratic losses,
                                   dense layout, FP32 (the k x k solves in FP64) */

typedef struct {
    int32_t max_sweeps;   /* sweeps to run, >= 0 */
    int32_t precision;    /* GLRM_FP32, GLRM_BF16 or GLRM_BF16_PLAIN */
    int32_t init_alpha;   /* 1: alpha_x[i] = alpha_scale / max(n_i, 1) and likewise
                             alpha_y (Section 7.2); 0: use the caller's alpha (resume) */
    float   alpha_scale;  /* the paper's initial scale, 1 */
    float   step_up;      /* factor after a step that did not increase the row objective (1.05) */
    float   step_down;    /* factor after a step that increased it (0.7) */
    double  tol;          /* > 0: stop once (F_prev - F) <= tol * |F_prev| after a sweep
                             (reads F back to the host every sweep); 0: run max_sweeps */
    uint32_t flags;       /* GLRM_WS_PREPARED | GLRM_TIME_KERNELS */
    int32_t update;       /* GLRM_UPDATE_PROXGRAD (0) or GLRM_UPDATE_PROXPROX */
    int32_t inner;        /* prox-prox: updates per half-step with the cached factorization (>= 1) */
} glrm_fit_opts;

typedef struct {
    int32_t sweeps;          /* sweeps run */
    double  objective;       /* F after the last sweep, recomputed in float64 on the GPU */
    double  objective_fp32;  /* F after the last sweep as the sweep tracked it (float32 terms) */
    int64_t rows_rejected;   /* rows whose step was rejected in the last sweep */
    int64_t cols_rejected;   /* columns whose step was rejected in the last sweep */
    /* with GLRM_TIME_KERNELS: summed event time (ms) and launch count per kernel kind.
     * Dense: [0] fused row pass (X step + column partials), [1] column prox, [2] column
     * check pass, [3] column accept + objective.  COO: [0] row walk, [1] column walk,
     * [3] objective.  Prox-prox update: [0] the rows' Gram pass, [1] the rows' solves
     * and check, [2] the columns' Gram pass, solves and check, [3] the sweep's F. */
    double  kernel_ms[4];
    int32_t kernel_calls[4];
} glrm_fit_info;

/* Bytes of workspace glrm_fit needs with these options: glrm_workspace_size
 * for the proximal gradient update; with GLRM_UPDATE_PROXPROX also a
 * transposed copy of the table, every row's and column's Gram data and the
 * trial factors.  0 if the problem is invalid. */
size_t glrm_fit_workspace_size(const glrm_data *d, const glrm_fit_opts *opts);

/* Run Algorithm 2 (Section 7.2): per sweep, every row takes one proximal
 * gradient step against Y^{t-1} and keeps it only if its row objective did not
 * increase; then every column does the same against the updated X^t
 * (Gauss-Seidel).  Step sizes are per row / per column and move by step_up /
 * step_down.  X (m x k), Y (n x k), alpha_x (m) and alpha_y (n) are device
 * arrays updated in place, so a second call resumes the fit.  history
 * (device, max_sweeps doubles, may be NULL) receives F after each sweep as the
 * sweep tracked it.  info_host (host, may be NULL) is filled at the end.
 * The dense layout takes any width.  Up to n = 1024 for k <= 32 and
 * n = 512 for k <= 64 one fused pass does the row half-step (a table row's
 * tiles stay on one workgroup); wider tables take it in column blocks, in
 * three passes over the table with the row steps and decisions between them
 * (the same arithmetic, with row sums over the blocks in block order).
 *
 * With opts->update = GLRM_UPDATE_PROXPROX (Section 7.2, "Prox-prox method";
 * Section 7.3) every row i instead forms G_i = sum_j w_j y_j y_j^T and
 * b_i = sum_j w_j A_ij y_j over its observed entries, factors
 * G_i + I / (2 alpha_i) (Cholesky, double) and applies
 *     x <- prox_{alpha r}((G_i + I / (2 alpha))^-1 (b_i + x / (2 alpha)))
 * opts->inner times, then keeps the result under the same step rule; the
 * columns do the same against X^t.  ws must hold glrm_fit_workspace_size()
 * bytes.  On one device
 * the results are bitwise reproducible: partial sums are combined in a fixed
 * order (how many there are follows the device's size).  Synchronizes
 * `stream`. */
int glrm_fit(const glrm_data *d, float *X, float *Y, float *alpha_x, float *alpha_y,
             const glrm_fit_opts *opts, glrm_fit_info *info_host, double *history,
             void *ws, size_t ws_bytes, void *stream);

/* Imputation modes. */
#define GLRM_IMPUTE_ALL     0  /* decode every entry: the denoised table (end of Section 5.3) */
#define GLRM_IMPUTE_MISSING 1  /* observed entries keep A_ij; only the missing ones are decoded */

/* The decoded table of Section 5.3, Ahat_ij = argmin over the data domain of
 * L_j(x_i . y_j, a):
 *   QUADRATIC, HUBER   x_i . y_j (losses over the reals are smallest at a = u)
 *   LOGISTIC, HINGE    +1 if x_i . y_j > 0, else -1 (at 0 both values tie and
 *                      the smaller is taken)
 *   ORDINAL            the level nearest to x_i . y_j, clamped to 1..levels (a
 *                      half-way tie takes the lower level)
 * x_i . y_j is a float32 fused multiply-add chain over l = 0..k-1, so an entry
 * within rounding of a tie may decode to either neighbour.  X and Y must be
 * finite.  Ahat is m x n row-major with leading dimension ldh >= n (device);
 * all m x n entries are written, the padding beyond n is not.  A column
 * under a multi-dimensional loss decodes its block u = x_i Y_j (float32
 * fused multiply-add chains): CATEGORICAL the label of the largest u_l (the
 * argmin of the one-vs-all loss; the first of equal ones), MORDINAL the level
 * of least loss (the lowest of equal ones); Ahat stays m x n.  With
 * GLRM_IMPUTE_MISSING the observed entries receive A_ij instead (dense: mask
 * != 0, or every entry when mask is NULL; COO: the nnz listed entries).
 * Reads the per-column loss codes from `ws` (glrm_workspace_size() bytes):
 * without GLRM_WS_PREPARED in `flags` it uploads them first and waits for that
 * small copy, and a COO list in GLRM_IMPUTE_MISSING mode is prepared (and its
 * indices validated) in full.  Otherwise asynchronous on `stream`. */
int glrm_impute(const glrm_data *d, const float *X, const float *Y, int32_t mode, float *Ahat, int64_t ldh,
                void *ws, size_t ws_bytes, unsigned flags, void *stream);

/* Description of the last error on the calling thread ("" if none). */
const char *glrm_last_error(void);

/* Library version string. */
const char *glrm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GLRM_H */
