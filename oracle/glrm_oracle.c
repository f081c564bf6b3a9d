/*
 * Plain FP64 CPU oracle for the alternating proximal-gradient fit of a
 * generalized low rank model (Udell, Horn, Zadeh, Boyd: "Generalized Low Rank
 * Models", arXiv 1410.0342).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * Everything is double precision, sequential, and walks only the observed
 * entries, in the order rows → entries of the row.  No blocking, fusion or
 * reordering beyond what the paper's definitions state.
 *
 * Problem (eq. gpca, Section 4; abstract form eq. apca, Section 5):
 *     minimize  sum_{(i,j) in Omega} L_ij(x_i . y_j, A_ij)
 *               + sum_i r(x_i) + sum_j rt(y_j)
 * X is m x k (row x_i), Y is stored n x k (row j holds the paper's column y_j).
 *
 * The observed set is handed over as a row-compressed list of entries
 * (row_ptr / col / val / ecode, ecode = index into the loss table).  The
 * column half-step is the row half-step on the transposed problem, which is
 * exactly how Section 7.2 defines it: swap the roles of X and Y, use rt for r,
 * transpose every matrix argument.  The caller builds the transposed list.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

enum { OR_QUAD = 0, OR_HUBER = 1, OR_LOGISTIC = 2, OR_HINGE = 3, OR_ORDINAL = 4 };
enum { OR_RZERO = 0, OR_RQUAD = 1, OR_RL1 = 2, OR_RNONNEG = 3 };

typedef struct {
    int32_t kind;
    int32_t levels;   /* ordinal: number of levels d (data in 1..d) */
    double param;     /* Huber: threshold delta */
} oracle_loss_t;

typedef struct {
    int64_t m, n;                 /* rows of the updated factor, rows of the fixed factor */
    int32_t k;
    const int64_t *row_ptr;       /* m+1 */
    const int32_t *col;           /* nnz, index into the fixed factor */
    const double *val;            /* nnz, A_ij */
    const uint8_t *ecode;         /* nnz, loss of the entry (its column's loss) */
    const oracle_loss_t *losses;  /* table */
    const double *ew;             /* nnz, weight of the entry's loss (its column's), or NULL for 1 */
} oracle_problem_t;

/* the weight of entry e: the scaled losses L_ij / sigma_j^2 of eq. sgpca (Section 4.3) */
static double ew(const oracle_problem_t *P, int64_t e) { return P->ew ? P->ew[e] : 1.0; }

static double pos(double t) { return t > 0.0 ? t : 0.0; }

/* ---- losses, value (Section 4 and Section 5.2) ----------------------- */
double oracle_loss(const oracle_loss_t *L, double u, double a)
{
    switch (L->kind) {
    case OR_QUAD:          /* (a-u)^2, eq. qpca */
        return (a - u) * (a - u);
    case OR_HUBER: {       /* huber(u-a): half r^2 inside the threshold, linear outside */
        double r = u - a, d = L->param, ar = fabs(r);
        return ar <= d ? 0.5 * r * r : d * ar - 0.5 * d * d;
    }
    case OR_LOGISTIC: {    /* log(1 + exp(-a u)), written without overflow */
        double t = -a * u;
        return pos(t) + log1p(exp(-fabs(t)));
    }
    case OR_HINGE:         /* (1 - a u)_+ */
        return pos(1.0 - a * u);
    case OR_ORDINAL: {     /* eq. ord-pca: one hinge per level below and above a */
        double s = 0.0;
        for (int lv = 1; lv <= L->levels; ++lv) {
            if ((double)lv < a) s += pos(1.0 - u + (double)lv);
            else if ((double)lv > a) s += pos(1.0 + u - (double)lv);
        }
        return s;
    }
    }
    return NAN;
}

/* ---- losses, derivative in u (a subgradient at kinks, Section 7.2 gradient
 * method: any subgradient may be used; the strict-inequality branch is taken,
 * so a kink contributes 0) --------------------------------------------------- */
double oracle_dloss(const oracle_loss_t *L, double u, double a)
{
    switch (L->kind) {
    case OR_QUAD:
        return 2.0 * (u - a);
    case OR_HUBER: {
        double r = u - a, d = L->param;
        return r > d ? d : (r < -d ? -d : r);
    }
    case OR_LOGISTIC:      /* d/du log(1+exp(-au)) = -a / (1 + exp(a u)) */
        return -a / (1.0 + exp(a * u));
    case OR_HINGE:
        return (a * u < 1.0) ? -a : 0.0;
    case OR_ORDINAL: {
        double g = 0.0;
        for (int lv = 1; lv <= L->levels; ++lv) {
            if ((double)lv < a) { if (1.0 - u + (double)lv > 0.0) g -= 1.0; }
            else if ((double)lv > a) { if (1.0 + u - (double)lv > 0.0) g += 1.0; }
        }
        return g;
    }
    }
    return NAN;
}

/* ---- regularizers (Section 3) and their proximal operators (Section 7.2,
 * prox_f(z) = argmin_x f(x) + 1/2 ||x - z||^2).  `offset` applies the offset
 * of Section 3.3 to coordinate 0: 1 = r'(x) = r(x_2..) plus the indicator of
 * x_1 = 1 (the rows of X), 2 = rt'(y) = rt(y_2..) (the columns of Y); 0 = none. */
double oracle_reg(int32_t kind, double w, int32_t offset, const double *x, int32_t k)
{
    double s = 0.0;
    int c0 = 0;
    if (offset) {
        if (offset == 1 && x[0] != 1.0) return INFINITY;
        c0 = 1;
    }
    switch (kind) {
    case OR_RZERO: return 0.0;
    case OR_RQUAD: for (int c = c0; c < k; ++c) s += x[c] * x[c]; return w * s;
    case OR_RL1:   for (int c = c0; c < k; ++c) s += fabs(x[c]); return w * s;
    case OR_RNONNEG:
        for (int c = c0; c < k; ++c) if (x[c] < 0.0) return INFINITY;
        return 0.0;
    }
    return NAN;
}

void oracle_prox(int32_t kind, double w, int32_t offset, double alpha, double *v, int32_t k)
{
    int c0 = 0;
    if (offset) {
        if (offset == 1) v[0] = 1.0;   /* projection onto {x_1 = 1} */
        c0 = 1;                         /* offset 2: unpenalized, unchanged */
    }
    for (int c = c0; c < k; ++c) {
        switch (kind) {
        case OR_RZERO: break;
        case OR_RQUAD: v[c] = v[c] / (1.0 + 2.0 * alpha * w); break;
        case OR_RL1: {
            double t = fabs(v[c]) - alpha * w;
            v[c] = t > 0.0 ? (v[c] > 0.0 ? t : -t) : 0.0;
            break;
        }
        case OR_RNONNEG: v[c] = v[c] > 0.0 ? v[c] : 0.0; break;
        }
    }
}

/* The minimum-norm element of the subdifferential of r at x, coordinate by
 * coordinate (every r here is a sum over coordinates): the projection of 0
 * onto the interval of subgradients.  quadratic {2 w x}; l1 {w sign x}, and
 * [-w, w] at 0, so 0; nonnegative {0} for x > 0 and (-inf, 0] at 0, so 0;
 * none {0}.  Outside r's domain (r = +inf: x < 0 under the nonnegative
 * constraint, x_1 != 1 under the offset of the rows of X) there is no
 * subgradient and the coordinate gets NaN.  The offset coordinate is
 * otherwise unpenalized: 0. */
void oracle_reg_subgrad(int32_t kind, double w, int32_t offset, const double *x, int32_t k, double *g)
{
    int c0 = 0;
    if (offset) {
        g[0] = (offset == 1 && x[0] != 1.0) ? NAN : 0.0;
        c0 = 1;
    }
    for (int c = c0; c < k; ++c) {
        switch (kind) {
        case OR_RQUAD: g[c] = 2.0 * w * x[c]; break;
        case OR_RL1: g[c] = x[c] > 0.0 ? w : (x[c] < 0.0 ? -w : 0.0); break;
        case OR_RNONNEG: g[c] = x[c] < 0.0 ? NAN : 0.0; break;
        default: g[c] = 0.0; break;
        }
    }
}

static double dot(const double *a, const double *b, int32_t k)
{
    double s = 0.0;
    for (int c = 0; c < k; ++c) s += a[c] * b[c];
    return s;
}

/* Loss part of one row's objective: sum over the row's observed entries. */
static double row_loss(const oracle_problem_t *P, int64_t i, const double *u, const double *V)
{
    double f = 0.0;
    for (int64_t e = P->row_ptr[i]; e < P->row_ptr[i + 1]; ++e)
        f += ew(P, e) * oracle_loss(&P->losses[P->ecode[e]], dot(u, V + (int64_t)P->col[e] * P->k, P->k), P->val[e]);
    return f;
}

/* Sum of the loss over all observed entries (the first term of eq. gpca). */
double oracle_loss_sum(const oracle_problem_t *P, const double *U, const double *V)
{
    double s = 0.0;
    for (int64_t i = 0; i < P->m; ++i) s += row_loss(P, i, U + i * P->k, V);
    return s;
}

/* Gradient of the loss sum with respect to the rows of U:
 * dU_i = sum_j dL(u_i . v_j, A_ij) v_j.  Calling it on the transposed problem
 * with the factors swapped gives the gradient with respect to Y. */
void oracle_loss_grad_rows(const oracle_problem_t *P, const double *U, const double *V, double *dU)
{
    const int32_t k = P->k;
    for (int64_t i = 0; i < P->m; ++i) {
        double *g = dU + i * k;
        for (int c = 0; c < k; ++c) g[c] = 0.0;
        for (int64_t e = P->row_ptr[i]; e < P->row_ptr[i + 1]; ++e) {
            const double *v = V + (int64_t)P->col[e] * k;
            double d = ew(P, e) * oracle_dloss(&P->losses[P->ecode[e]], dot(U + i * k, v, k), P->val[e]);
            for (int c = 0; c < k; ++c) g[c] += d * v[c];
        }
    }
}

/* The loss derivative of every observed entry, dL(u_i . v_j, A_ij), in the
 * order of the list (the matrix G of Section 7.6 on the observed set). */
void oracle_dloss_entries(const oracle_problem_t *P, const double *U, const double *V, double *out)
{
    const int32_t k = P->k;
    for (int64_t i = 0; i < P->m; ++i)
        for (int64_t e = P->row_ptr[i]; e < P->row_ptr[i + 1]; ++e)
            out[e] = ew(P, e) * oracle_dloss(&P->losses[P->ecode[e]], dot(U + i * k, V + (int64_t)P->col[e] * k, k), P->val[e]);
}

/* Sum of the absolute terms of that gradient, dU_i = sum_j |dL(u_i . v_j, A_ij)| |v_j|
 * (coordinate-wise).  Not part of the method: it scales the rounding bound
 * of a gradient computed in finite precision, which the tests use to tell a
 * decision that rounding may flip from one that it cannot. */
void oracle_loss_grad_abs_rows(const oracle_problem_t *P, const double *U, const double *V, double *dU)
{
    const int32_t k = P->k;
    for (int64_t i = 0; i < P->m; ++i) {
        double *g = dU + i * k;
        for (int c = 0; c < k; ++c) g[c] = 0.0;
        for (int64_t e = P->row_ptr[i]; e < P->row_ptr[i + 1]; ++e) {
            const double *v = V + (int64_t)P->col[e] * k;
            double d = ew(P, e) * fabs(oracle_dloss(&P->losses[P->ecode[e]], dot(U + i * k, v, k), P->val[e]));
            for (int c = 0; c < k; ++c) g[c] += d * fabs(v[c]);
        }
    }
}

/* Sum of the squared terms of that gradient, dU_i = sum_j (dL(u_i . v_j, A_ij) v_j)^2
 * (coordinate-wise): independent rounding errors of the terms add in
 * quadrature, so its square root scales their typical sum.  Test use only. */
void oracle_loss_grad_sq_rows(const oracle_problem_t *P, const double *U, const double *V, double *dU)
{
    const int32_t k = P->k;
    for (int64_t i = 0; i < P->m; ++i) {
        double *g = dU + i * k;
        for (int c = 0; c < k; ++c) g[c] = 0.0;
        for (int64_t e = P->row_ptr[i]; e < P->row_ptr[i + 1]; ++e) {
            const double *v = V + (int64_t)P->col[e] * k;
            double d = ew(P, e) * oracle_dloss(&P->losses[P->ecode[e]], dot(U + i * k, v, k), P->val[e]);
            for (int c = 0; c < k; ++c) g[c] += (d * v[c]) * (d * v[c]);
        }
    }
}

/*
 * One half-step of Algorithm 2 with the proximal gradient update and the
 * per-row step-size rule of Section 7.2 ("Choosing a step size"):
 *   f    = sum_j L(u_i . v_j, A_ij) + r(u_i)
 *   g    = sum_j dL(u_i . v_j, A_ij) v_j
 *   u+   = prox_{alpha_i r}(u_i - alpha_i g)
 *   f+   = sum_j L(u+ . v_j, A_ij) + r(u+)
 *   (f+ = +inf when u+ has a non-finite coordinate)
 *   f+ <= f : keep u+ and multiply alpha_i by step_up
 *   else    : keep u_i and multiply alpha_i by step_down
 * Rows are independent.  Returns the number of rejected rows.  f_old / f_new
 * (length m) receive f and f+ when not NULL; accepted receives the decision.
 */
int64_t oracle_half_step(const oracle_problem_t *P, double *U, const double *V, double *alpha,
                         int32_t reg_kind, double reg_w, int32_t reg_offset, double step_up, double step_down,
                         double *f_old, double *f_new, uint8_t *accepted, double *scratch_2k)
{
    const int32_t k = P->k;
    double *g = scratch_2k, *up = scratch_2k + k;
    int64_t rejected = 0;
    for (int64_t i = 0; i < P->m; ++i) {
        double *u = U + i * k;
        double f = row_loss(P, i, u, V) + oracle_reg(reg_kind, reg_w, reg_offset, u, k);
        for (int c = 0; c < k; ++c) g[c] = 0.0;
        for (int64_t e = P->row_ptr[i]; e < P->row_ptr[i + 1]; ++e) {
            const double *v = V + (int64_t)P->col[e] * k;
            double d = ew(P, e) * oracle_dloss(&P->losses[P->ecode[e]], dot(u, v, k), P->val[e]);
            for (int c = 0; c < k; ++c) g[c] += d * v[c];
        }
        for (int c = 0; c < k; ++c) up[c] = u[c] - alpha[i] * g[c];
        oracle_prox(reg_kind, reg_w, reg_offset, alpha[i], up, k);
        double fp = row_loss(P, i, up, V) + oracle_reg(reg_kind, reg_w, reg_offset, up, k);
        /* the factors range over the reals (Section 2.1): a trial point with an
         * infinite or NaN coordinate (a step size that overflowed) is outside
         * the problem's domain, so its objective counts as +inf */
        for (int c = 0; c < k; ++c)
            if (!isfinite(up[c])) fp = INFINITY;
        int acc = (fp <= f);
        if (acc) {
            for (int c = 0; c < k; ++c) u[c] = up[c];
            alpha[i] *= step_up;
        } else {
            alpha[i] *= step_down;
            ++rejected;
        }
        if (f_old) f_old[i] = f;
        if (f_new) f_new[i] = fp;
        if (accepted) accepted[i] = (uint8_t)acc;
    }
    return rejected;
}

/* ---- the prox-prox update for quadratic losses (Sections 7.2 and 7.3) -------
 * For f_i(x) = sum_j w_j (A_ij - x . v_j)^2 over row i's observed entries, with
 * G_i = sum_j w_j v_j v_j^T and b_i = sum_j w_j A_ij v_j:
 *     prox_{alpha f_i}(x) = argmin_z f_i(z) + 1/(2 alpha) ||z - x||^2
 *                         = (G_i + I / (2 alpha))^-1 (b_i + x / (2 alpha)),
 * and the update is x <- prox_{alpha r}(prox_{alpha f_i}(x)), applied `inner`
 * times with Y fixed (the factorization is the same each time).  The step
 * rule is the one of the gradient step: keep the result only if the row
 * objective did not increase, and move alpha_i by step_up / step_down.
 * (The paper prints (G + I/alpha)^-1 (A Y^T + X/alpha); the factors 2 above
 * follow from the loss (A - u)^2 and the prox's 1/2 ||.||^2.) */
static void cholesky_solve(int k, double *M, double *rhs)
{
    /* M (k x k, row-major, SPD) = L L^T in place (lower), then rhs <- M^-1 rhs */
    for (int j = 0; j < k; ++j) {
        double d = M[j * k + j];
        for (int l = 0; l < j; ++l) d -= M[j * k + l] * M[j * k + l];
        d = sqrt(d);
        M[j * k + j] = d;
        for (int i = j + 1; i < k; ++i) {
            double s = M[i * k + j];
            for (int l = 0; l < j; ++l) s -= M[i * k + l] * M[j * k + l];
            M[i * k + j] = s / d;
        }
    }
    for (int j = 0; j < k; ++j) {       /* L y = rhs */
        double s = rhs[j];
        for (int l = 0; l < j; ++l) s -= M[j * k + l] * rhs[l];
        rhs[j] = s / M[j * k + j];
    }
    for (int j = k - 1; j >= 0; --j) {  /* L^T x = y */
        double s = rhs[j];
        for (int l = j + 1; l < k; ++l) s -= M[l * k + j] * rhs[l];
        rhs[j] = s / M[j * k + j];
    }
}

int64_t oracle_half_step_proxprox(const oracle_problem_t *P, double *U, const double *V, double *alpha,
                                  int32_t reg_kind, double reg_w, int32_t reg_offset, int32_t inner,
                                  double step_up, double step_down, double *f_old, double *f_new,
                                  uint8_t *accepted, double *trial, double *scratch)
{
    const int32_t k = P->k;
    double *G = scratch, *M = G + k * k, *b = M + k * k, *x = b + k, *rhs = x + k;
    int64_t rejected = 0;
    for (int64_t i = 0; i < P->m; ++i) {
        double *u = U + i * k;
        for (int c = 0; c < k * k; ++c) G[c] = 0.0;
        for (int c = 0; c < k; ++c) b[c] = 0.0;
        for (int64_t e = P->row_ptr[i]; e < P->row_ptr[i + 1]; ++e) {
            const double *v = V + (int64_t)P->col[e] * k, w = ew(P, e);
            for (int r = 0; r < k; ++r) {
                b[r] += w * P->val[e] * v[r];
                for (int c = 0; c < k; ++c) G[r * k + c] += w * v[r] * v[c];
            }
        }
        const double h = 1.0 / (2.0 * alpha[i]);
        for (int c = 0; c < k; ++c) x[c] = u[c];
        for (int q = 0; q < inner; ++q) {
            for (int c = 0; c < k * k; ++c) M[c] = G[c];
            for (int c = 0; c < k; ++c) { M[c * k + c] += h; rhs[c] = b[c] + h * x[c]; }
            cholesky_solve(k, M, rhs);
            for (int c = 0; c < k; ++c) x[c] = rhs[c];
            oracle_prox(reg_kind, reg_w, reg_offset, alpha[i], x, k);
        }
        const double f = row_loss(P, i, u, V) + oracle_reg(reg_kind, reg_w, reg_offset, u, k);
        double fp = row_loss(P, i, x, V) + oracle_reg(reg_kind, reg_w, reg_offset, x, k);
        for (int c = 0; c < k; ++c)
            if (!isfinite(x[c])) fp = INFINITY;
        const int acc = (fp <= f);
        if (trial)
            for (int c = 0; c < k; ++c) trial[i * k + c] = x[c];
        if (acc) {
            for (int c = 0; c < k; ++c) u[c] = x[c];
            alpha[i] *= step_up;
        } else {
            alpha[i] *= step_down;
            ++rejected;
        }
        if (f_old) f_old[i] = f;
        if (f_new) f_new[i] = fp;
        if (accepted) accepted[i] = (uint8_t)acc;
    }
    return rejected;
}

/* Initial step sizes (Section 7.2): alpha_i = s / n_i, n_i the number of
 * observations in row i; an empty row takes s. */
void oracle_init_alpha(const oracle_problem_t *P, double s, double *alpha)
{
    for (int64_t i = 0; i < P->m; ++i) {
        int64_t ni = P->row_ptr[i + 1] - P->row_ptr[i];
        alpha[i] = s / (double)(ni > 0 ? ni : 1);
    }
}

/* Sum of r over the rows of U (the regularizer terms of eq. gpca). */
double oracle_reg_sum(int32_t kind, double w, int32_t offset, const double *U, int64_t rows, int32_t k)
{
    double s = 0.0;
    for (int64_t i = 0; i < rows; ++i) s += oracle_reg(kind, w, offset, U + i * k, k);
    return s;
}

/* The full objective of eq. gpca: loss over the observed entries plus both
 * regularizer sums.  P is the row view (U = X, V = Y). */
double oracle_objective(const oracle_problem_t *P, const double *X, const double *Y,
                        int32_t rx_kind, double rx_w, int32_t ry_kind, double ry_w, int32_t offset)
{
    return oracle_loss_sum(P, X, Y) + oracle_reg_sum(rx_kind, rx_w, offset ? 1 : 0, X, P->m, P->k)
         + oracle_reg_sum(ry_kind, ry_w, offset ? 2 : 0, Y, P->n, P->k);
}

/* ---- automatic loss scaling (Section 4.3) ----------------------------------
 * On the column view (each "row" is a column of A): for column j,
 *   mu_j     = argmin over mu of f(mu) = sum_e L_j(mu, A_ej)
 *   sigma2_j = f(mu_j) / (n_j - 1).
 * f is convex, so its minimizers are where the subgradient sum changes sign:
 * bisection on the sign of sum_e dL_j(mu, A_ej) over [min A - 1, max A + 1]
 * (which holds a minimizer of every loss here), 200 halvings, to double
 * rounding.  Readings: an empty column takes mu = 0; sigma2 = 1 when n_j < 2
 * or f(mu_j) = 0 (nothing to scale by). */
static double col_loss_at(const oracle_problem_t *C, int64_t j, double mu)
{
    double f = 0.0;
    for (int64_t e = C->row_ptr[j]; e < C->row_ptr[j + 1]; ++e)
        f += oracle_loss(&C->losses[C->ecode[e]], mu, C->val[e]);
    return f;
}

static double col_dloss_at(const oracle_problem_t *C, int64_t j, double mu)
{
    double g = 0.0;
    for (int64_t e = C->row_ptr[j]; e < C->row_ptr[j + 1]; ++e)
        g += oracle_dloss(&C->losses[C->ecode[e]], mu, C->val[e]);
    return g;
}

void oracle_column_loss_at(const oracle_problem_t *C, const double *mu, double *out)
{
    for (int64_t j = 0; j < C->m; ++j) out[j] = col_loss_at(C, j, mu[j]);
}

void oracle_column_scaling(const oracle_problem_t *C, double *mu, double *sigma2)
{
    for (int64_t j = 0; j < C->m; ++j) {
        const int64_t nj = C->row_ptr[j + 1] - C->row_ptr[j];
        if (nj == 0) { mu[j] = 0.0; sigma2[j] = 1.0; continue; }
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t e = C->row_ptr[j]; e < C->row_ptr[j + 1]; ++e) {
            if (C->val[e] < lo) lo = C->val[e];
            if (C->val[e] > hi) hi = C->val[e];
        }
        lo -= 1.0;
        hi += 1.0;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (col_dloss_at(C, j, mid) < 0.0) lo = mid;   /* f still decreasing: the minimum lies above */
            else hi = mid;
        }
        mu[j] = 0.5 * (lo + hi);
        const double S = col_loss_at(C, j, mu[j]);
        sigma2[j] = (nj >= 2 && S > 0.0) ? S / (double)(nj - 1) : 1.0;
    }
}

/* ---- imputation (Section 5.3): the entry of the column's data domain whose
 * loss at u = x_i . y_j is smallest, a_hat = argmin_a L_j(u, a).  The
 * quadratic and Huber losses are defined for every real a and are smallest at
 * a = u, which the paper states as the decoded value for them.  The Boolean
 * losses range over {-1, +1} and the ordinal hinge over {1..levels}: the
 * argmin is taken by evaluating the loss at every value of the domain in
 * increasing order and keeping the first smallest one, so a tie goes to the
 * smaller value. ------------------------------------------------------------- */
double oracle_decode(const oracle_loss_t *L, double u)
{
    switch (L->kind) {
    case OR_QUAD:
    case OR_HUBER:
        return u;
    case OR_LOGISTIC:
    case OR_HINGE:
        return oracle_loss(L, u, 1.0) < oracle_loss(L, u, -1.0) ? 1.0 : -1.0;
    case OR_ORDINAL: {
        double best = 1.0, fbest = oracle_loss(L, u, 1.0);
        for (int lv = 2; lv <= L->levels; ++lv) {
            double f = oracle_loss(L, u, (double)lv);
            if (f < fbest) { fbest = f; best = (double)lv; }
        }
        return best;
    }
    }
    return NAN;
}

/* a_hat for every entry of an m x n matrix of products Z (row-major), column j
 * decoded with losses[col_code[j]]. */
void oracle_decode_matrix(const oracle_loss_t *losses, const uint8_t *col_code, const double *Z,
                          int64_t m, int64_t n, double *out)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            out[i * n + j] = oracle_decode(&losses[col_code[j]], Z[i * n + j]);
}

/* ---- multi-dimensional losses (Section 6) ------------------------------------
 * Feature j of the table has embedding dimension d_j and owns rows
 * fcol[j] .. fcol[j+1]-1 of Y (stored d x k: those rows are the columns of
 * the paper's block Y_j), so u = x_i Y_j has d_j entries (eq. mpca).
 *   categorical, labels 1..d (one-vs-all, Section 6.1), d_j = d:
 *       L(u, a) = (1 - u_a)_+ + sum_{a' != a} (1 + u_a')_+
 *   multi-dimensional ordinal, levels 1..d (eq. ord-mpca), d_j = d - 1:
 *       L(u, a) = sum_{l=1}^{d-1} (1 - s_l(a) u_l)_+,  s_l(a) = +1 if a > l, else -1
 *   (the paper prints the factor as the indicator of a > l; it is read as
 *   this sign, the form under which each term is the SVM that separates the
 *   levels up to l from those above, which is how the paper describes it)
 * Every other kind is the scalar loss of u_0 (d_j = 1).  Feature j's loss is
 * scaled by fw[j] (NULL = 1).  At a kink the derivative takes the
 * strict-inequality branch, as everywhere in this file.  The regularizers
 * r on the rows of X and rt on the columns of every Y_j are the ones of
 * eq. gpca; r~_j(Y_j) is rt summed over the block's columns. */
enum { OR_CATEGORICAL = 5, OR_MORDINAL = 6 };
#define OR_MD_MAXD 1024

typedef struct {
    int64_t rows;                 /* rows of the view: rows of A (row view) or features (feature view) */
    int32_t k;
    const int64_t *row_ptr;       /* rows + 1 */
    const int32_t *other;         /* per entry: its feature (row view) or its row of A (feature view) */
    const double *val;            /* per entry: A_ij */
    const int32_t *fkind, *flev;  /* per feature */
    const double *fpar, *fw;      /* per feature (fw may be NULL) */
    const int64_t *fcol;          /* features + 1 */
} oracle_md_t;

int32_t oracle_md_dim(int32_t kind, int32_t lev)
{
    return kind == OR_CATEGORICAL ? lev : (kind == OR_MORDINAL ? lev - 1 : 1);
}

double oracle_md_loss(int32_t kind, int32_t lev, double par, const double *u, double a)
{
    if (kind == OR_CATEGORICAL) {
        double s = 0.0;
        for (int l = 1; l <= lev; ++l) s += (l == (int)a) ? pos(1.0 - u[l - 1]) : pos(1.0 + u[l - 1]);
        return s;
    }
    if (kind == OR_MORDINAL) {
        double s = 0.0;
        for (int l = 1; l <= lev - 1; ++l) s += pos(1.0 - (a > (double)l ? 1.0 : -1.0) * u[l - 1]);
        return s;
    }
    oracle_loss_t L = {kind, lev, par};
    return oracle_loss(&L, u[0], a);
}

void oracle_md_dloss(int32_t kind, int32_t lev, double par, const double *u, double a, double *g)
{
    if (kind == OR_CATEGORICAL) {
        for (int l = 1; l <= lev; ++l)
            g[l - 1] = (l == (int)a) ? (1.0 - u[l - 1] > 0.0 ? -1.0 : 0.0) : (1.0 + u[l - 1] > 0.0 ? 1.0 : 0.0);
        return;
    }
    if (kind == OR_MORDINAL) {
        for (int l = 1; l <= lev - 1; ++l) {
            const double sg = a > (double)l ? 1.0 : -1.0;
            g[l - 1] = 1.0 - sg * u[l - 1] > 0.0 ? -sg : 0.0;
        }
        return;
    }
    oracle_loss_t L = {kind, lev, par};
    g[0] = oracle_dloss(&L, u[0], a);
}

/* Section 5.3 for a block: argmin over the feature's values of L(u, a),
 * by enumeration of the labels (the first of equal minima). */
double oracle_md_decode(int32_t kind, int32_t lev, double par, const double *u)
{
    if (kind == OR_CATEGORICAL || kind == OR_MORDINAL) {
        double best = 1.0, fbest = oracle_md_loss(kind, lev, par, u, 1.0);
        for (int a = 2; a <= lev; ++a) {
            const double f = oracle_md_loss(kind, lev, par, u, (double)a);
            if (f < fbest) { fbest = f; best = a; }
        }
        return best;
    }
    oracle_loss_t L = {kind, lev, par};
    return oracle_decode(&L, u[0]);
}

static int md_d(const oracle_md_t *P, int64_t j) { return oracle_md_dim(P->fkind[j], P->flev[j]); }
static double md_w(const oracle_md_t *P, int64_t j) { return P->fw ? P->fw[j] : 1.0; }

/* loss of one entry: feature j, value a, row x, block B (d_j rows of k) */
static double md_entry_loss(const oracle_md_t *P, int64_t j, const double *x, const double *B, double a, double *u)
{
    const int d = md_d(P, j);
    for (int l = 0; l < d; ++l) u[l] = dot(x, B + (int64_t)l * P->k, P->k);
    return md_w(P, j) * oracle_md_loss(P->fkind[j], P->flev[j], P->fpar[j], u, a);
}

/* its derivatives with respect to u (scaled by the weight) */
static void md_entry_dloss(const oracle_md_t *P, int64_t j, const double *x, const double *B, double a, double *u,
                           double *g)
{
    const int d = md_d(P, j);
    for (int l = 0; l < d; ++l) u[l] = dot(x, B + (int64_t)l * P->k, P->k);
    oracle_md_dloss(P->fkind[j], P->flev[j], P->fpar[j], u, a, g);
    for (int l = 0; l < d; ++l) g[l] *= md_w(P, j);
}

/* losses of row i (row view) at x against Y */
static double md_row_loss(const oracle_md_t *R, int64_t i, const double *x, const double *Y, double *u)
{
    double f = 0.0;
    for (int64_t e = R->row_ptr[i]; e < R->row_ptr[i + 1]; ++e) {
        const int32_t j = R->other[e];
        f += md_entry_loss(R, j, x, Y + R->fcol[j] * R->k, R->val[e], u);
    }
    return f;
}

/* losses of feature j (feature view) with block B against X */
static double md_feat_loss(const oracle_md_t *F, int64_t j, const double *B, const double *X, double *u)
{
    double f = 0.0;
    for (int64_t e = F->row_ptr[j]; e < F->row_ptr[j + 1]; ++e)
        f += md_entry_loss(F, j, X + (int64_t)F->other[e] * F->k, B, F->val[e], u);
    return f;
}

static double md_block_reg(int32_t kind, double w, int32_t offset, const double *B, int d, int32_t k)
{
    double r = 0.0;
    for (int l = 0; l < d; ++l) r += oracle_reg(kind, w, offset, B + (int64_t)l * k, k);
    return r;
}

/* the objective of eq. mpca, from the row view; nf features */
double oracle_md_objective(const oracle_md_t *R, int64_t nf, const double *X, const double *Y, int32_t rx_kind,
                           double rx_w, int32_t ry_kind, double ry_w, int32_t offset)
{
    double u[OR_MD_MAXD];
    double f = 0.0;
    for (int64_t i = 0; i < R->rows; ++i)
        f += md_row_loss(R, i, X + i * R->k, Y, u) + oracle_reg(rx_kind, rx_w, offset ? 1 : 0, X + i * R->k, R->k);
    f += oracle_reg_sum(ry_kind, ry_w, offset ? 2 : 0, Y, R->fcol[nf], R->k);
    return f;
}

/* loss-part gradients from the row view: dX_i = sum_j (dL/du) Y_j^T and
 * the rows of dY of block j, sum_i x_i^T (dL/du) */
void oracle_md_grad(const oracle_md_t *R, int64_t nf, const double *X, const double *Y, double *dX, double *dY)
{
    const int k = R->k;
    double u[OR_MD_MAXD], g[OR_MD_MAXD];
    for (int64_t t = 0; t < R->rows * k; ++t) dX[t] = 0.0;
    for (int64_t t = 0; t < R->fcol[nf] * k; ++t) dY[t] = 0.0;
    for (int64_t i = 0; i < R->rows; ++i)
        for (int64_t e = R->row_ptr[i]; e < R->row_ptr[i + 1]; ++e) {
            const int32_t j = R->other[e];
            md_entry_dloss(R, j, X + i * k, Y + R->fcol[j] * k, R->val[e], u, g);
            for (int l = 0; l < md_d(R, j); ++l) {
                const double *y = Y + (R->fcol[j] + l) * k;
                double *dy = dY + (R->fcol[j] + l) * k;
                for (int c = 0; c < k; ++c) {
                    dX[i * k + c] += g[l] * y[c];
                    dy[c] += g[l] * X[i * k + c];
                }
            }
        }
}

/* Initial step sizes of Algorithm 2: s over the entries of each row's loss
 * terms (a feature of dimension d_j counts d_j) and s / n_j per feature. */
void oracle_md_init_alpha(const oracle_md_t *R, const oracle_md_t *F, int64_t nf, double s, double *ax, double *af)
{
    for (int64_t i = 0; i < R->rows; ++i) {
        int64_t c = 0;
        for (int64_t e = R->row_ptr[i]; e < R->row_ptr[i + 1]; ++e) c += md_d(R, R->other[e]);
        ax[i] = s / (double)(c > 0 ? c : 1);
    }
    for (int64_t j = 0; j < nf; ++j) {
        const int64_t c = F->row_ptr[j + 1] - F->row_ptr[j];
        af[j] = s / (double)(c > 0 ? c : 1);
    }
}

/* X half-step of Algorithm 2 (proximal gradient step and step rule of
 * Section 7.2) on the row view, in place. */
int64_t oracle_md_half_step_x(const oracle_md_t *R, double *X, const double *Y, double *alpha, int32_t reg_kind,
                              double reg_w, int32_t offset, double step_up, double step_down, double *f_old,
                              double *f_new, uint8_t *accepted)
{
    const int k = R->k;
    double u[OR_MD_MAXD], g[OR_MD_MAXD], gx[64], xp[64];
    int64_t rejected = 0;
    for (int64_t i = 0; i < R->rows; ++i) {
        double *x = X + i * k;
        const double f = md_row_loss(R, i, x, Y, u) + oracle_reg(reg_kind, reg_w, offset, x, k);
        for (int c = 0; c < k; ++c) gx[c] = 0.0;
        for (int64_t e = R->row_ptr[i]; e < R->row_ptr[i + 1]; ++e) {
            const int32_t j = R->other[e];
            md_entry_dloss(R, j, x, Y + R->fcol[j] * k, R->val[e], u, g);
            for (int l = 0; l < md_d(R, j); ++l)
                for (int c = 0; c < k; ++c) gx[c] += g[l] * Y[(R->fcol[j] + l) * k + c];
        }
        for (int c = 0; c < k; ++c) xp[c] = x[c] - alpha[i] * gx[c];
        oracle_prox(reg_kind, reg_w, offset, alpha[i], xp, k);
        double fp = md_row_loss(R, i, xp, Y, u) + oracle_reg(reg_kind, reg_w, offset, xp, k);
        for (int c = 0; c < k; ++c)
            if (!isfinite(xp[c])) fp = INFINITY;
        const int acc = fp <= f;
        if (acc) {
            for (int c = 0; c < k; ++c) x[c] = xp[c];
            alpha[i] *= step_up;
        } else {
            alpha[i] *= step_down;
            ++rejected;
        }
        if (f_old) f_old[i] = f;
        if (f_new) f_new[i] = fp;
        if (accepted) accepted[i] = (uint8_t)acc;
    }
    return rejected;
}

/* Y half-step on the feature view: the block Y_j of feature j takes one
 * proximal gradient step with the feature's one step size and is kept or
 * rejected whole (the column update of Algorithm 2, with Y_j in the place of
 * y_j).  scratch: 2 * OR_MD_MAXD * k doubles. */
int64_t oracle_md_half_step_y(const oracle_md_t *F, double *Y, const double *X, double *alpha, int32_t reg_kind,
                              double reg_w, int32_t offset, double step_up, double step_down, double *f_old,
                              double *f_new, uint8_t *accepted, double *scratch)
{
    const int k = F->k;
    double u[OR_MD_MAXD], g[OR_MD_MAXD];
    double *gb = scratch, *bp = scratch + OR_MD_MAXD * k;
    int64_t rejected = 0;
    for (int64_t j = 0; j < F->rows; ++j) {
        const int d = md_d(F, j);
        double *B = Y + F->fcol[j] * k;
        const double f = md_feat_loss(F, j, B, X, u) + md_block_reg(reg_kind, reg_w, offset, B, d, k);
        for (int t = 0; t < d * k; ++t) gb[t] = 0.0;
        for (int64_t e = F->row_ptr[j]; e < F->row_ptr[j + 1]; ++e) {
            const double *x = X + (int64_t)F->other[e] * k;
            md_entry_dloss(F, j, x, B, F->val[e], u, g);
            for (int l = 0; l < d; ++l)
                for (int c = 0; c < k; ++c) gb[l * k + c] += g[l] * x[c];
        }
        for (int l = 0; l < d; ++l) {
            for (int c = 0; c < k; ++c) bp[l * k + c] = B[l * k + c] - alpha[j] * gb[l * k + c];
            oracle_prox(reg_kind, reg_w, offset, alpha[j], bp + l * k, k);
        }
        double fp = md_feat_loss(F, j, bp, X, u) + md_block_reg(reg_kind, reg_w, offset, bp, d, k);
        for (int t = 0; t < d * k; ++t)
            if (!isfinite(bp[t])) fp = INFINITY;
        const int acc = fp <= f;
        if (acc) {
            for (int t = 0; t < d * k; ++t) B[t] = bp[t];
            alpha[j] *= step_up;
        } else {
            alpha[j] *= step_down;
            ++rejected;
        }
        if (f_old) f_old[j] = f;
        if (f_new) f_new[j] = fp;
        if (accepted) accepted[j] = (uint8_t)acc;
    }
    return rejected;
}

/* Imputation (Section 5.3) of every entry: out is rows x nf */
void oracle_md_impute(const oracle_md_t *R, int64_t nf, const double *X, const double *Y, double *out)
{
    const int k = R->k;
    double u[OR_MD_MAXD];
    for (int64_t i = 0; i < R->rows; ++i)
        for (int64_t j = 0; j < nf; ++j) {
            for (int l = 0; l < md_d(R, j); ++l) u[l] = dot(X + i * k, Y + (R->fcol[j] + l) * k, k);
            out[i * nf + j] = oracle_md_decode(R->fkind[j], R->flev[j], R->fpar[j], u);
        }
}
