// Host side of the C ABI declared in include/glrm.h: argument validation,
// workspace layout, and the sweep driver of Algorithm 2 (Section 7.2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/glrm.h"
#include "glrm_kernels.h"
#include "coo.h"
#include "impute.h"
#include "linalg.h"
#include "proxprox.h"
#include "smallmat.h"

using namespace glrm;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(GLRM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int P_MAX = 1024;    // workgroups (and partials) of the persistent dense fit passes, at most
constexpr int64_t P_BYTES = 64ll << 20;  // ... and the Y-gradient partials within this (256 at least)
constexpr int P_GRAD = 256;    // row chunks of the one-pass loss gradient
constexpr int REG_BLOCKS = 1024; // partials of a regularizer sum (workgroups: four per CU)
constexpr int OBJ64_BLOCKS = 2048;  // workgroups (and partials) of the FP64 objective
constexpr int AUX_SMALL = 16 * LA_MAXB * LA_MAXB;  // doubles of small matrices in the linear-algebra region

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Tiles per wavefront of the gradient pass at kp = 64 (its instances stop at 2).
constexpr int GRAD_TMAX64 = 2;

int kp_of(int k) { return k <= 16 ? 16 : (k <= 32 ? 32 : 64); }

// Tiles per wavefront of the two passes of the fit: the fused row pass runs
// xstep_waves(kp) wavefronts of up to 16 tiles (8 at kp = 64), the trial-column
// pass ycheck_waves(kp) wavefronts of up to 8 tiles.
int tpw_xstep(int64_t ntiles, int kp)
{
    for (int t : {1, 2, 4, 8, 16})
        if ((kp < 64 || t <= 8) && (int64_t)xstep_waves(kp) * t >= ntiles) return t;
    return 0;
}

int tpw_ycheck(int64_t ntiles, int kp)
{
    for (int t : {1, 2, 4, 8})
        if ((int64_t)ycheck_waves(kp) * t >= ntiles) return t;
    return 0;
}

struct Layout {
    int64_t m, n, k, kp, mp, ldp;
    int pmax = 0;               // partial slots of the dense fit passes
    size_t total = 0;
    // offsets
    size_t codes, colw, row_count, col_count, Ap;
    size_t emb_src, emb_thr, emb_kind, blk0, blk1, hpc;   // embedded columns (Section 6)
    size_t feat;                                          // per column of A: block start, kind, levels
    size_t part_dy, part_h, part_hp, part_rowreg, part_rej, part_dx, part_obj;
    size_t ycur_f32, ycur_t32, ycur_hi, ycur_lo, ycur_tb;
    size_t yp_f32, yp_t32, yp_hi, yp_lo, yp_tb;
    size_t Yplus, h_old, ry_plus, ry_old, part_F, part_rejc, stats, istats, regpart, scal, part_obj64;
    size_t coo;            // start of the COO region
    CooLayout cl;
    int64_t cb_grad;       // column blocks of the gradient kernel
    int tpw_grad;
    // dense fits wider than the fused row pass takes: the row half-step in
    // column blocks (tiles per wavefront, blocks, per-block row sums, trial rows)
    bool wide = false;
    int wide_tpw = 0;
    int64_t wide_ncb = 0;
    size_t wd_f = 0, wd_fp = 0, wd_xp = 0, wd_rsum = 0;
    // linear-algebra region (certificate, SVD initialization), when requested
    int aux_b = 0;                       // vector block width
    size_t aux_V = 0, aux_V2 = 0;        // entry-wise matrix (dense: mp x ldp; COO: row and column order)
    size_t aux_m1 = 0, aux_m2 = 0;       // m x aux_b doubles
    size_t aux_n1 = 0, aux_n2 = 0;       // n x aux_b doubles
    size_t aux_part = 0;                 // partial sums
    size_t aux_small = 0;                // AUX_SMALL doubles of small matrices
    size_t aux_cols = 0;                 // 8 n doubles of per-column state
    size_t aux_colout = 0;               // COL_SLOTS n doubles: the column passes' results
    // prox-prox region (dense fits with the prox-prox update)
    bool pp = false;
    int pp_gsz = 0;
    size_t pp_At = 0, pp_gram = 0, pp_gpart = 0, pp_trial = 0, pp_fpart = 0;
    size_t pp_objx = 0, pp_objy = 0, pp_rejx = 0, pp_rejy = 0, pp_fin = 0;

    size_t take(size_t bytes)
    {
        size_t off = total;
        total += round_up((int64_t)bytes, 256);
        return off;
    }
};

// grad_only: the layout of the gradient entry points alone, whose Y-gradient
// partials never exceed P_GRAD rows (the fit's run up to P_MAX).
bool make_layout(const glrm_data *d, Layout &L, bool grad_only = false, int aux_b = 0, bool proxprox = false)
{
    L = Layout();
    L.m = d->m;
    L.n = d->n;
    L.k = d->k;
    L.kp = kp_of(d->k);
    L.mp = round_up(d->m, 16);
    L.ldp = round_up(d->n, 16);
    const int64_t ntiles = L.ldp / 16;
    // the gradient pass: grad_waves(kp) wavefronts of up to 16 tiles (2 at
    // kp = 64); wider tables take several column blocks
    {
        const int tmax = L.kp == 64 ? GRAD_TMAX64 : 16, nw = grad_waves((int)L.kp);
        int t = 1;
        while (t < tmax && (int64_t)nw * t < ntiles) t *= 2;
        L.tpw_grad = t;
        L.cb_grad = (ntiles + nw * t - 1) / (nw * t);
    }
    const int64_t kp = L.kp, ldp = L.ldp, n = L.n, m = L.m;
    if (d->layout == GLRM_DENSE && !grad_only && !proxprox && tpw_xstep(ntiles, (int)kp) == 0) {
        L.wide = true;
        L.wide_tpw = kp == 64 ? 4 : 16;
        const int64_t per = (int64_t)xstep_waves((int)kp) * L.wide_tpw;
        L.wide_ncb = (ntiles + per - 1) / per;
    }
    L.codes = L.take(ldp);
    L.colw = L.take(sizeof(float) * ldp);
    L.emb_src = L.take(sizeof(int32_t) * ldp);
    L.emb_thr = L.take(sizeof(int32_t) * ldp);
    L.emb_kind = L.take(ldp);
    L.blk0 = L.take(sizeof(int32_t) * ldp);
    L.blk1 = L.take(sizeof(int32_t) * ldp);
    L.hpc = L.take(sizeof(float) * ldp);
    L.feat = L.take(sizeof(int32_t) * 3 * ldp);
    L.row_count = L.take(sizeof(int32_t) * m);
    L.col_count = L.take(sizeof(int32_t) * n);
    L.stats = L.take(sizeof(double) * 8);
    L.istats = L.take(sizeof(long long) * 8);
    L.scal = L.take(sizeof(double) * 8);
    L.regpart = L.take(sizeof(double) * 2 * REG_BLOCKS);
    L.part_obj64 = L.take(sizeof(double) * OBJ64_BLOCKS);
    L.ycur_f32 = L.take(sizeof(float) * ldp * kp);
    L.ycur_t32 = L.take(sizeof(float) * ldp * kp);
    L.ycur_hi = L.take(2 * ldp * kp);
    L.ycur_lo = L.take(2 * ldp * kp);
    L.ycur_tb = L.take(2 * ldp * kp);
    L.yp_f32 = L.take(sizeof(float) * ldp * kp);
    L.yp_t32 = L.take(sizeof(float) * ldp * kp);
    L.yp_hi = L.take(2 * ldp * kp);
    L.yp_lo = L.take(2 * ldp * kp);
    L.yp_tb = L.take(2 * ldp * kp);
    L.Yplus = L.take(sizeof(float) * n * L.k);
    L.h_old = L.take(sizeof(float) * n);
    L.ry_plus = L.take(sizeof(float) * n);
    L.ry_old = L.take(sizeof(float) * n);
    const int64_t ya_blocks = (n * kp + 255) / 256;
    L.part_F = L.take(sizeof(double) * ya_blocks);
    L.part_rejc = L.take(sizeof(int32_t) * ya_blocks);
    if (d->layout == GLRM_DENSE) {
        L.Ap = L.take(sizeof(float) * L.mp * ldp);
        L.pmax = grad_only ? P_GRAD
                           : (int)std::clamp<int64_t>(P_BYTES / ((int64_t)sizeof(float) * ldp * kp), 256, P_MAX);
        L.part_dy = L.take(sizeof(float) * L.pmax * ldp * kp);
        L.part_h = L.take(sizeof(float) * L.pmax * ldp);
        L.part_hp = L.take(sizeof(float) * L.pmax * ldp);
        L.part_rowreg = L.take(sizeof(float) * L.pmax);
        L.part_rej = L.take(sizeof(int32_t) * L.pmax);
        const int64_t cbx = std::max<int64_t>(L.cb_grad > 1 ? L.cb_grad : 0, L.wide_ncb);
        L.part_dx = cbx > 0 ? L.take(sizeof(float) * cbx * m * L.k) : 0;
        if (L.wide) {
            L.wd_f = L.take(sizeof(float) * L.wide_ncb * L.mp);
            L.wd_fp = L.take(sizeof(float) * L.wide_ncb * L.mp);
            L.wd_xp = L.take(sizeof(float) * m * L.k);
            L.wd_rsum = L.take(sizeof(float) * 3 * L.mp);
        }
        L.part_obj = L.take(sizeof(double) * P_GRAD * std::max<int64_t>(L.cb_grad, 1));
    } else {
        L.coo = L.take(0);
        coo_layout(d, L.kp, L.cl);
        L.coo = L.take(L.cl.total);
    }
    if (aux_b > 0) {
        const int64_t b = aux_b;
        L.aux_b = aux_b;
        if (d->layout == GLRM_DENSE) {
            L.aux_V = L.take(sizeof(float) * L.mp * ldp);
        } else {
            L.aux_V = L.take(sizeof(float) * std::max<int64_t>(d->nnz, 1));
            L.aux_V2 = L.take(sizeof(float) * std::max<int64_t>(d->nnz, 1));
        }
        L.aux_m1 = L.take(sizeof(double) * m * b);
        L.aux_m2 = L.take(sizeof(double) * m * b);
        L.aux_n1 = L.take(sizeof(double) * n * b);
        L.aux_n2 = L.take(sizeof(double) * n * b);
        const int64_t kb = std::max<int64_t>(kp, b);
        const int64_t parts = std::max<int64_t>({(int64_t)LA_TCHUNKS * n * b,
                                                 (int64_t)tall_tmul_blocks(std::max(m, n)) * kb * kb, 256,
                                                 d->layout == GLRM_DENSE ? col_part_doubles(m, n) : 0});
        L.aux_part = L.take(sizeof(double) * parts);
        L.aux_small = L.take(sizeof(double) * AUX_SMALL);
        L.aux_cols = L.take(sizeof(double) * 8 * n);
        L.aux_colout = L.take(sizeof(double) * COL_SLOTS * n);
    }
    if (proxprox && d->layout == GLRM_DENSE) {
        const int64_t rmax = std::max(m, n);
        L.pp = true;
        L.pp_gsz = pp_gram_floats((int)kp);
        L.pp_At = L.take(sizeof(float) * ldp * L.mp);
        L.pp_gram = L.take(sizeof(float) * round_up(rmax, 16) * L.pp_gsz);
        L.pp_gpart = L.take(sizeof(float) * PP_SPLITS_MAX * round_up(n, 16) * L.pp_gsz);
        L.pp_trial = L.take(sizeof(float) * rmax * L.k);
        L.pp_fpart = L.take(sizeof(float) * 2 * std::max<int64_t>(m, (int64_t)PP_SPLITS_MAX * n));
        L.pp_objx = L.take(sizeof(double) * m);
        L.pp_objy = L.take(sizeof(double) * n);
        L.pp_rejx = L.take(sizeof(int32_t) * m);
        L.pp_rejy = L.take(sizeof(int32_t) * n);
        L.pp_fin = L.take(sizeof(double) * pp_finalize_part_doubles());
    }
    return true;
}

template <typename T>
T *at(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

int validate_data(const glrm_data *d)
{
    if (!d) return fail(GLRM_EINVAL, "data is NULL");
    if (d->m < 1 || d->n < 1) return fail(GLRM_EINVAL, "m and n must be >= 1 (got %lld, %lld)", (long long)d->m, (long long)d->n);
    if (d->m > (int64_t)INT32_MAX || d->n > (int64_t)INT32_MAX) return fail(GLRM_EUNSUPPORTED, "m and n must fit in int32");
    if (d->k < 1) return fail(GLRM_EINVAL, "k must be >= 1 (got %d)", d->k);
    if (d->k > GLRM_MAX_K) return fail(GLRM_EUNSUPPORTED, "k = %d exceeds GLRM_MAX_K = %d", d->k, GLRM_MAX_K);
    if (d->layout == GLRM_DENSE) {
        if (!d->A) return fail(GLRM_EINVAL, "A is NULL");
        if (d->lda < d->n) return fail(GLRM_EINVAL, "lda (%lld) < n (%lld)", (long long)d->lda, (long long)d->n);
    } else if (d->layout == GLRM_COO_ROWSORTED) {
        if (d->nnz < 0) return fail(GLRM_EINVAL, "nnz < 0");
        // an empty observed set needs no arrays
        if (d->nnz > 0 && (!d->A || !d->row || !d->col)) return fail(GLRM_EINVAL, "COO A / row / col is NULL");
        if (d->nnz > (int64_t)INT32_MAX) return fail(GLRM_EUNSUPPORTED, "nnz must fit in int32 for this build");
    } else {
        return fail(GLRM_EINVAL, "unknown layout %d", d->layout);
    }
    if (d->n_losses < 1 || d->n_losses > GLRM_MAX_LOSSES)
        return fail(GLRM_EINVAL, "n_losses must be in 1..%d (got %d)", GLRM_MAX_LOSSES, d->n_losses);
    if (!d->losses) return fail(GLRM_EINVAL, "losses is NULL");
    for (int q = 0; q < d->n_losses; ++q) {
        const glrm_loss &l = d->losses[q];
        if (l.kind < GLRM_LOSS_QUADRATIC || l.kind > GLRM_LOSS_MORDINAL) return fail(GLRM_EINVAL, "loss %d: unknown kind %d", q, l.kind);
        if (l.kind == GLRM_LOSS_HUBER && !(l.param > 0.0f && std::isfinite(l.param)))
            return fail(GLRM_EINVAL, "loss %d: Huber threshold must be finite and > 0", q);
        if (l.kind == GLRM_LOSS_ORDINAL && (l.levels < 2 || l.levels > 1000000))
            return fail(GLRM_EINVAL, "loss %d: ordinal levels must be in 2..1e6", q);
        if ((l.kind == GLRM_LOSS_CATEGORICAL || l.kind == GLRM_LOSS_MORDINAL) && (l.levels < 2 || l.levels > GLRM_MAX_LEVELS))
            return fail(GLRM_EINVAL, "loss %d: a multi-dimensional loss needs 2..%d levels", q, GLRM_MAX_LEVELS);
    }
    if (d->col_loss) {
        for (int64_t j = 0; j < d->n; ++j)
            if (d->col_loss[j] >= d->n_losses) return fail(GLRM_EINVAL, "col_loss[%lld] = %d >= n_losses", (long long)j, d->col_loss[j]);
    }
    if (d->offset != 0 && d->offset != 1) return fail(GLRM_EINVAL, "offset must be 0 or 1 (got %d)", d->offset);
    for (const glrm_reg *r : {&d->rx, &d->ry}) {
        if (r->kind < GLRM_REG_ZERO || r->kind > GLRM_REG_NONNEG) return fail(GLRM_EINVAL, "unknown regularizer kind %d", r->kind);
        if (!(r->weight >= 0.0f) || !std::isfinite(r->weight)) return fail(GLRM_EINVAL, "regularizer weight must be finite and >= 0");
    }
    return GLRM_OK;
}

// ---- multi-dimensional losses (Section 6) ----------------------------------
// A column of A under the categorical or multi-dimensional ordinal loss with
// d levels is a feature of embedding dimension d or d - 1.  Both losses are
// sums of hinge losses (1 - s u_l)_+ over their embedded columns with a sign
// s = +-1 fixed by the value (one-vs-all: s = +1 on the value's own label;
// ordinal: s = +1 on the thresholds below the value), so every pass runs
// unchanged on the embedded table of +-1 entries under the hinge loss, and
// only the column step decides per block (one decision for the block Y_j).
struct Embed {
    bool active = false;
    glrm_data e;                        // the problem over the embedded columns
    std::vector<uint8_t> codes;         // loss code per embedded column
    std::vector<glrm_loss> losses;      // the caller's table (+ a hinge entry)
    std::vector<int32_t> src, thr, blk0, blk1;
    std::vector<uint8_t> kind;
};

bool is_md(int kind) { return kind == GLRM_LOSS_CATEGORICAL || kind == GLRM_LOSS_MORDINAL; }

int md_dim(const glrm_loss &l)
{
    return l.kind == GLRM_LOSS_CATEGORICAL ? l.levels : (l.kind == GLRM_LOSS_MORDINAL ? l.levels - 1 : 1);
}

// Validates d and points *out at the problem the passes run on: d itself, or
// its embedding in E.
int embed(const glrm_data *d, Embed &E, const glrm_data **out)
{
    int rc = validate_data(d);
    if (rc) return rc;
    *out = d;
    E.active = false;
    bool any = false;
    int64_t total = 0;
    for (int64_t j = 0; j < d->n; ++j) {
        const glrm_loss &l = d->losses[d->col_loss ? d->col_loss[j] : 0];
        any = any || is_md(l.kind);
        total += md_dim(l);
    }
    if (!any) return GLRM_OK;
    if (d->layout != GLRM_DENSE) return fail(GLRM_EUNSUPPORTED, "multi-dimensional losses are built for the dense layout");
    if (total > (int64_t)INT32_MAX) return fail(GLRM_EUNSUPPORTED, "the embedded table must have < 2^31 columns");
    E.losses.assign(d->losses, d->losses + d->n_losses);
    int hinge = -1;
    for (int q = 0; q < d->n_losses && hinge < 0; ++q)
        if (d->losses[q].kind == GLRM_LOSS_HINGE) hinge = q;
    if (hinge < 0) {
        if (d->n_losses >= GLRM_MAX_LOSSES)
            return fail(GLRM_EUNSUPPORTED, "multi-dimensional losses need a free loss slot (n_losses < %d) or a hinge entry",
                        GLRM_MAX_LOSSES);
        hinge = d->n_losses;
        E.losses.push_back(glrm_loss{GLRM_LOSS_HINGE, 0, 0.0f});
    }
    E.codes.clear(); E.src.clear(); E.thr.clear(); E.kind.clear(); E.blk0.clear(); E.blk1.clear();
    for (int64_t j = 0; j < d->n; ++j) {
        const int q = d->col_loss ? d->col_loss[j] : 0;
        const glrm_loss &l = d->losses[q];
        const int dj = md_dim(l);
        const int32_t b0 = (int32_t)E.src.size();
        for (int t = 0; t < dj; ++t) {
            E.src.push_back((int32_t)j);
            E.blk0.push_back(b0);
            E.blk1.push_back(b0 + dj);
            if (l.kind == GLRM_LOSS_CATEGORICAL) {          // label t + 1 against the rest
                E.codes.push_back((uint8_t)hinge); E.kind.push_back(EMB_EQ); E.thr.push_back(t + 1);
            } else if (l.kind == GLRM_LOSS_MORDINAL) {      // levels above t + 1 against the rest
                E.codes.push_back((uint8_t)hinge); E.kind.push_back(EMB_GT); E.thr.push_back(t + 1);
            } else {
                E.codes.push_back((uint8_t)q); E.kind.push_back(EMB_COPY); E.thr.push_back(0);
            }
        }
    }
    E.e = *d;
    E.e.n = total;
    E.e.col_loss = E.codes.data();
    E.e.losses = E.losses.data();
    E.e.n_losses = (int32_t)E.losses.size();
    E.active = true;
    *out = &E.e;
    return GLRM_OK;
}

// Uploads the embedding map (padding columns repeat the last column, as the
// codes do); the caller synchronizes before the vectors go.
int upload_embed(const Embed &E, const Layout &L, void *ws, std::vector<int32_t> (&pad)[4], std::vector<uint8_t> &kpad,
                 hipStream_t st)
{
    const std::vector<int32_t> *v[4] = {&E.src, &E.thr, &E.blk0, &E.blk1};
    const size_t off[4] = {L.emb_src, L.emb_thr, L.blk0, L.blk1};
    for (int q = 0; q < 4; ++q) {
        pad[q] = *v[q];
        pad[q].resize((size_t)L.ldp, v[q]->back());
        HIP_TRY(hipMemcpyAsync(at<int32_t>(ws, off[q]), pad[q].data(), sizeof(int32_t) * L.ldp, hipMemcpyHostToDevice,
                               st));
    }
    kpad = E.kind;
    kpad.resize((size_t)L.ldp, E.kind.back());
    HIP_TRY(hipMemcpyAsync(at<uint8_t>(ws, L.emb_kind), kpad.data(), (size_t)L.ldp, hipMemcpyHostToDevice, st));
    return GLRM_OK;
}

EmbedMap embed_map(const Embed &E, const Layout &L, void *ws)
{
    if (!E.active) return EmbedMap{nullptr, nullptr, nullptr};
    return EmbedMap{at<int32_t>(ws, L.emb_src), at<int32_t>(ws, L.emb_thr), at<uint8_t>(ws, L.emb_kind)};
}

// The loss table as the kernels take it.  With per-column weights the table
// points at the workspace's padded copy of them (written by prepare) and is
// never treated as uniform, so the weighted per-column path runs.
LossTab make_losstab(const glrm_data *d, const Layout &L, void *ws)
{
    LossTab t;
    memset(&t, 0, sizeof t);
    t.n = d->n_losses;
    for (int q = 0; q < d->n_losses; ++q) {
        t.kind[q] = d->losses[q].kind;
        t.levels[q] = d->losses[q].levels;
        t.param[q] = d->losses[q].param;
    }
    t.uniform = -1;
    if (!d->col_loss) t.uniform = 0;
    else {
        int u = d->col_loss[0];
        for (int64_t j = 1; j < d->n; ++j)
            if (d->col_loss[j] != u) { u = -1; break; }
        t.uniform = u;
    }
    t.colw = at<float>(ws, L.colw);   // all 1 unless the caller gave weights
    if (d->col_weight) t.uniform = -1;
    return t;
}

Reg make_reg(const glrm_reg &r, int32_t offset = 0) { return Reg{r.kind, r.weight, offset}; }
// The regularizers of the rows of X and of the columns of Y; with the offset
// (Section 3.3) coordinate 0 is the constant 1 in X and a free offset in Y.
Reg reg_x(const glrm_data *d) { return make_reg(d->rx, d->offset ? 1 : 0); }
Reg reg_y(const glrm_data *d) { return make_reg(d->ry, d->offset ? 2 : 0); }

LossU make_lossu(const LossTab &t)
{
    LossU u;
    if (t.uniform >= 0) {
        u.kind = t.kind[t.uniform];
        u.levels = t.levels[t.uniform];
        u.param = t.param[t.uniform];
    } else {
        u.kind = -1;
        u.levels = 0;
        u.param = 0.0f;
    }
    return u;
}

YShadow shadow(void *ws, const Layout &L, bool plus)
{
    YShadow s;
    s.f32 = at<float>(ws, plus ? L.yp_f32 : L.ycur_f32);
    s.t32 = at<float>(ws, plus ? L.yp_t32 : L.ycur_t32);
    s.hi = at<__bf16>(ws, plus ? L.yp_hi : L.ycur_hi);
    s.lo = at<__bf16>(ws, plus ? L.yp_lo : L.ycur_lo);
    s.tb = at<__bf16>(ws, plus ? L.yp_tb : L.ycur_tb);
    return s;
}

int check_ws(const Layout &L, void *ws, size_t ws_bytes)
{
    if (!ws) return fail(GLRM_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(GLRM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(GLRM_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    return GLRM_OK;
}

// Per-column loss codes: host -> workspace.  Padding columns repeat the last
// column's code, so the last tile keeps one loss.  Without a code list every
// column gets code 0.  The caller keeps `codes` alive until the copy is done.
int upload_codes(const glrm_data *d, const Layout &L, void *ws, std::string &codes, hipStream_t st)
{
    codes.assign((size_t)L.ldp, '\0');
    if (d->col_loss) {
        memcpy(&codes[0], d->col_loss, (size_t)d->n);
        for (int64_t j = d->n; j < L.ldp; ++j) codes[(size_t)j] = (char)d->col_loss[d->n - 1];
    }
    HIP_TRY(hipMemcpyAsync(at<uint8_t>(ws, L.codes), codes.data(), (size_t)L.ldp, hipMemcpyHostToDevice, st));
    return GLRM_OK;
}

int prepare(const glrm_data *d, const Layout &L, void *ws, hipStream_t st, const Embed &E)
{
    std::string codes;
    int rc0 = upload_codes(d, L, ws, codes, st);
    if (rc0) return rc0;
    std::vector<int32_t> pad[4];
    std::vector<uint8_t> kpad;
    if (E.active && (rc0 = upload_embed(E, L, ws, pad, kpad, st))) return rc0;
    const EmbedMap em = embed_map(E, L, ws);
    HIP_TRY(launch_pad_weights(d->col_weight, em.src, L.n, L.ldp, at<float>(ws, L.colw), st));
    if (d->layout == GLRM_DENSE) {
        HIP_TRY(launch_fill_i32(at<int32_t>(ws, L.col_count), L.n, 0, st));
        PackArgs p;
        p.m = L.m; p.n = L.n; p.lda = d->lda; p.mp = L.mp; p.ldp = L.ldp;
        p.A = d->A; p.mask = d->mask;
        p.emb = em;
        p.Ap = at<float>(ws, L.Ap);
        p.row_count = at<int32_t>(ws, L.row_count);
        p.col_count = at<int32_t>(ws, L.col_count);
        HIP_TRY(launch_pack_dense(p, st));
    } else {
        int rc = coo_prepare(d, L.kp, L.cl, at<char>(ws, L.coo), at<int32_t>(ws, L.row_count),
                             at<int32_t>(ws, L.col_count), st);
        if (rc != GLRM_OK) return rc;
    }
    // the host vectors must outlive the copies
    HIP_TRY(hipStreamSynchronize(st));
    if (d->layout != GLRM_DENSE) {
        int bad = coo_check_result(L.cl, at<char>(ws, L.coo), st);
        if (bad) return fail(GLRM_EINVAL, "COO indices are out of range, unsorted or duplicated");
    }
    return GLRM_OK;
}

int write_shadows(const Layout &L, const float *Y, void *ws, int prec, bool clear_plus, hipStream_t st)
{
    YShadowArgs a;
    a.n = L.n; a.ldp = L.ldp; a.k = (int32_t)L.k; a.Y = Y;
    a.ys = shadow(ws, L, false);
    a.yp = clear_plus ? shadow(ws, L, true) : YShadow{nullptr, nullptr, nullptr, nullptr, nullptr};
    HIP_TRY(launch_yshadow(a, (int)L.kp, prec, st));
    return GLRM_OK;
}

// Regularizer sums of X and Y into regpart[0..2*REG_BLOCKS).
int reg_sums(const glrm_data *d, const Layout &L, const float *X, const float *Y, void *ws, hipStream_t st)
{
    double *rp = at<double>(ws, L.regpart);
    HIP_TRY(launch_regsum(reg_x(d), X, L.m, (int32_t)L.k, rp, REG_BLOCKS, st));
    HIP_TRY(launch_regsum(reg_y(d), Y, L.n, (int32_t)L.k, rp + REG_BLOCKS, REG_BLOCKS, st));
    return GLRM_OK;
}

int objective64(const glrm_data *d, const Layout &L, const float *X, const float *Y, void *ws, double *out_dev,
                hipStream_t st)
{
    double *po = at<double>(ws, d->layout == GLRM_DENSE ? L.part_obj64 : L.scal);
    int nparts = 0;
    if (d->layout == GLRM_DENSE) {
        Obj64Args a;
        a.m = L.m; a.n = L.n; a.mp = L.mp; a.ldp = L.ldp; a.k = (int32_t)L.k;
        a.Ap = at<float>(ws, L.Ap);
        a.codes = at<uint8_t>(ws, L.codes);
        a.lt = make_losstab(d, L, ws);
        a.X = X; a.Y = Y;
        a.part_obj = po;
        const int64_t tiles = (L.mp / 16) * ((L.ldp + 255) / 256);
        nparts = (int)std::min<int64_t>(OBJ64_BLOCKS, std::max<int64_t>(1, tiles));
        HIP_TRY(launch_objective64(a, nparts, st));
    } else {
        int rc = coo_objective(d, L.cl, at<char>(ws, L.coo), at<uint8_t>(ws, L.codes), make_losstab(d, L, ws), X, Y,
                               GLRM_FP64, &po, &nparts, st);
        if (rc != GLRM_OK) return rc;
    }
    int rc = reg_sums(d, L, X, Y, ws, st);
    if (rc != GLRM_OK) return rc;
    double *rp = at<double>(ws, L.regpart);
    double *tmp = at<double>(ws, L.scal) + 4;
    HIP_TRY(launch_sum_doubles(po, nparts, rp, 2 * REG_BLOCKS, tmp, st));
    HIP_TRY(hipMemcpyAsync(out_dev, tmp, sizeof(double), hipMemcpyDeviceToDevice, st));
    return GLRM_OK;
}

// Row chunks of the loss pass.  With the gradient, P_GRAD workgroups in all,
// so a table cut into several column blocks takes fewer, longer row chunks
// (and fewer Y-gradient partials to reduce); the objective alone has no
// partials to spare and keeps P_GRAD row chunks per column block.
int grad_rows(const Layout &L, bool want_grad)
{
    const int64_t per = want_grad ? (P_GRAD + L.cb_grad - 1) / L.cb_grad : P_GRAD;
    return (int)std::max<int64_t>(1, std::min<int64_t>(per, L.mp / 16));
}

// Dense loss (+ gradient) pass at fp32 / bf16 precision.
int dense_lossgrad(const glrm_data *d, const Layout &L, const float *X, const float *Y, int prec, float *dX,
                   float *dY, bool want_grad, void *ws, hipStream_t st)
{
    int rc = write_shadows(L, Y, ws, prec, false, st);
    if (rc != GLRM_OK) return rc;
    const int gx = grad_rows(L, want_grad);
    const int gy = (int)L.cb_grad;
    LossGradArgs a;
    a.m = L.m; a.mp = L.mp; a.ldp = L.ldp; a.k = (int32_t)L.k;
    a.Ap = at<float>(ws, L.Ap);
    a.codes = at<uint8_t>(ws, L.codes);
    a.lt = make_losstab(d, L, ws);
    a.lu = make_lossu(a.lt);
    a.X = X;
    a.ycur = shadow(ws, L, false);
    a.dX = dX;
    a.part_dx = (want_grad && gy > 1) ? at<float>(ws, L.part_dx) : nullptr;
    a.part_dy = at<float>(ws, L.part_dy);
    a.part_obj = at<double>(ws, L.part_obj);
    HIP_TRY(launch_lossgrad(a, (int)L.kp, L.tpw_grad, prec, want_grad, gx, gy, st));
    if (want_grad) {
        ReduceArgs r;
        r.m = L.m; r.n = L.n; r.ldp = L.ldp; r.k = (int32_t)L.k; r.P = gx; r.CB = gy;
        r.part_dy = a.part_dy; r.part_dx = a.part_dx; r.dY = dY; r.dX = dX;
        HIP_TRY(launch_reduce_dy(r, (int)L.kp, st));
        if (gy > 1) HIP_TRY(launch_reduce_dx(r, st));
    }
    return GLRM_OK;
}

// Optional per-kernel event timing of a fit (GLRM_TIME_KERNELS).
struct KernelTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    size_t used = 0;
    int init(bool enable, size_t launches)
    {
        on = enable;
        if (!on) return GLRM_OK;
        ev.resize(2 * launches);
        kind.resize(launches);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(GLRM_EHIP, "hipEventCreate failed");
        return GLRM_OK;
    }
    hipError_t start(int k, hipStream_t st)
    {
        if (!on || used >= kind.size()) return hipSuccess;
        kind[used] = k;
        return hipEventRecord(ev[2 * used], st);
    }
    hipError_t stop(hipStream_t st)
    {
        if (!on || used >= kind.size()) return hipSuccess;
        hipError_t e = hipEventRecord(ev[2 * used + 1], st);
        ++used;
        return e;
    }
    void report(glrm_fit_info *info)
    {
        if (!on) return;
        for (size_t i = 0; i < used; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess && info) {
                info->kernel_ms[kind[i]] += ms;
                info->kernel_calls[kind[i]] += 1;
            }
        }
    }
    ~KernelTimer()
    {
        for (auto &e : ev) hipEventDestroy(e);
    }
};

int check_prec(int prec, bool allow64)
{
    if (prec == GLRM_FP32 || prec == GLRM_BF16 || prec == GLRM_BF16_PLAIN) return GLRM_OK;
    if (prec == GLRM_FP64 && allow64) return GLRM_OK;
    return fail(GLRM_EINVAL, "unsupported precision %d for this call", prec);
}

}  // namespace

namespace glrm {
int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
}  // namespace glrm

namespace {
// The gradient entry points after their checks: prepare unless told the
// workspace holds it, one loss-and-gradient pass, the objective if asked.
int grad_run(const glrm_data *d, const Layout &L, const float *X, const float *Y, int precision, float *dX,
             float *dY, double *obj_host, void *ws, unsigned flags, hipStream_t st, const Embed &E)
{
    int rc;
    if (!(flags & GLRM_WS_PREPARED) && (rc = prepare(d, L, ws, st, E))) return rc;
    double *po = nullptr;
    int nparts = 0;
    if (d->layout == GLRM_DENSE) {
        if ((rc = dense_lossgrad(d, L, X, Y, precision, dX, dY, true, ws, st))) return rc;
        po = at<double>(ws, L.part_obj);
        nparts = (int)(grad_rows(L, true) * L.cb_grad);
    } else {
        if ((rc = coo_grad(d, L.kp, L.cl, at<char>(ws, L.coo), at<uint8_t>(ws, L.codes), make_losstab(d, L, ws), X, Y,
                           precision, dX, dY, &po, &nparts, st)))
            return rc;
    }
    if (flags & GLRM_GRAD_WITH_REG) {
        HIP_TRY(launch_reg_grad(reg_x(d), X, L.m, (int32_t)L.k, dX, st));
        HIP_TRY(launch_reg_grad(reg_y(d), Y, L.n, (int32_t)L.k, dY, st));
    }
    if (obj_host) {
        double *res = at<double>(ws, L.scal);
        if ((rc = reg_sums(d, L, X, Y, ws, st))) return rc;
        HIP_TRY(launch_sum_doubles(po, nparts, at<double>(ws, L.regpart), 2 * REG_BLOCKS, res, st));
        HIP_TRY(hipMemcpyAsync(obj_host, res, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return GLRM_OK;
}


// The workspace of glrm_grad_noalloc: a file-scope device array, one copy on
// every device the library runs on, held until the process ends.  In host
// code its name stands for a host-side symbol, not a device address: the
// address comes from hipGetSymbolAddress, once per device with that device
// current, and only that address is handed to kernels.
__device__ __align__(256) unsigned char scratch[GLRM_NOALLOC_MAX_BYTES];

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_DEVICES] = {};

int scratch_address(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_DEVICES) return fail(GLRM_EUNSUPPORTED, "device %d is beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(GLRM_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GLRM_OK;
}
// The entry-wise matrix of the loss derivatives at (X, Y) in the aux region:
// dense, in the padded table's layout; COO, per entry in row order (aux_V) and
// in the column-grouped order (aux_V2).
int grad_matrix(const glrm_data *d, const Layout &L, const float *X, const float *Y, void *ws, hipStream_t st)
{
    EntryArgs ea;
    memset(&ea, 0, sizeof ea);
    ea.m = L.m; ea.n = L.n; ea.mp = L.mp; ea.ldp = L.ldp; ea.k = (int32_t)L.k;
    ea.Ap = d->layout == GLRM_DENSE ? at<float>(ws, L.Ap) : nullptr;
    ea.codes = at<uint8_t>(ws, L.codes);
    ea.lt = make_losstab(d, L, ws);
    ea.colw = ea.lt.colw;
    ea.X = X; ea.Y = Y;
    if (d->layout == GLRM_DENSE) {
        HIP_TRY(launch_dense_grad_matrix(ea, at<float>(ws, L.aux_V), st));
    } else {
        HIP_TRY(launch_coo_grad_values(ea, d->row, d->col, d->A, d->nnz, at<float>(ws, L.aux_V), st));
        HIP_TRY(launch_permute(coo_perm(L.cl, at<char>(ws, L.coo)), at<float>(ws, L.aux_V), d->nnz,
                               at<float>(ws, L.aux_V2), st));
    }
    return GLRM_OK;
}

// out (m x b) = alpha V B, or out (n x b) = alpha V^T B (transposed)
int apply_matrix(const glrm_data *d, const Layout &L, void *ws, bool transposed, const double *B, int32_t b,
                 double alpha, double *out, hipStream_t st)
{
    if (d->layout == GLRM_DENSE) {
        if (!transposed) HIP_TRY(launch_dense_apply(at<float>(ws, L.aux_V), L.m, L.n, L.ldp, B, b, alpha, out, st));
        else HIP_TRY(launch_dense_apply_t(at<float>(ws, L.aux_V), L.m, L.n, L.ldp, B, b, alpha,
                                          at<double>(ws, L.aux_part), out, st));
    } else {
        const CooView cv = coo_view(L.cl, at<char>(ws, L.coo));
        if (!transposed) HIP_TRY(launch_seg_apply(cv.row_ptr, d->col, at<float>(ws, L.aux_V), L.m, B, b, alpha, out, st));
        else HIP_TRY(launch_seg_apply(cv.col_ptr, cv.csc_row, at<float>(ws, L.aux_V2), L.n, B, b, alpha, out, st));
    }
    return GLRM_OK;
}

// Gram matrices of both factors, to the host.
int gram_pair(const Layout &L, const float *X, const float *Y, void *ws, std::vector<double> &Gx,
              std::vector<double> &Gy, hipStream_t st)
{
    const int k = (int)L.k;
    double *part = at<double>(ws, L.aux_part), *sm = at<double>(ws, L.aux_small);
    HIP_TRY(launch_gram_f(X, L.m, k, part, sm, st));
    HIP_TRY(launch_gram_f(Y, L.n, k, part, sm + k * k, st));
    Gx.assign((size_t)k * k, 0.0);
    Gy.assign((size_t)k * k, 0.0);
    HIP_TRY(hipMemcpyAsync(Gx.data(), sm, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(Gy.data(), sm + k * k, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GLRM_OK;
}

// Orthonormal basis of the columns of Q (rows x b, double) into Qo: with
// Q^T Q = E diag(l) E^T, Qo = Q E_r diag(l_r)^-1/2 over the eigenvalues above
// 1e-12 of the largest (a column space of rank r <= b); done twice, as in
// CholeskyQR2, so the second pass repairs the rounding of the first.  Returns
// r through *r; the basis ends in *Q (the buffers swap).
int orthonormalize(const Layout &L, void *ws, double **Q, double **Qo, int64_t rows, int *b, hipStream_t st)
{
    double *part = at<double>(ws, L.aux_part), *sm = at<double>(ws, L.aux_small);
    for (int pass = 0; pass < 2; ++pass) {
        const int bb = *b;
        if (bb == 0) return GLRM_OK;
        HIP_TRY(launch_tall_tmul_d(*Q, rows, bb, bb, *Q, bb, part, sm, st));
        std::vector<double> G((size_t)bb * bb), w(bb), E((size_t)bb * bb);
        HIP_TRY(hipMemcpyAsync(G.data(), sm, sizeof(double) * bb * bb, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        glrm_host::sym_eig(bb, G.data(), w.data(), E.data());
        int r = 0;
        while (r < bb && w[r] > 1e-12 * std::max(w[0], 0.0) && w[r] > 0.0) ++r;
        std::vector<double> T((size_t)bb * std::max(r, 1));
        for (int a = 0; a < bb; ++a)
            for (int c = 0; c < r; ++c) T[a * r + c] = E[a * bb + c] / std::sqrt(w[c]);
        if (r > 0) {
            HIP_TRY(hipMemcpyAsync(sm, T.data(), sizeof(double) * bb * r, hipMemcpyHostToDevice, st));
            HIP_TRY(launch_tall_mul_d(*Q, rows, bb, bb, sm, r, 1.0, 0.0, *Qo, st));
            HIP_TRY(hipStreamSynchronize(st));   // T lives on this host stack
        }
        std::swap(*Q, *Qo);
        *b = r;
    }
    return GLRM_OK;
}

}  // namespace

extern "C" {

const char *glrm_last_error(void) { return g_err.c_str(); }

const char *glrm_version(void) { return "glrm-gfx950 0.1"; }

size_t glrm_workspace_size(const glrm_data *d0)
{
    Embed E;
    const glrm_data *d = nullptr;
    if (embed(d0, E, &d) != GLRM_OK) return 0;
    Layout L;
    make_layout(d, L);
    return L.total;
}

int64_t glrm_embed_dim(const glrm_data *d0)
{
    Embed E;
    const glrm_data *d = nullptr;
    if (embed(d0, E, &d) != GLRM_OK) return -1;
    return d->n;
}

size_t glrm_fit_workspace_size(const glrm_data *d0, const glrm_fit_opts *o)
{
    Embed E;
    const glrm_data *d = nullptr;
    if (embed(d0, E, &d) != GLRM_OK) return 0;
    Layout L;
    make_layout(d, L, false, 0, o && o->update == GLRM_UPDATE_PROXPROX);
    return L.total;
}

int glrm_prepare(const glrm_data *d0, void *ws, size_t ws_bytes, void *stream)
{
    g_err.clear();
    Embed E;
    const glrm_data *d = nullptr;
    int rc = embed(d0, E, &d);
    if (rc) return rc;
    Layout L;
    make_layout(d, L);
    if ((rc = check_ws(L, ws, ws_bytes))) return rc;
    return prepare(d, L, ws, (hipStream_t)stream, E);
}

int glrm_objective(const glrm_data *d0, const float *X, const float *Y, int precision, double *obj_host, void *ws,
                   size_t ws_bytes, unsigned flags, void *stream)
{
    g_err.clear();
    Embed E;
    const glrm_data *d = nullptr;
    int rc = embed(d0, E, &d);
    if (rc) return rc;
    if (!X || !Y || !obj_host) return fail(GLRM_EINVAL, "X, Y and obj_host must not be NULL");
    if ((rc = check_prec(precision, true))) return rc;
    Layout L;
    make_layout(d, L);
    if ((rc = check_ws(L, ws, ws_bytes))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (!(flags & GLRM_WS_PREPARED) && (rc = prepare(d, L, ws, st, E))) return rc;
    double *res = at<double>(ws, L.scal);
    if (precision == GLRM_FP64) {
        if ((rc = objective64(d, L, X, Y, ws, res, st))) return rc;
    } else {
        double *po = nullptr;
        int nparts = 0;
        if (d->layout == GLRM_DENSE) {
            if ((rc = dense_lossgrad(d, L, X, Y, precision, nullptr, nullptr, false, ws, st))) return rc;
            po = at<double>(ws, L.part_obj);
            nparts = (int)(grad_rows(L, false) * L.cb_grad);
        } else {
            if ((rc = coo_objective(d, L.cl, at<char>(ws, L.coo), at<uint8_t>(ws, L.codes), make_losstab(d, L, ws), X, Y,
                                    precision, &po, &nparts, st)))
                return rc;
        }
        if ((rc = reg_sums(d, L, X, Y, ws, st))) return rc;
        HIP_TRY(launch_sum_doubles(po, nparts, at<double>(ws, L.regpart), 2 * REG_BLOCKS, res, st));
    }
    HIP_TRY(hipMemcpyAsync(obj_host, res, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GLRM_OK;
}

int glrm_grad(const glrm_data *d0, const float *X, const float *Y, int precision, float *dX, float *dY,
              double *obj_host, void *ws, size_t ws_bytes, unsigned flags, void *stream)
{
    g_err.clear();
    Embed E;
    const glrm_data *d = nullptr;
    int rc = embed(d0, E, &d);
    if (rc) return rc;
    if (!X || !Y || !dX || !dY) return fail(GLRM_EINVAL, "X, Y, dX and dY must not be NULL");
    if ((rc = check_prec(precision, false))) return rc;
    Layout L;
    make_layout(d, L);
    if ((rc = check_ws(L, ws, ws_bytes))) return rc;
    return grad_run(d, L, X, Y, precision, dX, dY, obj_host, ws, flags, (hipStream_t)stream, E);
}

int glrm_grad_noalloc(const glrm_data *d0, const float *X, const float *Y, int precision, float *dX, float *dY,
                      double *obj_host, unsigned flags, void *stream)
{
    g_err.clear();
    Embed E;
    const glrm_data *d = nullptr;
    int rc = embed(d0, E, &d);
    if (rc) return rc;
    if (!X || !Y || !dX || !dY) return fail(GLRM_EINVAL, "X, Y, dX and dY must not be NULL");
    if ((rc = check_prec(precision, false))) return rc;
    Layout L;
    make_layout(d, L, true);
    if (L.total > (size_t)GLRM_NOALLOC_MAX_BYTES)
        return fail(GLRM_ENOMEM, "glrm_grad_noalloc: this problem needs %zu bytes of scratch; the static scratch "
                    "holds %zu (use glrm_grad with a workspace)", L.total, (size_t)GLRM_NOALLOC_MAX_BYTES);
    void *ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    return grad_run(d, L, X, Y, precision, dX, dY, obj_host, ws, flags, (hipStream_t)stream, E);
}
size_t glrm_linalg_workspace_size(const glrm_data *d0, int32_t block)
{
    Embed E;
    const glrm_data *d = nullptr;
    if (embed(d0, E, &d) != GLRM_OK) return 0;
    if (block < 1 || block > LA_MAXB) {
        fail(GLRM_EINVAL, "block must be in 1..%d", LA_MAXB);
        return 0;
    }
    Layout L;
    make_layout(d, L, false, block);
    return L.total;
}

int glrm_certificate(const glrm_data *d0, const float *X, const float *Y, int32_t iters, glrm_cert_info *info,
                     void *ws, size_t ws_bytes, unsigned flags, void *stream)
{
    g_err.clear();
    Embed E;
    const glrm_data *d = nullptr;
    int rc = embed(d0, E, &d);
    if (rc) return rc;
    if (!X || !Y || !info) return fail(GLRM_EINVAL, "X, Y and info must not be NULL");
    if (iters < 1 || iters > 1000000) return fail(GLRM_EINVAL, "iters must be in 1..1e6");
    if (d->rx.kind != GLRM_REG_QUADRATIC || d->ry.kind != GLRM_REG_QUADRATIC || d->rx.weight != d->ry.weight ||
        !(d->rx.weight > 0.0f))
        return fail(GLRM_EINVAL, "the certificate needs the quadratic regularizer with one weight > 0 on both factors");
    Layout L;
    make_layout(d, L, false, 1);
    if ((rc = check_ws(L, ws, ws_bytes))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (!(flags & GLRM_WS_PREPARED) && (rc = prepare(d, L, ws, st, E))) return rc;
    const int k = (int)L.k;
    // weight w on ||x||^2 is the factored problem's gamma / 2
    const double inv_gamma = 1.0 / (2.0 * (double)d->rx.weight);
    if ((rc = grad_matrix(d, L, X, Y, ws, st))) return rc;
    std::vector<double> Gx, Gy;
    if ((rc = gram_pair(L, X, Y, ws, Gx, Gy, st))) return rc;
    std::vector<double> P((size_t)k * k), Pt((size_t)k * k), sv(k);
    const int rank = glrm_host::polar_map(k, Gx.data(), Gy.data(), 1e-6, P.data(), sv.data());
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) Pt[j * k + i] = P[i * k + j];
    double *sm = at<double>(ws, L.aux_small);
    double *Pd = sm, *Ptd = sm + k * k, *tv = sm + 2 * k * k, *sv_d = tv + LA_MAXB, *nrm = sv_d + LA_MAXB;
    double *est = nrm + 4;
    HIP_TRY(hipMemcpyAsync(Pd, P.data(), sizeof(double) * k * k, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(Ptd, Pt.data(), sizeof(double) * k * k, hipMemcpyHostToDevice, st));
    double *part = at<double>(ws, L.aux_part);
    double *u = at<double>(ws, L.aux_m1), *v = at<double>(ws, L.aux_n1), *w = at<double>(ws, L.aux_n2);
    HIP_TRY(launch_start_vector(v, L.n, 0x14100342ull, st));
    HIP_TRY(launch_sumsq(v, L.n, part, nrm, st));
    HIP_TRY(launch_normalize(v, L.n, nrm, nullptr, 0, st));
    for (int it = 0; it < iters; ++it) {
        // u = M v = G v / gamma + X P Y^T v
        if ((rc = apply_matrix(d, L, ws, false, v, 1, inv_gamma, u, st))) return rc;
        HIP_TRY(launch_tall_tmul_f(Y, L.n, k, k, v, 1, part, tv, st));
        HIP_TRY(launch_tall_mul_d(Pd, k, k, k, tv, 1, 1.0, 0.0, sv_d, st));
        HIP_TRY(launch_tall_mul_f(X, L.m, k, k, sv_d, 1, 1.0, 1.0, u, st));
        HIP_TRY(launch_sumsq(u, L.m, part, nrm, st));
        HIP_TRY(launch_normalize(nullptr, 0, nrm, est, it & 1, st));
        // w = M^T u = G^T u / gamma + Y P^T X^T u, then v = w / ||w||
        if ((rc = apply_matrix(d, L, ws, true, u, 1, inv_gamma, w, st))) return rc;
        HIP_TRY(launch_tall_tmul_f(X, L.m, k, k, u, 1, part, tv, st));
        HIP_TRY(launch_tall_mul_d(Ptd, k, k, k, tv, 1, 1.0, 0.0, sv_d, st));
        HIP_TRY(launch_tall_mul_f(Y, L.n, k, k, sv_d, 1, 1.0, 1.0, w, st));
        HIP_TRY(launch_sumsq(w, L.n, part, nrm + 1, st));
        HIP_TRY(launch_normalize(w, L.n, nrm + 1, nullptr, 0, st));
        std::swap(v, w);
    }
    double e2[2] = {0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(e2, est, sizeof e2, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    info->norm = e2[(iters - 1) & 1];
    info->norm_prev = iters > 1 ? e2[iters & 1] : NAN;
    info->rank = rank;
    info->iters = iters;
    return GLRM_OK;
}

int glrm_column_scaling(const glrm_data *d0, float *mu, float *sigma2, void *ws, size_t ws_bytes, unsigned flags,
                        void *stream)
{
    g_err.clear();
    Embed E;
    const glrm_data *d = nullptr;
    int rc = embed(d0, E, &d);
    if (rc) return rc;
    if (E.active) return fail(GLRM_EUNSUPPORTED, "column scaling is built for scalar losses only");
    if (!mu || !sigma2) return fail(GLRM_EINVAL, "mu and sigma2 must not be NULL");
    Layout L;
    make_layout(d, L, false, 1);
    if ((rc = check_ws(L, ws, ws_bytes))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (!(flags & GLRM_WS_PREPARED) && (rc = prepare(d, L, ws, st, E))) return rc;
    const bool coo = d->layout != GLRM_DENSE;
    ColArgs a;
    memset(&a, 0, sizeof a);
    a.m = L.m; a.n = L.n; a.mp = L.mp; a.ldp = L.ldp;
    if (coo) {
        const CooView cv = coo_view(L.cl, at<char>(ws, L.coo));
        a.col_ptr = cv.col_ptr;
        a.csc_val = cv.csc_val;
    } else {
        a.Ap = at<float>(ws, L.Ap);
    }
    a.codes = at<uint8_t>(ws, L.codes);
    a.lt = make_losstab(d, L, ws);
    // per column: the bracket and its midpoint, and the passes' results
    double *lo = at<double>(ws, L.aux_cols), *hi = lo + L.n, *mid = hi + L.n;
    double *out = at<double>(ws, L.aux_colout);
    a.lo = lo; a.hi = hi; a.mid = mid;
    double *part = at<double>(ws, L.aux_part);
    const int32_t *count = at<int32_t>(ws, L.col_count);
    HIP_TRY(launch_col_pass(a, 0, coo, part, out, st));
    HIP_TRY(launch_bracket(lo, hi, mid, out, count, L.n, true, st));
    // a search on the sign of the derivative sum: the bracket [min a - 1,
    // max a + 1] holds a minimizer of every loss here; each pass keeps one of
    // COL_PTS + 1 sub-intervals, so COL_PASSES passes take it as far as 64
    // halvings, to double rounding
    for (int it = 0; it < COL_PASSES; ++it) {
        HIP_TRY(launch_col_pass(a, 1, coo, part, out, st));
        HIP_TRY(launch_bracket(lo, hi, mid, out, count, L.n, false, st));
    }
    HIP_TRY(launch_col_pass(a, 2, coo, part, out, st));
    HIP_TRY(launch_scaling_finish(mid, out, count, L.n, mu, sigma2, st));
    return GLRM_OK;
}

int glrm_init_svd(const glrm_data *d0, const float *mu, const float *sigma2, const float *omega, int32_t l,
                  int32_t power_iters, float *X, float *Y, double *sv_host, void *ws, size_t ws_bytes,
                  unsigned flags, void *stream)
{
    g_err.clear();
    Embed E;
    const glrm_data *d = nullptr;
    int rc = embed(d0, E, &d);
    if (rc) return rc;
    if (E.active) return fail(GLRM_EUNSUPPORTED, "the SVD initialization is built for scalar losses only");
    const int k = d->k, off = d->offset ? 1 : 0, ks = k - off;
    if (!X || !Y) return fail(GLRM_EINVAL, "X and Y must not be NULL");
    if (off && !mu) return fail(GLRM_EINVAL, "the offset row needs the column means mu");
    if (ks > 0 && !omega) return fail(GLRM_EINVAL, "omega (the n x l test matrix) must not be NULL");
    if (l < ks || l < 1 || l > LA_MAXB) return fail(GLRM_EINVAL, "l must be in max(k', 1)..%d (k' = %d)", LA_MAXB, ks);
    if (power_iters < 0 || power_iters > 32) return fail(GLRM_EINVAL, "power_iters must be in 0..32");
    Layout L;
    make_layout(d, L, false, l);
    if ((rc = check_ws(L, ws, ws_bytes))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (!(flags & GLRM_WS_PREPARED) && (rc = prepare(d, L, ws, st, E))) return rc;
    const int64_t m = L.m, n = L.n;
    const int32_t *count = at<int32_t>(ws, L.col_count);
    float *cs = at<float>(ws, L.aux_cols), *mu0 = cs + n;
    HIP_TRY(launch_svd_scales(mu, sigma2, count, m, n, cs, mu0, st));
    for (int c = 0; c < k; ++c) {
        HIP_TRY(launch_fill_column(X, m, k, c, c < off ? 1.0f : 0.0f, nullptr, st));
        HIP_TRY(launch_fill_column(Y, n, k, c, 0.0f, c < off ? mu0 : nullptr, st));
    }
    std::vector<double> svals(std::max(ks, 1), 0.0);
    if (ks > 0) {
        // the standardized table of Section 7.5 in the aux region
        EntryArgs ea;
        memset(&ea, 0, sizeof ea);
        ea.m = m; ea.n = n; ea.mp = L.mp; ea.ldp = L.ldp; ea.k = k;
        ea.Ap = d->layout == GLRM_DENSE ? at<float>(ws, L.Ap) : nullptr;
        ea.mu = mu0; ea.cs = cs;
        if (d->layout == GLRM_DENSE) {
            HIP_TRY(launch_dense_scaled_matrix(ea, at<float>(ws, L.aux_V), st));
        } else {
            HIP_TRY(launch_coo_scaled_values(ea, d->col, d->A, d->nnz, at<float>(ws, L.aux_V), st));
            HIP_TRY(launch_permute(coo_perm(L.cl, at<char>(ws, L.coo)), at<float>(ws, L.aux_V), d->nnz,
                                   at<float>(ws, L.aux_V2), st));
        }
        double *Qa = at<double>(ws, L.aux_m1), *Qb = at<double>(ws, L.aux_m2);
        double *Za = at<double>(ws, L.aux_n1), *Zb = at<double>(ws, L.aux_n2);
        double *sm = at<double>(ws, L.aux_small);
        // randomized range finder (Halko, Martinsson, Tropp 2011): Q = orth(A~ Omega),
        // then power_iters rounds of Q = orth(A~ orth(A~^T Q))
        int b = l;
        HIP_TRY(launch_to_double(omega, n * (int64_t)l, Za, st));
        if ((rc = apply_matrix(d, L, ws, false, Za, b, 1.0, Qa, st))) return rc;
        if ((rc = orthonormalize(L, ws, &Qa, &Qb, m, &b, st))) return rc;
        for (int it = 0; it < power_iters && b > 0; ++it) {
            if ((rc = apply_matrix(d, L, ws, true, Qa, b, 1.0, Za, st))) return rc;
            if ((rc = orthonormalize(L, ws, &Za, &Zb, n, &b, st))) return rc;
            if (b == 0) break;
            if ((rc = apply_matrix(d, L, ws, false, Za, b, 1.0, Qa, st))) return rc;
            if ((rc = orthonormalize(L, ws, &Qa, &Qb, m, &b, st))) return rc;
        }
        if (b > 0) {
            // B = Q^T A~ (kept transposed, n x b); B B^T = U_B diag(s^2) U_B^T
            if ((rc = apply_matrix(d, L, ws, true, Qa, b, 1.0, Za, st))) return rc;
            double *part = at<double>(ws, L.aux_part);
            HIP_TRY(launch_tall_tmul_d(Za, n, b, b, Za, b, part, sm, st));
            std::vector<double> C((size_t)b * b), s2(b), U((size_t)b * b);
            HIP_TRY(hipMemcpyAsync(C.data(), sm, sizeof(double) * b * b, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            glrm_host::sym_eig(b, C.data(), s2.data(), U.data());
            const double smax = std::sqrt(std::max(s2[0], 0.0));
            int r = 0;
            while (r < ks && r < b && s2[r] > 0.0 && std::sqrt(s2[r]) > 1e-6 * smax) ++r;
            if (r > 0) {
                // X = Q U_B,r diag(s^1/2);  Y = diag(sigma) B^T U_B,r diag(s^-1/2) (= V diag(s^1/2))
                std::vector<double> S1((size_t)b * r), S2((size_t)b * r);
                for (int a = 0; a < b; ++a)
                    for (int t = 0; t < r; ++t) {
                        const double sv = std::sqrt(s2[t]);
                        S1[a * r + t] = U[a * b + t] * std::sqrt(sv);
                        S2[a * r + t] = U[a * b + t] / std::sqrt(sv);
                    }
                for (int t = 0; t < r; ++t) svals[t] = std::sqrt(s2[t]);
                double *S1d = sm, *S2d = sm + (size_t)b * r;
                HIP_TRY(hipMemcpyAsync(S1d, S1.data(), sizeof(double) * b * r, hipMemcpyHostToDevice, st));
                HIP_TRY(hipMemcpyAsync(S2d, S2.data(), sizeof(double) * b * r, hipMemcpyHostToDevice, st));
                HIP_TRY(launch_tall_mul_d(Qa, m, b, b, S1d, r, 1.0, 0.0, Qb, st));
                HIP_TRY(launch_tall_mul_d(Za, n, b, b, S2d, r, 1.0, 0.0, Zb, st));
                HIP_TRY(launch_to_float_scaled(Qb, m, r, r, nullptr, X, k, off, st));
                HIP_TRY(launch_to_float_scaled(Zb, n, r, r, sigma2, Y, k, off, st));
                HIP_TRY(hipStreamSynchronize(st));   // S1, S2 live on this host stack
            }
        }
    }
    if (sv_host)
        for (int t = 0; t < ks; ++t) sv_host[t] = svals[t];
    HIP_TRY(hipStreamSynchronize(st));
    return GLRM_OK;
}

int glrm_impute(const glrm_data *d0, const float *X, const float *Y, int32_t mode, float *Ahat, int64_t ldh, void *ws,
                size_t ws_bytes, unsigned flags, void *stream)
{
    g_err.clear();
    Embed E;
    const glrm_data *d = nullptr;
    int rc = embed(d0, E, &d);
    if (rc) return rc;
    if (!X || !Y || !Ahat) return fail(GLRM_EINVAL, "X, Y and Ahat must not be NULL");
    if (mode != GLRM_IMPUTE_ALL && mode != GLRM_IMPUTE_MISSING) return fail(GLRM_EINVAL, "unknown imputation mode %d", mode);
    if (ldh < d0->n) return fail(GLRM_EINVAL, "ldh (%lld) < n (%lld)", (long long)ldh, (long long)d0->n);
    Layout L;
    make_layout(d, L);
    if ((rc = check_ws(L, ws, ws_bytes))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (E.active) {
        // feature by feature: the block's first row of Y, the loss kind and levels
        std::vector<int32_t> info(3 * (size_t)d0->n);
        for (int64_t j = 0, c = 0; j < d0->n; ++j) {
            const glrm_loss &l = d0->losses[d0->col_loss ? d0->col_loss[j] : 0];
            info[(size_t)j] = (int32_t)c;
            info[(size_t)(d0->n + j)] = l.kind;
            info[(size_t)(2 * d0->n + j)] = l.levels;
            c += md_dim(l);
        }
        int32_t *fi = at<int32_t>(ws, L.feat);
        HIP_TRY(hipMemcpyAsync(fi, info.data(), sizeof(int32_t) * info.size(), hipMemcpyHostToDevice, st));
        ImputeMDArgs a;
        a.m = d0->m; a.nf = d0->n; a.ldh = ldh; a.lda = d0->lda; a.k = d0->k;
        a.keep_observed = (mode == GLRM_IMPUTE_MISSING && d0->mask) ? 1 : 0;
        a.fcol = fi; a.fkind = fi + d0->n; a.flev = fi + 2 * d0->n;
        if (mode == GLRM_IMPUTE_MISSING && !d0->mask) {
            HIP_TRY(hipMemcpy2DAsync(Ahat, (size_t)ldh * sizeof(float), d0->A, (size_t)d0->lda * sizeof(float),
                                     (size_t)d0->n * sizeof(float), (size_t)d0->m, hipMemcpyDeviceToDevice, st));
        } else {
            HIP_TRY(launch_impute_md(a, X, Y, d0->A, d0->mask, Ahat, st));
        }
        // the host vector must outlive the copy
        HIP_TRY(hipStreamSynchronize(st));
        return GLRM_OK;
    }
    // the pass needs only the loss codes; a COO list that is about to be
    // written into the output is validated by the full preparation
    if (!(flags & GLRM_WS_PREPARED)) {
        if (d->layout == GLRM_COO_ROWSORTED && mode == GLRM_IMPUTE_MISSING) {
            if ((rc = prepare(d, L, ws, st, E))) return rc;
        } else {
            std::string codes;
            if ((rc = upload_codes(d, L, ws, codes, st))) return rc;
            HIP_TRY(launch_pad_weights(d->col_weight, nullptr, L.n, L.ldp, at<float>(ws, L.colw), st));
            HIP_TRY(hipStreamSynchronize(st));
        }
    }
    const bool dense_keep = d->layout == GLRM_DENSE && mode == GLRM_IMPUTE_MISSING;
    if (dense_keep && !d->mask) {
        // every entry is observed: the table itself
        HIP_TRY(hipMemcpy2DAsync(Ahat, (size_t)ldh * sizeof(float), d->A, (size_t)d->lda * sizeof(float),
                                 (size_t)d->n * sizeof(float), (size_t)d->m, hipMemcpyDeviceToDevice, st));
        return GLRM_OK;
    }
    ImputeArgs a;
    a.m = d->m; a.n = d->n; a.ldh = ldh; a.lda = dense_keep ? d->lda : 0;
    a.k = d->k;
    a.rows_per_block = impute_rows_per_block(d->m, d->n);
    a.keep_observed = dense_keep ? 1 : 0;
    a.codes = at<uint8_t>(ws, L.codes);
    a.lt = make_losstab(d, L, ws);
    HIP_TRY(launch_impute(a, X, Y, dense_keep ? d->A : nullptr, dense_keep ? d->mask : nullptr, Ahat, st));
    if (d->layout == GLRM_COO_ROWSORTED && mode == GLRM_IMPUTE_MISSING)
        HIP_TRY(launch_scatter_observed(d->nnz, d->m, d->n, ldh, d->row, d->col, d->A, Ahat, st));
    return GLRM_OK;
}

int glrm_prox(const glrm_reg *reg, float *V, int64_t rows, int32_t k, int64_t ldv, const float *alpha, void *stream)
{
    g_err.clear();
    if (!reg) return fail(GLRM_EINVAL, "reg is NULL");
    if (reg->kind < GLRM_REG_ZERO || reg->kind > GLRM_REG_NONNEG) return fail(GLRM_EINVAL, "unknown regularizer kind %d", reg->kind);
    if (!(reg->weight >= 0.0f) || !std::isfinite(reg->weight)) return fail(GLRM_EINVAL, "regularizer weight must be finite and >= 0");
    if (rows < 0 || k < 1 || ldv < k) return fail(GLRM_EINVAL, "need rows >= 0, k >= 1, ldv >= k");
    if (rows > 0 && !V) return fail(GLRM_EINVAL, "V is NULL");
    HIP_TRY(launch_prox(make_reg(*reg), V, rows, k, ldv, alpha, (hipStream_t)stream));
    return GLRM_OK;
}

int glrm_fit(const glrm_data *d0, float *X, float *Y, float *alpha_x, float *alpha_y, const glrm_fit_opts *o,
             glrm_fit_info *info, double *history, void *ws, size_t ws_bytes, void *stream)
{
    g_err.clear();
    Embed E;
    const glrm_data *d = nullptr;
    int rc = embed(d0, E, &d);
    if (rc) return rc;
    if (!X || !Y || !alpha_x || !alpha_y || !o) return fail(GLRM_EINVAL, "X, Y, alpha_x, alpha_y and opts must not be NULL");
    if (o->max_sweeps < 0) return fail(GLRM_EINVAL, "max_sweeps < 0");
    if ((rc = check_prec(o->precision, false))) return rc;
    if (!(o->step_up > 0.0f) || !(o->step_down > 0.0f) || !std::isfinite(o->step_up) || !std::isfinite(o->step_down))
        return fail(GLRM_EINVAL, "step factors must be finite and > 0");
    if (o->init_alpha && !(o->alpha_scale > 0.0f && std::isfinite(o->alpha_scale)))
        return fail(GLRM_EINVAL, "alpha_scale must be finite and > 0");
    if (!(o->tol >= 0.0)) return fail(GLRM_EINVAL, "tol must be >= 0");
    if (o->update != GLRM_UPDATE_PROXGRAD && o->update != GLRM_UPDATE_PROXPROX)
        return fail(GLRM_EINVAL, "unknown update rule %d", o->update);
    const bool proxprox = o->update == GLRM_UPDATE_PROXPROX;
    if (proxprox) {
        if (d->layout != GLRM_DENSE) return fail(GLRM_EUNSUPPORTED, "the prox-prox update is built for the dense layout");
        if (o->precision != GLRM_FP32) return fail(GLRM_EUNSUPPORTED, "the prox-prox update computes in FP32 (and FP64 for the solves)");
        if (o->inner < 1 || o->inner > 10000) return fail(GLRM_EINVAL, "inner must be in 1..10000");
        for (int64_t j = 0; j < d->n; ++j) {
            const int q = d->col_loss ? d->col_loss[j] : 0;
            if (d->losses[q].kind != GLRM_LOSS_QUADRATIC)
                return fail(GLRM_EUNSUPPORTED, "the prox-prox update needs the quadratic loss on every column (column %lld)",
                            (long long)j);
        }
    }
    Layout L;
    make_layout(d, L, false, 0, proxprox);
    if ((rc = check_ws(L, ws, ws_bytes))) return rc;
    const int prec = o->precision;
    int tpw = 0, tpw_y = 0;
    if (proxprox) {
        // no pass-shape limits: the Gram, solve and check passes take any width
    } else if (d->layout == GLRM_DENSE) {
        // tpw == 0: too wide for the fused row pass, which then runs in column blocks
        tpw = tpw_xstep(L.ldp / 16, (int)L.kp);
        tpw_y = tpw_ycheck(L.ldp / 16, (int)L.kp);
    } else {
        if ((rc = coo_fit_supported(d, L.kp, L.cl, prec))) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    if (info) memset(info, 0, sizeof *info);
    KernelTimer timer;
    if ((rc = timer.init((o->flags & GLRM_TIME_KERNELS) != 0, (size_t)o->max_sweeps * 4))) return rc;
    if (!(o->flags & GLRM_WS_PREPARED) && (rc = prepare(d, L, ws, st, E))) return rc;
    if (o->init_alpha) {
        HIP_TRY(launch_init_alpha(at<int32_t>(ws, L.row_count), L.m, o->alpha_scale, alpha_x, st));
        HIP_TRY(launch_init_alpha(at<int32_t>(ws, L.col_count), L.n, o->alpha_scale, alpha_y, st));
    }
    const LossTab lt = make_losstab(d, L, ws);
    double *stats = at<double>(ws, L.stats);
    long long *istats = at<long long>(ws, L.istats);
    int sweeps = 0;
    double F_prev = NAN;

    if (proxprox) {
        // the transposed table serves the column half-step as rows
        HIP_TRY(launch_transpose(at<float>(ws, L.Ap), L.mp, L.ldp, at<float>(ws, L.pp_At), st));
        PPArgs px;
        memset(&px, 0, sizeof px);
        px.rows = L.m; px.cols = L.n; px.ldt = L.ldp; px.k = (int32_t)L.k; px.kp = (int32_t)L.kp;
        px.T = at<float>(ws, L.Ap);
        px.wcol = at<float>(ws, L.colw);
        px.wrow = nullptr;
        px.U = X; px.V = Y; px.alpha = alpha_x; px.reg = reg_x(d);
        px.inner = o->inner; px.step_up = o->step_up; px.step_down = o->step_down;
        px.gram = at<float>(ws, L.pp_gram); px.gpart = at<float>(ws, L.pp_gpart); px.splits = 1;
        px.trial = at<float>(ws, L.pp_trial); px.fpart = at<float>(ws, L.pp_fpart);
        px.rowobj = at<double>(ws, L.pp_objx); px.obj_with_loss = 0; px.rej = at<int32_t>(ws, L.pp_rejx);
        PPArgs py = px;
        py.rows = L.n; py.cols = L.m; py.ldt = L.mp;
        py.T = at<float>(ws, L.pp_At);
        py.wcol = nullptr;
        py.wrow = at<float>(ws, L.colw);
        py.U = Y; py.V = X; py.alpha = alpha_y; py.reg = reg_y(d);
        py.splits = (int32_t)std::min<int64_t>(PP_SPLITS_MAX, std::max<int64_t>(1, L.m / 1024));
        py.rowobj = at<double>(ws, L.pp_objy); py.obj_with_loss = 1; py.rej = at<int32_t>(ws, L.pp_rejy);
        for (int t = 0; t < o->max_sweeps; ++t) {
            HIP_TRY(timer.start(0, st));
            HIP_TRY(launch_pp_gram(px, st));
            HIP_TRY(timer.stop(st));
            HIP_TRY(timer.start(1, st));
            HIP_TRY(launch_pp_solve(px, st));
            HIP_TRY(launch_pp_check(px, st));
            HIP_TRY(timer.stop(st));
            HIP_TRY(timer.start(2, st));
            HIP_TRY(launch_pp_gram(py, st));
            HIP_TRY(launch_pp_solve(py, st));
            HIP_TRY(launch_pp_check(py, st));
            HIP_TRY(timer.stop(st));
            HIP_TRY(timer.start(3, st));
            HIP_TRY(launch_pp_finalize(px.rowobj, px.rej, L.m, py.rowobj, py.rej, L.n, at<double>(ws, L.pp_fin), stats,
                                       istats, history, t, st));
            HIP_TRY(timer.stop(st));
            sweeps = t + 1;
            if (o->tol > 0.0) {
                double F;
                HIP_TRY(hipMemcpyAsync(&F, stats, sizeof(double), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                if (t > 0 && (F_prev - F) <= o->tol * std::fabs(F_prev)) break;
                F_prev = F;
            }
        }
    } else if (d->layout == GLRM_DENSE) {
        if ((rc = write_shadows(L, Y, ws, prec, true, st))) return rc;
        const int64_t npanels = L.mp / 16;
        // persistent grids: as many workgroups as fit on the device at once
        int dev = 0, cus = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const bool quad = make_lossu(lt).kind == L_QUAD;
        const bool wide = L.wide;
        // the row half-step in column blocks: row chunks of the two row-sum
        // passes, of the column pass (its Y-gradient partials, P_GRAD in
        // all) and of the decisions
        const int ncb_w = (int)L.wide_ncb;
        const int gx_rows = (int)std::min<int64_t>(P_GRAD, npanels);
        // the column pass fills the device once (its partials, one per row
        // chunk, are reduced by yprox)
        const int gx_cols = wide ? (int)std::max<int64_t>(1, std::min<int64_t>(
                                       {(int64_t)L.pmax, npanels,
                                        (int64_t)cus * xwide_blocks((int)L.kp, L.wide_tpw, prec, quad) / ncb_w}))
                                 : 0;
        const int grid_dec = (int)std::min<int64_t>(L.pmax, (L.m + 63) / 64);
        const int grid = wide ? gx_cols
                              : (int)std::min<int64_t>({(int64_t)L.pmax, npanels,
                                                        (int64_t)cus * xstep_blocks((int)L.kp, tpw, prec, quad)});
        // A table wider than 4 tiles per wavefront runs the trial-column pass
        // in column blocks of 4 tiles per wavefront, so two workgroups fit on
        // a CU; the partial rows stay one per panel stream.
        int ncb_y = 1;
        if (tpw_y > 4 || tpw_y == 0) {
            tpw_y = 4;
            ncb_y = (int)((L.ldp / 16 + 4 * ycheck_waves((int)L.kp) - 1) / (4 * ycheck_waves((int)L.kp)));
        }
        const int grid_y = ncb_y * (int)std::max<int64_t>(1, std::min<int64_t>(
            {(int64_t)L.pmax, npanels, (int64_t)cus * ycheck_blocks((int)L.kp, tpw_y, prec, quad) / ncb_y}));
        XStepArgs xa;
        xa.m = L.m; xa.mp = L.mp; xa.ldp = L.ldp; xa.k = (int32_t)L.k;
        xa.Ap = at<float>(ws, L.Ap);
        xa.codes = at<uint8_t>(ws, L.codes);
        xa.lt = lt;
        xa.lu = make_lossu(lt);
        xa.rx = reg_x(d);
        xa.X = X;
        xa.alpha = alpha_x;
        xa.step_up = o->step_up; xa.step_down = o->step_down;
        xa.ycur = shadow(ws, L, false);
        xa.part_dy = at<float>(ws, L.part_dy);
        xa.part_h = at<float>(ws, L.part_h);
        xa.part_rowreg = at<float>(ws, L.part_rowreg);
        xa.part_rej = at<int32_t>(ws, L.part_rej);

        XWideArgs wa0;
        memset(&wa0, 0, sizeof wa0);
        wa0.m = L.m; wa0.mp = L.mp; wa0.ldp = L.ldp; wa0.k = (int32_t)L.k;
        wa0.Ap = xa.Ap; wa0.codes = xa.codes; wa0.lt = lt; wa0.lu = xa.lu;
        wa0.X = X; wa0.ycur = xa.ycur;
        wa0.part_f = wide ? at<float>(ws, L.wd_f) : nullptr;
        wa0.part_dx = wide ? at<float>(ws, L.part_dx) : nullptr;
        XWideArgs wa1 = wa0;
        wa1.X = wide ? at<float>(ws, L.wd_xp) : nullptr;
        wa1.part_f = wide ? at<float>(ws, L.wd_fp) : nullptr;
        wa1.part_dx = nullptr;
        XWideArgs wa2 = wa0;
        wa2.part_f = nullptr; wa2.part_dx = nullptr;
        wa2.part_dy = xa.part_dy; wa2.part_h = xa.part_h;
        XWideRowArgs ra;
        memset(&ra, 0, sizeof ra);
        ra.m = L.m; ra.mp = L.mp; ra.k = (int32_t)L.k; ra.ncb = ncb_w;
        ra.rx = xa.rx; ra.X = X; ra.alpha = alpha_x;
        ra.part_f = wa0.part_f; ra.part_fp = wa1.part_f; ra.part_dx = wa0.part_dx;
        ra.Xp = wide ? at<float>(ws, L.wd_xp) : nullptr;
        ra.rsum = wide ? at<float>(ws, L.wd_rsum) : nullptr;
        ra.step_up = o->step_up; ra.step_down = o->step_down;
        ra.part_rowreg = xa.part_rowreg; ra.part_rej = xa.part_rej;

        YProxArgs pa;
        pa.n = L.n; pa.ldp = L.ldp; pa.k = (int32_t)L.k; pa.P = grid;
        pa.part_dy = xa.part_dy; pa.part_h = xa.part_h;
        pa.ry = reg_y(d);
        pa.Y = Y; pa.alpha = alpha_y;
        pa.Yplus = at<float>(ws, L.Yplus);
        pa.yplus = shadow(ws, L, true);
        pa.h_old = at<float>(ws, L.h_old);
        pa.ry_plus = at<float>(ws, L.ry_plus);
        pa.ry_old = at<float>(ws, L.ry_old);

        YCheckArgs ca;
        ca.m = L.m; ca.mp = L.mp; ca.ldp = L.ldp; ca.k = (int32_t)L.k;
        ca.Ap = xa.Ap; ca.codes = xa.codes; ca.lt = lt; ca.lu = xa.lu; ca.X = X;
        ca.yplus = pa.yplus;
        ca.part_hp = at<float>(ws, L.part_hp);
        ca.ncb = ncb_y;

        YAcceptArgs aa;
        aa.n = L.n; aa.ldp = L.ldp; aa.k = (int32_t)L.k; aa.P = grid_y / ncb_y;
        aa.part_hp = ca.part_hp; aa.ry_plus = pa.ry_plus; aa.h_old = pa.h_old;
        aa.alpha = alpha_y; aa.step_up = o->step_up; aa.step_down = o->step_down;
        aa.Yplus = pa.Yplus; aa.Y = Y;
        aa.yplus = pa.yplus; aa.ycur = xa.ycur;
        aa.part_F = at<double>(ws, L.part_F);
        aa.part_rejc = at<int32_t>(ws, L.part_rejc);
        aa.phase = E.active ? 2 : 0;
        aa.hpc = at<float>(ws, L.hpc);
        aa.blk0 = E.active ? at<int32_t>(ws, L.blk0) : nullptr;
        aa.blk1 = E.active ? at<int32_t>(ws, L.blk1) : nullptr;
        YAcceptArgs aa1 = aa;
        aa1.phase = 1;
        const int ya_blocks = yaccept_blocks(L.n, (int)L.kp);

        FinalizeArgs fa;
        fa.part_F = aa.part_F; fa.part_rejc = aa.part_rejc; fa.n_colparts = ya_blocks;
        fa.part_rowreg = xa.part_rowreg; fa.part_rej = xa.part_rej; fa.n_rowparts = wide ? grid_dec : grid;
        fa.stats = stats; fa.istats = istats; fa.history = history;

        for (int t = 0; t < o->max_sweeps; ++t) {
            HIP_TRY(timer.start(0, st));
            if (wide) {
                HIP_TRY(launch_xwide(wa0, 0, (int)L.kp, L.wide_tpw, prec, gx_rows, ncb_w, st));
                HIP_TRY(launch_xwide_step(ra, st));
                HIP_TRY(launch_xwide(wa1, 1, (int)L.kp, L.wide_tpw, prec, gx_rows, ncb_w, st));
                HIP_TRY(launch_xwide_decide(ra, grid_dec, st));
                HIP_TRY(launch_xwide(wa2, 2, (int)L.kp, L.wide_tpw, prec, gx_cols, ncb_w, st));
            } else {
                HIP_TRY(launch_xstep(xa, (int)L.kp, tpw, prec, grid, st));
            }
            HIP_TRY(timer.stop(st));
            HIP_TRY(timer.start(1, st));
            HIP_TRY(launch_yprox(pa, (int)L.kp, prec, st));
            HIP_TRY(timer.stop(st));
            HIP_TRY(timer.start(2, st));
            HIP_TRY(launch_ycheck(ca, (int)L.kp, tpw_y, prec, grid_y, st));
            HIP_TRY(timer.stop(st));
            HIP_TRY(timer.start(3, st));
            if (E.active) HIP_TRY(launch_yaccept(aa1, (int)L.kp, prec, ya_blocks, st));
            HIP_TRY(launch_yaccept(aa, (int)L.kp, prec, ya_blocks, st));
            fa.sweep = t;
            HIP_TRY(launch_finalize(fa, st));
            HIP_TRY(timer.stop(st));
            sweeps = t + 1;
            if (o->tol > 0.0) {
                double F;
                HIP_TRY(hipMemcpyAsync(&F, stats, sizeof(double), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                if (t > 0 && (F_prev - F) <= o->tol * std::fabs(F_prev)) break;
                F_prev = F;
            }
        }
    } else {
        rc = coo_fit(d, L.kp, L.cl, at<char>(ws, L.coo), at<uint8_t>(ws, L.codes), lt, X, Y, alpha_x, alpha_y, o,
                     history, stats, istats, &sweeps, st,
                     [&](int k) { return timer.start(k, st); }, [&]() { return timer.stop(st); });
        if (rc != GLRM_OK) return rc;
    }

    double *obj64 = at<double>(ws, L.scal) + 1;
    if ((rc = objective64(d, L, X, Y, ws, obj64, st))) return rc;
    double hs[2] = {0, 0};
    long long is[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&hs[0], obj64, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&hs[1], stats, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(is, istats, 2 * sizeof(long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    timer.report(info);
    if (info) {
        info->sweeps = sweeps;
        info->objective = hs[0];
        info->objective_fp32 = sweeps > 0 ? hs[1] : NAN;
        info->rows_rejected = sweeps > 0 ? is[0] : 0;
        info->cols_rejected = sweeps > 0 ? is[1] : 0;
    }
    return GLRM_OK;
}

}  // extern "C"
