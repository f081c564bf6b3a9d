"""Shared set-up for the GPU parity tests: the same seeded case goes to the
HIP library (through the C ABI binding) and to the FP64 oracle."""
import numpy as np

import oracle


def _f32(x):
    return float(np.float32(x))


def oracle_problem(case):
    """The oracle receives exactly what the C ABI carries: float32 weights and
    loss parameters."""
    losses = [(int(a), int(b), _f32(c)) for a, b, c in case.losses]
    rx = (int(case.rx[0]), _f32(case.rx[1]))
    ry = (int(case.ry[0]), _f32(case.ry[1]))
    if case.layout == "coo":
        return oracle.Problem.from_coo(case.m, case.n, case.k, case.rows, case.cols, case.vals, case.col_loss,
                                       losses, rx, ry)
    return oracle.Problem.from_dense(case.A, case.mask, case.k, case.col_loss, losses, rx, ry)


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel_fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---- decisions near a tie ------------------------------------------------------
#
# The GPU forms its step x+ = prox(x - alpha g) from a gradient g that carries
# rounding error (bound: grad_eps below).  A gradient coordinate is a sum of
# terms G_ij y_jc; its error is bounded by the four sources listed below, in
# units of the sum of their magnitudes S_c = sum_j |G_ij| |y_jc| (the oracle's
# grad_abs) and of their root sum of squares R_c (grad_rss).  The prox
# operators are nonexpansive, so each coordinate of the GPU's trial point lies
# within eps_c = 2 alpha (that bound) of the oracle's.  The trial objective
# then moves by at most sum_c S+_c eps_c to first order (S+ is the same
# magnitude sum at the trial point, plus the regularizer's slope); the band
# doubles that for the second-order term and adds the float32 rounding of the
# objective sums themselves (sqrt(n) 2^-24 relative for n <= 2e4 terms).  A
# decision whose margin |f+ - f| lies inside the band may legitimately go
# either way; every other decision must match the oracle's.

GRAD_REL = {"fp32": 0.0, "bf16": 2.0 ** -8, "coo_bf16": 0.0}
SUM_REL = 1e-5
# Four sources.  (1) The derivative operand: the BF16 form rounds every
# G_ij to bfloat16 (round to nearest even).  These errors are not independent:
# a derivative that saturates (the logistic one near +-1)
# piles up just below a power of two and always rounds the same way.  So
# their sum E_c = sum_j (bf16(G_ij) - G_ij) v_jc is computed exactly from the
# oracle's derivatives.  (2) The factor operand, also rounded to bfloat16:
# worst case 2^-8 of S_c (all errors of one sign); factor values spread over
# many units in the last place, so their rounding errors are independent and
# uniform within half a unit, 2^-8 relative at most: the sum's standard
# deviation is at most 2^-8 / sqrt(3) of the root of the squared terms R_c,
# and 2^-6 R_c is about seven of them; the smaller bound is taken.  FP32
# products are exact to 2^-24, below (3).  (3) The float32 accumulation: a sum
# of N terms added in sequence errs by at most (N - 1) 2^-24 of S_c, and the
# kernels add runs of at most about 2^10 terms in sequence (a workgroup's rows
# or a wavefront's chunk) before fixed-order reductions of the partials, so
# the accumulated error stays below min(N, 2^10) 2^-24 of S_c, N the row's
# (column's) observed count; a float32 product's own rounding adds 2^-24.
# (4) The rounding of z = x . y itself, |z_gpu - z| <= z_rel sum_c |x_c||y_c|
# (FP32: k float32 products and their sum, (k + 1) 2^-24; BF16: three
# bfloat16 products per coordinate, whose dropped lo*lo term and rounded lo
# parts leave about 3 2^-18, and the float32 sums, under 2^-14 in all).  A smooth loss passes it on to G scaled by its curvature
# (quadratic 2, Huber 1, logistic 1/4); a kinked loss (hinge, ordinal hinge)
# passes nothing on, except where a kink lies within that distance of z: there
# the derivative may take either side, a step of 1 per term that kinks there.
RSS_REL = {"fp32": None, "bf16": 2.0 ** -6, "coo_bf16": None}
ACC_RUN = 2 ** 10
CURVATURE = {0: 2.0, 1: 1.0, 2: 0.25, 3: 0.0, 4: 0.0}


def bf16_round(a):
    """float64 -> float32 -> bfloat16 (round to nearest even) -> float64."""
    b = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def acc_rel(P, which):
    """Source (3) per row (which = "x") or column: (min(N, 2^10) + 1) 2^-24."""
    a = P.init_alpha(1.0)[0 if which == "x" else 1]      # 1 / max(N, 1)
    return (np.minimum(np.rint(1.0 / a), ACC_RUN) + 1.0) * 2.0 ** -24


def _kink_steps(kind, levels, a, u, dz):
    """Size of the derivative's jumps within dz of u (0 where there are none)."""
    out = np.zeros_like(u)
    h = kind == 3                                   # hinge: kink at u = a (a = +-1)
    out[h] = (np.abs(u[h] - a[h]) <= dz[h]).astype(np.float64)
    o = kind == 4                                   # ordinal hinge: kinks at 2..a and a..levels-1
    if o.any():
        uo, ao, lo, do = u[o], a[o], levels[o].astype(np.float64), dz[o]
        t = np.clip(np.rint(uo), 1.0, lo)           # the nearest integer in range
        is_kink = ((t >= 2) & (t <= ao)) | ((t >= ao) & (t <= lo - 1))
        steps = np.where((t == ao) & (ao >= 2) & (ao <= lo - 1), 2.0, 1.0)
        out[o] = np.where(is_kink & (np.abs(uo - t) <= do), steps, 0.0)
    return out


def z_terms(P, which, X, Y, prec):
    """Source (4) per coordinate: sum over the row's (column's) observed
    entries of w (curvature dz + kink steps) |v_c|."""
    view = P.row if which == "x" else P.colv
    U, V = (np.asarray(X, np.float64), np.asarray(Y, np.float64))
    if which != "x":
        U, V = V, U
    rows = np.repeat(np.arange(view.m), np.diff(view.row_ptr))
    other = view.col.astype(np.int64)
    Ur, Vo = U[rows], V[other]
    u = np.einsum("ij,ij->i", Ur, Vo)
    z_rel = (U.shape[1] + 1) * 2.0 ** -24 if prec in ("fp32", "coo_bf16") else 2.0 ** -14
    dz = z_rel * np.einsum("ij,ij->i", np.abs(Ur), np.abs(Vo))
    kinds = np.array([l[0] for l in P.losses], np.int64)[view.ecode]
    levels = np.array([l[1] for l in P.losses], np.int64)[view.ecode]
    curv = np.array([CURVATURE[int(l[0])] for l in P.losses])[view.ecode]
    term = curv * dz + _kink_steps(kinds, levels, view.val, u, dz)
    if view.ew is not None:
        term = term * view.ew
    out = np.zeros((view.m, U.shape[1]))
    for c in range(U.shape[1]):
        out[:, c] = np.bincount(rows, weights=term * np.abs(Vo[:, c]), minlength=view.m)
    return out


def grad_eps(P, which, X, Y, alpha, prec):
    """Per-coordinate bound on |x+_gpu - x+_oracle| from the gradient's rounding."""
    S = P.grad_abs(X, Y)[0 if which == "x" else 1]
    bound = GRAD_REL[prec] * S
    if RSS_REL[prec] is not None:
        R = P.grad_rss(X, Y)[0 if which == "x" else 1]
        bound = np.minimum(bound, RSS_REL[prec] * R)
        G = P.grad_matrix(X, Y)
        dG = bf16_round(G) - G
        X64, Y64 = np.asarray(X, np.float64), np.asarray(Y, np.float64)
        bound = bound + np.abs(dG @ Y64 if which == "x" else dG.T @ X64)
    bound = bound + acc_rel(P, which)[:, None] * S + z_terms(P, which, X, Y, prec)
    return 2.0 * np.asarray(alpha, np.float64)[:, None] * bound


def _reg_slope(reg, V, offset=0):
    kind, w = reg
    if kind == 1:
        out = 2.0 * w * np.abs(V)
    elif kind == 2:
        out = np.full_like(V, w)
    else:
        out = np.zeros_like(V)
    if offset:
        out[:, 0] = 0.0      # the offset coordinate carries no penalty
    return out


def _trial(reg, V, g, alpha, offset=0):
    out = np.empty_like(V)
    for i in range(V.shape[0]):
        out[i] = oracle.prox(reg[0], reg[1], float(alpha[i]), V[i] - alpha[i] * g[i], offset)
    return out


def _offsets(P):
    """Offset codes of the X and Y regularizers (Section 3.3)."""
    return (1, 2) if getattr(P, "offset", False) else (0, 0)


# The sparse layout's BF16 form computes the gradient and the trial point as
# FP32 does ("coo_bf16" takes the FP32 bounds above), but evaluates the trial
# objective from z_ij + d . v_j with the step d = u+ - u and the gathered row
# v_j both in bfloat16: each trial product errs by at most 2^-8 sum_c |d_c| |v_jc|
# (two roundings of 2^-9), which moves the trial objective by at most
# (|G(z+)| + a kink's step + curvature / 2 times that) times that error, entry by entry.
def trial_bf16_terms(P, which, U0, Ut, V):
    """Per row (which = "x") or column: the bound on the trial objective's
    error in the sparse BF16 form."""
    view = P.row if which == "x" else P.colv
    U0, Ut, V = (np.asarray(a, np.float64) for a in (U0, Ut, V))
    rows = np.repeat(np.arange(view.m), np.diff(view.row_ptr))
    other = view.col.astype(np.int64)
    D = np.abs(Ut - U0)
    dz = 2.0 ** -8 * np.einsum("ij,ij->i", D[rows], np.abs(V[other]))
    u = np.einsum("ij,ij->i", Ut[rows], V[other])
    G = P.grad_matrix(Ut, V) if which == "x" else P.grad_matrix(V, Ut).T
    kinds = np.array([l[0] for l in P.losses], np.int64)[view.ecode]
    levels = np.array([l[1] for l in P.losses], np.int64)[view.ecode]
    curv = np.array([CURVATURE[int(l[0])] for l in P.losses])[view.ecode]
    slope = np.abs(G[rows, other]) + _kink_steps(kinds, levels, view.val, u, dz) + 0.5 * curv * dz
    term = slope * dz
    if view.ew is not None:
        term = term * view.ew
    return np.bincount(rows, weights=term, minlength=view.m)


def band_rows(P, X, Y, ax, f_old, f_new, prec):
    """Decision band of every row of the X half-step at (X, Y) with step sizes ax."""
    X, Y = np.asarray(X, np.float64), np.asarray(Y, np.float64)
    g, _ = P.grad(X, Y)
    ox = _offsets(P)[0]
    Xp = _trial(P.rx, X, g, ax, ox)
    Sp, _ = P.grad_abs(Xp, Y)
    eps = grad_eps(P, "x", X, Y, ax, prec)
    first = np.sum((Sp + _reg_slope(P.rx, Xp, ox)) * eps, axis=1)
    if prec == "coo_bf16":
        first = first + trial_bf16_terms(P, "x", X, Xp, Y)
    return 2.0 * first + SUM_REL * (np.abs(f_old) + np.abs(f_new))


def band_cols(P, X, Y, ay, h_old, h_new, prec):
    """Decision band of every column of the Y half-step at (X^t, Y)."""
    X, Y = np.asarray(X, np.float64), np.asarray(Y, np.float64)
    _, g = P.grad(X, Y)
    oy = _offsets(P)[1]
    Yp = _trial(P.ry, Y, g, ay, oy)
    _, Sp = P.grad_abs(X, Yp)
    eps = grad_eps(P, "y", X, Y, ay, prec)
    first = np.sum((Sp + _reg_slope(P.ry, Yp, oy)) * eps, axis=1)
    if prec == "coo_bf16":
        first = first + trial_bf16_terms(P, "y", Y, Yp, X)
    return 2.0 * first + SUM_REL * (np.abs(h_old) + np.abs(h_new))


def clear_decisions(f_old, f_new, band):
    """True where the oracle's accept / reject decision has a margin beyond the band."""
    f_old, f_new = np.asarray(f_old), np.asarray(f_new)
    with np.errstate(invalid="ignore"):
        return ~(np.isfinite(f_old) & np.isfinite(f_new)) | (np.abs(f_new - f_old) > band)


def _check_half(P, which, U0, V, alpha0, Ugpu, alpha_gpu, prec, step_up=1.05, step_down=0.7, tag=""):
    """One half-step of the GPU checked against the oracle's from the same
    state.  `which` is "x" (rows of X against Y = V) or "y" (columns of Y
    against X^t = V).  Every row is checked:
      * its decision (read from the step size, which moved by step_up or
        step_down) equals the oracle's wherever the oracle's margin lies
        outside the band;
      * an accepted row equals the oracle's trial point within the rounding
        bound eps_c of its gradient (+ float32 rounding of the value);
      * a rejected row is bit-for-bit the old row.
    Returns (number of decisions inside the band, number of them the GPU took
    the other way)."""
    U0 = np.asarray(U0, np.float64)
    V = np.asarray(V, np.float64)
    alpha0 = np.asarray(alpha0, np.float64)
    Uo = U0.copy()
    ao = alpha0.copy()
    if which == "x":
        X0, Y0 = U0, V
        _, f_old, f_new, acc_o = P.half_step_x(Uo, V, ao, step_up, step_down)
        band = band_rows(P, X0, Y0, alpha0, f_old, f_new, prec)
        g, _ = P.grad(X0, Y0)
        reg, off = P.rx, _offsets(P)[0]
    else:
        X0, Y0 = V, U0
        _, f_old, f_new, acc_o = P.half_step_y(V, Uo, ao, step_up, step_down)
        band = band_cols(P, X0, Y0, alpha0, f_old, f_new, prec)
        _, g = P.grad(X0, Y0)
        reg, off = P.ry, _offsets(P)[1]
    trial = _trial(reg, U0, g, alpha0, off)
    # the float32 rounding of x - alpha g and of the prox adds 2^-22 of |x| + |x+|
    eps = grad_eps(P, which, X0, Y0, alpha0, prec) + 2.0 ** -22 * (np.abs(trial) + np.abs(U0)) + 1e-30
    return compare_half(tag, "rows" if which == "x" else "columns", U0, Ugpu, alpha0, alpha_gpu, acc_o, f_old, f_new,
                        band, trial, eps, step_up, step_down)


def compare_half(tag, what, U0, Ugpu, alpha0, alpha_gpu, acc_o, f_old, f_new, band, trial, eps, step_up=1.05,
                 step_down=0.7, blocks=None):
    """The checks of one half-step, given the oracle's outcome: decisions
    (read from the GPU's step sizes) equal wherever the oracle's margin
    clears the band; rejected rows bit-for-bit unchanged; accepted rows within
    eps of the oracle's trial point.  With ``blocks`` (the first row of each
    block, then the end) the rows move in blocks: acc_o, f_old, f_new and band
    are per block, and every row of a block must take the block's decision.
    Returns (decisions inside the band, of them taken the other way, GPU
    decisions)."""
    U0 = np.asarray(U0, np.float64)
    alpha0 = np.asarray(alpha0, np.float64)
    Ugpu = np.asarray(Ugpu, np.float32)
    alpha_gpu = np.asarray(alpha_gpu, np.float64)
    ratio = alpha_gpu / np.maximum(alpha0, 1e-300)
    acc_g = np.abs(ratio - step_up) <= 1e-6 * step_up
    rej_g = np.abs(ratio - step_down) <= 1e-6 * step_down
    assert np.all(acc_g | rej_g), "%s: step sizes moved by neither factor" % tag
    acc_r = acc_g
    if blocks is not None:
        blocks = np.asarray(blocks)
        sizes = np.diff(blocks)
        cnt = np.add.reduceat(acc_g.astype(np.int64), blocks[:-1])
        assert np.all((cnt == 0) | (cnt == sizes)), "%s: a block's columns took different decisions" % tag
        acc_g = cnt == sizes
    clear = clear_decisions(f_old, f_new, band)
    acc_o = np.asarray(acc_o).astype(bool)
    bad = np.nonzero(clear & (acc_g != acc_o))[0]
    assert bad.size == 0, "%s: decisions differ on clear %s %s (margin %s, band %s)" % (
        tag, what, bad[:8], (np.asarray(f_new) - np.asarray(f_old))[bad[:8]], np.asarray(band)[bad[:8]])
    U0_32 = U0.astype(np.float32)
    rej_r = ~acc_r
    assert np.array_equal(Ugpu[rej_r], U0_32[rej_r]), "%s: a rejected row changed" % tag
    if acc_r.any():
        diff = np.abs(Ugpu[acc_r].astype(np.float64) - trial[acc_r])
        worst = np.max(diff / eps[acc_r])
        assert worst <= 1.0, "%s: accepted trial point off by %.3g of its rounding bound" % (tag, worst)
    return int((~clear).sum()), int((~clear & (acc_g != acc_o)).sum()), acc_g


def guided_half(P, which, U, V, alpha, gpu_acc, prec, step_up=1.05, step_down=0.7):
    """The oracle's half-step from (U, alpha) against V, except that every
    decision inside its rounding band takes the branch the GPU took
    (gpu_acc).  Either branch is a correct outcome there; following the GPU's
    lets a multi-sweep comparison isolate the arithmetic error.  Returns the
    new (U, alpha)."""
    U = np.asarray(U, np.float64)
    alpha = np.asarray(alpha, np.float64)
    Uo, ao = U.copy(), alpha.copy()
    if which == "x":
        _, f_old, f_new, acc_o = P.half_step_x(Uo, V, ao, step_up, step_down)
        band = band_rows(P, U, V, alpha, f_old, f_new, prec)
        g, _ = P.grad(U, V)
        reg, off = P.rx, _offsets(P)[0]
    else:
        _, f_old, f_new, acc_o = P.half_step_y(V, Uo, ao, step_up, step_down)
        band = band_cols(P, V, U, alpha, f_old, f_new, prec)
        _, g = P.grad(V, U)
        reg, off = P.ry, _offsets(P)[1]
    acc = np.where(clear_decisions(f_old, f_new, band), acc_o.astype(bool), np.asarray(gpu_acc, bool))
    trial = _trial(reg, U, g, alpha, off)
    return np.where(acc[:, None], trial, U), alpha * np.where(acc, step_up, step_down)


def check_sweep(P, X0, Y0, ax0, ay0, Xg, Yg, axg, ayg, prec, tag=""):
    """A GPU sweep from (X0, Y0, ax0, ay0) to (Xg, Yg, axg, ayg) checked half by
    half: the rows against the oracle's X half-step from the same state, the
    columns against the oracle's Y half-step from the GPU's own X^t (so both
    halves are compared like for like).  Returns the near-tie counts."""
    nr = _check_half(P, "x", X0, Y0, ax0, Xg, axg, prec, tag=tag + " rows")
    nc = _check_half(P, "y", Y0, Xg, ay0, Yg, ayg, prec, tag=tag + " columns")
    return dict(band_rows=nr[0], band_cols=nc[0], flipped=nr[1] + nc[1], acc_rows=nr[2], acc_cols=nc[2])


def init_alpha32(P, scale):
    """The step sizes the GPU starts from: scale / max(n_i, 1) in float32."""
    ax, ay = P.init_alpha(1.0)          # 1 / max(n_i, 1)
    cx = np.rint(1.0 / ax).astype(np.float32)
    cy = np.rint(1.0 / ay).astype(np.float32)
    return (np.float32(scale) / cx).astype(np.float64), (np.float32(scale) / cy).astype(np.float64)
