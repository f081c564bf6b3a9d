"""Pins for the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
formulas: values come from hand-worked fixtures, closed forms, library
routines (SVD, norms, scalar minimisation) and invariants.
"""
import json
import os

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load_losses():
    rows = []
    for line in open(os.path.join(GOLD, "losses.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        kind, levels, param, u, a, val, der = line.split()
        rows.append((int(kind), int(levels), float(param), float(u), float(a), float(val), float(der)))
    return rows


@pytest.mark.parametrize("row", _load_losses())
def test_loss_hand_values(row):
    """Hand-worked values of each loss (Sections 2.2, 4.2, 5.2, eq. ord-pca)."""
    kind, levels, param, u, a, val, der = row
    assert oracle.loss(kind, u, a, levels, param) == pytest.approx(val, rel=1e-14, abs=1e-14)
    assert oracle.dloss(kind, u, a, levels, param) == pytest.approx(der, rel=1e-14, abs=1e-14)


SMOOTH = [(0, 0, 0.0), (1, 0, 1.0), (1, 0, 0.3), (2, 0, 0.0)]
KINKED = [(3, 0, 0.0), (4, 5, 0.0), (4, 7, 0.0)]


@pytest.mark.parametrize("loss", SMOOTH + KINKED)
def test_loss_derivative_matches_central_difference(loss):
    """dL/du against FP64 central differences away from kinks (Section 7.2
    uses the gradient of each loss)."""
    kind, levels, param = loss
    g = np.random.default_rng(7)
    h = 1e-6
    checked = 0
    for _ in range(400):
        if kind in (2, 3):
            a = float(g.choice([-1.0, 1.0]))
        elif kind == 4:
            a = float(g.integers(1, levels + 1))
        else:
            a = float(g.normal() * 3)
        u = float(g.normal() * 4)
        # stay off kinks: hinge at a*u = 1, ordinal at integers +- 1, Huber at |u-a| = param
        if kind == 3 and abs(a * u - 1.0) < 1e-3:
            continue
        if kind == 4 and abs(u - round(u)) < 1e-3:
            continue
        fd = (oracle.loss(kind, u + h, a, levels, param) - oracle.loss(kind, u - h, a, levels, param)) / (2 * h)
        assert oracle.dloss(kind, u, a, levels, param) == pytest.approx(fd, rel=1e-6, abs=1e-6)
        checked += 1
    assert checked > 300


@pytest.mark.parametrize("loss", KINKED + [(1, 0, 1.0)])
def test_subgradient_inequality_at_kinks(loss):
    """At a kink the chosen value must still be a subgradient (Section 7.2):
    L(u + t) >= L(u) + g t for t of both signs."""
    kind, levels, param = loss
    if kind == 3:
        pts = [(1.0, 1.0), (-1.0, -1.0)]
    elif kind == 1:
        pts = [(2.0 + param, 2.0), (2.0 - param, 2.0)]
    else:
        pts = [(float(u), float(a)) for a in range(1, levels + 1) for u in range(0, levels + 2)]
    for u, a in pts:
        g = oracle.dloss(kind, u, a, levels, param)
        for t in (1e-3, -1e-3, 0.5, -0.5, 2.0, -2.0):
            assert oracle.loss(kind, u + t, a, levels, param) >= oracle.loss(kind, u, a, levels, param) + g * t - 1e-12


def test_ordinal_hinge_is_zero_at_its_level_and_grows_one_per_level():
    """eq. ord-pca: zero at u = a, and one unit per level of error beyond the
    neighbouring level."""
    d = 7
    for a in range(1, d + 1):
        assert oracle.loss(4, float(a), float(a), d) == 0.0
        for s in range(1, d - a + 1):  # u = a + s: hinges a' = a+1 .. a+s contribute s, s-1, ..., 1
            assert oracle.loss(4, float(a + s), float(a), d) == pytest.approx(s * (s + 1) / 2)


@pytest.mark.parametrize("kind,w", [(0, 0.0), (1, 0.3), (1, 2.0), (2, 0.4), (2, 1.5), (3, 0.0)])
def test_prox_is_the_minimiser_of_its_definition(kind, w):
    """prox_{alpha r}(v) = argmin_x alpha r(x) + 1/2 ||x - v||^2 (Section 7.2),
    checked against bounded scalar minimisation coordinate by coordinate."""
    g = np.random.default_rng(11 + kind)
    for _ in range(40):
        v = g.normal(size=4) * 3
        alpha = float(g.uniform(0.05, 2.0))
        p = oracle.prox(kind, w, alpha, v)
        for c in range(v.size):
            def obj(x):
                return alpha * oracle.reg(kind, w, [x]) + 0.5 * (x - v[c]) ** 2
            lo, hi = (0.0, abs(v[c]) + 10) if kind == 3 else (-abs(v[c]) - 10, abs(v[c]) + 10)
            r = minimize_scalar(obj, bounds=(lo, hi), method="bounded", options={"xatol": 1e-12})
            assert p[c] == pytest.approx(r.x, abs=1e-7)
            assert obj(p[c]) <= obj(r.x) + 1e-12


def test_regularizer_values():
    """Section 3: quadratic w||x||^2, l1 w||x||_1, nonnegative indicator."""
    x = np.array([1.0, -2.0, 0.5])
    assert oracle.reg(0, 3.0, x) == 0.0
    assert oracle.reg(1, 0.5, x) == pytest.approx(0.5 * np.linalg.norm(x) ** 2)
    assert oracle.reg(2, 0.5, x) == pytest.approx(0.5 * np.linalg.norm(x, 1))
    assert oracle.reg(3, 0.0, x) == np.inf
    assert oracle.reg(3, 0.0, np.abs(x)) == 0.0


@pytest.mark.parametrize("kind,w", [(0, 0.0), (1, 0.7), (2, 0.4), (3, 0.0)])
def test_regularizer_subgradient_is_a_subgradient_of_least_norm(kind, w):
    """The subgradient the regularized autograd objective uses (Section 3 for
    r; the least-norm element of the subdifferential where r has a kink).
    Checked by the subgradient inequality r(y) >= r(x) + g . (y - x) against
    r's own values at random points (zeros included), by central differences
    where r is differentiable, and by least norm at the kinks: any other
    valid subgradient there is at least as long."""
    gen = np.random.default_rng(50 + kind)
    for _ in range(60):
        x = gen.normal(size=5)
        x[gen.random(5) < 0.3] = 0.0
        if kind == 3:
            x = np.abs(x)
        g = oracle.reg_subgrad(kind, w, x)[0]
        assert np.all(np.isfinite(g))
        for _ in range(20):
            y = gen.normal(size=5) * 2
            if kind == 3:
                y = np.abs(y)
            assert oracle.reg(kind, w, y) >= oracle.reg(kind, w, x) + g @ (y - x) - 1e-12
        h = 1e-6
        for c in range(5):
            if kind == 2 and x[c] == 0.0:
                # the kink: every t in [-w, w] passes the inequality; least norm is t = 0
                assert g[c] == 0.0
                for t in (-w, w):
                    gt = g.copy()
                    gt[c] = t
                    y = x.copy()
                    y[c] = gen.normal()
                    assert oracle.reg(kind, w, y) >= oracle.reg(kind, w, x) + gt @ (y - x) - 1e-12
                continue
            if kind == 3:
                assert g[c] == 0.0          # {0} inside the orthant, (-inf, 0] on its boundary
                continue
            xp, xm = x.copy(), x.copy()
            xp[c] += h
            xm[c] -= h
            fd = (oracle.reg(kind, w, xp) - oracle.reg(kind, w, xm)) / (2 * h)
            assert g[c] == pytest.approx(fd, abs=1e-6)


def test_regularizer_subgradient_outside_the_domain_and_at_the_offset():
    """Where r = +inf there is no subgradient (NaN); the offset coordinate of
    Section 3.3 is unpenalized (0) on the columns of Y and feasible only at 1
    on the rows of X."""
    g = oracle.reg_subgrad(3, 0.0, np.array([0.5, -1.0, 0.0]))[0]
    assert g[0] == 0.0 and np.isnan(g[1]) and g[2] == 0.0
    for kind in (1, 2, 3):
        gy = oracle.reg_subgrad(kind, 0.5, np.array([-3.0, 2.0]), offset=2)[0]
        assert gy[0] == 0.0 and gy[1] == oracle.reg_subgrad(kind, 0.5, np.array([2.0]))[0][0]
        gx = oracle.reg_subgrad(kind, 0.5, np.array([1.0, 2.0]), offset=1)[0]
        assert gx[0] == 0.0
        assert np.isnan(oracle.reg_subgrad(kind, 0.5, np.array([0.9, 2.0]), offset=1)[0][0])


def _problem(case):
    if case.layout == "coo":
        return oracle.Problem.from_coo(case.m, case.n, case.k, case.rows, case.cols, case.vals,
                                       case.col_loss, case.losses, case.rx, case.ry)
    return oracle.Problem.from_dense(case.A, case.mask, case.k, case.col_loss, case.losses, case.rx, case.ry)


def test_objective_reduces_to_frobenius_norm():
    """With quadratic loss, full Omega and gamma the objective is eq. qpca:
    ||A - XY||_F^2 + gamma ||X||_F^2 + gamma ||Y||_F^2 (library norms)."""
    c = synth.plain_pca(m=40, n=30, k=4)
    for gam in (0.0, 0.7):
        P = oracle.Problem.from_dense(c.A, None, c.k, c.col_loss, c.losses, (1, gam), (1, gam))
        X, Y = c.X0.astype(np.float64), c.Y0.astype(np.float64)
        ref = (np.linalg.norm(c.A.astype(np.float64) - X @ Y.T) ** 2
               + gam * np.linalg.norm(X) ** 2 + gam * np.linalg.norm(Y) ** 2)
        assert P.objective(X, Y) == pytest.approx(ref, rel=1e-13)


def test_objective_masked_matches_masked_norm():
    """Section 2.4 (matrix completion): only observed entries enter."""
    c = synth.dense_quadratic(m=50, n=40, k=3)
    P = _problem(c)
    X, Y = c.X0.astype(np.float64), c.Y0.astype(np.float64)
    R = (c.A.astype(np.float64) - X @ Y.T) * c.mask
    ref = np.linalg.norm(R) ** 2 + 0.1 * (np.linalg.norm(X) ** 2 + np.linalg.norm(Y) ** 2)
    assert P.objective(X, Y) == pytest.approx(ref, rel=1e-13)


def test_objective_invariant_under_orthogonal_change_of_basis():
    """(XT, T^T Y) gives the same product and, for quadratic or zero
    regularizers, the same objective (Section 2.3)."""
    c = synth.small_mixed(23, 17, 4, seed=3, rx=(1, 0.2), ry=(1, 0.3))
    P = _problem(c)
    X, Y = c.X0.astype(np.float64), c.Y0.astype(np.float64)
    Q, _ = np.linalg.qr(np.random.default_rng(1).normal(size=(4, 4)))
    assert P.objective(X @ Q, Y @ Q) == pytest.approx(P.objective(X, Y), rel=1e-12)


def test_objective_invariant_under_rescaling_without_regularizer():
    c = synth.small_mixed(23, 17, 3, seed=4, rx=(0, 0.0), ry=(0, 0.0))
    P = _problem(c)
    X, Y = c.X0.astype(np.float64), c.Y0.astype(np.float64)
    assert P.objective(2.5 * X, Y / 2.5) == pytest.approx(P.objective(X, Y), rel=1e-12)


def test_objective_equivariant_under_row_and_column_permutation():
    c = synth.small_mixed(19, 13, 3, seed=5)
    P = _problem(c)
    g = np.random.default_rng(2)
    pr, pc = g.permutation(c.m), g.permutation(c.n)
    P2 = oracle.Problem.from_dense(c.A[pr][:, pc], c.mask[pr][:, pc], c.k, c.col_loss[pc], c.losses, c.rx, c.ry)
    X, Y = c.X0.astype(np.float64), c.Y0.astype(np.float64)
    assert P2.objective(X[pr], Y[pc]) == pytest.approx(P.objective(X, Y), rel=1e-12)


@pytest.mark.parametrize("seed,kinds", [(1, (0, 1, 2)), (2, (0, 2)), (3, (1,))])
def test_gradient_matches_central_difference(seed, kinds):
    """Loss gradient (Section 7.2: g = sum_j dL(x_i y_j, A_ij) y_j) against FP64
    central differences of the loss sum, for smooth losses."""
    c = synth.small_mixed(9, 7, 3, seed=seed, kinds=kinds)
    P = _problem(c)
    X, Y = c.X0.astype(np.float64), c.Y0.astype(np.float64)
    dX, dY = P.grad(X, Y)
    h = 1e-6
    for M, D in ((X, dX), (Y, dY)):
        for idx in np.ndindex(M.shape):
            old = M[idx]
            M[idx] = old + h
            fp = P.loss_sum(X, Y)
            M[idx] = old - h
            fm = P.loss_sum(X, Y)
            M[idx] = old
            assert D[idx] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-7)


def test_hand_worked_sweeps():
    """Sweeps worked by hand from Algorithm 2 and the step rule of Section 7.2."""
    d = json.load(open(os.path.join(GOLD, "sweeps.json")))
    for case in d["cases"]:
        A = np.array(case["A"], dtype=np.float64)
        mask = None if case["mask"] is None else np.array(case["mask"], dtype=np.uint8)
        P = oracle.Problem.from_dense(A, mask, case["k"], np.array(case["col_loss"]), case["losses"],
                                      case["rx"], case["ry"])
        X = np.array(case["X0"], dtype=np.float64)
        Y = np.array(case["Y0"], dtype=np.float64)
        ax, ay = P.init_alpha(1.0)
        for t, exp in enumerate(case["sweeps"]):
            diag = P.sweep(X, Y, ax, ay)
            tag = "%s sweep %d" % (case["name"], t + 1)
            np.testing.assert_allclose(X, exp["X"], rtol=1e-12, atol=1e-12, err_msg=tag)
            np.testing.assert_allclose(Y, exp["Y"], rtol=1e-12, atol=1e-12, err_msg=tag)
            np.testing.assert_allclose(ax, exp["ax"], rtol=1e-12, err_msg=tag)
            np.testing.assert_allclose(ay, exp["ay"], rtol=1e-12, err_msg=tag)
            assert P.objective(X, Y) == pytest.approx(exp["F"], rel=1e-12), tag
            assert diag["rows_rejected"] == exp["rows_rejected"], tag
            assert diag["cols_rejected"] == exp["cols_rejected"], tag


def test_eckart_young_plain_pca():
    """Quadratic loss, no regularizer, full Omega, rank 5 on the 200 x 50
    table (Section 2.3): the fit reaches the truncated SVD, so the objective
    equals the sum of the trailing 45 squared singular values."""
    c = synth.plain_pca()
    P = _problem(c)
    X, Y, ax, ay, hist, _ = P.fit(c.X0, c.Y0, c.sweeps)
    s = np.linalg.svd(c.A.astype(np.float64), compute_uv=False)
    target = float(np.sum(s[c.k:] ** 2))
    assert hist[-1] == pytest.approx(target, rel=1e-8)
    assert np.all(np.diff(hist) <= 1e-12 * hist[:-1])


def test_quadratically_regularized_pca_closed_form():
    """eq. qpca with gamma > 0 and full Omega: soft-thresholded truncated SVD
    (Section 2.3 and Appendix A).  Optimal value sum_{i>k} s_i^2 +
    sum_{i<=k} (2 gamma s_i - gamma^2 if s_i >= gamma else s_i^2); Appendix A
    shows there are no other local minima."""
    c = synth.plain_pca(m=60, n=40, k=4, config=11)
    s = np.linalg.svd(c.A.astype(np.float64), compute_uv=False)
    gam = float(0.5 * (s[2] + s[3]))  # makes the 4th component inactive
    P = oracle.Problem.from_dense(c.A, None, c.k, c.col_loss, c.losses, (1, gam), (1, gam))
    X, Y, ax, ay, hist, _ = P.fit(c.X0, c.Y0, 3000)
    top = s[: c.k]
    target = float(np.sum(s[c.k:] ** 2) + np.sum(np.where(top >= gam, 2 * gam * top - gam ** 2, top ** 2)))
    assert hist[-1] == pytest.approx(target, rel=1e-8)
    # stationary points balance the factors: X^T X = Y Y^T (Appendix A)
    np.testing.assert_allclose(X.T @ X, Y.T @ Y, atol=1e-4 * np.abs(X.T @ X).max())


def test_objective_never_increases():
    """The step rule keeps every row and column objective from increasing
    (Section 7.2), so F is non-increasing after each half-step."""
    c = synth.small_mixed(40, 30, 3, seed=9, rx=(1, 0.1), ry=(2, 0.05))
    P = _problem(c)
    X, Y = c.X0.astype(np.float64).copy(), c.Y0.astype(np.float64).copy()
    ax, ay = P.init_alpha(4.0)  # large start: forces rejections
    F = P.objective(X, Y)
    rejected = 0
    for _ in range(60):
        r, *_ = P.half_step_x(X, Y, ax)
        F1 = P.objective(X, Y)
        assert F1 <= F * (1 + 1e-13) + 1e-13
        r2, *_ = P.half_step_y(X, Y, ay)
        F2 = P.objective(X, Y)
        assert F2 <= F1 * (1 + 1e-13) + 1e-13
        F = F2
        rejected += r + r2
    assert rejected > 0


def test_step_sizes_move_by_exact_factors_and_rejected_rows_stay():
    c = synth.small_mixed(30, 20, 3, seed=10)
    P = _problem(c)
    X, Y = c.X0.astype(np.float64).copy(), c.Y0.astype(np.float64).copy()
    ax, ay = P.init_alpha(3.0)
    for _ in range(5):
        X_old, ax_old = X.copy(), ax.copy()
        r, fo, fn, acc = P.half_step_x(X, Y, ax)
        acc = acc.astype(bool)
        assert np.all(ax[acc] == ax_old[acc] * 1.05)
        assert np.all(ax[~acc] == ax_old[~acc] * 0.7)
        assert np.array_equal(X[~acc], X_old[~acc])
        assert np.array_equal(acc, fn <= fo)
        P.half_step_y(X, Y, ay)


def test_a_trial_point_outside_the_reals_is_rejected():
    """The factors are real matrices (Section 2.1).  With an infinite step
    size the step of a row with no observations and no regularizer is
    x - inf * 0 = NaN: that trial point is outside the domain, so the row is
    rejected and keeps its (finite) value, where comparing a loss-free, zero
    trial objective with the old one would have accepted it.  An observed
    row with an overflowing step is rejected as well, and its old objective
    is untouched."""
    c = synth.small_mixed(8, 6, 2, seed=13, rx=(0, 0.0), ry=(0, 0.0), empty_row=2)
    P = _problem(c)
    X, Y = c.X0.astype(np.float64).copy(), c.Y0.astype(np.float64).copy()
    X0 = X.copy()
    ax = np.full(c.m, np.inf)
    r, fo, fn, acc = P.half_step_x(X, Y, ax)
    assert r == c.m and not acc.any()
    assert np.all(np.isinf(fn)) and np.all(np.isfinite(fo))
    np.testing.assert_array_equal(X, X0)
    assert fo[2] == 0.0          # the empty row's old objective: no loss, no regularizer
    # a finite step size leaves the empty row's step at exactly 0: accepted
    ax = np.full(c.m, 1e300)
    r, fo, fn, acc = P.half_step_x(X, Y, ax)
    assert acc[2] and fn[2] == 0.0
    np.testing.assert_array_equal(X, X0)


def test_initial_step_is_inverse_count():
    """alpha_i^0 = 1/n_i (Section 7.2), empty rows take the scale itself."""
    c = synth.small_mixed(12, 9, 2, seed=12, empty_row=3, empty_col=4)
    P = _problem(c)
    ax, ay = P.init_alpha(1.0)
    ni = c.mask.sum(1)
    mj = c.mask.sum(0)
    np.testing.assert_array_equal(ax, 1.0 / np.maximum(ni, 1))
    np.testing.assert_array_equal(ay, 1.0 / np.maximum(mj, 1))


def test_dense_and_coo_forms_agree():
    cd = synth.small_mixed(20, 15, 3, seed=13)
    cc = synth.small_mixed(20, 15, 3, seed=13, layout="coo")
    Pd, Pc = _problem(cd), _problem(cc)
    X, Y = cd.X0.astype(np.float64), cd.Y0.astype(np.float64)
    assert Pd.objective(X, Y) == Pc.objective(X, Y)


def test_certificate_at_zero_is_the_scaled_top_singular_value():
    """Section 7.6 at X = Y = 0: U V^T vanishes (rank 0) and, for the quadratic
    loss on a fully observed table, G = 2 (0 - A), so the certificate is
    2 sigma_1(A) / gamma with gamma = 2 w (numpy's SVD of A)."""
    c = synth.plain_pca(m=30, n=20, k=3)
    w = 0.7
    P = oracle.Problem.from_dense(c.A, None, c.k, c.col_loss, c.losses, (1, w), (1, w))
    val, r = P.certificate(np.zeros((c.m, c.k)), np.zeros((c.n, c.k)))
    s = np.linalg.svd(c.A.astype(np.float64), compute_uv=False)
    assert r == 0
    assert val == pytest.approx(2.0 * s[0] / (2.0 * w), rel=1e-12)


def test_certificate_at_the_quadratic_pca_optimum_is_the_next_singular_value():
    """Quadratic loss, full table, w ||.||^2 on both factors: the global optimum
    (Section 2.2, Appendix A) is X = U_k diag(sqrt(s_i - w)), Y = V_k diag(
    sqrt(s_i - w)).  Then G / (2w) = (Z - A) / w cancels U_k V_k^T and leaves
    -sum_{i>k} (s_i / w) u_i v_i^T, so the certificate equals s_{k+1} / w:
    <= 1 exactly when s_{k+1} <= w."""
    c = synth.plain_pca(m=40, n=25, k=4)
    A = c.A.astype(np.float64)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    for w in (0.5 * (s[c.k - 1] + s[c.k]), 0.5 * s[c.k]):
        X = U[:, :c.k] * np.sqrt(s[:c.k] - w)
        Y = Vt[:c.k].T * np.sqrt(s[:c.k] - w)
        P = oracle.Problem.from_dense(c.A, None, c.k, c.col_loss, c.losses, (1, w), (1, w))
        val, r = P.certificate(X, Y)
        assert r == c.k
        assert val == pytest.approx(s[c.k] / w, rel=1e-9)


def test_global_optimality_certificate_after_convergence():
    """Convex loss + quadratic regularizer with missing entries (Section 7.6):
    the converged fit certifies (norm <= 1); the random start does not."""
    c = synth.dense_quadratic(m=40, n=30, k=4, missing=0.3, gamma=2.0, config=12)
    P = _problem(c)
    X, Y, *_ = P.fit(c.X0, c.Y0, 4000)
    assert P.certificate(X, Y)[0] <= 1.0 + 1e-4
    assert P.certificate(c.X0, c.Y0)[0] > 1.0 + 1e-2


# ---- imputation decode (Section 5.3) ------------------------------------------
U_GRID = np.concatenate([np.linspace(-9.3, 9.3, 187), [-2.5, -0.5, 0.5, 1.5, 2.5, 3.5, 6.5, 7.5]])


@pytest.mark.parametrize("loss", [(0, 0, 0.0), (1, 0, 1.0), (1, 0, 0.25)])
def test_decode_real_losses_is_the_product(loss):
    """Section 5.3: for losses over the reals the decoded entry is x_i . y_j.
    Checked against a scalar minimiser of L(u, .) as well."""
    kind, levels, param = loss
    for u in U_GRID:
        assert oracle.decode(kind, u, levels, param) == u
    for u in (-3.7, 0.2, 5.1):
        r = minimize_scalar(lambda a: oracle.loss(kind, u, a, levels, param), bracket=(u - 2, u + 2), tol=1e-12)
        assert abs(r.x - u) < 1e-5


@pytest.mark.parametrize("kind", [2, 3])
def test_decode_boolean_losses_is_the_sign(kind):
    """Section 5.3: for logistic and hinge (MMMF) data the decoded entry is
    sign(x_i . y_j); at u = 0 both values tie and the smaller is taken."""
    for u in U_GRID[np.abs(U_GRID) > 1e-9]:
        assert oracle.decode(kind, u) == np.sign(u)
    for u in (1e-3, -1e-3, 4e-2):
        assert oracle.decode(kind, u) == np.sign(u)
    assert oracle.decode(kind, 0.0) == -1.0


@pytest.mark.parametrize("levels", [2, 5, 7])
def test_decode_ordinal_is_the_nearest_level(levels):
    """eq. ord-pca decoded by Section 5.3.  Going from level a to a+1 changes
    the loss by (1 + a - u)_+ - (u - a)_+, which is negative exactly when
    a < u - 1/2 and zero when a = u - 1/2; so the minimiser is the level
    nearest to u, clamped to 1..levels, with the lower level at a half-way
    tie: clamp(ceil(u - 1/2), 1, levels)."""
    for u in U_GRID:
        want = min(max(np.ceil(u - 0.5), 1.0), float(levels))
        assert oracle.decode(4, u, levels) == want, u


def test_impute_table_keeps_observed_entries_and_decodes_the_rest():
    """Section 5.3 on a mixed table: missing entries take the decoded value of
    their column's loss, observed entries keep A_ij when asked to; with no
    mask every entry is decoded (the denoised table)."""
    rng = np.random.default_rng(5)
    m, n, k = 7, 6, 3
    X, Y = rng.normal(size=(m, k)), rng.normal(size=(n, k))
    losses = [(0, 0, 0.0), (3, 0, 0.0), (4, 4, 0.0)]
    col_loss = np.array([0, 1, 2, 0, 2, 1], np.uint8)
    A = rng.normal(size=(m, n))
    mask = rng.random((m, n)) < 0.6
    Z, full = oracle.impute(X, Y, col_loss, losses)
    assert np.allclose(Z, np.einsum("ik,jk->ij", X, Y), rtol=0, atol=1e-12)
    for i in range(m):
        for j in range(n):
            u = sum(X[i, l] * Y[j, l] for l in range(k))
            kind = losses[col_loss[j]][0]
            want = u if kind == 0 else (np.sign(u) if kind == 3 else min(max(np.ceil(u - 0.5), 1), 4))
            assert full[i, j] == pytest.approx(want, abs=1e-12)
    _, part = oracle.impute(X, Y, col_loss, losses, A=A, mask=mask)
    assert np.array_equal(part[mask], A[mask])
    assert np.array_equal(part[~mask], full[~mask])


# ---- automatic loss scaling (Section 4.3) ------------------------------------------

def _scaling_case(kinds, seed, m=300, n=12, missing=0.2, levels=5):
    c = synth.small_mixed(m, n, 3, seed=seed, missing=missing, kinds=kinds, levels=levels)
    return c, _problem(c)


def test_scaling_of_quadratic_columns_is_mean_and_sample_variance():
    """Section 2.6 / 4.3: for (u - a)^2, mu_j is the mean and sigma_j^2 the
    sample variance of the observed entries (numpy)."""
    c, P = _scaling_case((0,), 21)
    mu, s2 = P.column_scaling()
    for j in range(c.n):
        a = c.A[c.mask[:, j].astype(bool), j].astype(np.float64)
        assert mu[j] == pytest.approx(a.mean(), abs=1e-12 * (1 + abs(a).max()))
        assert s2[j] == pytest.approx(a.var(ddof=1), rel=1e-10)


def test_scaling_of_logistic_columns_is_the_log_odds():
    """For log(1 + exp(-a u)) the minimizer is log(p / (1 - p)), p the share of
    +1 labels (set the derivative sum to zero)."""
    c, P = _scaling_case((2,), 22)
    mu, s2 = P.column_scaling()
    for j in range(c.n):
        a = c.A[c.mask[:, j].astype(bool), j].astype(np.float64)
        p = np.mean(a > 0)
        want = np.log(p / (1 - p))
        assert abs(want) < 2.0
        assert mu[j] == pytest.approx(want, abs=1e-12)
        f = np.sum(np.log1p(np.exp(-a * want)))
        assert s2[j] == pytest.approx(f / (a.size - 1), rel=1e-10)


def test_scaling_of_huber_columns_matches_a_scalar_minimizer():
    c, P = _scaling_case((1,), 23)
    mu, s2 = P.column_scaling()
    for j in range(c.n):
        a = c.A[c.mask[:, j].astype(bool), j].astype(np.float64)
        f = lambda u: sum(oracle.loss(1, u, x, 0, 1.0) for x in a)  # noqa: E731
        r = minimize_scalar(f, bounds=(a.min() - 1, a.max() + 1), method="bounded", options={"xatol": 1e-10})
        assert mu[j] == pytest.approx(r.x, abs=1e-6)
        assert s2[j] * (a.size - 1) == pytest.approx(r.fun, rel=1e-9)


@pytest.mark.parametrize("kind", [3, 4])
def test_scaling_of_piecewise_linear_columns_reaches_the_minimum(kind):
    """Hinge and ordinal hinge: sum_i L(mu, a_i) is convex and piecewise linear
    with kinks at integers (a' +- 1 for integer levels, +-1 for the Boolean
    labels), so its minimum over the bracket is attained at an integer or a
    bracket end: brute force over those candidates."""
    c, P = _scaling_case((kind,), 24 + kind)
    mu, s2 = P.column_scaling()
    vals = P.column_loss_at(mu)
    for j in range(c.n):
        a = c.A[c.mask[:, j].astype(bool), j].astype(np.float64)
        lo, hi = a.min() - 1, a.max() + 1
        cand = np.concatenate([[lo, hi], np.arange(np.ceil(lo), np.floor(hi) + 1)])
        best = min(sum(oracle.loss(kind, u, x, 5) for x in a) for u in cand)
        assert vals[j] == pytest.approx(best, rel=1e-12, abs=1e-12)
        assert s2[j] * (a.size - 1) == pytest.approx(best, rel=1e-12)


def test_scaling_readings_for_degenerate_columns():
    """An empty column: mu = 0, sigma^2 = 1; one entry: sigma^2 = 1; a constant
    quadratic column: zero minimum, sigma^2 = 1."""
    A = np.array([[1.0, 3.0, 2.0], [1.0, 0.0, 5.0], [1.0, 0.0, -1.0]])
    mask = np.array([[1, 1, 0], [1, 0, 0], [1, 0, 0]], bool)
    P = oracle.Problem.from_dense(A, mask, 1, np.zeros(3, np.uint8), [(0, 0, 0.0)], (0, 0.0), (0, 0.0))
    mu, s2 = P.column_scaling()
    assert mu[0] == pytest.approx(1.0) and s2[0] == 1.0
    assert mu[1] == pytest.approx(3.0) and s2[1] == 1.0
    assert mu[2] == 0.0 and s2[2] == 1.0


def test_svd_initialization_of_a_full_quadratic_table_is_its_best_rank_k_fit():
    """Section 7.5 on a fully observed quadratic table: At = (A - mu) / sigma,
    so X Y^T = U_k S_k V_k^T diag(sigma) is the Eckart-Young approximation of
    the standardized table, scaled back, plus the offset mu (numpy SVD of the
    standardized table)."""
    c = synth.plain_pca(m=60, n=15, k=4)
    P = oracle.Problem.from_dense(c.A, None, 5, c.col_loss, c.losses, (1, 0.1), (1, 0.1), offset=True)
    mu, s2 = P.column_scaling()
    A = c.A.astype(np.float64)
    np.testing.assert_allclose(mu, A.mean(0), atol=1e-12 * np.abs(A).max())
    X, Y, s = P.init_svd(mu, s2, 5)
    Z = (A - A.mean(0)) / A.std(0, ddof=1)
    U, sv, Vt = np.linalg.svd(Z, full_matrices=False)
    want = (U[:, :4] * sv[:4]) @ Vt[:4] * A.std(0, ddof=1) + A.mean(0)
    np.testing.assert_allclose(X @ Y.T, want, atol=1e-9 * np.abs(want).max())
    np.testing.assert_allclose(s, sv[:4], rtol=1e-12)
    assert np.all(X[:, 0] == 1.0) and np.allclose(Y[:, 0], mu)


def test_offset_regularizer_holds_the_constant_and_frees_the_offset():
    """Section 3.3: r'(x) = r(x_2..) + indicator(x_1 = 1) and rt'(y) = rt(y_2..);
    their proxes set x_1 = 1 and leave y_1 alone."""
    x = np.array([1.0, 2.0, -3.0])
    assert oracle.reg(1, 0.5, x, offset=1) == pytest.approx(0.5 * 13.0)
    assert oracle.reg(1, 0.5, np.array([0.9, 2.0, -3.0]), offset=1) == np.inf
    assert oracle.reg(1, 0.5, np.array([7.0, 2.0, -3.0]), offset=2) == pytest.approx(0.5 * 13.0)
    np.testing.assert_allclose(oracle.prox(1, 0.5, 2.0, np.array([4.0, 2.0, -3.0]), offset=1), [1.0, 2.0 / 3.0, -1.0])
    np.testing.assert_allclose(oracle.prox(2, 0.5, 2.0, np.array([4.0, 2.0, -3.0]), offset=2), [4.0, 1.0, -2.0])


# ---- prox-prox update for quadratic losses (Sections 7.2, 7.3) ---------------------

def _pp_case(rx=(0, 0.0), missing=0.3, seed=41):
    c = synth.small_mixed(50, 30, 4, seed=seed, missing=missing, kinds=(0,), rx=rx, ry=rx)
    return c, _problem(c)


def test_proxprox_with_a_huge_step_is_exact_least_squares():
    """alpha -> infinity, r = 0: prox_{alpha f}(x) -> argmin f, the row's least
    squares solution over its observed entries (numpy lstsq): the exact
    alternating-minimization update of Algorithm 1 (Section 7.1)."""
    c, P = _pp_case()
    X, Y = c.X0.astype(np.float64).copy(), c.Y0.astype(np.float64)
    ax = np.full(c.m, 1e15)
    P.half_step_x_pp(X, Y, ax)
    for i in range(c.m):
        obs = c.mask[i].astype(bool)
        want = np.linalg.lstsq(Y[obs], c.A[i, obs].astype(np.float64), rcond=None)[0]
        np.testing.assert_allclose(X[i], want, rtol=1e-8, atol=1e-9)


def test_proxprox_fixed_point_under_the_quadratic_regularizer():
    """Repeating the update with r = g ||x||^2 converges to its fixed point
    x = prox_r(prox_f(x)), which solves (G (1 + 2 alpha g) + g I) x = b
    (G, b the row's Gram matrix and A Y^T row; numpy solve) -- not the
    minimizer (G + g I)^-1 b unless alpha -> 0."""
    g_ = 0.3
    c, P = _pp_case(rx=(1, g_))
    X, Y = c.X0.astype(np.float64).copy(), c.Y0.astype(np.float64)
    alpha = 0.05
    ax = np.full(c.m, alpha)
    P.half_step_x_pp(X, Y, ax, inner=400)
    for i in range(0, c.m, 7):
        obs = c.mask[i].astype(bool)
        G = Y[obs].T @ Y[obs]
        b = Y[obs].T @ c.A[i, obs].astype(np.float64)
        want = np.linalg.solve(G * (1 + 2 * alpha * g_) + g_ * np.eye(c.k), b)
        np.testing.assert_allclose(X[i], want, rtol=1e-9, atol=1e-11)


def test_proxprox_agrees_with_the_gradient_step_to_second_order():
    """prox_{alpha f}(x) = x - alpha grad f(x) + O(alpha^2): the gap between the
    prox-prox and the proximal gradient trial points shrinks fourfold when
    alpha halves (r = 0)."""
    c, P = _pp_case()
    X0, Y = c.X0.astype(np.float64), c.Y0.astype(np.float64)
    g, _ = P.grad(X0, Y)
    gaps = []
    for alpha in (1e-3, 5e-4, 2.5e-4):
        X = X0.copy()
        ax = np.full(c.m, alpha)
        _, fo, fn, acc = P.half_step_x_pp(X, Y, ax)
        assert acc.all()
        gaps.append(np.linalg.norm(X - (X0 - alpha * g)))
    assert 3.6 < gaps[0] / gaps[1] < 4.4 and 3.6 < gaps[1] / gaps[2] < 4.4
