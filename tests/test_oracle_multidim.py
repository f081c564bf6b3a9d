"""Pins of the oracle's multi-dimensional losses (Section 6) against what the
paper and the mathematics fix: hand-worked values, the reduction of the
two-level ordinal loss to the Boolean hinge, the separability of one-vs-all
(Section 6.1), the argmax decoding the paper gives for categorical PCA,
zero-loss embeddings, central differences, and agreement with the scalar
oracle on the expanded table."""
import numpy as np
import pytest

import oracle
from md_helpers import expand, expanded_problem

CAT, MORD = oracle.CATEGORICAL, oracle.MORDINAL
HINGE, QUAD, HUBER, LOGISTIC, ORDINAL = 3, 0, 1, 2, 4


def test_hand_worked_values():
    u = [0.5, -2.0, 0.3]
    # one-vs-all, label 2 of 3: (1 - u_2)_+ + (1 + u_1)_+ + (1 + u_3)_+ = 3 + 1.5 + 1.3
    assert oracle.md_loss(CAT, u, 2, levels=3) == pytest.approx(5.8, abs=1e-15)
    # ordinal, level 3 of 4: thresholds 1 and 2 below (sign +1), 3 above (sign -1)
    assert oracle.md_loss(MORD, u, 3, levels=4) == pytest.approx(0.5 + 3.0 + 1.3, abs=1e-15)
    # level 1: every threshold above: (1 + 0.5) + (1 - 2)_+ + (1 + 0.3)
    assert oracle.md_loss(MORD, u, 1, levels=4) == pytest.approx(2.8, abs=1e-15)
    np.testing.assert_array_equal(oracle.md_dloss(MORD, u, 3, levels=4), [-1.0, -1.0, 1.0])
    np.testing.assert_array_equal(oracle.md_dloss(CAT, u, 2, levels=3), [1.0, -1.0, 1.0])


def test_dimensions():
    assert oracle.md_dim(CAT, 7) == 7
    assert oracle.md_dim(MORD, 7) == 6
    assert oracle.md_dim(HUBER, 0) == 1


@pytest.mark.parametrize("seed", range(5))
def test_one_vs_all_is_a_sum_of_boolean_hinges(seed):
    """Section 6.1: the one-vs-all loss is separable across the classes, one
    Boolean hinge per label with +1 on the value's own label."""
    rng = np.random.default_rng(seed)
    d = int(rng.integers(2, 9))
    u = rng.normal(scale=2.0, size=d)
    for a in range(1, d + 1):
        s = [1.0 if l == a else -1.0 for l in range(1, d + 1)]
        want = sum(oracle.loss(HINGE, u[l], s[l]) for l in range(d))
        assert oracle.md_loss(CAT, u, a, levels=d) == pytest.approx(want, rel=1e-15, abs=1e-15)
        gw = [oracle.dloss(HINGE, u[l], s[l]) for l in range(d)]
        np.testing.assert_array_equal(oracle.md_dloss(CAT, u, a, levels=d), gw)


def test_two_level_ordinal_is_the_boolean_hinge():
    """With two levels the multi-dimensional ordinal loss has one threshold:
    the hinge loss with level 2 as +1 and level 1 as -1."""
    for u in np.linspace(-3, 3, 25):
        assert oracle.md_loss(MORD, [u], 2, levels=2) == oracle.loss(HINGE, u, 1.0)
        assert oracle.md_loss(MORD, [u], 1, levels=2) == oracle.loss(HINGE, u, -1.0)


@pytest.mark.parametrize("seed", range(5))
def test_categorical_decoding_is_the_argmax(seed):
    """Section 6.1: the imputed label is the argmax of u."""
    rng = np.random.default_rng(10 + seed)
    for _ in range(50):
        d = int(rng.integers(2, 12))
        u = rng.normal(scale=2.0, size=d)
        assert oracle.md_decode(CAT, u, levels=d) == float(np.argmax(u) + 1)


@pytest.mark.parametrize("levels", [2, 3, 5, 8])
def test_ordinal_decoding_of_a_zero_loss_embedding(levels):
    """u_l > 1 on the thresholds below level a and u_l < -1 above it gives
    loss 0 at a and at least 1 anywhere else, so a is decoded."""
    rng = np.random.default_rng(levels)
    for a in range(1, levels + 1):
        u = np.array([1.0 + rng.uniform(0.01, 2) if l < a else -1.0 - rng.uniform(0.01, 2)
                      for l in range(1, levels)])
        assert oracle.md_loss(MORD, u, a, levels=levels) == 0.0
        for b in range(1, levels + 1):
            if b != a:
                assert oracle.md_loss(MORD, u, b, levels=levels) >= 1.0
        assert oracle.md_decode(MORD, u, levels=levels) == a


def _mixed(seed, m=40, k=3, missing=0.2):
    rng = np.random.default_rng(seed)
    feats = [(QUAD, 0, 0.0), (CAT, 4, 0.0), (MORD, 5, 0.0), (LOGISTIC, 0, 0.0), (CAT, 2, 0.0), (HUBER, 0, 1.0),
             (ORDINAL, 4, 0.0), (MORD, 3, 0.0)]
    nf = len(feats)
    A = np.empty((m, nf))
    for j, (kind, lev, _) in enumerate(feats):
        if kind in (CAT, MORD, ORDINAL):
            A[:, j] = rng.integers(1, lev + 1, m)
        elif kind == LOGISTIC:
            A[:, j] = rng.choice([-1.0, 1.0], m)
        else:
            A[:, j] = rng.normal(size=m)
    mask = (rng.random((m, nf)) >= missing).astype(np.uint8)
    d = sum(oracle.md_dim(a, b) for a, b, _ in feats)
    X = rng.normal(size=(m, k))
    Y = rng.normal(size=(d, k))
    return A, mask, feats, X, Y


def test_gradient_matches_central_difference():
    A, mask, feats, X, Y = _mixed(1, m=12)
    M = oracle.MDProblem(A, mask, 3, feats, (0, 0.0), (0, 0.0))
    dX, dY = M.grad(X, Y)
    h = 1e-6
    for (V, dV) in ((X, dX), (Y, dY)):
        for idx in np.ndindex(*V.shape):
            save = V[idx]
            V[idx] = save + h
            fp = M.objective(X, Y)
            V[idx] = save - h
            fm = M.objective(X, Y)
            V[idx] = save
            assert dV[idx] == pytest.approx((fp - fm) / (2 * h), abs=1e-6)


@pytest.mark.parametrize("offset", [False, True])
def test_objective_and_gradient_equal_the_expanded_scalar_problem(offset):
    A, mask, feats, X, Y = _mixed(2)
    w = np.linspace(0.5, 2.0, len(feats))
    M = oracle.MDProblem(A, mask, 3, feats, (1, 0.3), (2, 0.2), offset=offset, weight=w)
    P, fcol, owner = expanded_problem(A, mask, 3, feats, (1, 0.3), (2, 0.2), offset=offset, weight=w)
    np.testing.assert_array_equal(fcol, M.fcol)
    if offset:
        X[:, 0] = 1.0
    assert M.objective(X, Y) == pytest.approx(P.objective(X, Y), rel=1e-13)
    for a, b in zip(M.grad(X, Y), P.grad(X, Y)):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_row_half_step_equals_the_expanded_scalar_problem():
    """The row objective is the same sum either way, and the row counts n_i
    count the embedded entries, so the X half-steps coincide."""
    A, mask, feats, X, Y = _mixed(3)
    M = oracle.MDProblem(A, mask, 3, feats, (1, 0.1), (1, 0.1))
    P, _, _ = expanded_problem(A, mask, 3, feats, (1, 0.1), (1, 0.1))
    ax, _ = M.init_alpha(1.0)
    axp, _ = P.init_alpha(1.0)
    np.testing.assert_array_equal(ax, axp)
    X1, X2 = X.copy(), X.copy()
    r1 = M.half_step_x(X1, Y, ax.copy())
    r2 = P.half_step_x(X2, Y, axp.copy())
    np.testing.assert_allclose(X1, X2, rtol=1e-12, atol=1e-13)
    np.testing.assert_array_equal(r1[3], r2[3])
    assert r1[0] == r2[0]


def test_block_step_decides_on_the_sum_over_the_block():
    """The column step of a feature keeps or rejects its whole block on the sum
    of its columns' objectives, each column stepping with the block's step
    size: the block's old and trial objectives are the sums the scalar oracle
    computes per expanded column, and a block of mixed column outcomes
    follows the sum."""
    A, mask, feats, X, Y = _mixed(5, m=60)
    M = oracle.MDProblem(A, mask, 3, feats, (1, 0.1), (1, 0.1))
    P, fcol, owner = expanded_problem(A, mask, 3, feats, (1, 0.1), (1, 0.1))
    _, af = M.init_alpha(8.0)           # long steps: plenty of rejections
    ay = af[owner]
    Ym, Yp = Y.copy(), Y.copy()
    _, fo, fn, acc = M.half_step_y(X, Ym, af.copy())
    _, ho, hn, accp = P.half_step_y(X, Yp, ay.copy())
    np.testing.assert_allclose(fo, np.add.reduceat(ho, fcol[:-1]), rtol=1e-12)
    np.testing.assert_allclose(fn, np.add.reduceat(hn, fcol[:-1]), rtol=1e-12)
    np.testing.assert_array_equal(acc.astype(bool), fn <= fo)
    mixed = 0
    for j in range(len(feats)):
        blk = slice(fcol[j], fcol[j + 1])
        if acc[j]:
            # accepted: every column of the block holds its trial point, which
            # the scalar oracle kept wherever that column alone improved
            np.testing.assert_allclose(Ym[blk][accp[blk].astype(bool)], Yp[blk][accp[blk].astype(bool)],
                                       rtol=1e-12, atol=1e-13)
        else:
            np.testing.assert_array_equal(Ym[blk], Y[blk])
        mixed += int(0 < accp[blk].sum() < fcol[j + 1] - fcol[j])
    assert mixed > 0, "the seeded case must exercise a block of mixed column outcomes"


def test_fit_never_increases_the_objective():
    A, mask, feats, X, Y = _mixed(5, m=80)
    M = oracle.MDProblem(A, mask, 3, feats, (1, 0.1), (1, 0.1))
    f0 = M.objective(X, Y)
    *_, hist = M.fit(X, Y, 30)
    assert hist[0] <= f0
    assert np.all(np.diff(hist) <= 1e-12 * np.abs(hist[:-1]))
    assert hist[-1] < 0.5 * f0


def test_impute_decodes_every_feature_by_its_loss():
    A, mask, feats, X, Y = _mixed(6, m=30)
    M = oracle.MDProblem(A, mask, 3, feats, (1, 0.1), (1, 0.1))
    out = M.impute(X, Y)
    for j, (kind, lev, par) in enumerate(feats):
        U = X @ Y[M.fcol[j]:M.fcol[j + 1]].T
        if kind == CAT:
            np.testing.assert_array_equal(out[:, j], np.argmax(U, axis=1) + 1)
        elif kind in (QUAD, HUBER):
            np.testing.assert_allclose(out[:, j], U[:, 0], rtol=1e-14, atol=1e-15)
        elif kind == LOGISTIC:
            np.testing.assert_array_equal(out[:, j], np.where(U[:, 0] > 0, 1.0, -1.0))
        else:
            for i in range(X.shape[0]):
                f = [oracle.md_loss(kind, U[i], a, levels=lev) for a in range(1, lev + 1)]
                assert out[i, j] == float(np.argmin(f) + 1)
