"""Test-side tools for the multi-dimensional losses of Section 6.

``expand`` writes out, with numpy, the table of +-1 values on which the
categorical and multi-dimensional ordinal losses become sums of hinge losses
(the separability Section 6.1 states for one-vs-all; the ordinal loss is one
hinge per threshold by its definition), so the scalar oracle can serve as an
independent second opinion on the feature-level oracle."""
import numpy as np

import oracle

HINGE = 3


def feature_losses(col_loss, losses):
    """Per-feature (kind, levels, param) from a code list and a loss table."""
    return [tuple(losses[int(c)]) for c in col_loss]


def expand(A, mask, feat_losses):
    """(expanded table, expanded mask, loss table, codes, first column of each
    feature, feature of each expanded column).  The expanded losses are the
    caller's scalar losses followed by one hinge entry."""
    A = np.asarray(A, np.float64)
    m, nf = A.shape
    scal = []
    cols, masks, codes, owner = [], [], [], []
    for j, (kind, lev, par) in enumerate(feat_losses):
        obs = np.ones(m, bool) if mask is None else np.asarray(mask)[:, j] != 0
        a = A[:, j]
        if kind == oracle.CATEGORICAL:
            for l in range(1, lev + 1):
                cols.append(np.where(a == l, 1.0, -1.0)); masks.append(obs); codes.append(-1); owner.append(j)
        elif kind == oracle.MORDINAL:
            for l in range(1, lev):
                cols.append(np.where(a > l, 1.0, -1.0)); masks.append(obs); codes.append(-1); owner.append(j)
        else:
            if (kind, lev, par) not in scal:
                scal.append((kind, lev, par))
            cols.append(a); masks.append(obs); codes.append(scal.index((kind, lev, par))); owner.append(j)
    hinge_code = len(scal)
    table = scal + [(HINGE, 0, 0.0)]
    codes = np.array([hinge_code if c < 0 else c for c in codes], np.uint8)
    Ae = np.stack(cols, axis=1)
    Me = np.stack(masks, axis=1).astype(np.uint8)
    owner = np.array(owner, np.int64)
    fcol = np.concatenate([[0], np.cumsum(np.bincount(owner, minlength=nf))]).astype(np.int64)
    Ae = np.where(Me != 0, Ae, 0.0)
    return Ae, Me, table, codes, fcol, owner


def expanded_problem(A, mask, k, feat_losses, rx, ry, offset=False, weight=None):
    """The scalar oracle's problem on the expanded table."""
    Ae, Me, table, codes, fcol, owner = expand(A, mask, feat_losses)
    w = None if weight is None else np.asarray(weight, np.float64)[owner]
    P = oracle.Problem.from_dense(Ae, Me, k, codes, table, rx, ry, offset=offset, col_weight=w)
    return P, fcol, owner
