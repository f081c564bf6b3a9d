"""Plain FP64 CPU oracle for the alternating proximal-gradient GLRM fit.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product library never imports,
links or calls anything here, and this package imports nothing from the
product package.

The arithmetic lives in ``glrm_oracle.c`` (double precision, sequential loops
over the observed entries).  This module only marshals arrays: it turns a
dense table plus mask, or a row-sorted COO list, into the row-compressed list
of observed entries the C code walks, and builds the transposed list for the
column half-step (Section 7.2 defines the Y update as the X update with the
roles of X and Y swapped and every matrix argument transposed).

Loss kinds: 0 quadratic, 1 Huber(delta = param), 2 logistic, 3 hinge,
4 ordinal hinge over 1..levels; the multi-dimensional losses of Section 6
(``MDProblem``): 5 categorical one-vs-all over labels 1..levels, 6
multi-dimensional ordinal over levels 1..levels.  Regularizer kinds: 0 zero, 1 quadratic
w*||x||^2, 2 l1 w*||x||_1, 3 nonnegative indicator.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "glrm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build():
    """Compile the oracle with gcc (plain -O2, no fast-math: IEEE double)."""
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                           "-o", _LIB, _SRC, "-lm"])


class _Loss(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("levels", ctypes.c_int32), ("param", ctypes.c_double)]


class _Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("ecode", ctypes.c_void_p), ("losses", ctypes.c_void_p), ("ew", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P, D, I64, I32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int32
        L.oracle_loss.restype = D
        L.oracle_loss.argtypes = [P, D, D]
        L.oracle_dloss.restype = D
        L.oracle_dloss.argtypes = [P, D, D]
        L.oracle_reg.restype = D
        L.oracle_reg.argtypes = [I32, D, I32, P, I32]
        L.oracle_prox.restype = None
        L.oracle_prox.argtypes = [I32, D, I32, D, P, I32]
        L.oracle_reg_subgrad.restype = None
        L.oracle_reg_subgrad.argtypes = [I32, D, I32, P, I32, P]
        L.oracle_loss_sum.restype = D
        L.oracle_loss_sum.argtypes = [P, P, P]
        L.oracle_loss_grad_rows.restype = None
        L.oracle_loss_grad_rows.argtypes = [P, P, P, P]
        L.oracle_dloss_entries.restype = None
        L.oracle_dloss_entries.argtypes = [P, P, P, P]
        L.oracle_loss_grad_sq_rows.restype = None
        L.oracle_loss_grad_sq_rows.argtypes = [P, P, P, P]
        L.oracle_loss_grad_abs_rows.restype = None
        L.oracle_loss_grad_abs_rows.argtypes = [P, P, P, P]
        L.oracle_half_step.restype = I64
        L.oracle_half_step.argtypes = [P, P, P, P, I32, D, I32, D, D, P, P, P, P]
        L.oracle_half_step_proxprox.restype = I64
        L.oracle_half_step_proxprox.argtypes = [P, P, P, P, I32, D, I32, I32, D, D, P, P, P, P, P]
        L.oracle_init_alpha.restype = None
        L.oracle_init_alpha.argtypes = [P, D, P]
        L.oracle_reg_sum.restype = D
        L.oracle_reg_sum.argtypes = [I32, D, I32, P, I64, I32]
        L.oracle_objective.restype = D
        L.oracle_objective.argtypes = [P, P, P, I32, D, I32, D, I32]
        L.oracle_column_scaling.restype = None
        L.oracle_column_scaling.argtypes = [P, P, P]
        L.oracle_column_loss_at.restype = None
        L.oracle_column_loss_at.argtypes = [P, P, P]
        L.oracle_decode.restype = D
        L.oracle_decode.argtypes = [P, D]
        L.oracle_decode_matrix.restype = None
        L.oracle_decode_matrix.argtypes = [P, P, P, I64, I64, P]
        L.oracle_md_dim.restype = I32
        L.oracle_md_dim.argtypes = [I32, I32]
        L.oracle_md_loss.restype = D
        L.oracle_md_loss.argtypes = [I32, I32, D, P, D]
        L.oracle_md_dloss.restype = None
        L.oracle_md_dloss.argtypes = [I32, I32, D, P, D, P]
        L.oracle_md_decode.restype = D
        L.oracle_md_decode.argtypes = [I32, I32, D, P]
        L.oracle_md_objective.restype = D
        L.oracle_md_objective.argtypes = [P, I64, P, P, I32, D, I32, D, I32]
        L.oracle_md_grad.restype = None
        L.oracle_md_grad.argtypes = [P, I64, P, P, P, P]
        L.oracle_md_init_alpha.restype = None
        L.oracle_md_init_alpha.argtypes = [P, P, I64, D, P, P]
        L.oracle_md_half_step_x.restype = I64
        L.oracle_md_half_step_x.argtypes = [P, P, P, P, I32, D, I32, D, D, P, P, P]
        L.oracle_md_half_step_y.restype = I64
        L.oracle_md_half_step_y.argtypes = [P, P, P, P, I32, D, I32, D, D, P, P, P, P]
        L.oracle_md_impute.restype = None
        L.oracle_md_impute.argtypes = [P, I64, P, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---- scalar helpers (for pin tests) -----------------------------------------
def loss(kind, u, a, levels=0, param=1.0):
    L = _Loss(kind, levels, param)
    return lib().oracle_loss(ctypes.byref(L), float(u), float(a))


def dloss(kind, u, a, levels=0, param=1.0):
    L = _Loss(kind, levels, param)
    return lib().oracle_dloss(ctypes.byref(L), float(u), float(a))


def decode(kind, u, levels=0, param=1.0):
    """argmin over the loss's data domain of L(u, a) (Section 5.3)."""
    L = _Loss(kind, levels, param)
    return lib().oracle_decode(ctypes.byref(L), float(u))


def impute(X, Y, col_loss, losses, A=None, mask=None):
    """The decoded table a_hat_ij = argmin_a L_j(x_i . y_j, a) (Section 5.3).

    X is m x k, Y is n x k; ``col_loss`` gives each column's index into
    ``losses`` (None = all 0).  With ``mask`` (m x n bool) the observed entries
    keep their data A_ij and only the missing ones are decoded.  Returns the
    float64 products Z = X Y^T (the paper's XY) and the decoded table."""
    X, Y = _f64(X), _f64(Y)
    m, n = X.shape[0], Y.shape[0]
    Z = np.ascontiguousarray(X @ Y.T)
    code = np.zeros(n, np.uint8) if col_loss is None else np.ascontiguousarray(col_loss, dtype=np.uint8)
    tab = (_Loss * max(1, len(losses)))(*[_Loss(int(a), int(b), float(c)) for a, b, c in losses])
    out = np.empty((m, n))
    lib().oracle_decode_matrix(ctypes.byref(tab), _ptr(code), _ptr(Z), m, n, _ptr(out))
    if mask is not None:
        mask = np.asarray(mask, dtype=bool)
        out[mask] = np.asarray(A, dtype=np.float64)[mask]
    return Z, out


def reg(kind, w, x, offset=0):
    """r(x); offset 1 / 2 applies the offset of Section 3.3 to coordinate 0
    (held at 1 / free and unpenalized)."""
    x = _f64(x).ravel()
    return lib().oracle_reg(kind, float(w), int(offset), _ptr(x), x.size)


def reg_subgrad(kind, w, V, offset=0):
    """The minimum-norm subgradient of r at every row of V (rows x k; NaN
    where r is +inf)."""
    V = np.atleast_2d(_f64(V))
    out = np.empty_like(V)
    for i in range(V.shape[0]):
        row = np.ascontiguousarray(V[i])
        g = np.empty_like(row)
        lib().oracle_reg_subgrad(kind, float(w), int(offset), _ptr(row), row.size, _ptr(g))
        out[i] = g
    return out


def prox(kind, w, alpha, v, offset=0):
    v = _f64(v).ravel().copy()
    lib().oracle_prox(kind, float(w), int(offset), float(alpha), _ptr(v), v.size)
    return v


class _View:
    """One row-compressed list of observed entries (kept alive with its arrays)."""

    def __init__(self, m, n, k, row_ptr, col, val, ecode, loss_arr, ew=None):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = _f64(val)
        self.ecode = np.ascontiguousarray(ecode, dtype=np.uint8)
        self.ew = None if ew is None else _f64(ew)
        self._loss_arr = loss_arr
        self.s = _Problem(m, n, k, self.row_ptr.ctypes.data, self.col.ctypes.data,
                          self.val.ctypes.data, self.ecode.ctypes.data,
                          ctypes.addressof(loss_arr), None if self.ew is None else self.ew.ctypes.data)
        self.m, self.n = m, n


class Problem:
    """A GLRM instance in the oracle's form.

    Build it with :meth:`from_dense` (A m x n, mask m x n bool or None) or
    :meth:`from_coo` (row-sorted unique (i, j) pairs and values).
    ``col_loss`` holds one loss-table index per column; ``losses`` is a list of
    ``(kind, levels, param)``; ``rx`` / ``ry`` are ``(kind, weight)``.
    """

    def __init__(self, m, n, k, rows, cols, vals, col_loss, losses, rx, ry, col_order=None, row_sorted=False,
                 offset=False, col_weight=None):
        """rows / cols / vals list the observed entries.  ``row_sorted`` says they
        are already ordered by (row, column); ``col_order`` optionally gives the
        permutation that orders them by (column, row).  ``offset`` makes
        coordinate 0 the model's offset (Section 3.3: x_i0 = 1, y_j0 free and
        unpenalized); ``col_weight`` (n) scales column j's loss (Section 4.3)."""
        self.m, self.n, self.k = int(m), int(n), int(k)
        self.offset = bool(offset)
        self.col_weight = None if col_weight is None else np.asarray(col_weight, np.float64)
        self.rx, self.ry = (int(rx[0]), float(rx[1])), (int(ry[0]), float(ry[1]))
        self.losses = list(losses)
        self._loss_arr = (_Loss * max(1, len(losses)))(*[_Loss(int(a), int(b), float(c)) for a, b, c in losses])
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        vals = np.asarray(vals, dtype=np.float64)
        ecode = np.asarray(col_loss, dtype=np.uint8)[cols]
        ew = None if self.col_weight is None else self.col_weight[cols]
        # row view: entries ordered by (row, column)
        o = None if row_sorted else np.lexsort((cols, rows))
        pick = (lambda a: a) if o is None else (lambda a: a[o])
        rp = np.zeros(self.m + 1, dtype=np.int64)
        np.add.at(rp, rows + 1, 1) if rows.size < (1 << 22) else rp.__setitem__(
            slice(1, None), np.bincount(rows, minlength=self.m))
        self.row = _View(self.m, self.n, self.k, np.cumsum(rp), pick(cols), pick(vals), pick(ecode), self._loss_arr,
                         None if ew is None else pick(ew))
        # transposed view for the column half-step: ordered by (column, row)
        o = np.lexsort((rows, cols)) if col_order is None else col_order
        cp = np.zeros(self.n + 1, dtype=np.int64)
        cp[1:] = np.bincount(cols, minlength=self.n)
        self.colv = _View(self.n, self.m, self.k, np.cumsum(cp), rows[o], vals[o], ecode[o], self._loss_arr,
                          None if ew is None else ew[o])
        self.nnz = int(rows.size)

    @classmethod
    def from_dense(cls, A, mask, k, col_loss, losses, rx, ry, offset=False, col_weight=None):
        A = np.asarray(A)
        m, n = A.shape
        if mask is None:
            flat = np.arange(m * n, dtype=np.int64)
            rows, cols = np.divmod(flat, n)
            colflat = np.arange(m * n, dtype=np.int64)
            cj, ci = np.divmod(colflat, m)           # column-major walk
            order = ci * n + cj                      # position of (ci, cj) in the row-major list
        else:
            mask = np.asarray(mask).astype(bool, copy=False)
            rows, cols = np.nonzero(mask)
            # entries in column-major order, as positions in the row-major list
            rank = np.zeros(mask.shape, dtype=np.int64)
            rank[rows, cols] = np.arange(rows.size, dtype=np.int64)
            cj, ci = np.nonzero(mask.T)
            order = rank[ci, cj]
            del rank
        return cls(m, n, k, rows, cols, A[rows, cols], col_loss, losses, rx, ry, col_order=order, row_sorted=True,
                   offset=offset, col_weight=col_weight)

    @classmethod
    def from_coo(cls, m, n, k, rows, cols, vals, col_loss, losses, rx, ry, offset=False, col_weight=None):
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        row_sorted = bool(rows.size < 2 or np.all((rows[1:] > rows[:-1]) | ((rows[1:] == rows[:-1]) & (cols[1:] > cols[:-1]))))
        order = np.argsort(cols, kind="stable") if row_sorted else None
        return cls(m, n, k, rows, cols, vals, col_loss, losses, rx, ry, col_order=order, row_sorted=row_sorted,
                   offset=offset, col_weight=col_weight)

    # ---- the method ----------------------------------------------------------
    def objective(self, X, Y):
        X, Y = _f64(X), _f64(Y)
        return lib().oracle_objective(ctypes.byref(self.row.s), _ptr(X), _ptr(Y),
                                      self.rx[0], self.rx[1], self.ry[0], self.ry[1], 1 if self.offset else 0)

    def loss_sum(self, X, Y):
        X, Y = _f64(X), _f64(Y)
        return lib().oracle_loss_sum(ctypes.byref(self.row.s), _ptr(X), _ptr(Y))

    def grad(self, X, Y):
        """Loss-part gradients (dX m x k, dY n x k)."""
        X, Y = _f64(X), _f64(Y)
        dX = np.empty_like(X)
        dY = np.empty_like(Y)
        lib().oracle_loss_grad_rows(ctypes.byref(self.row.s), _ptr(X), _ptr(Y), _ptr(dX))
        lib().oracle_loss_grad_rows(ctypes.byref(self.colv.s), _ptr(Y), _ptr(X), _ptr(dY))
        return dX, dY

    def grad_abs(self, X, Y):
        """Sums of the absolute gradient terms, sum_j |dL_ij| |y_j| (m x k) and
        sum_i |dL_ij| |x_i| (n x k): the scale of a gradient's rounding error."""
        X, Y = _f64(X), _f64(Y)
        aX = np.empty_like(X)
        aY = np.empty_like(Y)
        lib().oracle_loss_grad_abs_rows(ctypes.byref(self.row.s), _ptr(X), _ptr(Y), _ptr(aX))
        lib().oracle_loss_grad_abs_rows(ctypes.byref(self.colv.s), _ptr(Y), _ptr(X), _ptr(aY))
        return aX, aY

    def grad_matrix(self, X, Y):
        """The m x n matrix G of loss derivatives dL_j(x_i . y_j, A_ij) on the
        observed set, 0 elsewhere (dense; small problems)."""
        X, Y = _f64(X), _f64(Y)
        g = np.empty(self.nnz)
        lib().oracle_dloss_entries(ctypes.byref(self.row.s), _ptr(X), _ptr(Y), _ptr(g))
        G = np.zeros((self.m, self.n))
        rows = np.repeat(np.arange(self.m), np.diff(self.row.row_ptr))
        G[rows, self.row.col] = g
        return G

    def certificate(self, X, Y, rtol=1e-6):
        """Section 7.6: ||G / gamma + U V^T||_2 with X Y^T = U S V^T (singular
        values above rtol times the largest) and gamma = 2 w for the
        regularizer w ||.||^2 on both factors (the factored problem carries
        gamma / 2).  At most 1 certifies (X, Y) globally optimal.  Returns
        (norm, rank)."""
        if self.rx[0] != 1 or self.ry[0] != 1 or self.rx[1] != self.ry[1] or not self.rx[1] > 0:
            raise ValueError("the certificate needs the quadratic regularizer with one weight on both factors")
        X, Y = _f64(X), _f64(Y)
        gamma = 2.0 * self.rx[1]
        U, s, Vt = np.linalg.svd(X @ Y.T, full_matrices=False)
        r = int(np.sum(s > rtol * s[0])) if s.size and s[0] > 0 else 0
        M = self.grad_matrix(X, Y) / gamma + U[:, :r] @ Vt[:r]
        return float(np.linalg.norm(M, 2)), r

    def column_scaling(self):
        """Section 4.3: (mu, sigma2) per column, from the unweighted losses."""
        mu, s2 = np.empty(self.n), np.empty(self.n)
        lib().oracle_column_scaling(ctypes.byref(self.colv_plain().s), _ptr(mu), _ptr(s2))
        return mu, s2

    def column_loss_at(self, mu):
        """sum over column j's observed entries of L_j(mu_j, A_ij), per column."""
        mu = _f64(mu)
        out = np.empty(self.n)
        lib().oracle_column_loss_at(ctypes.byref(self.colv_plain().s), _ptr(mu), _ptr(out))
        return out

    def colv_plain(self):
        """The column view without loss weights."""
        v = self.colv
        return _View(v.m, v.n, self.k, v.row_ptr, v.col, v.val, v.ecode, self._loss_arr)

    def dense_values(self):
        """The observed entries as a dense m x n array and the observation mask."""
        A = np.zeros((self.m, self.n))
        M = np.zeros((self.m, self.n), bool)
        rows = np.repeat(np.arange(self.m), np.diff(self.row.row_ptr))
        A[rows, self.row.col] = self.row.val
        M[rows, self.row.col] = True
        return A, M

    def init_svd(self, mu, sigma2, k):
        """Section 7.5: the exact top-k' SVD of the standardized table
        At_ij = m / (sigma_j m_j) (A_ij - mu_j) on the observed set (0
        elsewhere), X = U S^1/2, Y = diag(sigma) V S^1/2, with k' = k - 1 and
        the offset in coordinate 0 (x_i0 = 1, y_j0 = mu_j) when this problem
        has one.  Returns X, Y and the singular values."""
        A, M = self.dense_values()
        mu = np.asarray(mu, np.float64)
        sig = np.sqrt(np.asarray(sigma2, np.float64))
        cnt = M.sum(axis=0)
        scale = np.where(cnt > 0, self.m / (sig * np.maximum(cnt, 1)), 0.0)
        At = np.where(M, (A - mu[None, :]) * scale[None, :], 0.0)
        off = 1 if self.offset else 0
        ks = k - off
        U, s, Vt = np.linalg.svd(At, full_matrices=False)
        X = np.zeros((self.m, k))
        Y = np.zeros((self.n, k))
        if off:
            X[:, 0] = 1.0
            Y[:, 0] = mu
        r = min(ks, int(np.sum(s > 1e-6 * s[0])) if s.size and s[0] > 0 else 0)
        X[:, off:off + r] = U[:, :r] * np.sqrt(s[:r])
        Y[:, off:off + r] = sig[:, None] * (Vt[:r].T * np.sqrt(s[:r]))
        return X, Y, s[:ks]

    def grad_rss(self, X, Y):
        """Root of the sums of the squared gradient terms (m x k, n x k)."""
        X, Y = _f64(X), _f64(Y)
        aX = np.empty_like(X)
        aY = np.empty_like(Y)
        lib().oracle_loss_grad_sq_rows(ctypes.byref(self.row.s), _ptr(X), _ptr(Y), _ptr(aX))
        lib().oracle_loss_grad_sq_rows(ctypes.byref(self.colv.s), _ptr(Y), _ptr(X), _ptr(aY))
        return np.sqrt(aX), np.sqrt(aY)

    def init_alpha(self, s=1.0):
        ax = np.empty(self.m)
        ay = np.empty(self.n)
        lib().oracle_init_alpha(ctypes.byref(self.row.s), float(s), _ptr(ax))
        lib().oracle_init_alpha(ctypes.byref(self.colv.s), float(s), _ptr(ay))
        return ax, ay

    def half_step_x(self, X, Y, ax, step_up=1.05, step_down=0.7):
        """X half-step in place on float64 arrays; returns (rejected, f_old, f_new, accepted)."""
        fo, fn, acc = np.empty(self.m), np.empty(self.m), np.empty(self.m, dtype=np.uint8)
        scr = np.empty(2 * self.k)
        rej = lib().oracle_half_step(ctypes.byref(self.row.s), _ptr(X), _ptr(Y), _ptr(ax),
                                     self.rx[0], self.rx[1], 1 if self.offset else 0, float(step_up), float(step_down),
                                     _ptr(fo), _ptr(fn), _ptr(acc), _ptr(scr))
        return rej, fo, fn, acc

    def half_step_y(self, X, Y, ay, step_up=1.05, step_down=0.7):
        """Y half-step in place (the X half-step on the transposed problem)."""
        fo, fn, acc = np.empty(self.n), np.empty(self.n), np.empty(self.n, dtype=np.uint8)
        scr = np.empty(2 * self.k)
        rej = lib().oracle_half_step(ctypes.byref(self.colv.s), _ptr(Y), _ptr(X), _ptr(ay),
                                     self.ry[0], self.ry[1], 2 if self.offset else 0, float(step_up), float(step_down),
                                     _ptr(fo), _ptr(fn), _ptr(acc), _ptr(scr))
        return rej, fo, fn, acc

    def half_step_x_pp(self, X, Y, ax, inner=1, step_up=1.05, step_down=0.7, trial=None):
        """X half-step with the prox-prox update of Sections 7.2-7.3 (quadratic
        losses); in place, returns (rejected, f_old, f_new, accepted).  ``trial``
        (m x k float64) receives every row's trial point."""
        fo, fn, acc = np.empty(self.m), np.empty(self.m), np.empty(self.m, dtype=np.uint8)
        scr = np.empty(2 * self.k * self.k + 3 * self.k)
        rej = lib().oracle_half_step_proxprox(ctypes.byref(self.row.s), _ptr(X), _ptr(Y), _ptr(ax), self.rx[0],
                                              self.rx[1], 1 if self.offset else 0, int(inner), float(step_up),
                                              float(step_down), _ptr(fo), _ptr(fn), _ptr(acc),
                                              None if trial is None else _ptr(trial), _ptr(scr))
        return rej, fo, fn, acc

    def half_step_y_pp(self, X, Y, ay, inner=1, step_up=1.05, step_down=0.7, trial=None):
        """The same for the columns (the transposed problem)."""
        fo, fn, acc = np.empty(self.n), np.empty(self.n), np.empty(self.n, dtype=np.uint8)
        scr = np.empty(2 * self.k * self.k + 3 * self.k)
        rej = lib().oracle_half_step_proxprox(ctypes.byref(self.colv.s), _ptr(Y), _ptr(X), _ptr(ay), self.ry[0],
                                              self.ry[1], 2 if self.offset else 0, int(inner), float(step_up),
                                              float(step_down), _ptr(fo), _ptr(fn), _ptr(acc),
                                              None if trial is None else _ptr(trial), _ptr(scr))
        return rej, fo, fn, acc

    def fit_pp(self, X0, Y0, sweeps, inner=1, alpha_scale=1.0):
        """Algorithm 2 with the prox-prox update; returns X, Y, ax, ay, history."""
        X, Y = _f64(X0).copy(), _f64(Y0).copy()
        ax, ay = self.init_alpha(alpha_scale)
        hist = []
        for _ in range(int(sweeps)):
            self.half_step_x_pp(X, Y, ax, inner)
            self.half_step_y_pp(X, Y, ay, inner)
            hist.append(self.objective(X, Y))
        return X, Y, ax, ay, np.array(hist)

    def sweep(self, X, Y, ax, ay, step_up=1.05, step_down=0.7):
        """One iteration t of Algorithm 2 (Gauss-Seidel: the Y half-step sees X^t).

        Works in place on float64 arrays and returns a dict of diagnostics."""
        rx_, fxo, fxn, accx = self.half_step_x(X, Y, ax, step_up, step_down)
        ry_, fyo, fyn, accy = self.half_step_y(X, Y, ay, step_up, step_down)
        return dict(rows_rejected=rx_, cols_rejected=ry_, f_row_old=fxo, f_row_new=fxn, row_accepted=accx,
                    f_col_old=fyo, f_col_new=fyn, col_accepted=accy)

    def fit(self, X0, Y0, sweeps, alpha=None, alpha_scale=1.0, step_up=1.05, step_down=0.7):
        """Run ``sweeps`` iterations from (X0, Y0); alpha=None starts from s/n_i.

        Returns X, Y, ax, ay, history (objective after each sweep), rejects."""
        X, Y = _f64(X0).copy(), _f64(Y0).copy()
        if alpha is None:
            ax, ay = self.init_alpha(alpha_scale)
        else:
            ax, ay = _f64(alpha[0]).copy(), _f64(alpha[1]).copy()
        hist, rej = [], []
        for _ in range(int(sweeps)):
            d = self.sweep(X, Y, ax, ay, step_up, step_down)
            hist.append(self.objective(X, Y))
            rej.append((d["rows_rejected"], d["cols_rejected"]))
        return X, Y, ax, ay, np.array(hist), rej


# ---- multi-dimensional losses (Section 6) -----------------------------------
CATEGORICAL, MORDINAL = 5, 6


def md_dim(kind, levels):
    """Embedding dimension d_j of a feature with this loss."""
    return lib().oracle_md_dim(int(kind), int(levels))


def md_loss(kind, u, a, levels=0, param=1.0):
    u = _f64(np.atleast_1d(u))
    return lib().oracle_md_loss(int(kind), int(levels), float(param), _ptr(u), float(a))


def md_dloss(kind, u, a, levels=0, param=1.0):
    u = _f64(np.atleast_1d(u))
    g = np.empty(max(1, md_dim(kind, levels)))
    lib().oracle_md_dloss(int(kind), int(levels), float(param), _ptr(u), float(a), _ptr(g))
    return g


def md_decode(kind, u, levels=0, param=1.0):
    u = _f64(np.atleast_1d(u))
    return lib().oracle_md_decode(int(kind), int(levels), float(param), _ptr(u))


class _MD(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("k", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("other", ctypes.c_void_p), ("val", ctypes.c_void_p), ("fkind", ctypes.c_void_p),
                ("flev", ctypes.c_void_p), ("fpar", ctypes.c_void_p), ("fw", ctypes.c_void_p),
                ("fcol", ctypes.c_void_p)]


class MDProblem:
    """A table of features under the losses of eq. mpca: dense A (m x nf)
    with a mask (1 = observed), one loss (kind, levels, param) per feature,
    the regularizers r on the rows of X and rt on the columns of each Y_j.
    Y is stored d x k, d = sum_j d_j: feature j owns rows fcol[j] .. fcol[j+1]-1
    (the columns of the paper's block Y_j).  ``weight`` scales each feature's
    loss; ``offset`` is the offset coordinate 0 of Section 3.3."""

    def __init__(self, A, mask, k, feat_losses, rx, ry, offset=False, weight=None):
        A = np.asarray(A)
        self.m, self.nf = A.shape
        self.k = int(k)
        self.rx, self.ry = (int(rx[0]), float(rx[1])), (int(ry[0]), float(ry[1]))
        self.offset = bool(offset)
        self.fkind = np.array([int(l[0]) for l in feat_losses], np.int32)
        self.flev = np.array([int(l[1]) for l in feat_losses], np.int32)
        self.fpar = np.array([float(l[2]) for l in feat_losses], np.float64)
        self.fw = None if weight is None else _f64(weight)
        dims = np.array([md_dim(a, b) for a, b in zip(self.fkind, self.flev)], np.int64)
        self.dims = dims
        self.fcol = np.concatenate([[0], np.cumsum(dims)]).astype(np.int64)
        self.d = int(self.fcol[-1])
        obs = np.asarray(mask) != 0 if mask is not None else np.ones(A.shape, bool)
        ri, rj = np.nonzero(obs)                       # row-major: sorted by row
        self._keep = []
        self.row = self._view(self.m, ri, rj, A[ri, rj])
        order = np.lexsort((ri, rj))                   # sorted by feature, then row
        self.feat = self._view(self.nf, rj[order], ri[order], A[ri[order], rj[order]])
        self.nnz = int(ri.size)

    def _view(self, rows, key, other, val):
        ptr = np.zeros(rows + 1, np.int64)
        np.add.at(ptr, key + 1, 1)
        ptr = np.cumsum(ptr).astype(np.int64)
        oth = np.ascontiguousarray(other, np.int32)
        v = _f64(val)
        self._keep += [ptr, oth, v, self.fkind, self.flev, self.fpar, self.fcol]
        if self.fw is not None:
            self._keep.append(self.fw)
        return _MD(rows, self.k, _ptr(ptr).value, _ptr(oth).value, _ptr(v).value, _ptr(self.fkind).value,
                   _ptr(self.flev).value, _ptr(self.fpar).value,
                   None if self.fw is None else _ptr(self.fw).value, _ptr(self.fcol).value)

    def objective(self, X, Y):
        X, Y = _f64(X), _f64(Y)
        return lib().oracle_md_objective(ctypes.byref(self.row), self.nf, _ptr(X), _ptr(Y), self.rx[0], self.rx[1],
                                         self.ry[0], self.ry[1], 1 if self.offset else 0)

    def grad(self, X, Y):
        """Loss-part gradients (dX m x k, dY d x k)."""
        X, Y = _f64(X), _f64(Y)
        dX, dY = np.empty_like(X), np.empty_like(Y)
        lib().oracle_md_grad(ctypes.byref(self.row), self.nf, _ptr(X), _ptr(Y), _ptr(dX), _ptr(dY))
        return dX, dY

    def init_alpha(self, s=1.0):
        """(per row, per feature) initial step sizes."""
        ax, af = np.empty(self.m), np.empty(self.nf)
        lib().oracle_md_init_alpha(ctypes.byref(self.row), ctypes.byref(self.feat), self.nf, float(s), _ptr(ax),
                                   _ptr(af))
        return ax, af

    def half_step_x(self, X, Y, ax, step_up=1.05, step_down=0.7):
        fo, fn, acc = np.empty(self.m), np.empty(self.m), np.empty(self.m, dtype=np.uint8)
        rej = lib().oracle_md_half_step_x(ctypes.byref(self.row), _ptr(X), _ptr(Y), _ptr(ax), self.rx[0], self.rx[1],
                                          1 if self.offset else 0, float(step_up), float(step_down), _ptr(fo),
                                          _ptr(fn), _ptr(acc))
        return rej, fo, fn, acc

    def half_step_y(self, X, Y, af, step_up=1.05, step_down=0.7):
        """Block step of every feature (af: one step size per feature)."""
        fo, fn, acc = np.empty(self.nf), np.empty(self.nf), np.empty(self.nf, dtype=np.uint8)
        scr = np.empty(2 * 1024 * self.k)
        rej = lib().oracle_md_half_step_y(ctypes.byref(self.feat), _ptr(Y), _ptr(X), _ptr(af), self.ry[0],
                                          self.ry[1], 2 if self.offset else 0, float(step_up), float(step_down),
                                          _ptr(fo), _ptr(fn), _ptr(acc), _ptr(scr))
        return rej, fo, fn, acc

    def fit(self, X0, Y0, sweeps, alpha_scale=1.0, step_up=1.05, step_down=0.7):
        """Algorithm 2; returns X, Y, ax, af, history."""
        X, Y = _f64(X0).copy(), _f64(Y0).copy()
        ax, af = self.init_alpha(alpha_scale)
        hist = []
        for _ in range(int(sweeps)):
            self.half_step_x(X, Y, ax, step_up, step_down)
            self.half_step_y(X, Y, af, step_up, step_down)
            hist.append(self.objective(X, Y))
        return X, Y, ax, af, np.array(hist)

    def impute(self, X, Y):
        """Section 5.3 for every entry (m x nf): argmin over the feature's values."""
        X, Y = _f64(X), _f64(Y)
        out = np.empty((self.m, self.nf))
        lib().oracle_md_impute(ctypes.byref(self.row), self.nf, _ptr(X), _ptr(Y), _ptr(out))
        return out
