"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/glrm.h declares, and rejects bad arguments before
any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1410_0342_amd as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "glrm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(glrm_[a-z_0-9]+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(g.library_path())
    names = _declared()
    assert {"glrm_objective", "glrm_grad", "glrm_prox", "glrm_fit", "glrm_workspace_size", "glrm_prepare",
            "glrm_impute", "glrm_last_error"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def _data(**kw):
    s = g._Data()
    s.m, s.n, s.k, s.layout = kw.get("m", 10), kw.get("n", 8), kw.get("k", 3), kw.get("layout", g.DENSE)
    s.A = kw.get("A", 0x1000)
    s.lda = kw.get("lda", s.n)
    s.mask = None
    s.row = kw.get("row", None)
    s.col = kw.get("col", None)
    s.nnz = kw.get("nnz", 0)
    losses = kw.get("losses", [(0, 0, 0.0)])
    arr = (g._Loss * len(losses))(*[g._Loss(*x) for x in losses])
    s.losses = ctypes.addressof(arr)
    s.n_losses = kw.get("n_losses", len(losses))
    codes = kw.get("col_loss", None)
    if codes is not None:
        codes = np.ascontiguousarray(codes, np.uint8)
        s.col_loss = codes.ctypes.data
    s.rx = g._Reg(*kw.get("rx", (0, 0.0)))
    s.ry = g._Reg(*kw.get("ry", (0, 0.0)))
    return s, (arr, codes)


def test_workspace_size_of_a_valid_problem():
    s, keep = _data(m=1000, n=100, k=20)
    assert g._L().glrm_workspace_size(ctypes.byref(s)) >= 1000 * 112 * 4


@pytest.mark.parametrize("kw,msg", [
    (dict(m=0), "m and n"),
    (dict(k=0), "k must be"),
    (dict(k=65), "GLRM_MAX_K"),
    (dict(A=None), "A is NULL"),
    (dict(lda=3), "lda"),
    (dict(layout=7), "unknown layout"),
    (dict(layout=1, row=None, col=None, nnz=5), "COO A / row / col"),
    (dict(losses=[(9, 0, 0.0)]), "unknown kind"),
    (dict(losses=[(1, 0, 0.0)]), "Huber"),
    (dict(losses=[(4, 1, 0.0)]), "ordinal"),
    (dict(losses=[(5, 1, 0.0)]), "multi-dimensional"),
    (dict(losses=[(6, 1025, 0.0)]), "multi-dimensional"),
    (dict(n_losses=0), "n_losses"),
    (dict(col_loss=[0, 0, 0, 1, 0, 0, 0, 0]), "col_loss"),
    (dict(rx=(5, 0.0)), "regularizer"),
    (dict(ry=(1, -1.0)), "weight"),
])
def test_invalid_problems_are_rejected_on_the_host(kw, msg):
    s, keep = _data(**kw)
    assert g._L().glrm_workspace_size(ctypes.byref(s)) == 0
    assert msg in g.glrm_last_error()
    assert g._L().glrm_prepare(ctypes.byref(s), None, 0, None) in (g.EINVAL, g.EUNSUPPORTED)


def test_workspace_checks_before_any_launch():
    s, keep = _data()
    assert g._L().glrm_prepare(ctypes.byref(s), None, 0, None) == g.EINVAL
    assert "workspace is NULL" in g.glrm_last_error()
    assert g._L().glrm_prepare(ctypes.byref(s), ctypes.c_void_p(0x1001), 1 << 30, None) == g.EINVAL
    assert "aligned" in g.glrm_last_error()
    assert g._L().glrm_prepare(ctypes.byref(s), ctypes.c_void_p(0x1000), 16, None) == g.ENOMEM


def test_prox_and_fit_argument_errors():
    r = g._Reg(9, 0.0)
    assert g._L().glrm_prox(ctypes.byref(r), ctypes.c_void_p(0x1000), 4, 2, 2, None, None) == g.EINVAL
    r = g._Reg(1, 1.0)
    assert g._L().glrm_prox(ctypes.byref(r), ctypes.c_void_p(0x1000), 4, 2, 1, None, None) == g.EINVAL
    s, keep = _data()
    o = g._FitOpts(5, g.FP64, 1, 1.0, 1.05, 0.7, 0.0, 0)
    P = ctypes.c_void_p(0x1000)
    assert g._L().glrm_fit(ctypes.byref(s), P, P, P, P, ctypes.byref(o), None, None, P, 1 << 40, None) == g.EINVAL
    assert "precision" in g.glrm_last_error()
    o = g._FitOpts(-1, g.FP32, 1, 1.0, 1.05, 0.7, 0.0, 0)
    assert g._L().glrm_fit(ctypes.byref(s), P, P, P, P, ctypes.byref(o), None, None, P, 1 << 40, None) == g.EINVAL
    o = g._FitOpts(5, g.FP32, 1, 1.0, 1.05, 0.7, 0.0, 0)
    s, keep = _data(k=65)
    assert g._L().glrm_fit(ctypes.byref(s), P, P, P, P, ctypes.byref(o), None, None, P, 1 << 40, None) == g.EUNSUPPORTED


def test_wide_dense_fit_workspace_holds_the_column_blocked_row_pass():
    """A dense table wider than the fused row pass takes runs the row half-step
    in column blocks; its workspace adds the per-block row sums, the trial rows
    and the per-block row gradients (glrm_fit_workspace_size = glrm_workspace_size)."""
    L = g._L()
    for k, n_fused, n_wide in ((32, 1024, 1040), (64, 512, 528)):
        sizes = {}
        for n in (n_fused, n_wide):
            s, keep = _data(m=1000, n=n, k=k)
            sizes[n] = L.glrm_workspace_size(ctypes.byref(s))
            o = g._FitOpts(5, g.FP32, 1, 1.0, 1.05, 0.7, 0.0, 0)
            assert L.glrm_fit_workspace_size(ctypes.byref(s), ctypes.byref(o)) == sizes[n]
        # the wide one holds at least the trial rows (m x k floats) more
        assert sizes[n_wide] - sizes[n_fused] >= 4 * 1000 * k


def test_an_empty_coo_needs_no_arrays():
    """nnz = 0 is a valid (regularizer-only) problem: its arrays may be NULL."""
    s, keep = _data(layout=1, A=None, row=None, col=None, nnz=0)
    assert g._L().glrm_workspace_size(ctypes.byref(s)) > 0



def test_impute_argument_errors():
    s, keep = _data()
    P = ctypes.c_void_p(0x1000)
    L = g._L()
    assert L.glrm_impute(ctypes.byref(s), P, P, 0, None, 8, P, 1 << 40, 0, None) == g.EINVAL
    assert "NULL" in g.glrm_last_error()
    assert L.glrm_impute(ctypes.byref(s), P, P, 2, P, 8, P, 1 << 40, 0, None) == g.EINVAL
    assert "mode" in g.glrm_last_error()
    assert L.glrm_impute(ctypes.byref(s), P, P, 0, P, 7, P, 1 << 40, 0, None) == g.EINVAL
    assert "ldh" in g.glrm_last_error()
    assert L.glrm_impute(ctypes.byref(s), P, P, 0, P, 8, P, 16, 0, None) == g.ENOMEM
    bad, keep2 = _data(losses=[(7, 0, 0.0)])
    assert L.glrm_impute(ctypes.byref(bad), P, P, 0, P, 8, P, 1 << 40, 0, None) == g.EINVAL


def test_noalloc_gradient_rejects_a_problem_beyond_its_scratch():
    """The allocation-free gradient checks its static scratch limit before any
    HIP call: a 100,000 x 1,000 dense table needs far more than it holds."""
    s, keep = _data(m=100000, n=1000, k=20)
    rc = g._L().glrm_grad_noalloc(ctypes.byref(s), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), g.FP32,
                                  ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), None, 0, None)
    assert rc == g.ENOMEM
    assert "static scratch" in g.glrm_last_error()


def test_embedded_width_of_multidimensional_losses():
    """Section 6: a categorical column of d labels takes d rows of Y, a
    multi-dimensional ordinal column of d levels d - 1, a scalar column one."""
    L = g._L()
    s, keep = _data(n=5, losses=[(0, 0, 0.0), (5, 4, 0.0), (6, 7, 0.0)], col_loss=[0, 1, 2, 0, 1])
    assert L.glrm_embed_dim(ctypes.byref(s)) == 1 + 4 + 6 + 1 + 4
    s, keep = _data(n=5)
    assert L.glrm_embed_dim(ctypes.byref(s)) == 5
    # no free slot for the hinge loss the embedded columns use: refused
    losses = [(0, 0, 0.0)] * 15 + [(5, 3, 0.0)]
    s, keep = _data(n=2, losses=losses, col_loss=[0, 15])
    assert L.glrm_embed_dim(ctypes.byref(s)) == -1
    assert "free loss slot" in g.glrm_last_error()
    # ... unless the table has a hinge entry already
    losses = [(3, 0, 0.0)] + [(0, 0, 0.0)] * 14 + [(5, 3, 0.0)]
    s, keep = _data(n=2, losses=losses, col_loss=[0, 15])
    assert L.glrm_embed_dim(ctypes.byref(s)) == 4
    # the sparse layout has no embedding
    s, keep = _data(n=3, layout=g.COO_ROWSORTED, losses=[(5, 3, 0.0)])
    assert L.glrm_embed_dim(ctypes.byref(s)) == -1
    assert "dense layout" in g.glrm_last_error()
    assert L.glrm_workspace_size(ctypes.byref(s)) == 0
