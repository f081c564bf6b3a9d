"""Python binding of libglrm.so, the gfx950 alternating proximal-gradient fit of
a generalized low rank model (Udell et al., arXiv 1410.0342, Algorithm 2 of
Section 7.2).

This module only marshals arguments: it turns torch tensors into device
pointers, fills the C structs of ``include/glrm.h`` and calls the entry points
of the same names.  Every step of the method runs in the HIP kernels.  There
is no fallback: if the library is not built, importing the entry points raises.
"""
import ctypes
import os

import numpy as np

__all__ = [
    "GLRMError", "Data", "glrm_workspace_size", "glrm_prepare", "glrm_objective", "glrm_grad", "glrm_prox",
    "glrm_fit", "glrm_last_error", "library_path", "FP32", "BF16", "FP64", "BF16_PLAIN", "DENSE", "COO_ROWSORTED",
    "WS_PREPARED", "TIME_KERNELS", "glrm_impute", "IMPUTE_ALL", "IMPUTE_MISSING", "glrm_grad_noalloc",
    "NOALLOC_MAX_BYTES", "glrm_certificate", "glrm_linalg_workspace_size", "glrm_column_scaling",
    "glrm_init_svd", "fit_standardized", "UPDATE_PROXGRAD", "UPDATE_PROXPROX", "glrm_embed_dim",
    "LOSS_CATEGORICAL", "LOSS_MORDINAL",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libglrm.so")

FP32, BF16, FP64, BF16_PLAIN = 0, 1, 2, 3
DENSE, COO_ROWSORTED = 0, 1
WS_PREPARED = 1
TIME_KERNELS = 2
GRAD_WITH_REG = 4
IMPUTE_ALL, IMPUTE_MISSING = 0, 1
LOSS_QUADRATIC, LOSS_HUBER, LOSS_LOGISTIC, LOSS_HINGE, LOSS_ORDINAL, LOSS_CATEGORICAL, LOSS_MORDINAL = range(7)
UPDATE_PROXGRAD, UPDATE_PROXPROX = 0, 1
NOALLOC_MAX_BYTES = 64 << 20
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp64": FP64, "bf16_plain": BF16_PLAIN}

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP = 0, -1, -2, -3, -4


class GLRMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("glrm error %d: %s" % (code, msg))
        self.code = code


class _Loss(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("levels", ctypes.c_int32), ("param", ctypes.c_float)]


class _Reg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("weight", ctypes.c_float)]


class _Data(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("mask", ctypes.c_void_p),
                ("row", ctypes.c_void_p), ("col", ctypes.c_void_p), ("nnz", ctypes.c_int64),
                ("col_loss", ctypes.c_void_p), ("losses", ctypes.c_void_p), ("n_losses", ctypes.c_int32),
                ("rx", _Reg), ("ry", _Reg), ("offset", ctypes.c_int32), ("col_weight", ctypes.c_void_p)]


class _FitOpts(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("precision", ctypes.c_int32), ("init_alpha", ctypes.c_int32),
                ("alpha_scale", ctypes.c_float), ("step_up", ctypes.c_float), ("step_down", ctypes.c_float),
                ("tol", ctypes.c_double), ("flags", ctypes.c_uint32), ("update", ctypes.c_int32),
                ("inner", ctypes.c_int32)]


class _FitInfo(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("objective", ctypes.c_double), ("objective_fp32", ctypes.c_double),
                ("rows_rejected", ctypes.c_int64), ("cols_rejected", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double * 4), ("kernel_calls", ctypes.c_int32 * 4)]


class _CertInfo(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("norm_prev", ctypes.c_double), ("rank", ctypes.c_int32),
                ("iters", ctypes.c_int32)]


_lib = None


def library_path():
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libglrm.so is not built (%s); run __graft_entry__.build() first" % _LIB_PATH)
        L = ctypes.CDLL(_LIB_PATH)
        P, D = ctypes.c_void_p, ctypes.POINTER(_Data)
        L.glrm_workspace_size.restype = ctypes.c_size_t
        L.glrm_workspace_size.argtypes = [D]
        L.glrm_embed_dim.restype = ctypes.c_int64
        L.glrm_embed_dim.argtypes = [D]
        L.glrm_prepare.restype = ctypes.c_int
        L.glrm_prepare.argtypes = [D, P, ctypes.c_size_t, P]
        L.glrm_objective.restype = ctypes.c_int
        L.glrm_objective.argtypes = [D, P, P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), P, ctypes.c_size_t,
                                     ctypes.c_uint, P]
        L.glrm_grad.restype = ctypes.c_int
        L.glrm_grad.argtypes = [D, P, P, ctypes.c_int, P, P, ctypes.POINTER(ctypes.c_double), P, ctypes.c_size_t,
                                ctypes.c_uint, P]
        L.glrm_grad_noalloc.restype = ctypes.c_int
        L.glrm_grad_noalloc.argtypes = [D, P, P, ctypes.c_int, P, P, ctypes.POINTER(ctypes.c_double), ctypes.c_uint, P]
        L.glrm_linalg_workspace_size.restype = ctypes.c_size_t
        L.glrm_linalg_workspace_size.argtypes = [D, ctypes.c_int32]
        L.glrm_certificate.restype = ctypes.c_int
        L.glrm_certificate.argtypes = [D, P, P, ctypes.c_int32, ctypes.POINTER(_CertInfo), P, ctypes.c_size_t,
                                       ctypes.c_uint, P]
        L.glrm_column_scaling.restype = ctypes.c_int
        L.glrm_column_scaling.argtypes = [D, P, P, P, ctypes.c_size_t, ctypes.c_uint, P]
        L.glrm_init_svd.restype = ctypes.c_int
        L.glrm_init_svd.argtypes = [D, P, P, P, ctypes.c_int32, ctypes.c_int32, P, P,
                                    ctypes.POINTER(ctypes.c_double), P, ctypes.c_size_t, ctypes.c_uint, P]
        L.glrm_fit_workspace_size.restype = ctypes.c_size_t
        L.glrm_fit_workspace_size.argtypes = [D, ctypes.POINTER(_FitOpts)]
        L.glrm_prox.restype = ctypes.c_int
        L.glrm_prox.argtypes = [ctypes.POINTER(_Reg), P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, P, P]
        L.glrm_fit.restype = ctypes.c_int
        L.glrm_fit.argtypes = [D, P, P, P, P, ctypes.POINTER(_FitOpts), ctypes.POINTER(_FitInfo), P, P,
                               ctypes.c_size_t, P]
        L.glrm_impute.restype = ctypes.c_int
        L.glrm_impute.argtypes = [D, P, P, ctypes.c_int32, P, ctypes.c_int64, P, ctypes.c_size_t, ctypes.c_uint, P]
        L.glrm_last_error.restype = ctypes.c_char_p
        L.glrm_last_error.argtypes = []
        L.glrm_version.restype = ctypes.c_char_p
        L.glrm_version.argtypes = []
        _lib = L
    return _lib


def glrm_last_error():
    return _L().glrm_last_error().decode()


def _check(rc):
    if rc != OK:
        raise GLRMError(rc, glrm_last_error())


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, name, numel=None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements (got %d)" % (name, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


class Data:
    """A problem on the device: the ``glrm_data`` struct and the tensors and host
    arrays it points to (kept alive here), plus a cached workspace.

    ``losses`` is a list of ``(kind, levels, param)``; ``col_loss`` a host array
    of one loss index per column (None = all 0); ``rx`` / ``ry`` are
    ``(kind, weight)``.
    """

    def __init__(self, m, n, k, *, A, mask=None, row=None, col=None, layout=DENSE, lda=None, col_loss=None,
                 losses=((0, 0, 0.0),), rx=(0, 0.0), ry=(0, 0.0), offset=False, col_weight=None):
        torch = _torch()
        self.m, self.n, self.k, self.layout = int(m), int(n), int(k), int(layout)
        self.A, self.mask, self.row, self.col = A, mask, row, col
        self.losses = [tuple(x) for x in losses]
        self.rx, self.ry = (int(rx[0]), float(rx[1])), (int(ry[0]), float(ry[1]))
        self._loss_arr = (_Loss * len(self.losses))(*[_Loss(int(a), int(b), float(c)) for a, b, c in self.losses])
        self.col_loss = None if col_loss is None else np.ascontiguousarray(col_loss, dtype=np.uint8)
        s = _Data()
        s.m, s.n, s.k, s.layout = self.m, self.n, self.k, self.layout
        if self.layout == DENSE:
            s.A = _dev_ptr(A, torch.float32, "A")
            s.lda = int(lda if lda is not None else self.n)
            s.mask = _dev_ptr(mask, torch.uint8, "mask") if mask is not None else None
            s.nnz = 0
        else:
            s.A = _dev_ptr(A, torch.float32, "A (values)")
            s.row = _dev_ptr(row, torch.int32, "row")
            s.col = _dev_ptr(col, torch.int32, "col")
            s.nnz = int(A.numel())
            s.lda = 0
        s.col_loss = self.col_loss.ctypes.data if self.col_loss is not None else None
        s.losses = ctypes.addressof(self._loss_arr)
        s.n_losses = len(self.losses)
        s.rx = _Reg(*self.rx)
        s.ry = _Reg(*self.ry)
        self.offset = bool(offset)
        self.col_weight = col_weight
        s.offset = 1 if offset else 0
        s.col_weight = _dev_ptr(col_weight, torch.float32, "col_weight", self.n) if col_weight is not None else None
        self.s = s
        self._ws = None
        self.device = A.device
        # rows of Y: n, or the embedded width with multi-dimensional losses
        d = int(_L().glrm_embed_dim(ctypes.byref(s)))
        self.d = d if d > 0 else self.n

    @classmethod
    def from_case(cls, case, device="cuda"):
        """Upload a synthetic case (see ``synth.Case``) to the device."""
        torch = _torch()
        if case.layout == "coo":
            return cls(case.m, case.n, case.k, layout=COO_ROWSORTED,
                       A=torch.from_numpy(np.ascontiguousarray(case.vals, np.float32)).to(device),
                       row=torch.from_numpy(np.ascontiguousarray(case.rows, np.int32)).to(device),
                       col=torch.from_numpy(np.ascontiguousarray(case.cols, np.int32)).to(device),
                       col_loss=case.col_loss, losses=case.losses, rx=case.rx, ry=case.ry)
        mask = None if case.mask is None else torch.from_numpy(np.ascontiguousarray(case.mask, np.uint8)).to(device)
        return cls(case.m, case.n, case.k, layout=DENSE,
                   A=torch.from_numpy(np.ascontiguousarray(case.A, np.float32)).to(device), mask=mask,
                   col_loss=case.col_loss, losses=case.losses, rx=case.rx, ry=case.ry)

    def with_regs(self, rx, ry):
        """Same data and losses with other regularizers (shares the tensors)."""
        return self.variant(rx=rx, ry=ry)

    def variant(self, **kw):
        """The same data with some of k, rx, ry, offset, col_weight replaced
        (shares the tensors)."""
        args = dict(k=self.k, rx=self.rx, ry=self.ry, offset=self.offset, col_weight=self.col_weight)
        args.update(kw)
        return Data(self.m, self.n, args["k"], A=self.A, mask=self.mask, row=self.row, col=self.col,
                    layout=self.layout, lda=self.s.lda if self.layout == DENSE else None, col_loss=self.col_loss,
                    losses=self.losses, rx=args["rx"], ry=args["ry"], offset=args["offset"],
                    col_weight=args["col_weight"])

    def workspace(self, size=None):
        """Device workspace of at least glrm_workspace_size() (or `size`) bytes,
        256-byte aligned, cached.  Growing it copies the old contents over, so a
        prepared part stays valid (every layout extends the basic one)."""
        torch = _torch()
        size = max(glrm_workspace_size(self), size or 0)
        if self._ws is None or self._ws[1] < size:
            buf = torch.empty(size + 256, dtype=torch.uint8, device=self.device)
            off = (-buf.data_ptr()) % 256
            if self._ws is not None:
                # every larger layout keeps the smaller one as its prefix: carry the prepared part over
                old, osize, ooff = self._ws
                buf[off:off + osize].copy_(old[ooff:ooff + osize])
            self._ws = (buf, size, off)
        buf, size, off = self._ws
        return ctypes.c_void_p(buf.data_ptr() + off), size


def glrm_workspace_size(data):
    size = _L().glrm_workspace_size(ctypes.byref(data.s))
    if size == 0:
        # invalid data: glrm_prepare validates first and returns the reason's code
        rc = _L().glrm_prepare(ctypes.byref(data.s), None, 0, None)
        raise GLRMError(rc if rc < 0 else EINVAL, glrm_last_error())
    return size


def glrm_embed_dim(data):
    """Rows of Y for this problem: n, or sum_j d_j with multi-dimensional losses."""
    d = int(_L().glrm_embed_dim(ctypes.byref(data.s)))
    if d < 0:
        raise GLRMError(EINVAL, glrm_last_error())
    return d


def glrm_prepare(data, stream=None):
    ws, wsb = data.workspace()
    _check(_L().glrm_prepare(ctypes.byref(data.s), ws, wsb, _stream(stream)))


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def glrm_objective(data, X, Y, precision=FP32, flags=0, stream=None):
    """F(X, Y) of eq. gpca (loss over the observed entries + both regularizers)."""
    torch = _torch()
    ws, wsb = data.workspace()
    out = ctypes.c_double(0.0)
    _check(_L().glrm_objective(ctypes.byref(data.s), _dev_ptr(X, torch.float32, "X", data.m * data.k),
                               _dev_ptr(Y, torch.float32, "Y", data.d * data.k), _prec(precision),
                               ctypes.byref(out), ws, wsb, int(flags), _stream(stream)))
    return out.value


def glrm_grad(data, X, Y, precision=FP32, dX=None, dY=None, want_objective=False, flags=0, stream=None):
    """Loss-part gradients dX (m x k) and dY (n x k); optionally the objective.
    With GRAD_WITH_REG in flags the regularizers' least-magnitude subgradients
    are added."""
    torch = _torch()
    if dX is None:
        dX = torch.empty((data.m, data.k), dtype=torch.float32, device=X.device)
    if dY is None:
        dY = torch.empty((data.d, data.k), dtype=torch.float32, device=X.device)
    ws, wsb = data.workspace()
    out = ctypes.c_double(0.0)
    _check(_L().glrm_grad(ctypes.byref(data.s), _dev_ptr(X, torch.float32, "X", data.m * data.k),
                          _dev_ptr(Y, torch.float32, "Y", data.d * data.k), _prec(precision),
                          _dev_ptr(dX, torch.float32, "dX", data.m * data.k),
                          _dev_ptr(dY, torch.float32, "dY", data.d * data.k),
                          ctypes.byref(out) if want_objective else None, ws, wsb, int(flags), _stream(stream)))
    return (dX, dY, out.value) if want_objective else (dX, dY)


def glrm_grad_noalloc(data, X, Y, precision=FP32, dX=None, dY=None, want_objective=False, flags=0, stream=None):
    """glrm_grad with the library's static scratch instead of a workspace (the
    outputs are the caller's; pass dX / dY to allocate nothing here either)."""
    torch = _torch()
    if dX is None:
        dX = torch.empty((data.m, data.k), dtype=torch.float32, device=X.device)
    if dY is None:
        dY = torch.empty((data.d, data.k), dtype=torch.float32, device=X.device)
    out = ctypes.c_double(0.0)
    _check(_L().glrm_grad_noalloc(ctypes.byref(data.s), _dev_ptr(X, torch.float32, "X", data.m * data.k),
                                  _dev_ptr(Y, torch.float32, "Y", data.d * data.k), _prec(precision),
                                  _dev_ptr(dX, torch.float32, "dX", data.m * data.k),
                                  _dev_ptr(dY, torch.float32, "dY", data.d * data.k),
                                  ctypes.byref(out) if want_objective else None, int(flags), _stream(stream)))
    return (dX, dY, out.value) if want_objective else (dX, dY)


def glrm_linalg_workspace_size(data, block):
    size = _L().glrm_linalg_workspace_size(ctypes.byref(data.s), int(block))
    if size == 0:
        raise GLRMError(EINVAL, glrm_last_error())
    return size


def glrm_certificate(data, X, Y, iters=500, flags=0, stream=None):
    """The global-optimality certificate of Section 7.6: an estimate of
    ||G / gamma + U V^T||_2 by power iteration (<= 1 certifies (X, Y))."""
    torch = _torch()
    ws, wsb = data.workspace(glrm_linalg_workspace_size(data, 1))
    info = _CertInfo()
    _check(_L().glrm_certificate(ctypes.byref(data.s), _dev_ptr(X, torch.float32, "X", data.m * data.k),
                                 _dev_ptr(Y, torch.float32, "Y", data.d * data.k), int(iters), ctypes.byref(info),
                                 ws, wsb, int(flags), _stream(stream)))
    return dict(norm=info.norm, norm_prev=info.norm_prev, rank=info.rank, iters=info.iters)


def glrm_column_scaling(data, mu=None, sigma2=None, flags=0, stream=None):
    """mu_j and sigma_j^2 of every column (Section 4.3); two float32 GPU tensors."""
    torch = _torch()
    if mu is None:
        mu = torch.empty(data.n, dtype=torch.float32, device=data.device)
    if sigma2 is None:
        sigma2 = torch.empty(data.n, dtype=torch.float32, device=data.device)
    ws, wsb = data.workspace(glrm_linalg_workspace_size(data, 1))
    _check(_L().glrm_column_scaling(ctypes.byref(data.s), _dev_ptr(mu, torch.float32, "mu", data.n),
                                    _dev_ptr(sigma2, torch.float32, "sigma2", data.n), ws, wsb, int(flags),
                                    _stream(stream)))
    return mu, sigma2


def glrm_init_svd(data, omega, mu=None, sigma2=None, power_iters=2, X=None, Y=None, flags=0, stream=None):
    """X (m x k), Y (n x k) from the top singular triples of the standardized
    table (Section 7.5); omega is the caller's n x l float32 test matrix.
    Returns X, Y and the singular values."""
    torch = _torch()
    l = int(omega.shape[1]) if omega is not None else 1
    if X is None:
        X = torch.empty((data.m, data.k), dtype=torch.float32, device=data.device)
    if Y is None:
        Y = torch.empty((data.n, data.k), dtype=torch.float32, device=data.device)
    ks = data.k - (1 if data.offset else 0)
    sv = (ctypes.c_double * max(ks, 1))()
    ws, wsb = data.workspace(glrm_linalg_workspace_size(data, l))
    _check(_L().glrm_init_svd(ctypes.byref(data.s), _dev_ptr(mu, torch.float32, "mu", data.n) if mu is not None else None,
                              _dev_ptr(sigma2, torch.float32, "sigma2", data.n) if sigma2 is not None else None,
                              _dev_ptr(omega, torch.float32, "omega", data.n * l) if omega is not None else None,
                              l, int(power_iters), _dev_ptr(X, torch.float32, "X", data.m * data.k),
                              _dev_ptr(Y, torch.float32, "Y", data.d * data.k), sv, ws, wsb, int(flags),
                              _stream(stream)))
    return X, Y, np.array(sv[:ks])


def fit_standardized(data, k, sweeps, omega=None, oversample=10, power_iters=2, precision=BF16, seed=0, **fit_kw):
    """The fit as the paper's implementation runs it by default (Section 9.1):
    an offset in the model (Section 3.3) and losses scaled by 1 / sigma_j^2
    around mu_j (Section 4.3), started from the SVD initialization of
    Section 7.5.  ``k`` counts the offset coordinate.  ``omega`` (n x l,
    float32) defaults to i.i.d. N(0, 1) drawn by torch from ``seed``.  Returns
    (X, Y, info, mu, sigma2, model) with ``model`` the scaled, offset Data."""
    torch = _torch()
    mu, sigma2 = glrm_column_scaling(data)
    model = data.variant(k=int(k), offset=True, col_weight=1.0 / sigma2)
    if omega is None:
        gen = torch.Generator(device="cpu").manual_seed(int(seed))
        l = min(max(int(k) - 1 + int(oversample), 1), 96)
        omega = torch.randn((data.n, l), generator=gen, dtype=torch.float32).to(data.device)
    X, Y, sv = glrm_init_svd(model, omega, mu=mu, sigma2=sigma2, power_iters=power_iters)
    ax = torch.empty(data.m, dtype=torch.float32, device=data.device)
    ay = torch.empty(data.n, dtype=torch.float32, device=data.device)
    info = glrm_fit(model, X, Y, ax, ay, sweeps, precision=precision, **fit_kw)
    return X, Y, info, mu, sigma2, model


def glrm_prox(reg, V, alpha=None, stream=None):
    """In place V[i] <- prox_{alpha_i r}(V[i]) for a rows x k float32 tensor."""
    torch = _torch()
    rows, k = V.shape
    r = _Reg(int(reg[0]), float(reg[1]))
    _check(_L().glrm_prox(ctypes.byref(r), _dev_ptr(V, torch.float32, "V"), int(rows), int(k), int(k),
                          _dev_ptr(alpha, torch.float32, "alpha", rows) if alpha is not None else None,
                          _stream(stream)))
    return V


def glrm_fit(data, X, Y, alpha_x, alpha_y, max_sweeps, precision=BF16, init_alpha=True, alpha_scale=1.0,
             step_up=1.05, step_down=0.7, tol=0.0, history=None, flags=0, stream=None, update=UPDATE_PROXGRAD,
             inner=1):
    """Run Algorithm 2 in place on X, Y, alpha_x, alpha_y; returns the info dict.

    ``history`` (optional float64 GPU tensor of max_sweeps entries) receives F
    after each sweep.  ``update=UPDATE_PROXPROX`` takes the prox-prox update
    (quadratic losses, dense layout, FP32) with ``inner`` updates per
    half-step."""
    torch = _torch()
    o = _FitOpts(int(max_sweeps), _prec(precision), 1 if init_alpha else 0, float(alpha_scale), float(step_up),
                 float(step_down), float(tol), int(flags), int(update), int(inner))
    info = _FitInfo()
    size = _L().glrm_fit_workspace_size(ctypes.byref(data.s), ctypes.byref(o))
    ws, wsb = data.workspace(size)
    _check(_L().glrm_fit(ctypes.byref(data.s), _dev_ptr(X, torch.float32, "X", data.m * data.k),
                         _dev_ptr(Y, torch.float32, "Y", data.d * data.k),
                         _dev_ptr(alpha_x, torch.float32, "alpha_x", data.m),
                         _dev_ptr(alpha_y, torch.float32, "alpha_y", data.d), ctypes.byref(o), ctypes.byref(info),
                         _dev_ptr(history, torch.float64, "history") if history is not None else None,
                         ws, wsb, _stream(stream)))
    return dict(sweeps=info.sweeps, objective=info.objective, objective_fp32=info.objective_fp32,
                rows_rejected=info.rows_rejected, cols_rejected=info.cols_rejected,
                kernel_ms=list(info.kernel_ms), kernel_calls=list(info.kernel_calls))


def glrm_impute(data, X, Y, mode=IMPUTE_ALL, out=None, flags=0, stream=None):
    """The decoded table of Section 5.3 (m x n float32): every entry, or with
    ``mode=IMPUTE_MISSING`` only the missing ones (observed entries keep A).
    ``out`` may be a row-strided m x n float32 view (stride (ldh, 1))."""
    torch = _torch()
    if out is None:
        out = torch.empty((data.m, data.n), dtype=torch.float32, device=X.device)
    if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float32:
        raise TypeError("out must be a float32 GPU tensor")
    if out.dim() != 2 or tuple(out.shape) != (data.m, data.n) or out.stride(1) != 1 or out.stride(0) < data.n:
        raise ValueError("out must be m x n with stride (ldh >= n, 1)")
    ws, wsb = data.workspace()
    _check(_L().glrm_impute(ctypes.byref(data.s), _dev_ptr(X, torch.float32, "X", data.m * data.k),
                            _dev_ptr(Y, torch.float32, "Y", data.d * data.k), int(mode),
                            ctypes.c_void_p(out.data_ptr()), int(out.stride(0)), ws, wsb, int(flags),
                            _stream(stream)))
    return out
