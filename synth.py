"""Seeded synthetic GLRM inputs shaped like the paper's workloads.

This module only draws data: tables, observation patterns, loss tables,
regularizers and starting points.  It holds none of the fitting arithmetic and
is the one thing the HIP path and the oracle share.

Random streams: ``numpy.random.default_rng([14100342, config, stream])`` with
stream 0 = hidden factors, 1 = noise / outliers / flips, 2 = observation
pattern, 3 = starting point, 4 = sampled coordinates.

Loss kinds: 0 quadratic, 1 Huber, 2 logistic, 3 hinge, 4 ordinal hinge,
5 categorical one-vs-all, 6 multi-dimensional ordinal (Section 6; a column
under one of these owns levels resp. levels - 1 rows of Y0).
Regularizer kinds: 0 zero, 1 quadratic, 2 l1, 3 nonnegative.
"""
import os
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

SEED = 14100342

QUAD, HUBER, LOGISTIC, HINGE, ORDINAL, CATEGORICAL, MORDINAL = 0, 1, 2, 3, 4, 5, 6
RZERO, RQUAD, RL1, RNONNEG = 0, 1, 2, 3


def rng(config: int, stream: int, extra: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED, int(config), int(stream), int(extra)])


@dataclass
class Case:
    name: str
    m: int
    n: int
    k: int
    layout: str                          # "dense" or "coo"
    col_loss: np.ndarray                 # uint8 [n], index into losses
    losses: List[Tuple[int, int, float]]  # (kind, levels, param)
    rx: Tuple[int, float]
    ry: Tuple[int, float]
    X0: np.ndarray                       # float32 [m, k]
    Y0: np.ndarray                       # float32 [n, k]
    A: Optional[np.ndarray] = None       # dense float32 [m, n]
    mask: Optional[np.ndarray] = None    # dense uint8 [m, n], None = all observed
    rows: Optional[np.ndarray] = None    # coo int32, row-sorted, unique
    cols: Optional[np.ndarray] = None
    vals: Optional[np.ndarray] = None    # coo float32
    sweeps: int = 0
    notes: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        if self.layout == "coo":
            return int(self.rows.size)
        return self.m * self.n if self.mask is None else int(np.count_nonzero(self.mask))


def _normal32(g, shape, scale=1.0):
    return (g.standard_normal(shape, dtype=np.float32) * np.float32(scale)).astype(np.float32)


def _bernoulli_mask(g, m, n, p_obs):
    out = np.empty((m, n), dtype=np.uint8)
    step = max(1, (1 << 24) // max(n, 1))
    for r0 in range(0, m, step):
        r1 = min(m, r0 + step)
        out[r0:r1] = g.random((r1 - r0, n), dtype=np.float32) < np.float32(p_obs)
    return out


def _lowrank_plus_noise(g_f, g_n, m, n, r, noise, chunk_rows=1 << 14):
    U = g_f.standard_normal((m, r)).astype(np.float32)
    V = g_f.standard_normal((r, n)).astype(np.float32)
    A = np.empty((m, n), dtype=np.float32)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        A[r0:r1] = U[r0:r1] @ V + _normal32(g_n, (r1 - r0, n), noise)
    return A


# ---- the five workload shapes ------------------------------------------------

def plain_pca(m=200, n=50, k=5, sweeps=500, config=1):
    """Quadratic loss, no regularizer, fully observed, A = U V + 0.1 N."""
    A = _lowrank_plus_noise(rng(config, 0), rng(config, 1), m, n, k, 0.1)
    g = rng(config, 3)
    return Case("plain_pca_%dx%d_k%d" % (m, n, k), m, n, k, "dense",
                np.zeros(n, np.uint8), [(QUAD, 0, 0.0)], (RZERO, 0.0), (RZERO, 0.0),
                _normal32(g, (m, k)), _normal32(g, (n, k)), A=A, mask=None, sweeps=sweeps)


def dense_quadratic(m=100_000, n=1_000, k=20, missing=0.2, gamma=0.1, sweeps=200, config=2):
    """Rank-k Gaussian product + 0.1 N noise, entries missing at random."""
    A = _lowrank_plus_noise(rng(config, 0), rng(config, 1), m, n, k, 0.1)
    mask = _bernoulli_mask(rng(config, 2), m, n, 1.0 - missing)
    g = rng(config, 3)
    return Case("dense_quadratic_%dx%d_k%d" % (m, n, k), m, n, k, "dense",
                np.zeros(n, np.uint8), [(QUAD, 0, 0.0)], (RQUAD, gamma), (RQUAD, gamma),
                _normal32(g, (m, k)), _normal32(g, (n, k)), A=A, mask=mask, sweeps=sweeps)


def heterogeneous(m=1_000_000, n=200, k=10, missing=0.3, sweeps=200, config=3,
                  n_real=None, n_bool=None, levels=7):
    """Mixed table from a hidden rank-k model: Huber real columns with Laplace
    outliers, logistic Boolean columns with flips, ordinal-hinge columns made by
    cutting each standardized latent column into equal-width bins."""
    n_real = n // 2 if n_real is None else n_real
    n_bool = (3 * n) // 10 if n_bool is None else n_bool
    n_ord = n - n_real - n_bool
    gf, gn = rng(config, 0), rng(config, 1)
    Xt = gf.standard_normal((m, k)).astype(np.float32)
    Yt = gf.standard_normal((k, n)).astype(np.float32)
    A = np.empty((m, n), dtype=np.float32)
    chunk = max(1, (1 << 22) // n)
    # per-column spread of the latent, from a fixed sample of rows (data generation only)
    lat_std = (Xt[: min(m, 65536)] @ Yt).std(axis=0).astype(np.float32) + np.float32(1e-12)
    edges = np.linspace(-3.0, 3.0, levels + 1)[1:-1].astype(np.float32)
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        L = Xt[r0:r1] @ Yt
        rr = r1 - r0
        out = gn.random((rr, n_real), dtype=np.float32) < 0.05
        lap = gn.laplace(0.0, 10.0, (rr, n_real)).astype(np.float32)
        A[r0:r1, :n_real] = L[:, :n_real] + np.where(out, lap, 0).astype(np.float32)
        b = np.where(L[:, n_real:n_real + n_bool] >= 0, 1.0, -1.0).astype(np.float32)
        flip = gn.random((rr, n_bool), dtype=np.float32) < 0.05
        A[r0:r1, n_real:n_real + n_bool] = np.where(flip, -b, b)
        zs = L[:, n_real + n_bool:] / lat_std[n_real + n_bool:]
        A[r0:r1, n_real + n_bool:] = (np.searchsorted(edges, zs.ravel(), side="right").reshape(zs.shape) + 1).astype(np.float32)
    mask = _bernoulli_mask(rng(config, 2), m, n, 1.0 - missing)
    col_loss = np.zeros(n, np.uint8)
    col_loss[n_real:n_real + n_bool] = 1
    col_loss[n_real + n_bool:] = 2
    losses = [(HUBER, 0, 1.0), (LOGISTIC, 0, 0.0), (ORDINAL, levels, 0.0)]
    g = rng(config, 3)
    X0 = np.abs(_normal32(g, (m, k)))
    return Case("heterogeneous_%dx%d_k%d" % (m, n, k), m, n, k, "dense", col_loss, losses,
                (RNONNEG, 0.0), (RQUAD, 0.1), X0, _normal32(g, (n, k)), A=A, mask=mask, sweeps=sweeps)


def autograd_point(m=50_000, n=2_000, k=64, missing=0.1, config=4):
    """Logistic +-1 columns (a = +1 with probability sigmoid(latent)) next to
    quadratic columns (latent + N(0,1)); the evaluation point has entries of
    variance k^-1/2 so that x_i . y_j is of order one."""
    gf, gn = rng(config, 0), rng(config, 1)
    s = float(k) ** -0.25
    Xt = _normal32(gf, (m, k), s)
    Yt = _normal32(gf, (k, n), s)
    nl = n // 2
    A = np.empty((m, n), dtype=np.float32)
    chunk = max(1, (1 << 22) // n)
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        L = Xt[r0:r1] @ Yt
        p = 1.0 / (1.0 + np.exp(-L[:, :nl].astype(np.float64)))
        A[r0:r1, :nl] = np.where(gn.random(p.shape) < p, 1.0, -1.0)
        A[r0:r1, nl:] = L[:, nl:] + _normal32(gn, (r1 - r0, n - nl))
    mask = _bernoulli_mask(rng(config, 2), m, n, 1.0 - missing)
    col_loss = np.zeros(n, np.uint8)
    col_loss[:nl] = 1
    g = rng(config, 3)
    return Case("autograd_%dx%d_k%d" % (m, n, k), m, n, k, "dense", col_loss,
                [(QUAD, 0, 0.0), (LOGISTIC, 0, 0.0)], (RZERO, 0.0), (RZERO, 0.0),
                _normal32(g, (m, k), s), _normal32(g, (n, k), s), A=A, mask=mask)


def sparse_completion(m=2_000_000, n=20_000, k=32, density=0.01, noise=0.05, gamma=1.0,
                      sweeps=50, config=5, threads=None):
    """Each row observes each column independently with probability ``density``
    (drawn as geometric gaps), values from a rank-k Gaussian model plus noise;
    COO sorted by row then column, int32 indices.

    Rows are drawn in fixed chunks of CHUNK rows, each from its own seeded
    streams (pattern: ``rng(config, 2, c)``, noise: ``rng(config, 1, c)`` for
    chunk c), so the chunks can be drawn on several threads and the result
    does not depend on how many there are."""
    import concurrent.futures as cf
    import torch

    gf = rng(config, 0)
    Xt = gf.standard_normal((m, k)).astype(np.float32)
    Yt = gf.standard_normal((n, k)).astype(np.float32)
    Xt_t, Yt_t = torch.from_numpy(Xt), torch.from_numpy(Yt)
    chunk = 16384
    mean = n * density
    per = int(mean + 6.0 * np.sqrt(mean) + 16)   # gaps drawn per row up front

    def draw(c):
        r0 = c * chunk
        r1 = min(m, r0 + chunk)
        rr = r1 - r0
        gp, gn = rng(config, 2, c), rng(config, 1, c)
        # geometric gaps give an exact Bernoulli(density) pattern per row
        pos = np.cumsum(gp.geometric(density, size=(rr, per)), axis=1, dtype=np.int64) - 1
        short = np.nonzero(pos[:, -1] < n)[0]
        rows_extra = {}
        for i in short:   # rows whose gaps did not reach the end yet (rare)
            p = [pos[i]]
            last = p[0][-1]
            while last < n:
                more = last + np.cumsum(gp.geometric(density, size=per), dtype=np.int64)
                p.append(more)
                last = more[-1]
            rows_extra[i] = np.concatenate(p)
        keep = pos < n
        cnt = keep.sum(axis=1)
        cc = pos[keep]
        if rows_extra:
            parts, counts = [], cnt.copy()
            for i in range(rr):
                if i in rows_extra:
                    q = rows_extra[i]
                    q = q[q < n]
                    parts.append(q)
                    counts[i] = q.size
                else:
                    parts.append(pos[i][keep[i]])
            cc, cnt = np.concatenate(parts), counts
        rr_idx = np.repeat(np.arange(r0, r1, dtype=np.int64), cnt)
        with torch.no_grad():
            v = (Xt_t.index_select(0, torch.from_numpy(rr_idx)) *
                 Yt_t.index_select(0, torch.from_numpy(cc))).sum(1).numpy()
        v = v + _normal32(gn, cc.size, noise)
        return rr_idx.astype(np.int32), cc.astype(np.int32), v.astype(np.float32)

    nchunks = (m + chunk - 1) // chunk
    threads = threads or min(16, os.cpu_count() or 1)
    torch_threads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            out = list(ex.map(draw, range(nchunks)))
    finally:
        torch.set_num_threads(torch_threads)
    rows = np.concatenate([o[0] for o in out])
    cols = np.concatenate([o[1] for o in out])
    vals = np.concatenate([o[2] for o in out])
    del out
    g = rng(config, 3)
    return Case("sparse_completion_%dx%d_k%d" % (m, n, k), m, n, k, "coo",
                np.zeros(n, np.uint8), [(QUAD, 0, 0.0)], (RQUAD, gamma), (RQUAD, gamma),
                _normal32(g, (m, k)), _normal32(g, (n, k)), rows=rows, cols=cols, vals=vals,
                sweeps=sweeps)


# ---- a census-shaped table (Section 6.3) ----------------------------------------

def _y_rows(kind, levels):
    """Rows of Y a column takes (its embedding dimension)."""
    return levels if kind == CATEGORICAL else (levels - 1 if kind == MORDINAL else 1)


def census_like(m=3_132_796, k=10, missing=0.1, gamma=0.1, config=6, mordinal=False, offset=True):
    """A stand-in for the survey table of the paper's heterogeneous example:
    m responses to 21 questions of the four types its table lists (5 real, 9
    Boolean, 3 ordinal, 4 categorical), fitted at rank 10 with Huber, hinge,
    ordinal hinge and one-vs-all losses and gamma = 0.1.  The label and level
    counts (categorical 8, 50, 4, 5; ordinal 12, 8, 7) are this generator's
    choices.  Values come from a hidden rank-k Gaussian model: real columns
    are the latent plus N(0, 0.1^2) noise with 5% Laplace(0, 10) outliers,
    Boolean ones its sign with 5% flips, ordinal ones equal-width bins of the
    standardized latent over [-3, 3], categorical ones the argmax over the
    labels of latent scores plus Gumbel noise.  10% of entries are missing
    uniformly.  With ``mordinal`` the ordinal columns take the
    multi-dimensional ordinal loss instead.  With ``offset`` coordinate 0 of
    X0 is 1 (Section 3.3)."""
    kinds = ([(HUBER, 0)] * 5 + [(HINGE, 0)] * 9 + [(MORDINAL if mordinal else ORDINAL, lv) for lv in (12, 8, 7)]
             + [(CATEGORICAL, lv) for lv in (8, 50, 4, 5)])
    # interleave the types the way a survey mixes them (fixed order)
    order = [15, 17, 0, 5, 6, 1, 2, 3, 4, 7, 8, 9, 14, 16, 18, 10, 11, 12, 19, 13, 20]
    kinds = [kinds[i] for i in order]
    n = len(kinds)
    losses, col_loss = [], np.empty(n, np.uint8)
    for j, (kd, lv) in enumerate(kinds):
        entry = (kd, lv, 1.0 if kd == HUBER else 0.0)
        if entry not in losses:
            losses.append(entry)
        col_loss[j] = losses.index(entry)
    gf, gn = rng(config, 0), rng(config, 1)
    Xt = gf.standard_normal((m, k)).astype(np.float32)
    W = [gf.standard_normal((k, lv if kd == CATEGORICAL else 1)).astype(np.float32) / np.float32(np.sqrt(k))
         for kd, lv in kinds]
    A = np.empty((m, n), dtype=np.float32)
    chunk = 1 << 16
    edges = {lv: np.linspace(-3.0, 3.0, lv + 1)[1:-1].astype(np.float32) for kd, lv in kinds if kd in (ORDINAL, MORDINAL)}
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        xt = Xt[r0:r1]
        rr = r1 - r0
        for j, (kd, lv) in enumerate(kinds):
            z = xt @ W[j]
            if kd == HUBER:
                out = gn.random(rr, dtype=np.float32) < 0.05
                A[r0:r1, j] = z[:, 0] + 0.1 * gn.standard_normal(rr, dtype=np.float32) + np.where(
                    out, gn.laplace(0.0, 10.0, rr), 0.0).astype(np.float32)
            elif kd == HINGE:
                b = np.where(z[:, 0] >= 0, 1.0, -1.0).astype(np.float32)
                A[r0:r1, j] = np.where(gn.random(rr, dtype=np.float32) < 0.05, -b, b)
            elif kd in (ORDINAL, MORDINAL):
                A[r0:r1, j] = (np.searchsorted(edges[lv], z[:, 0], side="right") + 1).astype(np.float32)
            else:
                A[r0:r1, j] = (np.argmax(z + gn.gumbel(size=z.shape).astype(np.float32), axis=1) + 1).astype(np.float32)
    mask = _bernoulli_mask(rng(config, 2), m, n, 1.0 - missing)
    d = sum(_y_rows(kd, lv) for kd, lv in kinds)
    g = rng(config, 3)
    X0 = _normal32(g, (m, k))
    if offset:
        X0[:, 0] = 1.0
    return Case("census_like_%dx%d_k%d%s" % (m, n, k, "_mordinal" if mordinal else ""), m, n, k, "dense", col_loss,
                losses, (RQUAD, gamma), (RQUAD, gamma), X0, _normal32(g, (d, k)), A=A, mask=mask,
                notes=dict(d=d, offset=offset))


# ---- small mixed cases for tests -----------------------------------------------

def small_mixed(m, n, k, seed, missing=0.25, layout="dense", rx=(RQUAD, 0.1), ry=(RQUAD, 0.1),
                kinds=(QUAD, HUBER, LOGISTIC, HINGE, ORDINAL), levels=5, x_nonneg=False, empty_row=None,
                empty_col=None):
    """A table that mixes every requested loss kind column by column, with a
    hidden rank-k model under it.  Optional fully unobserved row / column."""
    gf, gn, gp, g0 = rng(100, 0, seed), rng(100, 1, seed), rng(100, 2, seed), rng(100, 3, seed)
    L = gf.standard_normal((m, k)) @ gf.standard_normal((k, n)) / np.sqrt(k)
    col_loss = np.array([i % len(kinds) for i in range(n)], dtype=np.uint8)
    losses = []
    for kd in kinds:
        losses.append((kd, levels if kd == ORDINAL else 0, 1.0 if kd == HUBER else 0.0))
    A = np.empty((m, n), dtype=np.float32)
    for j in range(n):
        kd = kinds[col_loss[j]]
        lj = L[:, j]
        if kd in (QUAD, HUBER):
            A[:, j] = lj + 0.1 * gn.standard_normal(m)
        elif kd in (LOGISTIC, HINGE):
            A[:, j] = np.where(lj + 0.3 * gn.standard_normal(m) >= 0, 1.0, -1.0)
        else:
            A[:, j] = np.clip(np.round(lj + (levels + 1) / 2.0), 1, levels)
    mask = (gp.random((m, n)) >= missing).astype(np.uint8)
    if empty_row is not None:
        mask[empty_row, :] = 0
    if empty_col is not None:
        mask[:, empty_col] = 0
    X0 = (g0.standard_normal((m, k)) / np.sqrt(k) ** 0.5).astype(np.float32)
    Y0 = (g0.standard_normal((n, k)) / np.sqrt(k) ** 0.5).astype(np.float32)
    if x_nonneg:
        X0 = np.abs(X0)
    c = Case("small_%s_%dx%d_k%d_s%d" % (layout, m, n, k, seed), m, n, k, "dense", col_loss, losses,
             tuple(rx), tuple(ry), X0, Y0, A=A, mask=mask)
    if layout == "coo":
        r, cidx = np.nonzero(mask)
        c.layout, c.rows, c.cols = "coo", r.astype(np.int32), cidx.astype(np.int32)
        c.vals = A[r, cidx].astype(np.float32)
        c.A = None
        c.mask = None
    return c


def sample_indices(config, count, upper, stream_extra=0):
    """Seeded sample of distinct indices in [0, upper)."""
    g = rng(config, 4, stream_extra)
    count = min(int(count), int(upper))
    return np.sort(g.choice(upper, size=count, replace=False))
