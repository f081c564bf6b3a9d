#!/usr/bin/env python3
"""Throughput of the alternating proximal-gradient GLRM sweep on one MI355X.

Workload (default): the dense quadratic GLRM, A = 100,000 x 1,000 = rank-20
Gaussian product + N(0, 0.1^2) noise, 20% of entries missing at random, rank
k = 20, quadratic regularizer 0.1 on both factors.  One step is one sweep of
Algorithm 2 (row half-step, column half-step, objective).  The split-BF16
matrix-core form and the FP32 form run the same number of sweeps from the same
seeded start; their final objectives (recomputed in float64 on the GPU) are
reported side by side.  Printed: one JSON line on stdout.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
IMPUTE_COUNTERS = {"impute": os.path.join(ROOT, "profiles", "impute_counters_heterogeneous.txt"),
                   "impute_dense": os.path.join(ROOT, "profiles", "impute_counters_dense_quadratic.txt")}
# HBM bytes per launch of each workload's dominant kernel, from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs scaled by a plain copy's reading; a line is used
# only while the kernel's sources and flags hash to what they were then.
HBM_COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters.txt")

# The dominant kernel of each sweep workload, its sources (for the hash) and
# its algorithmic bytes per launch (one read of every observed entry's data:
# dense 4 B value + 1 B mask per table entry, COO 4 + 4 B indices + 4 B value
# per entry; plus reading and writing the walked factor and its step sizes).
DOMINANT = {
    "dense": dict(kernel="xstep_kernel", desc="xstep (fused row pass)",
                  files=("dense_kernels.h", "dense_prec.hip", "glrm_device.h", "glrm_kernels.h"),
                  bytes=lambda c: 5.0 * c.m * c.n + 8.0 * c.m * c.k + 8.0 * c.m),
    "coo": dict(kernel="walk_kernel", desc="walk_kernel (row walk: gradient, step, trial, decision)",
                files=("coo.hip", "coo.h", "glrm_device.h"),
                bytes=lambda c: 12.0 * c.nnz + 8.0 * c.m * c.k + 8.0 * c.m),
    # a table too wide for the fused row pass: the whole row half-step (three
    # passes over the table in column blocks, the row steps and decisions)
    "dense_wide": dict(kernel="xwide_kernel", desc="row half-step in column blocks (three table passes)",
                       files=("dense_kernels.h", "dense_prec.hip", "dense.hip", "glrm_device.h", "glrm_kernels.h"),
                       bytes=lambda c: 3 * 5.0 * c.m * c.n + 3 * 8.0 * c.m * c.k + 8.0 * c.m),
    "grad": dict(kernel="lossgrad_kernel", desc="lossgrad (objective and both gradients, one pass)",
                 files=("dense_kernels.h", "dense_prec.hip", "glrm_device.h", "glrm_kernels.h"),
                 bytes=lambda c: 5.0 * c.m * c.n + 8.0 * c.m * c.k + 8.0 * c.n * c.k),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _code_only(text):
    """Source text without comments, trailing blanks and empty lines: what the
    compiler sees, so comment edits do not invalidate stored counters."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.splitlines() if l.strip())


def kernel_source_hash(read=None, unit="dense", files=None, prec_flags=None):
    """Hash of the code of a kernel's sources (comments ignored) and of the
    compiler flags it is built with (include paths left out).  ``unit`` is
    "dense" (the benchmark's split-BF16 instances) or "impute"; or give the
    ``files`` (and the dense precision's flags, ``prec_flags`` = (prec, lks))."""
    from paper_1410_0342_amd import build as B
    h = hashlib.sha256()
    if files is not None:
        extra = B.dense_prec_flags(*prec_flags) if prec_flags else []
        flags = [f for f in B.FLAGS + extra if not f.startswith("-I")]
    elif unit == "impute":
        flags = [f for f in B.FLAGS if not f.startswith("-I")]
        files = ("impute.hip", "impute.h", "glrm_device.h")
    else:
        flags = [f for f in B.FLAGS + B.dense_prec_flags(1, 0) if not f.startswith("-I")]
        files = ("dense_kernels.h", "dense_prec.hip", "glrm_device.h", "glrm_kernels.h")
    h.update(" ".join(flags).encode())
    for f in files:
        rel = "paper_1410_0342_amd/csrc/" + f
        if read is None:
            with open(os.path.join(ROOT, rel)) as fh:
                text = fh.read()
        else:
            text = read(rel)
        h.update(_code_only(text).encode())
    return h.hexdigest()[:16]


def _prec_flags(kind, pname, case):
    """(precision, loss set) of the dense instances a run uses, for the hash."""
    if kind == "coo":
        return None
    p = {"fp32": 0, "bf16": 1, "bf16_plain": 3}[pname]
    lks = 0 if (case.col_loss is None or len(case.losses) == 1) and case.losses[0][0] == 0 else 1
    return (p, lks)


def counter_traffic(kind, workload_name, pname, case):
    """HBM bytes per launch of the dominant kernel (fetched + written), if the
    committed counters match the current sources; else None."""
    d = DOMINANT[kind]
    if not os.path.exists(HBM_COUNTERS):
        return None
    h = kernel_source_hash(files=d["files"], prec_flags=_prec_flags(kind, pname, case))
    for line in open(HBM_COUNTERS).read().splitlines():
        f = dict(kv.split("=", 1) for kv in line.split() if "=" in kv)
        if (f.get("kernel") == d["kernel"] and f.get("workload") == workload_name and f.get("precision") == pname
                and f.get("hash") == h):
            return float(f["fetch_bytes"]) + float(f["write_bytes"])
    return None


def workload(name):
    import synth
    if name == "dense_quadratic":
        return synth.dense_quadratic()
    if name == "heterogeneous":
        return synth.heterogeneous()
    if name == "sparse_completion":
        return synth.sparse_completion()
    if name == "plain_pca":
        return synth.plain_pca()
    if name in ("autograd", "autograd_fit"):
        return synth.autograd_point()
    if name == "impute":
        return synth.heterogeneous()
    if name == "impute_dense":
        return synth.dense_quadratic()
    if name in ("proxprox", "linalg"):
        return synth.dense_quadratic()
    if name == "census":
        return synth.census_like()
    raise SystemExit("unknown workload " + name)


def run_adjacent(name, case, steps, warmup):
    """The adjacent steps on full-size workloads, timed with HIP events on
    the stream the calls run on.  proxprox: sweeps of the prox-prox update
    (FP32, one inner solve) beside prox-grad FP32 from the same start;
    linalg: column scaling, SVD initialization and the certificate on the
    dense quadratic table; census: sweeps of the multi-dimensional-loss fit."""
    import numpy as np
    import torch

    import paper_1410_0342_amd as g

    dev = torch.device("cuda:0")
    data = g.Data.from_case(case, dev)
    if case.notes.get("offset"):
        data = data.variant(offset=True)
    g.glrm_prepare(data)
    st = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    if name == "linalg":
        mu, s2 = g.glrm_column_scaling(data)
        out["column_scaling_ms"] = timed(lambda: g.glrm_column_scaling(data, mu, s2, flags=g.WS_PREPARED), 3)
        k = case.k
        gen = torch.Generator().manual_seed(0)
        omega = torch.randn((case.n, k + 10), generator=gen, dtype=torch.float32).to(dev)
        res = {}

        def init():
            res["X"], res["Y"], res["sv"] = g.glrm_init_svd(data, omega, mu, s2, power_iters=2, flags=g.WS_PREPARED)
        out["init_svd_ms"] = timed(init, 3)
        cdata = data.with_regs((1, 0.1), (1, 0.1))
        g.glrm_prepare(cdata)
        cert = {}

        def certify():
            cert["info"] = g.glrm_certificate(cdata, res["X"], res["Y"], iters=100, flags=g.WS_PREPARED)
        out["certificate_100_iters_ms"] = timed(certify, 3)
        out["certificate_norm"] = cert["info"]["norm"]
        out["top_singular_values"] = [float(v) for v in np.asarray(res["sv"])[:3]]
        for kname, v in out.items():
            if kname.endswith("_ms"):
                log("%s: %.3f ms" % (kname, v))
        return out
    precs = {"proxprox": [("proxprox_fp32", g.FP32, g.UPDATE_PROXPROX), ("proxgrad_fp32", g.FP32, g.UPDATE_PROXGRAD)],
             "census": [("bf16", g.BF16, g.UPDATE_PROXGRAD), ("fp32", g.FP32, g.UPDATE_PROXGRAD)]}[name]
    for tag, prec, upd in precs:
        X = torch.from_numpy(case.X0).to(dev)
        Y = torch.from_numpy(case.Y0).to(dev)
        ax = torch.empty(case.m, dtype=torch.float32, device=dev)
        ay = torch.empty(data.d, dtype=torch.float32, device=dev)
        g.glrm_fit(data, X, Y, ax, ay, warmup, precision=prec, init_alpha=True, flags=g.WS_PREPARED, update=upd)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        info = g.glrm_fit(data, X, Y, ax, ay, steps, precision=prec, init_alpha=False, flags=g.WS_PREPARED,
                          update=upd)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / max(steps, 1)
        out[tag] = dict(ms_per_step=ms, value=case.nnz / (ms * 1e-3), objective=info["objective"],
                        rows_rejected=info["rows_rejected"], cols_rejected=info["cols_rejected"])
        # the dominant launch (slot 0: the fused row pass, or the rows' Gram
        # pass of the prox-prox update), timed with HIP events around each
        # launch on the fit's stream, in a shorter fit from the same state
        kinfo = g.glrm_fit(data, X.clone(), Y.clone(), ax.clone(), ay.clone(), min(max(steps, 1), 10),
                           precision=prec, init_alpha=False, flags=g.WS_PREPARED | g.TIME_KERNELS, update=upd)
        out[tag]["launch0_ms"] = kinfo["kernel_ms"][0] / max(kinfo["kernel_calls"][0], 1)
        log("%s: %.4f ms/sweep, %.4g entries/s, F after %d sweeps = %.10g"
            % (tag, ms, out[tag]["value"], steps + warmup, info["objective"]))
    if name == "census":
        out["embedded_columns"] = int(data.d)   # the width of the table the row pass reads
    return out


def run_gpu(case, precisions, steps, warmup):
    import numpy as np
    import torch

    import paper_1410_0342_amd as g

    dev = torch.device("cuda:0")
    data = g.Data.from_case(case, dev)
    g.glrm_prepare(data)
    torch.cuda.synchronize()
    nnz = case.nnz
    out = {}
    for pname in precisions:
        prec = g.PRECISIONS[pname]
        X = torch.from_numpy(case.X0).to(dev)
        Y = torch.from_numpy(case.Y0).to(dev)
        ax = torch.empty(case.m, dtype=torch.float32, device=dev)
        ay = torch.empty(case.n, dtype=torch.float32, device=dev)
        if warmup > 0:
            g.glrm_fit(data, X, Y, ax, ay, warmup, precision=prec, init_alpha=True, flags=g.WS_PREPARED)
        else:
            g.glrm_fit(data, X, Y, ax, ay, 0, precision=prec, init_alpha=True, flags=g.WS_PREPARED)
        hist = torch.zeros(max(steps, 1), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = g.glrm_fit(data, X, Y, ax, ay, steps, precision=prec, init_alpha=False, flags=g.WS_PREPARED,
                          history=hist)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (t1 - t0) * 1e3 / max(steps, 1)
        # per-kernel durations (HIP events around every launch, on the fit's
        # stream) from a separate, shorter fit that continues from the same state
        kt_sweeps = min(max(steps, 1), 20)
        kinfo = g.glrm_fit(data, X.clone(), Y.clone(), ax.clone(), ay.clone(), kt_sweeps, precision=prec,
                           init_alpha=False, flags=g.WS_PREPARED | g.TIME_KERNELS)
        torch.cuda.synchronize()
        # Spread of the per-sweep time: each sample is the extra time of a
        # 25-sweep fit over a 5-sweep fit, divided by 20, which cancels a fit
        # call's fixed cost (set-up, final FP64 objective, synchronization).
        # HIP events on the stream the fits run on; the timed state is untouched.
        Xs, Ys, axs, ays = X.clone(), Y.clone(), ax.clone(), ay.clone()
        st = torch.cuda.current_stream()

        def fit_ms(sweeps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            g.glrm_fit(data, Xs, Ys, axs, ays, sweeps, precision=prec, init_alpha=False, flags=g.WS_PREPARED)
            e1.record(st)
            e1.synchronize()
            return e0.elapsed_time(e1)

        per = [(fit_ms(25) - fit_ms(5)) / 20.0 for _ in range(10)]
        pct = np.percentile(np.array(per), [10, 50, 90])
        del Xs, Ys, axs, ays
        out[pname] = dict(ms_per_step=ms, value=nnz / (ms * 1e-3), objective=info["objective"],
                          sweep_ms_p10_p50_p90=[float(v) for v in pct],
                          objective_tracked=info["objective_fp32"], rows_rejected=info["rows_rejected"],
                          cols_rejected=info["cols_rejected"],
                          kernel_ms=[v / kt_sweeps for v in kinfo["kernel_ms"]],
                          kernel_calls=[c / kt_sweeps for c in kinfo["kernel_calls"]],
                          history=hist.cpu().numpy()[:steps])
        log("%s: %.4f ms/sweep, %.4g entries/s, F = %.10g (tracked %.10g), kernel ms per sweep %s"
            % (pname, ms, out[pname]["value"], info["objective"], info["objective_fp32"],
               ["%.4f" % v for v in out[pname]["kernel_ms"]]))
        del X, Y, ax, ay
    return out


def run_grad(case, precisions, steps, warmup):
    """One step = one objective-and-gradient evaluation (glrm_grad with the
    objective) at a fixed point: the autograd forward and backward."""
    import torch

    import paper_1410_0342_amd as g

    dev = torch.device("cuda:0")
    data = g.Data.from_case(case, dev)
    g.glrm_prepare(data)
    X = torch.from_numpy(case.X0).to(dev)
    Y = torch.from_numpy(case.Y0).to(dev)
    dX = torch.empty_like(X)
    dY = torch.empty_like(Y)
    out = {}
    for pname in precisions:
        prec = g.PRECISIONS[pname]
        for _ in range(max(warmup, 1)):
            g.glrm_grad(data, X, Y, prec, dX=dX, dY=dY, flags=g.WS_PREPARED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.glrm_grad(data, X, Y, prec, dX=dX, dY=dY, flags=g.WS_PREPARED)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
        _, _, obj = g.glrm_grad(data, X, Y, prec, dX=dX, dY=dY, want_objective=True, flags=g.WS_PREPARED)
        out[pname] = dict(ms_per_step=ms, value=case.nnz / (ms * 1e-3), objective=obj)
        log("%s: %.4f ms per objective and gradient, %.4g entries/s, F = %.10g" % (pname, ms, out[pname]["value"], obj))
    return out


def run_impute(case, steps, warmup):
    """One step = one decoded table (glrm_impute, Section 5.3) from the case's
    seeded starting factors (the pass's work and data movement do not depend on
    their values), in each of the two forms; HIP events on the stream the calls
    run on bracket the timed calls."""
    import torch

    import paper_1410_0342_amd as g

    dev = torch.device("cuda:0")
    data = g.Data.from_case(case, dev)
    g.glrm_prepare(data)
    X = torch.from_numpy(case.X0).to(dev)
    Y = torch.from_numpy(case.Y0).to(dev)
    out = torch.empty((case.m, case.n), dtype=torch.float32, device=dev)
    m, n, k = case.m, case.n, case.k
    res = {}
    for name, mode, alg_bytes in (("all", g.IMPUTE_ALL, 4.0 * m * n + 4.0 * (m + n) * k),
                                  ("missing", g.IMPUTE_MISSING, 9.0 * m * n + 4.0 * (m + n) * k)):
        for _ in range(max(warmup, 1)):
            g.glrm_impute(data, X, Y, mode=mode, out=out, flags=g.WS_PREPARED)
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(steps):
            g.glrm_impute(data, X, Y, mode=mode, out=out, flags=g.WS_PREPARED)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / max(steps, 1)
        gbs = alg_bytes / (ms * 1e-3) / 1e9
        res[name] = dict(ms_per_step=ms, value=m * n / (ms * 1e-3), achieved=gbs, alg_bytes=alg_bytes)
        log("impute %s: %.4f ms per table, %.4g entries/s, %.0f GB/s algorithmic" % (name, ms, m * n / (ms * 1e-3), gbs))
    return res


def copy_calibration():
    """A plain device copy of known size (for scaling rocprofv3 byte counters)."""
    import torch
    src = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy calibration: 5 copies of %d bytes" % (src.numel() * 4))


def _sub_problem(case, rows):
    """The oracle's problem on the first `rows` rows of the workload."""
    import numpy as np

    import oracle
    if case.layout == "coo":
        hi = int(np.searchsorted(case.rows, rows))
        return oracle.Problem.from_coo(rows, case.n, case.k, case.rows[:hi], case.cols[:hi], case.vals[:hi],
                                       case.col_loss, case.losses, case.rx, case.ry)
    sub_mask = None if case.mask is None else case.mask[:rows]
    return oracle.Problem.from_dense(case.A[:rows], sub_mask, case.k, case.col_loss, case.losses, case.rx, case.ry)


def cpu_baseline(case, rows, sweeps, grad_only=False):
    """The FP64 oracle (as it stands, one thread) on the first `rows` rows of
    the same workload: `sweeps` sweeps of Algorithm 2, or with ``grad_only``
    that many objective-and-gradient evaluations."""
    import numpy as np

    P = _sub_problem(case, rows)
    X = case.X0[:rows].astype(np.float64).copy()
    Y = case.Y0.astype(np.float64).copy()
    ax, ay = P.init_alpha(1.0)
    t0 = time.perf_counter()
    for _ in range(sweeps):
        if grad_only:
            P.objective(X, Y)
            P.grad(X, Y)
        else:
            P.sweep(X, Y, ax, ay)
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), cpu)
    except OSError:
        pass
    what = "objective-and-gradient evaluation(s)" if grad_only else "sweep(s)"
    return dict(value=P.nnz * sweeps / dt, unit="entries/s", cores=1, kind="oracle",
                sample="first %d of %d rows (%d observed entries), %d %s of the FP64 oracle, "
                       "single thread, %.1f s" % (rows, case.m, P.nnz, sweeps, what, dt),
                cpu=cpu, host_cpus=os.cpu_count())


def _host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            return next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "unknown")
    except OSError:
        return "unknown"


def proxprox_cpu_baseline(case, rows, sweeps):
    """The FP64 oracle's prox-prox sweeps (one thread) on the first `rows` rows."""
    import numpy as np

    P = _sub_problem(case, rows)
    X = case.X0[:rows].astype(np.float64).copy()
    Y = case.Y0.astype(np.float64).copy()
    ax, ay = P.init_alpha(1.0)
    t0 = time.perf_counter()
    for _ in range(sweeps):
        P.half_step_x_pp(X, Y, ax)
        P.half_step_y_pp(X, Y, ay)
    dt = time.perf_counter() - t0
    return dict(value=P.nnz * sweeps / dt, unit="entries/s", cores=1, kind="oracle",
                sample="first %d of %d rows (%d observed entries), %d prox-prox sweep(s) of the FP64 oracle, "
                       "single thread, %.1f s" % (rows, case.m, P.nnz, sweeps, dt), cpu=_host_cpu())


def impute_cpu_baseline(case, rows):
    """The oracle's decode of every entry (one thread) on the first `rows` rows."""
    import numpy as np

    import oracle
    X = case.X0[:rows].astype(np.float64)
    Y = case.Y0.astype(np.float64)
    t0 = time.perf_counter()
    oracle.impute(X, Y, case.col_loss, case.losses)
    dt = time.perf_counter() - t0
    return dict(value=rows * case.n / dt, unit="entries/s", cores=1, kind="oracle",
                sample="first %d of %d rows (%d entries), every entry decoded by the oracle, single thread, "
                       "%.1f s" % (rows, case.m, rows * case.n, dt), cpu=_host_cpu())


def svd_cpu_baseline(case, rows):
    """The oracle's SVD initialization (its exact SVD, LAPACK held to one
    thread) on the first `rows` rows, scaled to the whole table by rows (the
    SVD of a tall rows x n table costs in proportion to rows)."""
    from threadpoolctl import threadpool_limits

    P = _sub_problem(case, rows)
    mu, s2 = P.column_scaling()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        P.init_svd(mu, s2, case.k)
        dt = time.perf_counter() - t0
    return dict(value=dt * 1e3 * case.m / rows, unit="ms", cores=1, kind="oracle",
                sample="first %d of %d rows: the oracle's exact SVD initialization, one thread, %.1f s, "
                       "scaled by %d / %d rows" % (rows, case.m, dt, case.m, rows), cpu=_host_cpu())


def census_cpu_baseline(case, rows, sweeps):
    """The feature-level FP64 oracle (one thread) on the first `rows` rows."""
    import numpy as np

    import oracle
    feats = [tuple(case.losses[int(c)]) for c in case.col_loss]
    M = oracle.MDProblem(case.A[:rows], case.mask[:rows], case.k, feats, case.rx, case.ry,
                         offset=bool(case.notes.get("offset")))
    X = case.X0[:rows].astype(np.float64).copy()
    Y = case.Y0.astype(np.float64).copy()
    ax, af = M.init_alpha(1.0)
    t0 = time.perf_counter()
    for _ in range(sweeps):
        M.half_step_x(X, Y, ax)
        M.half_step_y(X, Y, af)
    dt = time.perf_counter() - t0
    return dict(value=M.nnz * sweeps / dt, unit="entries/s", cores=1, kind="oracle",
                sample="first %d of %d rows (%d observed values), %d sweep(s) of the feature-level FP64 oracle, "
                       "single thread, %.1f s" % (rows, case.m, M.nnz, sweeps, dt))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dense_quadratic",
                    choices=["dense_quadratic", "heterogeneous", "sparse_completion", "plain_pca", "autograd",
                             "autograd_fit", "impute", "impute_dense", "proxprox", "linalg", "census"])
    ap.add_argument("--precision", default="both", choices=["both", "bf16", "fp32", "bf16_plain"])
    ap.add_argument("--cpu-rows", type=int, default=100000)
    ap.add_argument("--cpu-sweeps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the GLRM sweep here is built and measured on a single MI355X "
              "(the multi-GPU row sharding is designed, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    t0 = time.perf_counter()
    case = workload(args.workload)
    log("workload %s: m=%d n=%d k=%d observed=%d (generated in %.1f s)"
        % (case.name, case.m, case.n, case.k, case.nnz, time.perf_counter() - t0))
    if case.layout == "coo":
        # the sparse walks: FP32 (the faster form there) heads the line, BF16 beside it
        precisions = ["fp32", "bf16"] if args.precision == "both" else [args.precision]
    else:
        precisions = ["bf16", "fp32"] if args.precision == "both" else [args.precision]
    if args.workload in ("proxprox", "linalg", "census"):
        res = run_adjacent(args.workload, case, args.steps, args.warmup)
        if args.workload == "linalg":
            line = {"metric": "time per call of the linear-algebra steps (Sections 4.3, 7.5, 7.6)",
                    "value": res["init_svd_ms"], "unit": "ms", "higher_is_better": False, "n_gpus": 1,
                    "steps": 3, "warmup": 1, "data": "synthetic", "dtype": "f32/f64",
                    "config": {"workload": "linalg_" + case.name, "m": case.m, "n": case.n, "k": case.k}}
            line.update(res)
            if not args.no_cpu_baseline:
                line["cpu_baseline"] = svd_cpu_baseline(case, min(args.cpu_rows // 10, case.m))
        else:
            head = next(iter(res))
            line = {"metric": "observed entries/s per sweep", "value": res[head]["value"], "unit": "entries/s",
                    "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                    "ms_per_step": res[head]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                    "vs_baseline": None, "dtype": "bf16" if head == "bf16" else "f32", "data": "synthetic",
                    "config": {"workload": args.workload + "_" + case.name, "m": case.m, "n": case.n, "k": case.k,
                               "observed_entries": int(case.nnz), "precision": head}}
            line.update(res)
            t0 = res[head]["launch0_ms"]
            if args.workload == "proxprox":
                # the rows' Gram pass: per observed entry the upper triangle of
                # w v v^T (k (k + 1) / 2 multiply-adds) and w a v (k)
                flops = float(case.nnz) * (case.k * (case.k + 1) + 2 * case.k)
                line["roofline"] = {"bound": "mfma", "kernel": "pp_gram (the rows' Gram pass, fp32 matrix cores)",
                                    "achieved": flops / (t0 * 1e-3) / 1e12, "peak": 157.3, "unit": "TFLOP/s",
                                    "frac": flops / (t0 * 1e-3) / 1e12 / 157.3, "traffic": None,
                                    "avg_launch_ms": t0, "algorithmic_flops_per_launch": flops}
                if not args.no_cpu_baseline:
                    line["cpu_baseline"] = proxprox_cpu_baseline(case, min(args.cpu_rows // 5, case.m), 1)
            else:
                d = int(line.get("embedded_columns") or 0) or case.n
                alg = 5.0 * case.m * d + 8.0 * case.m * case.k + 8.0 * case.m
                line["roofline"] = {"bound": "hbm", "kernel": "xstep (fused row pass on the embedded table)",
                                    "achieved": alg / (t0 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": alg / (t0 * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                                    "avg_launch_ms": t0, "algorithmic_bytes_per_launch": alg}
                if not args.no_cpu_baseline:
                    line["cpu_baseline"] = census_cpu_baseline(case, min(args.cpu_rows * 10, case.m), args.cpu_sweeps)
        print(json.dumps(line), flush=True)
        return
    if args.workload in ("impute", "impute_dense"):
        res = run_impute(case, args.steps, args.warmup)
        if args.copy_calibration:
            copy_calibration()
        r = res["all"]
        traffic = {}
        counters = IMPUTE_COUNTERS[args.workload]
        if os.path.exists(counters):
            try:
                pc = dict(l.split(":", 1) for l in open(counters).read().splitlines() if ":" in l)
                pc = {k.strip(): v.strip() for k, v in pc.items()}
                if pc.get("kernel_source_hash") == kernel_source_hash(unit="impute") and case.name in pc.get("kernel", ""):
                    traffic = {"all": float(pc["traffic_bytes_per_launch_all"]),
                               "missing": float(pc["traffic_bytes_per_launch_missing"])}
            except (OSError, ValueError, KeyError):
                traffic = {}
        line = {
            "metric": "table entries decoded/s (Section 5.3 imputation)",
            "value": r["value"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "impute_" + case.name, "m": case.m, "n": case.n, "k": case.k,
                       "layout": "dense", "mode": "all"},
            "roofline": {"bound": "hbm", "kernel": "impute (every entry)", "achieved": r["achieved"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": r["achieved"] / HBM_PEAK_GBS,
                         "traffic": traffic.get("all"), "algorithmic_bytes_per_launch": r["alg_bytes"]},
            "missing_only": {"value": res["missing"]["value"], "ms_per_step": res["missing"]["ms_per_step"],
                             "traffic": traffic.get("missing"),
                             "achieved_GBs": res["missing"]["achieved"],
                             "frac": res["missing"]["achieved"] / HBM_PEAK_GBS,
                             "algorithmic_bytes_per_launch": res["missing"]["alg_bytes"]},
        }
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = impute_cpu_baseline(case, min(args.cpu_rows * 10, case.m))
        print(json.dumps(line), flush=True)
        return
    if args.workload == "autograd":
        res = run_grad(case, precisions, args.steps, args.warmup)
        head = precisions[0]
        r = res[head]
        m, n, k = case.m, case.n, case.k
        alg_bytes = DOMINANT["grad"]["bytes"](case)   # table and mask, X and dX, Y and dY
        achieved = alg_bytes / (r["ms_per_step"] * 1e-3) / 1e9
        line = {
            "metric": "observed entries/s per objective and gradient evaluation",
            "value": r["value"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16" if head.startswith("bf16") else "f32", "data": "synthetic",
            "config": {"workload": case.name, "m": m, "n": n, "k": k, "observed_entries": int(case.nnz),
                       "layout": "dense", "precision": head},
            "roofline": {"bound": "hbm", "kernel": "objective and gradient call (one lossgrad pass + reductions)",
                         "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": counter_traffic("grad", args.workload, head, case),
                         "algorithmic_bytes_per_launch": alg_bytes},
            "objective": {p: res[p]["objective"] for p in res},
        }
        if "fp32" in res and head != "fp32":
            line["fp32"] = {"value": res["fp32"]["value"], "ms_per_step": res["fp32"]["ms_per_step"]}
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline(case, min(args.cpu_rows // 10, case.m), args.cpu_sweeps,
                                                grad_only=True)
        print(json.dumps(line), flush=True)
        return
    res = run_gpu(case, precisions, args.steps, args.warmup)
    if args.copy_calibration:
        copy_calibration()

    head = precisions[0]
    r = res[head]
    m, n, k = case.m, case.n, case.k
    kind = "dense" if case.layout == "dense" else "coo"
    if args.workload == "autograd_fit":
        kind = "dense_wide"
    dom = DOMINANT[kind]
    # dominant kernel: the row pass (kernel kind 0), timed with HIP events on the fit's stream
    calls = max(r["kernel_calls"][0], 1)
    avg_ms = r["kernel_ms"][0] / calls
    alg_bytes = dom["bytes"](case)
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    line = {
        "metric": "observed entries/s per prox-grad sweep, bf16-MFMA vs fp32 at equal objective",
        "value": r["value"],
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if head.startswith("bf16") else "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "m": m, "n": n, "k": k, "observed_entries": case.nnz,
                   "layout": case.layout, "precision": head,
                   "sweeps_timed": args.steps, "sweeps_total": args.steps + args.warmup},
        "roofline": {"bound": "hbm", "kernel": dom["desc"], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counter_traffic(kind, args.workload, head, case), "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "objective": {p: res[p]["objective"] for p in res},
    }
    if len(res) == 2:
        other = precisions[1]
        # equal objective: both forms from the same seeded start for at least
        # CMP_SWEEPS sweeps (the timed run's own count when it is longer)
        cmp_sweeps = max(args.steps + args.warmup, 200 if kind.startswith("dense") else 50)
        if cmp_sweeps == args.steps + args.warmup:
            hist = {p: res[p]["history"] for p in res}
            fin = {p: res[p]["objective"] for p in res}
            offset = args.warmup
        else:
            hist, fin = compare_fits(case, precisions, cmp_sweeps)
            offset = 0
        fb, ff = fin.get("bf16"), fin.get("fp32")
        # time to equal objective: the sweeps each form needs to come within
        # 1e-3 of the FP32 fit's final objective, times its time per sweep
        target = ff + 1e-3 * abs(ff)

        def sweeps_to(h):
            reach = [i for i, v in enumerate(h) if v <= target]
            return (reach[0] + 1 + offset) if reach else None

        sb, sf = sweeps_to(hist["bf16"]), sweeps_to(hist["fp32"])
        line["equal_objective"] = {
            "sweeps": cmp_sweeps, "bf16": fb, "fp32": ff, "rel_diff": (fb - ff) / abs(ff),
            "bf16_no_worse_within_1e-3": fb <= target,
            "bf16_sweeps_to_fp32_objective": sb, "fp32_sweeps_to_fp32_objective": sf,
            "time_to_equal_objective_speedup": (
                (res["fp32"]["ms_per_step"] * sf) / (res["bf16"]["ms_per_step"] * sb) if sb and sf else None)}
        line[other] = {"value": res[other]["value"], "ms_per_step": res[other]["ms_per_step"]}
        line["rejected_last_sweep"] = {p: {"rows": res[p]["rows_rejected"], "cols": res[p]["cols_rejected"]}
                                       for p in res}
        line["bf16_over_fp32"] = res["bf16"]["value"] / res["fp32"]["value"]
    line["kernel_ms_per_sweep"] = {p: res[p]["kernel_ms"] for p in res}
    line["sweep_ms_p10_p50_p90"] = {p: res[p]["sweep_ms_p10_p50_p90"] for p in res}
    if not args.no_cpu_baseline:
        rows = min(args.cpu_rows, case.m)
        line["cpu_baseline"] = cpu_baseline(case, rows, args.cpu_sweeps)
    print(json.dumps(line), flush=True)


def compare_fits(case, precisions, sweeps):
    """Both forms from the seeded start for `sweeps` sweeps (untimed):
    per-sweep objective histories and the final FP64 objectives."""
    import torch

    import paper_1410_0342_amd as g

    dev = torch.device("cuda:0")
    data = g.Data.from_case(case, dev)
    g.glrm_prepare(data)
    hist, fin = {}, {}
    for pname in precisions:
        X = torch.from_numpy(case.X0).to(dev)
        Y = torch.from_numpy(case.Y0).to(dev)
        ax = torch.empty(case.m, dtype=torch.float32, device=dev)
        ay = torch.empty(case.n, dtype=torch.float32, device=dev)
        h = torch.zeros(sweeps, dtype=torch.float64, device=dev)
        info = g.glrm_fit(data, X, Y, ax, ay, sweeps, precision=g.PRECISIONS[pname], init_alpha=True,
                          flags=g.WS_PREPARED, history=h)
        hist[pname] = h.cpu().numpy()
        fin[pname] = info["objective"]
        log("equal-objective run, %s: F after %d sweeps = %.10g" % (pname, sweeps, info["objective"]))
    return hist, fin


if __name__ == "__main__":
    main()
