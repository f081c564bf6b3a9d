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
