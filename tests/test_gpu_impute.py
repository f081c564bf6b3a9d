"""GPU parity of the imputation decode (Section 5.3) against the FP64 oracle,
through the C ABI.

The kernel forms x_i . y_j as a float32 multiply-add chain of k terms, so it is
within k * 2^-24 * sum_l |x_il y_jl| of the exact product; the tests allow
BOUND = 1e-5 * sum_l |x_il y_jl| (k <= 64).  Real-valued columns (quadratic,
Huber) must agree to BOUND.  Boolean and ordinal columns are integer decisions
taken from that product: they must match the oracle exactly wherever the FP64
product is farther than BOUND from a decision boundary (0; the half-integers
between levels); within it, the kernel's value must be the decoded value of
some product in [u - BOUND, u + BOUND] (either neighbour).  Observed entries
in the missing-only form are bit-exact copies of A.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1410_0342_amd as g  # noqa: E402

DEV = torch.device("cuda:0")
F32 = lambda v: float(np.float32(v))  # noqa: E731


def _closed_form(u, kind, levels):
    """The decoded value of Section 5.3 by kind (arrays broadcast)."""
    boolean = np.where(u > 0, 1.0, -1.0)
    ordinal = np.clip(np.ceil(u - 0.5), 1.0, levels)
    return np.where(kind <= 1, u, np.where(kind <= 3, boolean, ordinal))


def check_decoded(X, Y, col_loss, losses, got, A=None, mask=None):
    """Compare the kernel's table with the oracle's; returns the number of
    entries that sat within rounding of a decision boundary."""
    X, Y = np.asarray(X, np.float64), np.asarray(Y, np.float64)
    Z, want = oracle.impute(X, Y, col_loss, losses, A=A, mask=mask)
    got = np.asarray(got, np.float64)
    bound = 1e-5 * (np.abs(X) @ np.abs(Y).T) + 1e-30
    kinds = np.array([losses[c][0] for c in col_loss])
    levels = np.array([max(losses[c][1], 1) for c in col_loss], np.float64)
    decoded = np.ones(Z.shape, bool) if mask is None else ~np.asarray(mask, bool)
    ties = 0
    real = (kinds <= 1)[None, :] & decoded
    assert np.all(np.abs(got[real] - Z[real]) <= bound[real]), np.max(np.abs(got - Z)[real] / bound[real])
    disc = (kinds >= 2)[None, :] & decoded
    lo = _closed_form(Z - bound, kinds[None, :], levels[None, :])
    hi = _closed_form(Z + bound, kinds[None, :], levels[None, :])
    sure = disc & (lo == hi)
    assert np.array_equal(got[sure], want[sure])
    near = disc & (lo != hi)
    ties += int(near.sum())
    assert np.all((got[near] == lo[near]) | (got[near] == hi[near]))
    if mask is not None:
        obs = np.asarray(mask, bool)
        assert np.array_equal(got[obs], np.asarray(A, np.float64)[obs])
    return ties


def _factors(m, n, k, seed):
    """Factors whose products spread over every level of a 5-level ordinal
    column: a constant first component shifts u to about 3."""
    r = np.random.default_rng([1410, 342, seed])
    X = r.standard_normal((m, k)).astype(np.float32)
    Y = (r.standard_normal((n, k)) * (2.0 / np.sqrt(k))).astype(np.float32)
    X[:, 0] = 1.0
    Y[:, 0] = 3.0
    return X, Y


CASES = [
    dict(m=1, n=1, k=1, seed=1),
    dict(m=37, n=23, k=3, seed=2),          # ragged rows and lanes, one column block
    dict(m=300, n=300, k=5, seed=3),        # a second, ragged column block of 256
    dict(m=130, n=517, k=20, seed=4),       # three column blocks, rank of the benchmark
    dict(m=77, n=64, k=64, seed=5),         # largest rank
    dict(m=1000, n=40, k=33, seed=6),       # many rows per workgroup, odd rank
    dict(m=50, n=1000, k=64, seed=10),      # unaligned rows of a 16-wavefront workgroup, largest rank
]


def _data(c, X, Y, layout="dense"):
    case = synth.small_mixed(c["m"], c["n"], c["k"], c["seed"], missing=0.3, layout=layout)
    return case, g.Data.from_case(case, DEV)


@pytest.mark.parametrize("c", CASES, ids=lambda c: "%dx%d_k%d" % (c["m"], c["n"], c["k"]))
@pytest.mark.parametrize("mode", [g.IMPUTE_ALL, g.IMPUTE_MISSING], ids=["all", "missing"])
def test_dense_impute_matches_the_oracle(c, mode):
    X, Y = _factors(c["m"], c["n"], c["k"], c["seed"])
    case, data = _data(c, X, Y)
    out = g.glrm_impute(data, to_dev(X, DEV), to_dev(Y, DEV), mode=mode)
    torch.cuda.synchronize()
    losses = [(a, b, F32(p)) for a, b, p in case.losses]
    kw = dict(A=case.A, mask=case.mask) if mode == g.IMPUTE_MISSING else {}
    check_decoded(X, Y, case.col_loss, losses, out.cpu().numpy(), **kw)


@pytest.mark.parametrize("mode", [g.IMPUTE_ALL, g.IMPUTE_MISSING], ids=["all", "missing"])
def test_coo_impute_matches_the_oracle(mode):
    c = dict(m=211, n=300, k=7, seed=7)
    X, Y = _factors(c["m"], c["n"], c["k"], c["seed"])
    case, data = _data(c, X, Y, layout="coo")
    out = g.glrm_impute(data, to_dev(X, DEV), to_dev(Y, DEV), mode=mode)
    torch.cuda.synchronize()
    losses = [(a, b, F32(p)) for a, b, p in case.losses]
    kw = {}
    if mode == g.IMPUTE_MISSING:
        mask = np.zeros((case.m, case.n), bool)
        mask[case.rows, case.cols] = True
        A = np.zeros((case.m, case.n), np.float32)
        A[case.rows, case.cols] = case.vals
        kw = dict(A=A, mask=mask)
    check_decoded(X, Y, case.col_loss, losses, out.cpu().numpy(), **kw)


def test_strided_output_leaves_the_padding_alone_and_a_second_call_overwrites():
    c = dict(m=90, n=70, k=4, seed=8)
    X, Y = _factors(c["m"], c["n"], c["k"], c["seed"])
    case, data = _data(c, X, Y)
    buf = torch.full((c["m"], 96), 12345.0, dtype=torch.float32, device=DEV)
    view = buf[:, :c["n"]]
    losses = [(a, b, F32(p)) for a, b, p in case.losses]
    for mode in (g.IMPUTE_MISSING, g.IMPUTE_ALL):
        g.glrm_impute(data, to_dev(X, DEV), to_dev(Y, DEV), mode=mode, out=view)
        torch.cuda.synchronize()
        host = buf.cpu().numpy()
        assert np.all(host[:, c["n"]:] == 12345.0)
    check_decoded(X, Y, case.col_loss, losses, host[:, :c["n"]])


def test_exact_ties_take_the_smaller_value():
    """k = 1 products that are exact in float32: u = 0 (Boolean tie) and
    u = 2.5 (ordinal tie between levels 2 and 3) decode to -1 and 2, and
    u = -0.0 to -1, on both sides."""
    losses = [(3, 0, 0.0), (2, 0, 0.0), (4, 5, 0.0), (0, 0, 0.0)]
    col_loss = np.array([0, 1, 2, 3], np.uint8)
    X = np.array([[0.0], [0.5], [-0.0], [1.5]], np.float32)
    Y = np.array([[1.0], [1.0], [5.0], [5.0]], np.float32)
    A = torch.zeros((4, 4), dtype=torch.float32, device=DEV)
    data = g.Data(4, 4, 1, A=A, col_loss=col_loss, losses=losses)
    out = g.glrm_impute(data, to_dev(X, DEV), to_dev(Y, DEV)).cpu().numpy()
    _, want = oracle.impute(X, Y, col_loss, losses)
    assert np.array_equal(out, want)
    assert out[0, 0] == -1.0 and out[0, 1] == -1.0 and out[1, 2] == 2.0 and out[3, 2] == 5.0


def test_missing_only_without_a_mask_returns_the_table():
    c = dict(m=50, n=33, k=2, seed=9)
    X, Y = _factors(c["m"], c["n"], c["k"], c["seed"])
    case = synth.small_mixed(c["m"], c["n"], c["k"], c["seed"])
    A = to_dev(case.A, DEV)
    data = g.Data(c["m"], c["n"], c["k"], A=A, col_loss=case.col_loss, losses=case.losses)
    out = g.glrm_impute(data, to_dev(X, DEV), to_dev(Y, DEV), mode=g.IMPUTE_MISSING)
    assert torch.equal(out, A)


@pytest.mark.parametrize("which", ["dense_quadratic", "heterogeneous"])
def test_full_size_sampled_rows(which):
    """The workloads of the benchmark at full size, in the launch the
    benchmark times (prepared workspace, missing-only and every-entry forms):
    300 seeded rows are decoded by the oracle one by one."""
    case = getattr(synth, which)()
    data = g.Data.from_case(case, DEV)
    g.glrm_prepare(data)
    X, Y = to_dev(case.X0, DEV), to_dev(case.Y0, DEV)
    rows = synth.sample_indices(9, 300, case.m)
    losses = [(a, b, F32(p)) for a, b, p in case.losses]
    for mode in (g.IMPUTE_ALL, g.IMPUTE_MISSING):
        out = g.glrm_impute(data, X, Y, mode=mode, flags=g.WS_PREPARED)
        torch.cuda.synchronize()
        got = out[torch.from_numpy(rows).to(DEV)].cpu().numpy()
        kw = {}
        if mode == g.IMPUTE_MISSING:
            kw = dict(A=case.A[rows], mask=case.mask[rows])
        ties = check_decoded(case.X0[rows], case.Y0, case.col_loss, losses, got, **kw)
        assert ties <= 0.001 * got.size
        del out
