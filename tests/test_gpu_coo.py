"""GPU parity of the sparse (row-sorted COO) path against the FP64 oracle."""
import numpy as np
import pytest

import synth
from gpu_helpers import check_sweep, init_alpha32, oracle_problem, rel_fro, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1410_0342_amd as g  # noqa: E402

DEV = torch.device("cuda:0")

CASES = [
    dict(m=37, n=23, k=3, seed=1),
    dict(m=130, n=70, k=5, seed=2, missing=0.7),
    dict(m=64, n=200, k=12, seed=3, missing=0.9),
    dict(m=300, n=45, k=20, seed=4, missing=0.5),
    dict(m=50, n=129, k=40, seed=5, missing=0.6),
    dict(m=33, n=17, k=7, seed=6, empty_row=5, empty_col=3),
    dict(m=1, n=1, k=1, seed=7, missing=0.0),
    dict(m=20000, n=40, k=6, seed=10, missing=0.3),
    dict(m=20, n=10, k=3, seed=11, missing=1.0),        # no entries at all
    # the row-blocked column step: blocks of 2^14 / 2^13 / 2^12 rows at kp = 16 / 32 / 64
    dict(m=60000, n=90, k=20, seed=12, missing=0.97),   # kp = 32: 8 row blocks, one per partial set
    dict(m=70000, n=30, k=40, seed=13, missing=0.95),   # kp = 64: 18 row blocks, 2-3 per partial set
    dict(m=9000, n=1500, k=10, seed=14, missing=0.99),  # several columns per wave
    dict(m=20000, n=1100, k=24, seed=15, missing=0.995),  # both
]


def _case(spec, **kw):
    spec = dict(spec)
    spec.update(kw)
    return synth.small_mixed(spec.pop("m"), spec.pop("n"), spec.pop("k"), layout="coo", **spec)


def _setup(case):
    data = g.Data.from_case(case, DEV)
    return data, to_dev(case.X0, DEV), to_dev(case.Y0, DEV), oracle_problem(case)


@pytest.mark.parametrize("spec", CASES)
@pytest.mark.parametrize("prec,tol", [(g.FP64, 1e-10), (g.FP32, 1e-5)])
def test_objective_matches_oracle(spec, prec, tol):
    case = _case(spec)
    data, X, Y, P = _setup(case)
    ref = P.objective(case.X0, case.Y0)
    assert abs(g.glrm_objective(data, X, Y, prec) - ref) <= tol * abs(ref)


@pytest.mark.parametrize("spec", CASES)
def test_gradient_matches_oracle(spec):
    case = _case(spec)
    data, X, Y, P = _setup(case)
    dXr, dYr = P.grad(case.X0, case.Y0)
    dX, dY, obj = g.glrm_grad(data, X, Y, g.FP32, want_objective=True)
    assert rel_fro(dX.cpu().numpy(), dXr) <= 1e-5
    assert rel_fro(dY.cpu().numpy(), dYr) <= 1e-5
    assert obj == pytest.approx(P.objective(case.X0, case.Y0), rel=1e-5)


@pytest.mark.parametrize("spec", CASES)
@pytest.mark.parametrize("prec", [g.FP32, g.BF16])
def test_one_sweep_matches_oracle(spec, prec):
    """One sweep from an identical state, every row and column checked (rows
    against the oracle's X half-step, columns against the oracle's Y
    half-step from the GPU's own X^t; see gpu_helpers.check_sweep).  BF16:
    the same trial points, decided on trial objectives from bfloat16 step
    products (the band carries their rounding)."""
    case = _case(spec, rx=(1, 0.1), ry=(2, 0.05))
    data, X, Y, P = _setup(case)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    info = g.glrm_fit(data, X, Y, ax, ay, 1, precision=prec, alpha_scale=2.0)
    ax0, ay0 = init_alpha32(P, 2.0)
    Xg, Yg = X.cpu().numpy(), Y.cpu().numpy()
    pname = "fp32" if prec == g.FP32 else "coo_bf16"
    r = check_sweep(P, case.X0, case.Y0, ax0, ay0, Xg, Yg, ax.cpu().numpy(), ay.cpu().numpy(), pname, tag=case.name)
    print("%s %s: decisions inside the rounding band: %d rows, %d columns"
          % (case.name, pname, r["band_rows"], r["band_cols"]))
    assert info["objective"] == pytest.approx(P.objective(Xg, Yg), rel=1e-10)


def test_fit_reaches_the_oracles_converged_objective():
    """Smooth convex losses + quadratic regularizers on a sparse pattern: the
    converged objectives agree, the first sweeps agree, F never increases."""
    case = synth.small_mixed(400, 150, 6, seed=31, missing=0.8, layout="coo", kinds=(0, 1, 2), rx=(1, 0.5),
                             ry=(1, 0.5))
    data, X, Y, P = _setup(case)
    T = 1500
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    hist = torch.zeros(T, dtype=torch.float64, device=DEV)
    info = g.glrm_fit(data, X, Y, ax, ay, T, precision=g.FP32, history=hist)
    *_, href, _ = P.fit(case.X0, case.Y0, T)
    assert abs(href[-1] - href[-50]) <= 1e-9 * abs(href[-1])
    assert abs(info["objective"] - href[-1]) <= 1e-5 * abs(href[-1])
    h = hist.cpu().numpy()
    np.testing.assert_allclose(h[:2], href[:2], rtol=1e-5)
    assert np.all(np.diff(h) <= 1e-5 * np.abs(h[:-1]))
    assert h[-1] == pytest.approx(info["objective"], rel=1e-5)


def test_dense_and_coo_layouts_agree():
    cd = synth.small_mixed(200, 90, 5, seed=61, missing=0.4)
    cc = synth.small_mixed(200, 90, 5, seed=61, missing=0.4, layout="coo")
    out = []
    for case in (cd, cc):
        data = g.Data.from_case(case, DEV)
        X, Y = to_dev(case.X0, DEV), to_dev(case.Y0, DEV)
        ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
        ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
        out.append(g.glrm_fit(data, X, Y, ax, ay, 15, precision=g.FP32)["objective"])
    assert out[0] == pytest.approx(out[1], rel=1e-4)


@pytest.mark.parametrize("bad", ["unsorted", "duplicate", "col_range", "row_range"])
def test_invalid_coo_is_rejected(bad):
    case = _case(CASES[0])
    rows, cols = case.rows.copy(), case.cols.copy()
    if bad == "unsorted":
        rows[[3, 10]] = rows[[10, 3]]
        cols[[3, 10]] = cols[[10, 3]]
    elif bad == "duplicate":
        rows[5], cols[5] = rows[4], cols[4]
    elif bad == "col_range":
        cols[-1] = case.n
    else:
        rows[-1] = case.m + 3
    data = g.Data(case.m, case.n, case.k, layout=g.COO_ROWSORTED, A=to_dev(case.vals, DEV), row=to_dev(rows, DEV),
                  col=to_dev(cols, DEV), col_loss=case.col_loss, losses=case.losses, rx=case.rx, ry=case.ry)
    with pytest.raises(g.GLRMError) as ei:
        g.glrm_prepare(data)
    assert ei.value.code == g.EINVAL


def test_bf16_plain_is_reported_unsupported_for_coo():
    case = _case(CASES[0])
    data, X, Y, P = _setup(case)
    with pytest.raises(g.GLRMError) as ei:
        g.glrm_objective(data, X, Y, g.BF16_PLAIN)
    assert ei.value.code == g.EUNSUPPORTED
    # BF16 objective and gradient calls compute as FP32
    assert g.glrm_objective(data, X, Y, g.BF16) == g.glrm_objective(data, X, Y, g.FP32)


@pytest.mark.parametrize("spec", [CASES[7], CASES[9], CASES[12]])
def test_bf16_three_sweeps_checked_sweep_by_sweep(spec):
    """Three BF16 sweeps, each checked against the oracle from the GPU's
    state before it."""
    case = _case(spec, rx=(1, 0.1), ry=(1, 0.1))
    data, X, Y, P = _setup(case)
    g.glrm_prepare(data)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    Xp, Yp = case.X0.copy(), case.Y0.copy()
    axp, ayp = init_alpha32(P, 1.0)
    for t in range(3):
        g.glrm_fit(data, X, Y, ax, ay, 1, precision=g.BF16, init_alpha=(t == 0), flags=g.WS_PREPARED)
        Xg, Yg, axg, ayg = X.cpu().numpy(), Y.cpu().numpy(), ax.cpu().numpy(), ay.cpu().numpy()
        check_sweep(P, Xp, Yp, axp, ayp, Xg, Yg, axg, ayg, "coo_bf16", tag="%s sweep %d" % (case.name, t + 1))
        Xp, Yp, axp, ayp = Xg, Yg, axg.astype(np.float64), ayg.astype(np.float64)


def test_fit_is_bitwise_repeatable():
    """Two fits from the same state give the same bits: every partial sum of
    both walks (and of the row-blocked column passes) is combined in a fixed
    order."""
    case = _case(dict(m=60000, n=90, k=20, seed=12, missing=0.97))
    data = g.Data.from_case(case, DEV)
    g.glrm_prepare(data)
    out = []
    for _ in range(2):
        X, Y = to_dev(case.X0, DEV), to_dev(case.Y0, DEV)
        ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
        ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
        info = g.glrm_fit(data, X, Y, ax, ay, 4, precision=g.FP32, flags=g.WS_PREPARED)
        out.append((X.cpu().numpy(), Y.cpu().numpy(), info["objective_fp32"]))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]
