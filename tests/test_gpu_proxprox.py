"""The prox-prox update for quadratic losses (Sections 7.2 and 7.3) on the GPU
against the oracle's half-steps.

Each GPU sweep is checked row by row and column by column against the
oracle's prox-prox half-steps from the same state (the columns from the GPU's
own X^t).  The GPU forms the Gram data in float32 (relative error ~1e-6 of
the sum of the term magnitudes) and solves in double, so a trial point agrees
with the oracle's to ~1e-5 relative here (G + I / (2 alpha) is well
conditioned at alpha = scale / n_i); a decision whose margin |f+ - f| is
below 1e-4 |f| may go either way (counted), any other must match."""
import numpy as np
import pytest

import synth
from gpu_helpers import init_alpha32, oracle_problem, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1410_0342_amd as g  # noqa: E402

DEV = torch.device("cuda:0")

CASES = [
    dict(m=37, n=23, k=3, seed=401),
    dict(m=130, n=70, k=5, seed=402, missing=0.4),
    dict(m=64, n=200, k=12, seed=403),
    dict(m=300, n=45, k=20, seed=404),
    dict(m=50, n=129, k=40, seed=405),
    dict(m=33, n=17, k=7, seed=406, empty_row=5, empty_col=3),
    dict(m=3000, n=1300, k=9, seed=407, missing=0.5),
    # the solve's packed factor at its edges: one coordinate, a rank that
    # fills kp = 16 and kp = 32 exactly, and the largest rank
    dict(m=41, n=29, k=1, seed=408),
    dict(m=90, n=60, k=16, seed=409),
    dict(m=120, n=80, k=32, seed=410, missing=0.3),
    dict(m=150, n=110, k=64, seed=411, missing=0.2),
]
REGS = [((0, 0.0), (0, 0.0)), ((1, 0.2), (1, 0.2)), ((2, 0.05), (3, 0.0))]


def _check_half(P, which, U0, V, a0, Ug, ag, inner, tag):
    U0, V, a0 = np.asarray(U0, np.float64), np.asarray(V, np.float64), np.asarray(a0, np.float64)
    Uo, ao = U0.copy(), a0.copy()
    trial = np.empty_like(U0)
    if which == "x":
        _, fo, fn, acc = P.half_step_x_pp(Uo, V, ao, inner, trial=trial)
    else:
        _, fo, fn, acc = P.half_step_y_pp(V, Uo, ao, inner, trial=trial)
    ratio = np.asarray(ag, np.float64) / a0
    acc_g = np.abs(ratio - 1.05) <= 1e-6
    rej_g = np.abs(ratio - 0.7) <= 1e-6
    assert np.all(acc_g | rej_g), tag
    clear = np.abs(fn - fo) > 1e-4 * np.abs(fo) + 1e-12
    bad = np.nonzero(clear & (acc_g != acc.astype(bool)))[0]
    assert bad.size == 0, "%s: decisions differ at %s" % (tag, bad[:8])
    Ug = np.asarray(Ug, np.float32)
    assert np.array_equal(Ug[rej_g], U0.astype(np.float32)[rej_g]), tag
    if acc_g.any():
        d = np.abs(Ug[acc_g] - trial[acc_g])
        tol = 1e-4 * np.abs(trial[acc_g]) + 1e-5 * max(np.abs(trial).max(), 1e-30)
        assert np.all(d <= tol), "%s: trial points off by %.3g" % (tag, np.max(d / tol))
    return int((~clear).sum())


@pytest.mark.parametrize("spec", CASES)
@pytest.mark.parametrize("regs", REGS)
@pytest.mark.parametrize("inner", [1, 5])
def test_proxprox_sweeps_match_oracle(spec, regs, inner):
    sp = dict(spec)
    case = synth.small_mixed(sp.pop("m"), sp.pop("n"), sp.pop("k"), kinds=(0,), rx=regs[0], ry=regs[1],
                             x_nonneg=regs[1][0] == 3 or regs[0][0] == 3, **sp)
    if regs[1][0] == 3:
        case.Y0 = np.abs(case.Y0)
    P = oracle_problem(case)
    data = g.Data.from_case(case, DEV)
    X, Y = to_dev(case.X0, DEV), to_dev(case.Y0, DEV)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    Xp, Yp = case.X0.astype(np.float64), case.Y0.astype(np.float64)
    axp, ayp = init_alpha32(P, 1.0)
    for t in range(3):
        info = g.glrm_fit(data, X, Y, ax, ay, 1, precision=g.FP32, init_alpha=(t == 0), update=g.UPDATE_PROXPROX,
                          inner=inner)
        Xg, Yg, axg, ayg = X.cpu().numpy(), Y.cpu().numpy(), ax.cpu().numpy(), ay.cpu().numpy()
        tag = "%s sweep %d" % (case.name, t + 1)
        _check_half(P, "x", Xp, Yp, axp, Xg, axg, inner, tag + " rows")
        _check_half(P, "y", Yp, Xg, ayp, Yg, ayg, inner, tag + " columns")
        Xp, Yp, axp, ayp = Xg.astype(np.float64), Yg.astype(np.float64), axg.astype(np.float64), ayg.astype(np.float64)
        assert info["objective"] == pytest.approx(P.objective(Xg, Yg), rel=1e-10)


def test_proxprox_fit_reaches_the_oracles_objective():
    """Thirty sweeps of the prox-prox fit (three inner updates, quadratic
    regularizer) from a common start: the GPU's objective history equals the
    oracle's, and neither increases."""
    case = synth.small_mixed(400, 150, 6, seed=411, missing=0.3, kinds=(0,), rx=(1, 0.3), ry=(1, 0.3))
    P = oracle_problem(case)
    data = g.Data.from_case(case, DEV)
    X, Y = to_dev(case.X0, DEV), to_dev(case.Y0, DEV)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    hist = torch.zeros(30, dtype=torch.float64, device=DEV)
    info = g.glrm_fit(data, X, Y, ax, ay, 30, precision=g.FP32, update=g.UPDATE_PROXPROX, inner=3, history=hist)
    *_, href = P.fit_pp(case.X0, case.Y0, 30, inner=3)
    h = hist.cpu().numpy()
    np.testing.assert_allclose(h, href, rtol=1e-5)
    assert info["objective"] == pytest.approx(href[-1], rel=1e-5)
    assert np.all(np.diff(href) <= 0)


@pytest.mark.parametrize("what", ["coo", "bf16", "logistic"])
def test_proxprox_limits_are_reported(what):
    kinds = (0, 2) if what == "logistic" else (0,)
    case = synth.small_mixed(30, 20, 3, seed=412, kinds=kinds, layout="coo" if what == "coo" else "dense")
    data = g.Data.from_case(case, DEV)
    X, Y = to_dev(case.X0, DEV), to_dev(case.Y0, DEV)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    with pytest.raises(g.GLRMError) as e:
        g.glrm_fit(data, X, Y, ax, ay, 1, precision=g.BF16 if what == "bf16" else g.FP32, update=g.UPDATE_PROXPROX)
    assert e.value.code == g.EUNSUPPORTED
