"""GPU parity of the dense path against the FP64 oracle, through the C ABI.

Tolerances: objective rel. err <= 1e-5 in FP32 and <= 1e-3 in BF16 (split);
gradients <= 1e-4 rel. (Frobenius) in FP32.  FP64 objectives agree to 1e-10
(only summation order differs).
"""
import json
import os

import numpy as np
import pytest

import synth
from gpu_helpers import check_sweep, guided_half, init_alpha32, oracle_problem, rel_fro, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1410_0342_amd as g  # noqa: E402

DEV = torch.device("cuda:0")
GOLD = os.path.join(os.path.dirname(__file__), "golden")

CASES = [
    dict(m=37, n=23, k=3, seed=1),                      # ragged rows and columns, one tile
    dict(m=130, n=70, k=5, seed=2, missing=0.4),        # several panels and tiles
    dict(m=64, n=200, k=12, seed=3),                    # kp = 16, 13 tiles
    dict(m=300, n=45, k=20, seed=4),                    # kp = 32
    dict(m=50, n=129, k=40, seed=5),                    # kp = 64
    dict(m=33, n=17, k=7, seed=6, empty_row=5, empty_col=3),
    dict(m=1, n=1, k=1, seed=7, missing=0.0),           # one entry, one ragged panel and tile
    dict(m=40, n=1024, k=20, seed=8),                   # widest fit at kp = 32: every tile slot used
    dict(m=24, n=512, k=64, seed=9),                    # widest fit at kp = 64
    dict(m=20000, n=40, k=6, seed=10, missing=0.3),     # narrow and tall: several workgroups per CU
    dict(m=20, n=10, k=3, seed=11, missing=1.0),        # nothing observed: regularizers only
    # wider than the fused row pass: the row half-step in column blocks
    dict(m=40, n=1025, k=20, seed=12),                  # kp = 32: a second block of one ragged tile
    dict(m=24, n=513, k=64, seed=13),                   # kp = 64: three blocks of 16 tiles, the last of one
    dict(m=70, n=2100, k=10, seed=14, missing=0.4),     # kp = 16: three blocks, 132 tiles, ragged rows
]


def _case(spec, **kw):
    spec = dict(spec)
    spec.update(kw)
    return synth.small_mixed(spec.pop("m"), spec.pop("n"), spec.pop("k"), **spec)


def _setup(case):
    data = g.Data.from_case(case, DEV)
    X = to_dev(case.X0, DEV)
    Y = to_dev(case.Y0, DEV)
    return data, X, Y, oracle_problem(case)


@pytest.mark.parametrize("spec", CASES)
def test_objective_fp64_matches_oracle(spec):
    case = _case(spec)
    data, X, Y, P = _setup(case)
    ref = P.objective(case.X0, case.Y0)
    got = g.glrm_objective(data, X, Y, g.FP64)
    assert got == pytest.approx(ref, rel=1e-10)


@pytest.mark.parametrize("spec", CASES)
@pytest.mark.parametrize("prec,tol", [(g.FP32, 1e-5), (g.BF16, 1e-4), (g.BF16_PLAIN, 3e-2)])
def test_objective_matches_oracle(spec, prec, tol):
    case = _case(spec)
    data, X, Y, P = _setup(case)
    ref = P.objective(case.X0, case.Y0)
    got = g.glrm_objective(data, X, Y, prec)
    assert abs(got - ref) <= tol * abs(ref)


def _coord_err(got, ref):
    """Largest per-coordinate error, scaled by max(|ref|, RMS of ref)."""
    ref = np.asarray(ref, np.float64)
    rms = np.sqrt(np.mean(ref ** 2)) if ref.size else 0.0
    return float(np.max(np.abs(np.asarray(got, np.float64) - ref) / np.maximum(np.abs(ref), max(rms, 1e-300))))


@pytest.mark.parametrize("spec", CASES)
@pytest.mark.parametrize("prec,tol,ctol", [(g.FP32, 1e-4, 1e-4), (g.BF16, 2e-2, 5e-2)])
def test_gradient_matches_oracle(spec, prec, tol, ctol):
    """Frobenius error and per-coordinate error (scale max(|ref|, RMS)) of both
    gradients.  BF16: each term of a gradient coordinate is one bfloat16
    product, 2^-8 relative, so a coordinate whose terms cancel carries up to
    2^-8 of the sum of their magnitudes; 5e-2 of the RMS covers it."""
    case = _case(spec)
    data, X, Y, P = _setup(case)
    dXr, dYr = P.grad(case.X0, case.Y0)
    dX, dY, obj = g.glrm_grad(data, X, Y, prec, want_objective=True)
    dX, dY = dX.cpu().numpy(), dY.cpu().numpy()
    assert rel_fro(dX, dXr) <= tol
    assert rel_fro(dY, dYr) <= tol
    assert _coord_err(dX, dXr) <= ctol
    assert _coord_err(dY, dYr) <= ctol
    assert obj == pytest.approx(P.objective(case.X0, case.Y0), rel=1e-5 if prec == g.FP32 else 1e-3)


def test_gradient_wide_table_uses_column_blocks():
    """n = 700 > 512 columns per gradient block: partial dX over blocks."""
    case = synth.small_mixed(90, 700, 8, seed=21, kinds=(0, 2))
    data, X, Y, P = _setup(case)
    dXr, dYr = P.grad(case.X0, case.Y0)
    dX, dY = g.glrm_grad(data, X, Y, g.FP32)
    assert rel_fro(dX.cpu().numpy(), dXr) <= 1e-4
    assert rel_fro(dY.cpu().numpy(), dYr) <= 1e-4


@pytest.mark.parametrize("kind,w", [(0, 0.0), (1, 0.3), (2, 0.4), (3, 0.0)])
def test_prox_matches_oracle(kind, w):
    import oracle
    rng = np.random.default_rng(kind)
    V = rng.normal(size=(1000, 7)).astype(np.float32) * 2
    al = rng.uniform(0.01, 3.0, size=1000).astype(np.float32)
    Vd = to_dev(V, DEV)
    g.glrm_prox((kind, w), Vd, to_dev(al, DEV))
    ref = np.stack([oracle.prox(kind, w, float(al[i]), V[i].astype(np.float64)) for i in range(V.shape[0])])
    np.testing.assert_allclose(Vd.cpu().numpy(), ref, rtol=2e-6, atol=1e-7)


def test_hand_worked_sweeps_on_the_gpu():
    """The sweeps worked by hand from Algorithm 2 (tests/golden/sweeps.json)."""
    d = json.load(open(os.path.join(GOLD, "sweeps.json")))
    for case in d["cases"]:
        A = np.array(case["A"], dtype=np.float32)
        m, n = A.shape
        k = case["k"]
        mask = None if case["mask"] is None else to_dev(np.array(case["mask"], dtype=np.uint8), DEV)
        data = g.Data(m, n, k, A=to_dev(A, DEV), mask=mask, col_loss=np.array(case["col_loss"]),
                      losses=[tuple(x) for x in case["losses"]], rx=tuple(case["rx"]), ry=tuple(case["ry"]))
        X = to_dev(np.array(case["X0"], dtype=np.float32), DEV)
        Y = to_dev(np.array(case["Y0"], dtype=np.float32), DEV)
        ax = torch.empty(m, dtype=torch.float32, device=DEV)
        ay = torch.empty(n, dtype=torch.float32, device=DEV)
        for t, exp in enumerate(case["sweeps"]):
            info = g.glrm_fit(data, X, Y, ax, ay, 1, precision=g.FP32, init_alpha=(t == 0))
            tag = "%s sweep %d" % (case["name"], t + 1)
            np.testing.assert_allclose(X.cpu().numpy(), exp["X"], rtol=1e-6, atol=1e-6, err_msg=tag)
            np.testing.assert_allclose(Y.cpu().numpy(), exp["Y"], rtol=1e-6, atol=1e-6, err_msg=tag)
            np.testing.assert_allclose(ax.cpu().numpy(), exp["ax"], rtol=1e-6, err_msg=tag)
            np.testing.assert_allclose(ay.cpu().numpy(), exp["ay"], rtol=1e-6, err_msg=tag)
            assert info["objective"] == pytest.approx(exp["F"], rel=1e-6), tag
            assert info["rows_rejected"] == exp["rows_rejected"], tag
            assert info["cols_rejected"] == exp["cols_rejected"], tag


PNAME = {g.FP32: "fp32", g.BF16: "bf16"}


@pytest.mark.parametrize("spec", CASES)
@pytest.mark.parametrize("prec", [g.FP32, g.BF16])
def test_one_sweep_matches_oracle(spec, prec):
    """One sweep from an identical state, every row and column checked: the
    rows against the oracle's X half-step, the columns against the oracle's Y
    half-step taken from the GPU's own X^t.  A decision whose margin lies
    outside its rounding band matches the oracle's; one inside it is either
    an accepted step equal to the oracle's trial point within the gradient's
    rounding bound, or a rejected step that left the row untouched (the band
    and bounds are derived in gpu_helpers)."""
    case = _case(spec, rx=(1, 0.1), ry=(2, 0.05))
    data, X, Y, P = _setup(case)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    info = g.glrm_fit(data, X, Y, ax, ay, 1, precision=prec, init_alpha=True, alpha_scale=2.0)
    ax0, ay0 = init_alpha32(P, 2.0)
    Xg, Yg = X.cpu().numpy(), Y.cpu().numpy()
    check_sweep(P, case.X0, case.Y0, ax0, ay0, Xg, Yg, ax.cpu().numpy(), ay.cpu().numpy(), PNAME[prec],
                tag=case.name)
    # the reported objective is F at the state the GPU reached (FP64 recompute)
    assert info["objective"] == pytest.approx(P.objective(Xg, Yg), rel=1e-10)


NONSMOOTH = [
    # hinge and ordinal columns, l1 on X, nonnegative Y
    dict(m=90, n=40, k=5, seed=71, kinds=(3, 4), rx=(2, 0.05), ry=(3, 0.0)),
    # every loss kind, nonnegative X from a nonnegative start, l1 on Y
    dict(m=120, n=33, k=4, seed=72, x_nonneg=True, rx=(3, 0.0), ry=(2, 0.1)),
    # ordinal only, l1 on both, a wider table (several tiles, kp = 16)
    dict(m=70, n=150, k=9, seed=73, kinds=(4,), rx=(2, 0.02), ry=(2, 0.02)),
]


@pytest.mark.parametrize("spec", NONSMOOTH)
@pytest.mark.parametrize("prec", [g.FP32, g.BF16])
def test_three_sweeps_nonsmooth_match_oracle(spec, prec):
    """Three sweeps on hinge / ordinal losses with l1 and nonnegative
    regularizers.  Each GPU sweep is checked against the oracle's sweep from
    the GPU's previous state (every row and column, as in the one-sweep
    test).  After three sweeps the GPU's objective equals, within the
    precision's tolerance, that of the oracle's three sweeps from the common
    start in which each decision inside its rounding band took the GPU's
    branch (either branch is correct there).  Where FP32 took every such
    decision the oracle's way, the oracle's own trajectory is compared too.

    BF16 on these kinked losses: each sweep is asserted as above, and the
    objectives are reported, not bounded.  Every accepted BF16 step is the
    oracle's within 2^-7 of its gradient's term magnitudes, but where a row's
    products sit near a hinge or an ordinal level that rounding moves them
    across the kink, which changes the next sweep's subgradient by a whole
    step; over three sweeps the trajectories part by up to ~0.2% of F even
    with every band decision taken the GPU's way (measured on the third
    table).  Smooth losses do not amplify it: their BF16 multi-sweep
    objectives are bounded (full-size dense quadratic, converged fits)."""
    sp = dict(spec)
    case = synth.small_mixed(sp.pop("m"), sp.pop("n"), sp.pop("k"), **sp)
    data, X, Y, P = _setup(case)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    Xp, Yp = case.X0.copy(), case.Y0.copy()
    axp, ayp = init_alpha32(P, 1.0)
    Xo, Yo, axo, ayo = case.X0.astype(np.float64), case.Y0.astype(np.float64), axp.copy(), ayp.copy()
    band = flipped = 0
    pn = PNAME[prec]
    for t in range(3):
        info = g.glrm_fit(data, X, Y, ax, ay, 1, precision=prec, init_alpha=(t == 0))
        Xg, Yg, axg, ayg = X.cpu().numpy(), Y.cpu().numpy(), ax.cpu().numpy(), ay.cpu().numpy()
        r = check_sweep(P, Xp, Yp, axp, ayp, Xg, Yg, axg, ayg, pn, tag="%s sweep %d" % (case.name, t + 1))
        band += r["band_rows"] + r["band_cols"]
        flipped += r["flipped"]
        Xo, axo = guided_half(P, "x", Xo, Yo, axo, r["acc_rows"], pn)
        Yo, ayo = guided_half(P, "y", Yo, Xo, ayo, r["acc_cols"], pn)
        Xp, Yp, axp, ayp = Xg, Yg, axg.astype(np.float64), ayg.astype(np.float64)
    *_, href, _ = P.fit(case.X0, case.Y0, 3)
    F_guided = P.objective(Xo, Yo)
    print("%s %s: %d decisions in the band, %d took the other branch; F gpu %.10g, guided oracle %.10g, "
          "oracle %.10g" % (case.name, pn, band, flipped, info["objective"], F_guided, href[-1]))
    if prec == g.FP32:
        assert info["objective"] == pytest.approx(F_guided, rel=1e-5)
        if flipped == 0:
            assert info["objective"] == pytest.approx(href[-1], rel=1e-5)
    F0 = P.objective(case.X0, case.Y0)
    assert info["objective"] < F0


@pytest.mark.parametrize("n", [60, 1100])
@pytest.mark.parametrize("prec,tol", [(g.FP32, 1e-5), (g.BF16, 1e-4)])
def test_fit_reaches_the_oracles_converged_objective(prec, tol, n):
    """Smooth convex losses with quadratic regularizers: after enough sweeps
    both the GPU and the oracle have converged (the oracle's last sweeps change
    F by < 1e-9 relative), and the objectives agree.  The first sweeps, before
    any near-tie decision can separate the trajectories, agree closely too.
    n = 1100 takes the row half-step in column blocks."""
    case = synth.small_mixed(200, n, 4, seed=31, missing=0.3, kinds=(0, 1, 2), rx=(1, 0.5), ry=(1, 0.5))
    data, X, Y, P = _setup(case)
    T = 1500
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    hist = torch.zeros(T, dtype=torch.float64, device=DEV)
    info = g.glrm_fit(data, X, Y, ax, ay, T, precision=prec, history=hist)
    *_, href, _ = P.fit(case.X0, case.Y0, T)
    assert abs(href[-1] - href[-50]) <= 1e-9 * abs(href[-1])
    assert abs(info["objective"] - href[-1]) <= tol * abs(href[-1])
    h = hist.cpu().numpy()
    np.testing.assert_allclose(h[:2], href[:2], rtol=1e-5 if prec == g.FP32 else 1e-3)
    assert np.all(np.diff(h) <= 1e-5 * np.abs(h[:-1]))
    assert info["objective"] == pytest.approx(P.objective(X.cpu().numpy(), Y.cpu().numpy()), rel=1e-12)


def test_eckart_young_on_the_gpu():
    """Plain PCA, 200 x 50, k = 5, 500 sweeps: the objective reaches the sum of
    the trailing squared singular values (Section 2.3)."""
    case = synth.plain_pca()
    data, X, Y, P = _setup(case)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    info = g.glrm_fit(data, X, Y, ax, ay, case.sweeps, precision=g.FP32)
    s = np.linalg.svd(case.A.astype(np.float64), compute_uv=False)
    target = float(np.sum(s[case.k:] ** 2))
    assert info["objective"] == pytest.approx(target, rel=1e-5)


def test_step_sizes_move_by_exact_factors_and_rejected_rows_stay():
    case = synth.small_mixed(120, 40, 4, seed=41)
    data, X, Y, P = _setup(case)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    g.glrm_fit(data, X, Y, ax, ay, 1, precision=g.FP32, alpha_scale=3.0)
    for _ in range(4):
        X0, ax0, ay0, Y0 = X.cpu().numpy(), ax.cpu().numpy(), ay.cpu().numpy(), Y.cpu().numpy()
        g.glrm_fit(data, X, Y, ax, ay, 1, precision=g.FP32, init_alpha=False)
        X1, ax1, ay1, Y1 = X.cpu().numpy(), ax.cpu().numpy(), ay.cpu().numpy(), Y.cpu().numpy()
        up = ax1 == (ax0 * np.float32(1.05)).astype(np.float32)
        dn = ax1 == (ax0 * np.float32(0.7)).astype(np.float32)
        assert np.all(up | dn)
        assert np.array_equal(X1[dn], X0[dn])
        upc = ay1 == (ay0 * np.float32(1.05)).astype(np.float32)
        dnc = ay1 == (ay0 * np.float32(0.7)).astype(np.float32)
        assert np.all(upc | dnc)
        assert np.array_equal(Y1[dnc], Y0[dnc])


@pytest.mark.parametrize("n", [90, 1300])
def test_fit_is_deterministic(n):
    case = synth.small_mixed(150, n, 6, seed=51)
    outs = []
    for _ in range(2):
        data, X, Y, P = _setup(case)
        ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
        ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
        g.glrm_fit(data, X, Y, ax, ay, 7, precision=g.BF16)
        outs.append((X.cpu().numpy(), Y.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_fit_beyond_the_rank_limit_is_reported():
    """k > 64 is reported as unsupported before any launch, with nothing
    written."""
    case = synth.small_mixed(10, 10, 65, seed=12)
    data, X, Y, _ = _setup(case)
    ax = torch.zeros(case.m, dtype=torch.float32, device=DEV)
    ay = torch.zeros(case.n, dtype=torch.float32, device=DEV)
    X0 = X.clone()
    with pytest.raises(g.GLRMError) as err:
        g.glrm_fit(data, X, Y, ax, ay, 1, precision=g.FP32)
    assert err.value.code == g.EUNSUPPORTED
    assert torch.equal(X, X0)



@pytest.mark.parametrize("layout", ["dense", "coo", "dense_wide"])
@pytest.mark.parametrize("prec", [g.FP32, g.BF16])
def test_overflowing_step_sizes_leave_the_factors_finite(layout, prec):
    """Step sizes that overflow float32 (alpha_scale 3e38, zero regularizers,
    an unobserved row and column whose gradient is exactly 0): a trial point
    with an infinite or NaN coordinate, or whose products overflow, is never
    accepted, so X and Y stay finite and every observed row and column keeps
    its start, as in the oracle; the objective equals the oracle's."""
    n = 1030 if layout == "dense_wide" else 30      # 1030: the row half-step in column blocks
    case = synth.small_mixed(60, n, 4, seed=81, missing=0.3, layout=layout.split("_")[0], rx=(0, 0.0), ry=(0, 0.0),
                             empty_row=3, empty_col=7)
    data = g.Data.from_case(case, DEV)
    X, Y = to_dev(case.X0, DEV), to_dev(case.Y0, DEV)
    P = oracle_problem(case)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    info = g.glrm_fit(data, X, Y, ax, ay, 4, precision=prec, alpha_scale=3.0e38)
    Xg, Yg = X.cpu().numpy(), Y.cpu().numpy()
    assert np.all(np.isfinite(Xg)) and np.all(np.isfinite(Yg))
    *_, href, _ = P.fit(case.X0, case.Y0, 4, alpha_scale=3.0e38)
    assert np.isfinite(info["objective"])
    assert info["objective"] == pytest.approx(href[-1], rel=1e-9)
    np.testing.assert_array_equal(Xg, case.X0)
    np.testing.assert_array_equal(Yg, case.Y0)
