"""The global-optimality certificate of Section 7.6 (glrm_certificate) against
the oracle's: the oracle forms G / gamma + U V^T densely and takes its
spectral norm from numpy's SVD; the GPU estimates it by power iteration, a
lower bound that converges at the rate (s2 / s1)^2 per iteration (at most
0.967 on these cases, so 600 iterations settle to double rounding)."""
import numpy as np
import pytest

import synth
from gpu_helpers import oracle_problem, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1410_0342_amd as g  # noqa: E402

DEV = torch.device("cuda:0")

SPECS = [
    dict(m=120, n=50, k=4, seed=201, kinds=(0, 1, 2), rx=(1, 0.5), ry=(1, 0.5), missing=0.3),
    dict(m=200, n=60, k=6, seed=202, kinds=(0,), rx=(1, 2.0), ry=(1, 2.0), missing=0.2),
    dict(m=64, n=130, k=12, seed=203, kinds=(0, 1, 2, 3, 4), rx=(1, 0.3), ry=(1, 0.3), missing=0.5),
    # a table smaller than one tile in both directions
    dict(m=9, n=7, k=2, seed=206, kinds=(0,), rx=(1, 0.5), ry=(1, 0.5), missing=0.2),
    # a rank whose Gram products take three 16-wide tiles (ragged at 36)
    dict(m=300, n=80, k=36, seed=205, kinds=(0, 1), rx=(1, 0.5), ry=(1, 0.5), missing=0.3),
]


@pytest.mark.parametrize("layout", ["dense", "coo"])
@pytest.mark.parametrize("spec", SPECS)
def test_certificate_matches_oracle(layout, spec):
    """At the seeded start and at the oracle's 3000-sweep fit: the same rank
    of X Y^T, the norm within 2e-5 (G is formed in float32 from float32 z),
    and the iteration settled."""
    sp = dict(spec)
    case = synth.small_mixed(sp.pop("m"), sp.pop("n"), sp.pop("k"), layout=layout, **sp)
    P = oracle_problem(case)
    data = g.Data.from_case(case, DEV)
    Xf, Yf, *_ = P.fit(case.X0, case.Y0, 3000)
    for name, X, Y in (("start", case.X0, case.Y0), ("fit", Xf, Yf)):
        X32, Y32 = np.asarray(X, np.float32), np.asarray(Y, np.float32)
        ref, r = P.certificate(X32, Y32)
        info = g.glrm_certificate(data, to_dev(X32, DEV), to_dev(Y32, DEV), iters=600)
        assert info["rank"] == r, name
        assert info["norm"] == pytest.approx(ref, rel=2e-5), name
        assert abs(info["norm"] - info["norm_prev"]) <= 1e-7 * ref, name
        assert (info["norm"] <= 1.0) == (ref <= 1.0) or abs(ref - 1.0) < 1e-4, name


def test_certificate_needs_one_quadratic_regularizer_on_both_factors():
    case = synth.small_mixed(30, 20, 3, seed=204, rx=(1, 0.5), ry=(1, 0.25))
    data = g.Data.from_case(case, DEV)
    with pytest.raises(g.GLRMError) as e:
        g.glrm_certificate(data, to_dev(case.X0, DEV), to_dev(case.Y0, DEV))
    assert e.value.code == g.EINVAL


def test_dense_quadratic_certificate_full_size():
    """The 100,000 x 1,000 rank-20 table with 20% missing, with the quadratic
    regularizer at gamma = 50 on both factors, so that the convex problem's
    solution has rank <= 20 (the noise part of G is about 0.2 (sqrt(m) +
    sqrt(n)) ~ 70 in spectral norm, below gamma' = 100).  From the seeded
    start the certificate fails by far; after 1500 FP32 sweeps the fit
    certifies itself globally optimal."""
    case = synth.dense_quadratic(gamma=50.0)
    data = g.Data.from_case(case, DEV)
    g.glrm_prepare(data)
    X, Y = to_dev(case.X0, DEV), to_dev(case.Y0, DEV)
    start = g.glrm_certificate(data, X, Y, iters=100)
    ax = torch.empty(case.m, dtype=torch.float32, device=DEV)
    ay = torch.empty(case.n, dtype=torch.float32, device=DEV)
    info = g.glrm_fit(data, X, Y, ax, ay, 1500, precision=g.FP32, flags=g.WS_PREPARED)
    cert = g.glrm_certificate(data, X, Y, iters=300)
    print("start %.6g; after 1500 sweeps (F = %.10g) %.8g (previous iterate %.8g), rank %d"
          % (start["norm"], info["objective"], cert["norm"], cert["norm_prev"], cert["rank"]))
    assert start["norm"] > 10.0
    assert cert["rank"] == case.k
    assert cert["norm"] <= 1.0 + 1e-3


@pytest.mark.parametrize("layout", ["dense", "coo"])
def test_certificate_with_factors_off_16_byte_alignment(layout):
    """The COO derivative values load the factors four floats at a time only
    when both start on 16 bytes; factors one float past an aligned start take
    the float path and give the same norm (the same sums in the same order,
    up to how the compiler fuses them)."""
    case = synth.small_mixed(120, 50, 4, seed=207, kinds=(0, 1, 2), rx=(1, 0.5), ry=(1, 0.5), missing=0.3,
                             layout=layout)
    data = g.Data.from_case(case, DEV)
    X32, Y32 = np.asarray(case.X0, np.float32), np.asarray(case.Y0, np.float32)
    ref = g.glrm_certificate(data, to_dev(X32, DEV), to_dev(Y32, DEV), iters=200)
    Xb = torch.zeros(X32.size + 1, dtype=torch.float32, device=DEV)
    Yb = torch.zeros(Y32.size + 1, dtype=torch.float32, device=DEV)
    Xb[1:] = to_dev(X32, DEV).reshape(-1)
    Yb[1:] = to_dev(Y32, DEV).reshape(-1)
    Xo, Yo = Xb[1:].view(X32.shape), Yb[1:].view(Y32.shape)
    assert Xo.data_ptr() % 16 != 0 and Yo.data_ptr() % 16 != 0
    off = g.glrm_certificate(data, Xo, Yo, iters=200)
    assert off["rank"] == ref["rank"]
    assert off["norm"] == pytest.approx(ref["norm"], rel=1e-12)
