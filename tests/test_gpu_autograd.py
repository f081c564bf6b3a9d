"""The loss as a torch.autograd.Function whose backward is the hand-written
gradient kernel, checked against the oracle's gradient and against FP64
central finite differences of the oracle's row / column objective."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import oracle_problem, rel_fro, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1410_0342_amd as g  # noqa: E402
from paper_1410_0342_amd.torch_ops import glrm_loss, glrm_objective  # noqa: E402

DEV = torch.device("cuda:0")


def _fd_row(case, X, Y, i, c, h=1e-6, by_col=False):
    """Central difference of the loss restricted to row i (or column i) with
    respect to coordinate c of x_i (or y_i), from the FP64 oracle on the
    one-row sub-problem."""
    if not by_col:
        obs = np.nonzero(case.mask[i])[0]
        P = oracle.Problem.from_coo(1, case.n, case.k, np.zeros(obs.size, np.int64), obs, case.A[i, obs],
                                    case.col_loss, case.losses, (0, 0.0), (0, 0.0))
        u, V = X[i:i + 1].astype(np.float64).copy(), Y.astype(np.float64)
        up, um = u.copy(), u.copy()
        up[0, c] += h
        um[0, c] -= h
        return (P.loss_sum(up, V) - P.loss_sum(um, V)) / (2 * h)
    obs = np.nonzero(case.mask[:, i])[0]
    P = oracle.Problem.from_coo(case.m, 1, case.k, obs, np.zeros(obs.size, np.int64), case.A[obs, i],
                                case.col_loss[i:i + 1], case.losses, (0, 0.0), (0, 0.0))
    v, U = Y[i:i + 1].astype(np.float64).copy(), X.astype(np.float64)
    vp, vm = v.copy(), v.copy()
    vp[0, c] += h
    vm[0, c] -= h
    return (P.loss_sum(U, vp) - P.loss_sum(U, vm)) / (2 * h)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 2e-2)])
def test_autograd_matches_oracle_gradient(prec, tol):
    case = synth.autograd_point(m=3000, n=300, k=64, config=104)
    data = g.Data.from_case(case, DEV)
    X = to_dev(case.X0, DEV).requires_grad_(True)
    Y = to_dev(case.Y0, DEV).requires_grad_(True)
    f = glrm_loss(X, Y, data, prec)
    f.backward()
    P = oracle_problem(case)
    dXr, dYr = P.grad(case.X0, case.Y0)
    assert rel_fro(X.grad.cpu().numpy(), dXr) <= tol
    assert rel_fro(Y.grad.cpu().numpy(), dYr) <= tol
    assert float(f) == pytest.approx(P.loss_sum(case.X0, case.Y0), rel=1e-5 if prec == "fp32" else 1e-3)


def test_autograd_matches_finite_differences_and_chains():
    case = synth.autograd_point(m=2000, n=200, k=64, config=105)
    data = g.Data.from_case(case, DEV)
    X = to_dev(case.X0, DEV).requires_grad_(True)
    Y = to_dev(case.Y0, DEV).requires_grad_(True)
    loss = 3.0 * glrm_loss(X, Y, data, "fp32")      # chain rule through a scale
    loss.backward()
    gX, gY = X.grad.cpu().numpy(), Y.grad.cpu().numpy()
    rng = synth.rng(105, 4)
    for _ in range(60):
        i, c = int(rng.integers(case.m)), int(rng.integers(case.k))
        fd = 3.0 * _fd_row(case, case.X0, case.Y0, i, c)
        assert gX[i, c] == pytest.approx(fd, rel=2e-4, abs=2e-4 * np.sqrt(np.mean(gX ** 2)))
        j, c = int(rng.integers(case.n)), int(rng.integers(case.k))
        fd = 3.0 * _fd_row(case, case.X0, case.Y0, j, c, by_col=True)
        assert gY[j, c] == pytest.approx(fd, rel=2e-4, abs=2e-4 * np.sqrt(np.mean(gY ** 2)))


def test_autograd_full_size_sampled():
    """50,000 x 2,000, k = 64, 1,000 logistic and 1,000 quadratic columns, 10%
    missing: GPU gradients against FP64 finite differences of the oracle's row
    and column objectives at 1,000 sampled coordinates (500 in X, 500 in Y)."""
    case = synth.autograd_point()
    data = g.Data.from_case(case, DEV)
    X = to_dev(case.X0, DEV).requires_grad_(True)
    Y = to_dev(case.Y0, DEV).requires_grad_(True)
    glrm_loss(X, Y, data, "fp32").backward()
    gX, gY = X.grad.cpu().numpy(), Y.grad.cpu().numpy()
    rng = synth.rng(4, 4)
    rmsx, rmsy = np.sqrt(np.mean(gX ** 2)), np.sqrt(np.mean(gY ** 2))
    bad = 0
    for t in range(500):
        i, c = int(rng.integers(case.m)), int(rng.integers(case.k))
        fd = _fd_row(case, case.X0, case.Y0, i, c)
        bad += abs(gX[i, c] - fd) > 1e-4 * max(abs(fd), rmsx)
    for t in range(500):
        j, c = int(rng.integers(case.n)), int(rng.integers(case.k))
        fd = _fd_row(case, case.X0, case.Y0, j, c, by_col=True)
        bad += abs(gY[j, c] - fd) > 1e-4 * max(abs(fd), rmsy)
    assert bad == 0


def test_forward_without_grad_uses_the_objective_only():
    case = synth.autograd_point(m=500, n=100, k=16, config=106)
    data = g.Data.from_case(case, DEV)
    X, Y = to_dev(case.X0, DEV), to_dev(case.Y0, DEV)
    with torch.no_grad():
        f = glrm_loss(X, Y, data, "fp32")
    assert float(f) == pytest.approx(oracle_problem(case).loss_sum(case.X0, case.Y0), rel=1e-5)


REGS = [
    # quadratic on X, l1 on Y (a few exact zeros in Y: the l1 kink)
    dict(rx=(1, 0.3), ry=(2, 0.2), zeros=True),
    # nonnegative X from a nonnegative start, quadratic on Y
    dict(rx=(3, 0.0), ry=(1, 0.5), x_nonneg=True),
    # no regularizer: the objective is the loss
    dict(rx=(0, 0.0), ry=(0, 0.0)),
]


@pytest.mark.parametrize("layout", ["dense", "coo"])
@pytest.mark.parametrize("spec", REGS)
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 2e-2)])
def test_objective_with_regularizers_matches_the_oracle(spec, prec, tol, layout):
    """All of eq. gpca: the value is the oracle's objective, the gradient the
    oracle's loss gradient plus its least-magnitude regularizer subgradient."""
    sp = dict(spec)
    zeros = sp.pop("zeros", False)
    case = synth.small_mixed(400, 70, 6, seed=120, layout=layout, **sp)
    if zeros:
        case.Y0[::7, 2] = 0.0
    data = g.Data.from_case(case, DEV)
    X = to_dev(case.X0, DEV).requires_grad_(True)
    Y = to_dev(case.Y0, DEV).requires_grad_(True)
    f = glrm_objective(X, Y, data, prec)
    (2.0 * f).backward()
    P = oracle_problem(case)
    dXr, dYr = P.grad(case.X0, case.Y0)
    dXr = 2.0 * (dXr + oracle.reg_subgrad(case.rx[0], case.rx[1], case.X0))
    dYr = 2.0 * (dYr + oracle.reg_subgrad(case.ry[0], case.ry[1], case.Y0))
    assert rel_fro(X.grad.cpu().numpy(), dXr) <= tol
    assert rel_fro(Y.grad.cpu().numpy(), dYr) <= tol
    if zeros:
        # at the kink the least-magnitude subgradient adds nothing to the loss gradient
        gl = g.glrm_grad(data.with_regs((0, 0.0), (0, 0.0)), X.detach(), Y.detach(), prec)[1]
        np.testing.assert_array_equal(Y.grad[::7, 2].cpu().numpy(), 2.0 * gl[::7, 2].cpu().numpy())
    assert float(f) == pytest.approx(P.objective(case.X0, case.Y0), rel=1e-5 if prec == "fp32" else 1e-3)
    with torch.no_grad():
        assert float(glrm_objective(X, Y, data, prec)) == pytest.approx(float(f), rel=1e-12)


def test_objective_outside_the_regularizer_domain_is_infinite_with_nan_subgradients():
    """A negative coordinate under the nonnegative constraint: F = +inf (as
    the oracle's), and exactly those coordinates of the gradient are NaN."""
    case = synth.small_mixed(120, 40, 4, seed=121, rx=(1, 0.1), ry=(3, 0.0))
    data = g.Data.from_case(case, DEV)
    X = to_dev(case.X0, DEV).requires_grad_(True)
    Y = to_dev(case.Y0, DEV).requires_grad_(True)
    f = glrm_objective(X, Y, data, "fp32")
    f.backward()
    assert float(f) == np.inf == oracle_problem(case).objective(case.X0, case.Y0)
    gy = Y.grad.cpu().numpy()
    np.testing.assert_array_equal(np.isnan(gy), case.Y0 < 0)
    assert np.all(np.isfinite(X.grad.cpu().numpy()))


def test_objective_with_the_offset_matches_the_oracle():
    """The offset of Section 3.3 (x_i0 = 1, y_j0 free and unpenalized): the
    offset coordinates get the loss gradient alone."""
    case = synth.small_mixed(300, 50, 5, seed=122, rx=(1, 0.4), ry=(2, 0.3))
    case.X0[:, 0] = 1.0
    data = g.Data.from_case(case, DEV).variant(offset=True)
    X = to_dev(case.X0, DEV).requires_grad_(True)
    Y = to_dev(case.Y0, DEV).requires_grad_(True)
    f = glrm_objective(X, Y, data, "fp32")
    f.backward()
    r, c = np.nonzero(case.mask)
    P = oracle.Problem.from_coo(case.m, case.n, case.k, r, c, case.A[r, c], case.col_loss, case.losses,
                                case.rx, case.ry, offset=True)
    dXr, dYr = P.grad(case.X0, case.Y0)
    dXr = dXr + oracle.reg_subgrad(case.rx[0], case.rx[1], case.X0, offset=1)
    dYr = dYr + oracle.reg_subgrad(case.ry[0], case.ry[1], case.Y0, offset=2)
    assert rel_fro(X.grad.cpu().numpy(), dXr) <= 1e-4
    assert rel_fro(Y.grad.cpu().numpy(), dYr) <= 1e-4
    assert float(f) == pytest.approx(P.objective(case.X0, case.Y0), rel=1e-5)
