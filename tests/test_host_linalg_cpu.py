"""The host-side small eigenproblems behind the certificate (Section 7.6) and
the SVD initialization (Section 7.5), built from the library's own source with
g++ and checked against numpy's SVD: X P Y^T must be U V^T of the thin SVD of
X Y^T, with the same rank and singular values, also for a rank-deficient X."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1410_0342_amd", "csrc", "smallmat.cpp")

DRIVER = r"""
#include <cstdio>
#include "smallmat.h"
int main() {
    int k; if (scanf("%d", &k) != 1) return 1;
    double *Gx = new double[k * k], *Gy = new double[k * k], *P = new double[k * k], *sv = new double[k];
    for (int i = 0; i < k * k; ++i) if (scanf("%lf", &Gx[i]) != 1) return 1;
    for (int i = 0; i < k * k; ++i) if (scanf("%lf", &Gy[i]) != 1) return 1;
    printf("%d\n", glrm_host::polar_map(k, Gx, Gy, 1e-6, P, sv));
    for (int i = 0; i < k * k; ++i) printf("%.17g\n", P[i]);
    for (int i = 0; i < k; ++i) printf("%.17g\n", sv[i]);
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "driver.cpp")
    with open(src, "w") as fh:
        fh.write(DRIVER)
    exe = os.path.join(d, "driver")
    subprocess.check_call(["g++", "-O2", "-I", os.path.dirname(SRC), "-o", exe, src, SRC])
    return exe


@pytest.mark.parametrize("m,n,k,rank_x", [(50, 40, 5, 5), (30, 20, 7, 7), (30, 20, 6, 4), (60, 8, 3, 3),
                                         (100, 90, 64, 64), (40, 40, 64, 40)])
def test_polar_map_gives_the_svd_factor_product(driver, m, n, k, rank_x):
    rng = np.random.default_rng(m * 1000 + k)
    X = rng.standard_normal((m, k))
    Y = rng.standard_normal((n, k))
    if rank_x < k:
        X[:, rank_x:] = X[:, :k - rank_x] @ rng.standard_normal((k - rank_x, k - rank_x)) if k - rank_x <= rank_x else 0.0
    inp = "%d\n%s\n%s\n" % (k, " ".join("%.17g" % v for v in (X.T @ X).ravel()),
                            " ".join("%.17g" % v for v in (Y.T @ Y).ravel()))
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout.split()
    r = int(out[0])
    P = np.array(out[1:1 + k * k], float).reshape(k, k)
    sv = np.array(out[1 + k * k:], float)
    U, s, Vt = np.linalg.svd(X @ Y.T, full_matrices=False)
    rr = int(np.sum(s > 1e-6 * s[0]))
    assert r == rr
    np.testing.assert_allclose(X @ P @ Y.T, U[:, :rr] @ Vt[:rr], atol=1e-8)
    # the singular values come from eigenvalues of Gram-type matrices: a
    # backward-stable eigensolver leaves an absolute error of order
    # n eps s_1^2 in s_i^2, so about n eps s_1^2 / s_i in s_i
    eps = np.finfo(float).eps
    allow = 1e-10 * s[:rr] + 64 * eps * s[0] ** 2 / s[:rr]
    assert np.all(np.abs(sv[:rr] - s[:rr]) <= allow)
    assert np.all(sv[rr:] == 0.0)


EIG_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "smallmat.h"
int main() {
    int n;
    while (scanf("%d", &n) == 1) {
        std::vector<double> A((size_t)n * n), w(n), V((size_t)n * n);
        for (auto &x : A) if (scanf("%lf", &x) != 1) return 1;
        glrm_host::sym_eig(n, A.data(), w.data(), V.data());
        for (double x : w) printf("%.17g\n", x);
        for (double x : V) printf("%.17g\n", x);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def eig_driver():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "eig.cpp")
    with open(src, "w") as fh:
        fh.write(EIG_DRIVER)
    exe = os.path.join(d, "eig")
    subprocess.check_call(["g++", "-O2", "-I", os.path.dirname(SRC), "-o", exe, src, SRC])
    return exe


def _eig_cases():
    rng = np.random.default_rng(41)
    cases = []
    for n in (1, 2, 3, 5, 16, 30, 64, 96):
        B = rng.standard_normal((n, n + 3))
        cases.append(B @ B.T)                      # positive definite
        M = rng.standard_normal((n, n))
        cases.append(M + M.T)                      # indefinite
    B = rng.standard_normal((30, 4))
    cases.append(B @ B.T)                          # rank 4
    Q, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    cases.append(Q @ np.diag([3.0] * 7 + [1.0] * 7 + [0.0] * 6) @ Q.T)   # repeated eigenvalues
    cases.append(np.diag(rng.standard_normal(12)))                      # already diagonal
    cases.append(np.zeros((6, 6)))
    cases.append(np.ones((9, 9)))
    cases.append(1e-200 * (B @ B.T))               # entries whose squares underflow
    cases.append(1e200 * (B @ B.T))                # and overflow
    D = np.diag(10.0 ** np.arange(-8, 8))
    M = rng.standard_normal((16, 16))
    cases.append(D @ (M + M.T) @ D)                # graded
    return cases


def test_symmetric_eigensolver_matches_numpy(eig_driver):
    """V diag(w) V^T = A with V orthonormal and w descending, the eigenvalues
    equal to numpy's: all to a small multiple of eps times the largest |w|
    (the bound of a backward-stable method)."""
    cases = _eig_cases()
    inp = "".join("%d\n%s\n" % (c.shape[0], " ".join("%.17g" % x for x in c.ravel())) for c in cases)
    out = subprocess.run([eig_driver], input=inp, capture_output=True, text=True, check=True).stdout.split()
    pos = 0
    eps = np.finfo(float).eps
    for c in cases:
        n = c.shape[0]
        w = np.array(out[pos:pos + n], float)
        pos += n
        V = np.array(out[pos:pos + n * n], float).reshape(n, n)
        pos += n * n
        ref = np.sort(np.linalg.eigvalsh(c))[::-1]
        scale = max(np.abs(ref).max(), np.finfo(float).tiny)
        assert np.all(np.diff(w) <= 0.0)
        assert np.abs(w - ref).max() <= 64 * n * eps * scale
        assert np.abs(V @ np.diag(w) @ V.T - c).max() <= 64 * n * eps * scale
        assert np.abs(V.T @ V - np.eye(n)).max() <= 64 * n * eps
    assert pos == len(out)
