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
    np.testing.assert_allclose(sv[:rr], s[:rr], rtol=1e-10)
    assert np.all(sv[rr:] == 0.0)
