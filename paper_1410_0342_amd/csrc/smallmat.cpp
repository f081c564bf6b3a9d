// Small dense symmetric eigenproblems on the host, in double: the k x k Gram
// matrices behind the global-optimality certificate (Section 7.6) and the
// l x l problems of the randomized SVD (Section 7.5).  Plain C++, no HIP, so
// the same file builds into a CPU test.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "smallmat.h"

namespace glrm_host {

void sym_eig(int n, const double *A, double *w, double *V)
{
    if (n <= 0) return;
    std::vector<double> a(A, A + (size_t)n * n), u(n), p(n), d(n), e(n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = i == j ? 1.0 : 0.0;
    // work on A / max |a_ij| (squares of tiny or huge entries neither
    // underflow nor overflow); the eigenvalues are scaled back at the end
    double scale = 0.0;
    for (double x : a) scale = std::max(scale, std::fabs(x));
    if (scale > 0.0)
        for (double &x : a) x /= scale;
    // Householder reduction to tridiagonal form: step k reflects column k
    // below the diagonal onto its first coordinate with H = I - beta u u^T,
    // B <- H B H on the trailing block as B - u q^T - q u^T (p = beta B u,
    // q = p - (beta u^T p / 2) u), and V <- V H.
    for (int k = 0; k + 2 < n; ++k) {
        const int m0 = k + 1;
        double norm2 = 0.0;
        for (int i = m0; i < n; ++i) norm2 += a[i * n + k] * a[i * n + k];
        const double x0 = a[m0 * n + k];
        const double alpha = x0 >= 0.0 ? -std::sqrt(norm2) : std::sqrt(norm2);
        const double uu = 2.0 * (norm2 - alpha * x0);   // u^T u for u = x - alpha e1
        if (!(uu > 0.0)) continue;                      // the column is already reduced
        const double beta = 2.0 / uu;
        for (int i = m0; i < n; ++i) u[i] = a[i * n + k];
        u[m0] = x0 - alpha;
        double up = 0.0;
        for (int i = m0; i < n; ++i) {
            double s = 0.0;
            for (int j = m0; j < n; ++j) s += a[i * n + j] * u[j];
            p[i] = beta * s;
            up += u[i] * p[i];
        }
        const double K = 0.5 * beta * up;
        for (int i = m0; i < n; ++i) p[i] -= K * u[i];   // p now holds q
        for (int i = m0; i < n; ++i)
            for (int j = m0; j < n; ++j) a[i * n + j] -= u[i] * p[j] + p[i] * u[j];
        for (int i = m0; i < n; ++i) a[i * n + k] = a[k * n + i] = 0.0;
        a[m0 * n + k] = a[k * n + m0] = alpha;
        for (int r = 0; r < n; ++r) {
            double s = 0.0;
            for (int j = m0; j < n; ++j) s += V[r * n + j] * u[j];
            s *= beta;
            for (int j = m0; j < n; ++j) V[r * n + j] -= s * u[j];
        }
    }
    for (int i = 0; i < n; ++i) d[i] = a[i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = a[(i + 1) * n + i];
    // Implicit symmetric QR steps with the Wilkinson shift on the unreduced
    // block lo..hi (e[i] couples i and i + 1): a Givens rotation in the plane
    // (k, k + 1), G = [c -s; s c], takes T to G^T T G and chases the bulge
    // down the block; V <- V G.  A coupling is dropped once it is below the
    // rounding of its two diagonal entries.
    const double eps = 2.220446049250313e-16;
    int guard = 64 * n;
    for (int hi = n - 1; hi > 0 && guard > 0;) {
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
        --guard;
        const double delta = 0.5 * (d[hi - 1] - d[hi]), eh = e[hi - 1];
        const double mu = d[hi] - eh * eh / (delta + (delta >= 0.0 ? 1.0 : -1.0) * std::hypot(delta, eh));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? z / r : 0.0;
            if (k > lo) e[k - 1] = r;
            const double dk = d[k], dk1 = d[k + 1], ek = e[k];
            d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
            d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
            e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
            if (k + 1 < hi) {
                x = e[k];
                z = s * e[k + 1];
                e[k + 1] *= c;
            }
            for (int row = 0; row < n; ++row) {
                const double vk = V[row * n + k], vk1 = V[row * n + k + 1];
                V[row * n + k] = c * vk + s * vk1;
                V[row * n + k + 1] = c * vk1 - s * vk;
            }
        }
    }
    // eigenvalues in descending order, vectors permuted alike
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int x, int y) { return d[x] > d[y]; });
    std::vector<double> Vs((size_t)n * n);
    for (int c = 0; c < n; ++c) {
        w[c] = d[order[c]] * scale;
        for (int r = 0; r < n; ++r) Vs[r * n + c] = V[r * n + order[c]];
    }
    std::copy(Vs.begin(), Vs.end(), V);
}

// With X = Qx Rx (Gram Gx = X^T X = Ex Lx Ex^T, Qx = X Ex Lx^-1/2 over the
// eigenvalues above the rank threshold) and likewise Y, X Y^T = Qx C Qy^T with
// C = Lx^1/2 Ex^T Ey Ly^1/2.  The thin SVD C = Uc S Vc^T gives X Y^T = U S V^T
// with U = Qx Uc, V = Qy Vc, so U V^T = X P Y^T with
//     P = Ex Lx^-1/2 (Uc Vc^T) Ly^-1/2 Ey^T
// over the nonzero singular values.  Uc Vc^T = C (C^T C)^-1/2 on them, from the
// eigen-decomposition of C^T C.  Returns the rank of X Y^T.
int polar_map(int k, const double *Gx, const double *Gy, double rtol, double *P, double *sv)
{
    std::vector<double> lx(k), ex((size_t)k * k), ly(k), ey((size_t)k * k);
    sym_eig(k, Gx, lx.data(), ex.data());
    sym_eig(k, Gy, ly.data(), ey.data());
    const double lxmax = std::max(lx[0], 0.0), lymax = std::max(ly[0], 0.0);
    int rx = 0, ry = 0;
    while (rx < k && lx[rx] > rtol * rtol * lxmax && lx[rx] > 0.0) ++rx;
    while (ry < k && ly[ry] > rtol * rtol * lymax && ly[ry] > 0.0) ++ry;
    for (int i = 0; i < k * k; ++i) P[i] = 0.0;
    for (int i = 0; i < k; ++i) sv[i] = 0.0;
    if (rx == 0 || ry == 0) return 0;
    // C = Lx^1/2 Ex^T Ey Ly^1/2  (rx x ry), columns of E are eigenvectors
    std::vector<double> C((size_t)rx * ry);
    for (int a = 0; a < rx; ++a)
        for (int b = 0; b < ry; ++b) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) s += ex[l * k + a] * ey[l * k + b];
            C[a * ry + b] = std::sqrt(lx[a]) * s * std::sqrt(ly[b]);
        }
    // C^T C = Vc S^2 Vc^T
    std::vector<double> CtC((size_t)ry * ry), s2(ry), vc((size_t)ry * ry);
    for (int a = 0; a < ry; ++a)
        for (int b = 0; b < ry; ++b) {
            double s = 0.0;
            for (int l = 0; l < rx; ++l) s += C[l * ry + a] * C[l * ry + b];
            CtC[a * ry + b] = s;
        }
    sym_eig(ry, CtC.data(), s2.data(), vc.data());
    const double smax = std::sqrt(std::max(s2[0], 0.0));
    int r = 0;
    while (r < ry && r < rx && s2[r] > 0.0 && std::sqrt(s2[r]) > rtol * smax) ++r;
    for (int i = 0; i < r; ++i) sv[i] = std::sqrt(s2[i]);
    // W = C Vc_r S_r^-1 Vc_r^T  (rx x ry)
    std::vector<double> W((size_t)rx * ry, 0.0);
    for (int a = 0; a < rx; ++a)
        for (int b = 0; b < ry; ++b) {
            double s = 0.0;
            for (int q = 0; q < r; ++q) {
                double cv = 0.0;
                for (int l = 0; l < ry; ++l) cv += C[a * ry + l] * vc[l * ry + q];
                s += cv / sv[q] * vc[b * ry + q];
            }
            W[a * ry + b] = s;
        }
    // P = Ex_r Lx^-1/2 W Ly^-1/2 Ey_r^T  (k x k)
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            double s = 0.0;
            for (int a = 0; a < rx; ++a) {
                const double xa = ex[i * k + a] / std::sqrt(lx[a]);
                for (int b = 0; b < ry; ++b) s += xa * W[a * ry + b] * ey[j * k + b] / std::sqrt(ly[b]);
            }
            P[i * k + j] = s;
        }
    return r;
}

}  // namespace glrm_host
