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
    std::vector<double> a(A, A + (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = i == j ? 1.0 : 0.0;
    double frob = 0.0;
    for (double x : a) frob += x * x;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
        if (off <= 1e-32 * frob || off == 0.0) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[p * n + q];
                if (apq == 0.0) continue;
                // rotation in the (p, q) plane that zeroes a_pq: t = tan(phi)
                // is the smaller root of t^2 + 2 theta t - 1 = 0
                const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < n; ++r) {
                    const double arp = a[r * n + p], arq = a[r * n + q];
                    a[r * n + p] = c * arp - s * arq;
                    a[r * n + q] = s * arp + c * arq;
                }
                for (int r = 0; r < n; ++r) {
                    const double apr = a[p * n + r], aqr = a[q * n + r];
                    a[p * n + r] = c * apr - s * aqr;
                    a[q * n + r] = s * apr + c * aqr;
                }
                a[p * n + q] = a[q * n + p] = 0.0;
                for (int r = 0; r < n; ++r) {
                    const double vrp = V[r * n + p], vrq = V[r * n + q];
                    V[r * n + p] = c * vrp - s * vrq;
                    V[r * n + q] = s * vrp + c * vrq;
                }
            }
        }
    }
    // eigenvalues in descending order, vectors permuted alike
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int x, int y) { return a[x * n + x] > a[y * n + y]; });
    std::vector<double> Vs((size_t)n * n);
    for (int c = 0; c < n; ++c) {
        w[c] = a[order[c] * n + order[c]];
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
