// Host-side small dense linear algebra in double (see smallmat.cpp).
#pragma once

namespace glrm_host {

// A (n x n, symmetric, row-major) = V diag(w) V^T, w descending, V's columns
// the eigenvectors (Householder tridiagonalization, then implicit QR steps
// with the Wilkinson shift).
void sym_eig(int n, const double *A, double *w, double *V);

// For factors X (m x k) and Y (n x k) with Gram matrices Gx = X^T X and
// Gy = Y^T Y: the k x k matrix P with U V^T = X P Y^T, where X Y^T = U S V^T is
// the thin SVD restricted to singular values above rtol times the largest.
// sv (k) receives the singular values (zeros past the rank); returns the rank.
int polar_map(int k, const double *Gx, const double *Gy, double rtol, double *P, double *sv);

}  // namespace glrm_host
