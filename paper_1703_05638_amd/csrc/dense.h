// Small dense float64 linear algebra on the host (column-major).
#pragma once
#include <cstddef>
#include <functional>
#include <vector>

namespace lrp {

// C = alpha op(A) op(B) + beta C, op(A) m x k, op(B) k x n.
void matmul(int m, int n, int k, const double* A, int lda, bool ta, const double* B, int ldb, bool tb, double* C,
            int ldc, double alpha, double beta);
// G = R^T R; false when G is not numerically positive definite.
bool cholesky_upper(int n, const double* G, int ldg, double* R);
void upper_inverse(int n, const double* R, double* Ri);

// Symmetric eigensolver: eigenvalues ascending in w, eigenvectors in V (n x n).
bool syev(int n, const double* A, int lda, double* w, double* V);
// Thin SVD A = U diag(s) V^T (U m x r, V n x r, r = min(m, n)), s descending,
// by one-sided Jacobi (after a Householder QR when A is tall or wide).  With
// keep, U and V hold only their first keep(s) columns (keep sees s).
void svd(int m, int n, const double* A, int lda, std::vector<double>& s, std::vector<double>& U,
         std::vector<double>& V, const std::function<int(const std::vector<double>&)>& keep = nullptr);
// Householder QR A (m x n) = Q (m x K) R (K x n), K = min(m, n), R upper trapezoidal.
void householder_qr(int m, int n, const double* A, int lda, std::vector<double>& Q, std::vector<double>& R);
void householder_r(int m, int n, const double* A, int lda, std::vector<double>& R);
// Smallest r with sqrt(sum_{i>=r} s_i^2) <= tol ||s||, capped at cap (cap < 0: none).
int truncation_rank(const std::vector<double>& s, double tol, int cap, double* tail_out);

}  // namespace lrp
