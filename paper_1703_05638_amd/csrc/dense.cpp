// Small dense float64 linear algebra on the host: Cholesky, triangular
// inverse, symmetric eigensolver (Householder tridiagonalization followed by
// implicit QR steps with Wilkinson shifts), one-sided Jacobi SVD and a
// Householder QR.  Sizes are the ranks of low-rank factors and the projected
// problems (a few hundred at most).  All matrices are column-major.
#include "dense.h"

#include <algorithm>
#include <functional>
#include <cmath>
#include <limits>
#include <numeric>

namespace lrp {

namespace {
inline double dot4(const double* x, const double* y, int len);
void householder_reduce(int m, int n, std::vector<double>& W, std::vector<std::vector<double>>* vs,
                        std::vector<double>& betas);
}  // namespace

void matmul(int m, int n, int k, const double* A, int lda, bool ta, const double* B, int ldb, bool tb, double* C,
            int ldc, double alpha, double beta) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      for (int p = 0; p < k; ++p) {
        const double a = ta ? A[(size_t)i * lda + p] : A[(size_t)p * lda + i];
        const double b = tb ? B[(size_t)p * ldb + j] : B[(size_t)j * ldb + p];
        s += a * b;
      }
      C[(size_t)j * ldc + i] = alpha * s + (beta == 0.0 ? 0.0 : beta * C[(size_t)j * ldc + i]);
    }
}

bool cholesky_upper(int n, const double* G, int ldg, double* R) {
  // G = R^T R, R upper triangular (column-major n x n, zero below the diagonal)
  std::fill(R, R + (size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i <= j; ++i) {
      double s = G[(size_t)j * ldg + i];
      for (int p = 0; p < i; ++p) s -= R[(size_t)i * n + p] * R[(size_t)j * n + p];
      if (i == j) {
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        R[(size_t)j * n + j] = std::sqrt(s);
      } else {
        R[(size_t)j * n + i] = s / R[(size_t)i * n + i];
      }
    }
  }
  return true;
}

void upper_inverse(int n, const double* R, double* Ri) {
  std::fill(Ri, Ri + (size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    Ri[(size_t)j * n + j] = 1.0 / R[(size_t)j * n + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int p = i + 1; p <= j; ++p) s += R[(size_t)p * n + i] * Ri[(size_t)j * n + p];
      Ri[(size_t)j * n + i] = -s / R[(size_t)i * n + i];
    }
  }
}

// sqrt(x^2 + z^2) without the cost of std::hypot unless a square could
// overflow or underflow.
static inline double fast_hypot(double x, double z) {
  const double ax = std::fabs(x), az = std::fabs(z);
  const double m = ax > az ? ax : az;
  if (m < 1e-150 || m > 1e150) return std::hypot(x, z);
  return std::sqrt(x * x + z * z);
}

// Householder reduction of symmetric A (n x n, both triangles stored) to
// tridiagonal form A = Q T Q^T.  On return d (n) and e (n-1) hold T and Q is
// written to Z (n x n).
static void tridiagonalize(int n, double* A, double* d, double* e, double* Z) {
  std::vector<double> v(n), p(n), q(n);
  for (int i = 0; i < n * n; ++i) Z[i] = 0.0;
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)j * n + i]; };
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of x = A[k+1:, k]
    double amax = 0.0;
    for (int i = 0; i < m; ++i) amax = std::max(amax, std::fabs(a(k + 1 + i, k)));
    if (amax == 0.0) continue;
    double ss = 0.0;  // scaled sum of squares
    for (int i = 0; i < m; ++i) {
      const double t = a(k + 1 + i, k) / amax;
      ss += t * t;
    }
    const double xnorm = amax * std::sqrt(ss);
    const double x0 = a(k + 1, k);
    const double alpha = x0 >= 0 ? -xnorm : xnorm;  // new subdiagonal value
    for (int i = 0; i < m; ++i) v[i] = a(k + 1 + i, k);
    v[0] -= alpha;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // p = beta * A22 v, accumulated column by column (contiguous access)
    for (int i = 0; i < m; ++i) p[i] = 0.0;
    for (int j = 0; j < m; ++j) {
      const double vj = beta * v[j];
      const double* col = &A[(size_t)(k + 1 + j) * n + (k + 1)];
      for (int i = 0; i < m; ++i) p[i] += col[i] * vj;
    }
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double K = 0.5 * beta * pv;
    for (int i = 0; i < m; ++i) q[i] = p[i] - K * v[i];
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) a(k + 1 + i, k + 1 + j) -= v[i] * q[j] + q[i] * v[j];
    a(k + 1, k) = alpha;
    a(k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) { a(k + 1 + i, k) = 0.0; a(k, k + 1 + i) = 0.0; }
    // Z <- Z H with H = I - beta v v^T acting on columns k+1..n-1 (row sums
    // accumulated column by column: contiguous access)
    std::vector<double>& zs = p;  // p is free again: zs[r] = beta sum_i Z[r, k+1+i] v[i]
    zs.assign(n, 0.0);
    for (int i = 0; i < m; ++i) {
      const double vi = v[i];
      const double* zc = Z + (size_t)(k + 1 + i) * n;
      for (int r = 0; r < n; ++r) zs[r] += zc[r] * vi;
    }
    for (int r = 0; r < n; ++r) zs[r] *= beta;
    for (int i = 0; i < m; ++i) {
      const double vi = v[i];
      double* zc = Z + (size_t)(k + 1 + i) * n;
      for (int r = 0; r < n; ++r) zc[r] -= zs[r] * vi;
    }
  }
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
}

// Implicit symmetric QR steps with Wilkinson shifts on the tridiagonal (d, e);
// rotations are accumulated into the columns of Z (n x n).
static bool tridiagonal_qr(int n, double* d, double* e, double* Z) {
  const double eps = std::numeric_limits<double>::epsilon();
  int hi = n - 1;
  int guard = 0;
  while (hi > 0) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    if (++guard > 60 * n) return false;
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    // Wilkinson shift: eigenvalue of the trailing 2x2 closer to d[hi]
    const double dd = 0.5 * (d[hi - 1] - d[hi]);
    const double b = e[hi - 1];
    const double den = dd + (dd >= 0 ? std::hypot(dd, b) : -std::hypot(dd, b));
    const double mu = d[hi] - b * b / den;
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      // rotation G in plane (k, k+1) with c*x - s*z = r, s*x + c*z = 0
      const double r = fast_hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) { c = x / r; s = -z / r; }
      if (k > lo) e[k - 1] = r;
      const double p = d[k], q = e[k], t = d[k + 1];
      d[k] = c * c * p - 2.0 * c * s * q + s * s * t;
      d[k + 1] = s * s * p + 2.0 * c * s * q + c * c * t;
      e[k] = c * s * (p - t) + (c * c - s * s) * q;
      if (k + 1 < hi) {
        x = e[k];
        z = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      for (int i = 0; i < n; ++i) {
        const double zk = Z[(size_t)k * n + i], zk1 = Z[(size_t)(k + 1) * n + i];
        Z[(size_t)k * n + i] = c * zk - s * zk1;
        Z[(size_t)(k + 1) * n + i] = s * zk + c * zk1;
      }
    }
  }
  return true;
}

bool syev(int n, const double* A, int lda, double* w, double* V) {
  if (n == 0) return true;
  std::vector<double> a((size_t)n * n), d(n), e(std::max(n - 1, 1));
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) a[(size_t)j * n + i] = 0.5 * (A[(size_t)j * lda + i] + A[(size_t)i * lda + j]);
  tridiagonalize(n, a.data(), d.data(), e.data(), V);
  if (!tridiagonal_qr(n, d.data(), e.data(), V)) return false;
  // sort ascending
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  std::vector<double> Vs((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    w[j] = d[idx[j]];
    std::copy(V + (size_t)idx[j] * n, V + (size_t)idx[j] * n + n, Vs.begin() + (size_t)j * n);
  }
  std::copy(Vs.begin(), Vs.end(), V);
  return true;
}

// One-sided Jacobi on the columns of A (m x n, m >= n): A V = U diag(s).
static void jacobi_columns(int m, int n, double* A, double* V) {
  for (int i = 0; i < n * n; ++i) V[i] = 0.0;
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  const double eps = std::numeric_limits<double>::epsilon();
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double al = 0.0, be = 0.0, ga = 0.0;
        double* ap = A + (size_t)p * m;
        double* aq = A + (size_t)q * m;
        for (int i = 0; i < m; ++i) { al += ap[i] * ap[i]; be += aq[i] * aq[i]; ga += ap[i] * aq[i]; }
        if (std::fabs(ga) <= eps * std::sqrt(al * be) || ga == 0.0) continue;
        rotated = true;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          const double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        double* vp = V + (size_t)p * n;
        double* vq = V + (size_t)q * n;
        for (int i = 0; i < n; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
}

void svd(int m, int n, const double* A, int lda, std::vector<double>& s, std::vector<double>& U,
         std::vector<double>& V, const std::function<int(const std::vector<double>&)>& keep) {
  // A = U diag(s) V^T, U: m x r, V: n x r, r = min(m, n), s descending; with
  // keep, only the first keep(s) columns of U and V are formed
  const bool tr = m < n;
  const int mm = tr ? n : m, nn = tr ? m : n;
  std::vector<double> W((size_t)mm * nn), Vw((size_t)nn * nn);
  for (int j = 0; j < nn; ++j)
    for (int i = 0; i < mm; ++i) W[(size_t)j * mm + i] = tr ? A[(size_t)i * lda + j] : A[(size_t)j * lda + i];
  // precondition by a Householder QR when tall, so Jacobi works on nn x nn;
  // the reflectors are kept and applied to the left vectors that are wanted
  const bool tall = mm > 2 * nn;
  std::vector<std::vector<double>> refl;
  std::vector<double> betas;
  if (tall) {
    householder_reduce(mm, nn, W, &refl, betas);
    std::vector<double> R((size_t)nn * nn, 0.0);
    for (int j = 0; j < nn; ++j)
      for (int i = 0; i <= j; ++i) R[(size_t)j * nn + i] = W[(size_t)j * mm + i];
    W.swap(R);
    jacobi_columns(nn, nn, W.data(), Vw.data());
  } else {
    jacobi_columns(mm, nn, W.data(), Vw.data());
  }
  const int wrows = tall ? nn : mm;
  std::vector<double> sv(nn);
  for (int j = 0; j < nn; ++j) {
    double t = 0.0;
    for (int i = 0; i < wrows; ++i) t = std::hypot(t, W[(size_t)j * wrows + i]);
    sv[j] = t;
  }
  std::vector<int> idx(nn);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return sv[x] > sv[y]; });
  s.assign(nn, 0.0);
  for (int jj = 0; jj < nn; ++jj) s[jj] = sv[idx[jj]];
  const int k = keep ? std::max(0, std::min(nn, keep(s))) : nn;
  // the first k left vectors of the (possibly reduced) matrix and right vectors
  std::vector<double> Ufull((size_t)mm * k, 0.0), Vr((size_t)nn * k);
  for (int jj = 0; jj < k; ++jj) {
    const int j = idx[jj];
    for (int i = 0; i < wrows; ++i) Ufull[(size_t)jj * mm + i] = sv[j] > 0 ? W[(size_t)j * wrows + i] / sv[j] : 0.0;
    for (int i = 0; i < nn; ++i) Vr[(size_t)jj * nn + i] = Vw[(size_t)j * nn + i];
  }
  // (zero singular values: the left vectors stay zero; callers do not need
  // them completed to an orthonormal basis)
  if (tall) {
    // Q [Ul; 0]: the reflectors applied last to first
    for (int r = nn - 1; r >= 0; --r) {
      if (betas[r] == 0.0) continue;
      const std::vector<double>& v = refl[r];
      const int len = mm - r;
      for (int jj = 0; jj < k; ++jj) {
        double* x = Ufull.data() + (size_t)jj * mm + r;
        const double sdot = betas[r] * dot4(v.data(), x, len);
        for (int i = 0; i < len; ++i) x[i] -= sdot * v[i];
      }
    }
  }
  if (!tr) {
    U.swap(Ufull);
    V.swap(Vr);
  } else {
    U.swap(Vr);
    V.swap(Ufull);
  }
}

namespace {
// four partial sums, so that the loops vectorize
inline double dot4(const double* x, const double* y, int len) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = 0;
  for (; i + 3 < len; i += 4) {
    s0 += x[i] * y[i];
    s1 += x[i + 1] * y[i + 1];
    s2 += x[i + 2] * y[i + 2];
    s3 += x[i + 3] * y[i + 3];
  }
  for (; i < len; ++i) s0 += x[i] * y[i];
  return (s0 + s1) + (s2 + s3);
}

// Householder reflections of W (m x n, leading dimension m) in place: W
// becomes R in its upper trapezoid; reflector k (I - beta_k v_k v_k^T, v_k of
// length m - k) is kept in vs[k] when keep_v.
void householder_reduce(int m, int n, std::vector<double>& W, std::vector<std::vector<double>>* vs,
                        std::vector<double>& betas) {
  const int K = std::min(m, n);
  betas.assign(K, 0.0);
  if (vs) vs->assign(K, {});
  std::vector<double> v(m);
  for (int k = 0; k < K; ++k) {
    const int len = m - k;
    double* wk = W.data() + (size_t)k * m + k;
    double amax = 0.0;
    for (int i = 0; i < len; ++i) amax = std::max(amax, std::fabs(wk[i]));
    if (amax == 0.0) continue;
    for (int i = 0; i < len; ++i) v[i] = wk[i] / amax;
    const double xn = std::sqrt(dot4(v.data(), v.data(), len));
    const double alpha = v[0] >= 0 ? -xn : xn;
    v[0] -= alpha;
    const double vv = dot4(v.data(), v.data(), len);
    if (!(vv > 0.0)) continue;
    const double beta = 2.0 / vv;
    for (int j = k; j < n; ++j) {
      double* wj = W.data() + (size_t)j * m + k;
      const double sdot = beta * dot4(v.data(), wj, len);
      for (int i = 0; i < len; ++i) wj[i] -= sdot * v[i];
    }
    betas[k] = beta;
    if (vs) (*vs)[k].assign(v.begin(), v.begin() + len);
  }
}
}  // namespace

// R factor only (K x n upper trapezoidal, K = min(m, n)) of A = Q R; Q is not formed.
void householder_r(int m, int n, const double* A, int lda, std::vector<double>& R) {
  const int K = std::min(m, n);
  std::vector<double> W((size_t)m * n), betas;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) W[(size_t)j * m + i] = A[(size_t)j * lda + i];
  householder_reduce(m, n, W, nullptr, betas);
  R.assign((size_t)K * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= std::min(j, K - 1); ++i) R[(size_t)j * K + i] = W[(size_t)j * m + i];
}

void householder_qr(int m, int n, const double* A, int lda, std::vector<double>& Q, std::vector<double>& R) {
  // A (m x n) = Q (m x K) R (K x n), K = min(m, n); R upper trapezoidal
  const int K = std::min(m, n);
  std::vector<double> W((size_t)m * n), betas;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) W[(size_t)j * m + i] = A[(size_t)j * lda + i];
  std::vector<std::vector<double>> vs;
  householder_reduce(m, n, W, &vs, betas);
  R.assign((size_t)K * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= std::min(j, K - 1); ++i) R[(size_t)j * K + i] = W[(size_t)j * m + i];
  Q.assign((size_t)m * K, 0.0);
  for (int j = 0; j < K; ++j) Q[(size_t)j * m + j] = 1.0;
  for (int k = K - 1; k >= 0; --k) {
    if (betas[k] == 0.0) continue;
    const std::vector<double>& v = vs[k];
    const int len = m - k;
    for (int j = 0; j < K; ++j) {
      double* qj = Q.data() + (size_t)j * m + k;
      const double sdot = betas[k] * dot4(v.data(), qj, len);
      for (int i = 0; i < len; ++i) qj[i] -= sdot * v[i];
    }
  }
}

int truncation_rank(const std::vector<double>& s, double tol, int cap, double* tail_out) {
  double total = 0.0;
  for (double x : s) total += x * x;
  if (total == 0.0) {
    if (tail_out) *tail_out = 0.0;
    return 0;
  }
  const int n = (int)s.size();
  std::vector<double> tail(n + 1, 0.0);
  for (int i = n - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
  int r = n;
  for (int i = 0; i <= n; ++i)
    if (std::sqrt(tail[i]) <= tol * std::sqrt(total)) { r = i; break; }
  if (cap >= 0 && r > cap) r = cap;
  if (tail_out) *tail_out = std::sqrt(tail[r] / total);
  return r;
}

}  // namespace lrp
