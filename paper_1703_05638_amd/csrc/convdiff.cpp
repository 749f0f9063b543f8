// The convection-diffusion operator of Sec. 6.3 in the space-time solves:
// L = nu K + w N + delta w^2 S on the tensor mesh, N the convection matrix of
// the wind (0, w) (along x2) and S its streamline-diffusion matrix (SUPG for
// bilinear elements: the Laplacian of a bilinear function vanishes inside
// each element, so only the streamline term remains).  With the 1D factors
// K1 = tridiag(-1, 2, -1) / h, M1 = h tridiag(1, 4, 1) / 6 and
// C1 = tridiag(-1/2, 0, 1/2) (first factor along x2):
//   L = D K1 (x) M1 + nu M1 (x) K1 + w C1 (x) M1,  D = nu + delta w^2.
// a L + b M is symmetric along x1, where K1 and M1 are diagonal in the
// orthonormal sine basis (eigenvalues kappa_j, mu_j), so a shifted solve is
// one tridiagonal system along x2 per sine mode (fast diagonalization).
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace lrp {

// Host settings of the operator on the N x N mesh with nt steps over [0, T]
// (no device work; exported for checks without a GPU).
CdParams cd_params(int N, int nt, double T, double nu, double w, double delta) {
  CdParams c{};
  const double h = 1.0 / N, tau = T / nt;
  if (delta < 0.0) {
    // element Peclet number of the square elements along the wind (the
    // element's length along the wind is h): delta = h / (2|w|) (1 - 1/Pe)
    // for Pe = |w| h / (2 nu) > 1, else 0
    const double wn = std::abs(w);
    const double pe = wn * h / (2.0 * nu);
    delta = (wn > 0.0 && pe > 1.0) ? h / (2.0 * wn) * (1.0 - 1.0 / pe) : 0.0;
  }
  c.delta = delta;
  // Spectrum of the symmetric part of M^{-1} L: D (M1^{-1} K1) along x2 plus
  // nu (M1^{-1} K1) along x1, so within [(D + nu) kappa_1 / mu_1, (D + nu) 12 / h^2);
  // the skew part w C1 (x) M1 has ||M^{-1/2} (C1 (x) M1) M^{-1/2}|| <=
  // ||C1|| / lambda_min(M1) < 3 / h.
  const double D = nu + delta * w * w;
  const double th = M_PI * h;
  const double kap1 = (4.0 / h) * std::sin(th / 2) * std::sin(th / 2), mu1 = (h / 3.0) * (2.0 + std::cos(th));
  c.lam_min = (D + nu) * kap1 / mu1;
  c.lam_sym = (D + nu) * 12.0 / (h * h);
  c.skew = 3.0 * std::abs(w) / h;
  // Newton-Schulz for the projected A = I + Kt, Kt = Q^T tau L Q with Q
  // M-orthonormal: the field of values of A lies in the rectangle
  // [1, 1 + s] x i[-b, b], s = tau lam_sym, b = tau skew (5% margin for the
  // rounding of the basis).  With X_0 = alpha I the error I - A X_k is
  // (I - alpha A)^(2^k), whose numerical radius is at most r^(2^k), r the
  // largest |1 - alpha z| over the rectangle (attained at a corner: the
  // modulus is convex), and its norm at most twice that.  alpha minimizes r.
  const double s = 1.05 * tau * c.lam_sym, b = 1.05 * tau * c.skew;
  c.fov_re = 1.0 + s;
  c.fov_im = b;
  auto radius = [&](double a) {
    double r2 = 0.0;
    for (double x : {1.0, 1.0 + s}) r2 = std::max(r2, (1.0 - a * x) * (1.0 - a * x) + a * a * b * b);
    return std::sqrt(r2);
  };
  double lo = 0.0, hi = 2.0 / (1.0 + s);
  for (int it = 0; it < 200; ++it) {
    const double m1 = lo + (hi - lo) / 3.0, m2 = hi - (hi - lo) / 3.0;
    if (radius(m1) < radius(m2)) hi = m2;
    else lo = m1;
  }
  c.ns_alpha = 0.5 * (lo + hi);
  c.ns_radius = radius(c.ns_alpha);
  // 2 r^(2^k) <= 1e-18, plus one step
  c.ns_iters = c.ns_radius > 0.0 && c.ns_radius < 1.0
                   ? std::max(1, (int)std::ceil(std::log2(std::log(5e-19) / std::log(c.ns_radius))) + 1)
                   : 1;
  return c;
}

void Problem::set_convection(double nu, double w, double delta) {
  sync();
  if (!(nu > 0.0)) {
    cd_on = false;
    cd_nu = cd_w = cd_delta = 0.0;
    poles_low_.clear();
    init_st_poles(2.0 * M_PI * M_PI, 24.0 / (h * h));
    return;
  }
  if (!std::isfinite(nu) || !std::isfinite(w) || !std::isfinite(delta))
    fail(LRPOST_EINVAL, "convection parameters must be finite");
  const CdParams cp = cd_params(N, nt, desc.T, nu, w, delta);
  if (!(cp.ns_radius < 1.0)) fail(LRPOST_EINVAL, "convection operator: no convergent Newton-Schulz start");
  delta = cp.delta;
  cd_nu = nu;
  cd_w = w;
  cd_delta = delta;
  cd_on = true;
  if (cd_mu_h_.empty()) {
    // orthonormal sine matrix S_ij = sqrt(2h) sin((i+1)(j+1) pi h) (the
    // argument reduced modulo 2 pi exactly in integers) and the 1D
    // eigenvalues on mode j: kappa_j = (4/h) sin^2(theta_j / 2),
    // mu_j = (h/3) (2 + cos theta_j), theta_j = (j+1) pi h
    std::vector<double> S((size_t)n * n);
    const long period = 2L * N;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const long k = ((long)(i + 1) * (j + 1)) % period;
        S[(size_t)i * n + j] = std::sqrt(2.0 * h) * std::sin((double)k * M_PI / (double)N);
      }
    cd_mu_h_.resize(n);
    cd_kap_h_.resize(n);
    for (int j = 0; j < n; ++j) {
      const double th = (j + 1) * M_PI * h;
      cd_kap_h_[j] = (4.0 / h) * std::sin(th / 2) * std::sin(th / 2);
      cd_mu_h_[j] = (h / 3.0) * (2.0 + std::cos(th));
    }
    cd_S_.ensure(sizeof(double) * S.size());
    cd_mu_.ensure(sizeof(double) * n);
    cd_kap_.ensure(sizeof(double) * n);
    to_device(cd_S_.as<double>(), S.data(), S.size());
    to_device(cd_mu_.as<double>(), cd_mu_h_.data(), n);
    to_device(cd_kap_.as<double>(), cd_kap_h_.data(), n);
    sync();
  }
  // Poles over the larger of the symmetric and skew scales (cd_params), more
  // than for the heat operator: transport keeps the space-time solutions'
  // rank higher (at 32^2, nt = 90 a rank-one initial state gives rank 21 at
  // 1e-8 against 11 for the heat equation), and a source of rank one gets
  // one basis column per pole.  Measured in a CPU emulation of the solver at
  // 32^2, nu = 1e-3 and 1e-2, nt = 90, tol 1e-8: rank-one sources keep a
  // relative error of 2e-3 with the heat operator's 13 poles, 5e-6 with 26
  // and 3-4e-7 with 52; the adjoint sources (rank 20-30) 3e-6 with 13 and
  // 3e-8 with 20.  So sources of rank <= 2 take four times the heat
  // operator's count, the others one and a half times.
  init_st_poles(cp.lam_min, std::max(cp.lam_sym, cp.skew), 4.0);
  poles_low_ = poles;
  init_st_poles(cp.lam_min, std::max(cp.lam_sym, cp.skew), 1.5);
  // Newton-Schulz start and step count of the non-symmetric projected problem
  cd_ns_alpha_ = cp.ns_alpha;
  cd_ns_iters_ = cp.ns_iters;
}

void Problem::cd_apply(int ncols, const double* X, double* Y, const std::vector<ShiftCoef>& ab, int sign) {
  if (ncols <= 0) return;
  if (!cd_on) fail(LRPOST_EINVAL, "no convection operator set");
  const double D = cd_nu + cd_delta * cd_w * cd_w;
  const double K1[3] = {-1.0 / h, 2.0 / h, -1.0 / h};
  const double M1[3] = {h / 6.0, 4.0 * h / 6.0, h / 6.0};
  const double C1[3] = {-0.5, 0.0, 0.5};
  const double sw = sign < 0 ? -cd_w : cd_w;
  const int nw = ab.size() == 1 ? 1 : ncols;
  std::vector<double> wt((size_t)6 * nw);
  for (int c = 0; c < nw; ++c) {
    const double a = ab[c].a, b = ab[c].b;
    for (int d2 = 0; d2 < 3; ++d2)
      for (int e = 0; e < 2; ++e) {
        const double mx = M1[1 - e], kx = K1[1 - e];  // e = 0: centre along x1, 1: side
        wt[(size_t)6 * c + 2 * d2 + e] =
            a * (D * K1[d2] * mx + cd_nu * M1[d2] * kx + sw * C1[d2] * mx) + b * M1[d2] * mx;
      }
  }
  cd_wt_.ensure(sizeof(double) * wt.size());
  to_device(cd_wt_.as<double>(), wt.data(), wt.size());
  timed(LRPOST_KERNEL_STENCIL, sizeof(double) * 2.0 * (double)nx * ncols,
        [&] { cd_stencil(st, n, ncols, X, nx, Y, nx, cd_wt_.as<double>(), nw == 1 ? 0 : 6); });
  LRP_HIP(hipGetLastError());
}

void Problem::cd_solve(int ncols, const double* B, double* X, const std::vector<ShiftCoef>& ab, int sign) {
  if (ncols <= 0) return;
  if (!cd_on) fail(LRPOST_EINVAL, "no convection operator set");
  std::vector<double> abh((size_t)2 * ncols);
  for (int c = 0; c < ncols; ++c) {
    const ShiftCoef& s = ab.size() == 1 ? ab[0] : ab[c];
    if (!(s.a >= 0.0) || !(s.b >= 0.0) || !(s.a + s.b > 0.0)) fail(LRPOST_EINVAL, "shifts must be a, b >= 0, a + b > 0");
    abh[(size_t)2 * c] = s.a;
    abh[(size_t)2 * c + 1] = s.b;
  }
  cd_ab_.ensure(sizeof(double) * abh.size());
  to_device(cd_ab_.as<double>(), abh.data(), abh.size());
  cd_tmp_.ensure(sizeof(double) * (size_t)nx * ncols);
  double* T = cd_tmp_.as<double>();
  const double D = cd_nu + cd_delta * cd_w * cd_w;
  const CdCoef k{D / h, 0.5 * (sign < 0 ? -cd_w : cd_w), cd_nu, h / 6.0};
  const double sbytes = sizeof(double) * 2.0 * (double)nx * ncols;
  const double sflops = 2.0 * (double)n * (double)nx * ncols;
  // B -> T (sine modes along x1), the x2 systems in place in T with X as the
  // elimination scratch, T -> X (the sine matrix is its own inverse)
  timed(LRPOST_KERNEL_SINE, sbytes, [&] { sine_x1(st, n, ncols, B, nx, T, nx, cd_S_.as<double>()); }, sflops);
  timed(LRPOST_KERNEL_TRIDIAG, sizeof(double) * 6.0 * (double)nx * ncols, [&] {
    tridiag_x2(st, n, ncols, T, nx, X, nx, cd_ab_.as<double>(), cd_mu_.as<double>(), cd_kap_.as<double>(), k);
  });
  timed(LRPOST_KERNEL_SINE, sbytes, [&] { sine_x1(st, n, ncols, T, nx, X, nx, cd_S_.as<double>()); }, sflops);
  LRP_HIP(hipGetLastError());
}

void Problem::st_apply(int ncols, const double* X, double* Y, const std::vector<ShiftCoef>& ab) {
  if (cd_on) cd_apply(ncols, X, Y, ab, cd_sign);
  else apply_op(ncols, X, Y, ab);
}

void Problem::st_spatial_solve(int ncols, const double* B, double* X, const std::vector<ShiftCoef>& ab, int cycles) {
  if (cd_on) cd_solve(ncols, B, X, ab, cd_sign);
  else mg_solve(ncols, B, X, ab, cycles);
}

}  // namespace lrp
