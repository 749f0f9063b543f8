// The initial-condition inverse problem of the paper's experiments (Sec. 6,
// eqs. pde, dis_obj, postvar, misfit; Sec. 6.2): the parameter is the initial
// state u = y(0), the state follows the source-free heat equation from it,
//   (M + tau K) y_1 = M u,  (M + tau K) y_k = M y_{k-1},
// i.e. the space-time system with right-hand side (M u) e_1^T, and the
// observations are the observed nodes at t_1..t_nt with noise sigma^2 I.
// With prior covariance c I the prior-preconditioned misfit Hessian of
// eq. misfit is G = c sigma^-2 C^T K^-T B^T B K^-1 C, C = e_1 kron M, which
// acts on nodal vectors: its eigenvectors are spatial fields, found by block
// Krylov steps with full re-orthogonalization and Rayleigh-Ritz (Sec. 4,
// Algorithm 1 for a self-adjoint operator), every step applying G to a
// block through the batched low-rank space-time solves.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "internal.h"

namespace lrp {

void Problem::set_obs_mask(const uint8_t* m) {
  std::vector<uint8_t> mh(nx, 0);
  int cnt = 0;
  for (long i = 0; i < nx; ++i) {
    mh[i] = m[i] ? 1 : 0;
    cnt += mh[i];
  }
  if (cnt == 0) fail(LRPOST_EINVAL, "observation mask selects no node");
  mask_h.swap(mh);
  nobs = cnt;
  mask.ensure(nx);
  to_device_bytes(mask.p, mask_h.data(), nx);
  sync();
}

// Y = G U for nvec initial states (U, Y: nx x nvec, device).
void Problem::ic_apply(int nvec, const double* U, double* Y, double c) {
  if (nvec <= 0) return;
  stats.applies += nvec;
  std::vector<LowRank> F(nvec), Yf(nvec), Zs(nvec), Pa(nvec);
  std::vector<const LowRank*> pF, pZ;
  std::vector<LowRank*> pY, pP;
  for (int j = 0; j < nvec; ++j) {
    F[j].resize(nx, nt, 1);
    apply_op(1, U + (size_t)j * nx, F[j].a(), {{0.0, 1.0}});  // M u_j
    F[j].B.assign(nt, 0.0);
    F[j].B[0] = 1.0;  // enters the first step only
    pF.push_back(&F[j]);
    pY.push_back(&Yf[j]);
  }
  spacetime_solve_batch(pF, pY, false);
  for (int j = 0; j < nvec; ++j) {
    Zs[j].resize(nx, nt, Yf[j].rank);
    if (Yf[j].rank > 0)
      mask_scale<double>(st, nx, Yf[j].rank, Yf[j].a(), nx, Zs[j].a(), nx, mask.as<uint8_t>(),
                         1.0 / (desc.sigma * desc.sigma));
    Zs[j].B = Yf[j].B;
    pZ.push_back(&Zs[j]);
    pP.push_back(&Pa[j]);
  }
  spacetime_solve_batch(pZ, pP, true);
  // C^T vec(P) = M p_1 with p_1 = W1 (first row of W2)^T, then the factor c
  DevMem p1, coef;
  p1.ensure(sizeof(double) * (size_t)nx * nvec);
  LRP_HIP(hipMemsetAsync(p1.p, 0, sizeof(double) * (size_t)nx * nvec, st));
  int rsum = 0;
  for (int j = 0; j < nvec; ++j) rsum += Pa[j].rank;
  std::vector<double> ch(std::max(rsum, 1));
  int off = 0;
  for (int j = 0; j < nvec; ++j) {
    for (int q = 0; q < Pa[j].rank; ++q) ch[off + q] = Pa[j].B[(size_t)q * nt];
    off += Pa[j].rank;
  }
  coef.ensure(sizeof(double) * ch.size());
  to_device(coef.as<double>(), ch.data(), ch.size());
  off = 0;
  for (int j = 0; j < nvec; ++j) {
    const int r = Pa[j].rank;
    if (r > 0)
      dense->gemm(false, false, (int)nx, 1, r, 1.0, Pa[j].a(), (int)nx, coef.as<double>() + off, r, 0.0,
                  p1.as<double>() + (size_t)j * nx, (int)nx);
    off += r;
  }
  apply_op(nvec, p1.as<double>(), Y, {{0.0, c}});
  sync();
}

// Orthonormalize the nb columns of W (nx x nb, device) against the first m
// columns of V (classical Gram-Schmidt twice) and among themselves (the
// eigenpairs of their Gram matrix, dropping directions below thresh of the
// largest squared norm the block had); the kept ones go to V[:, m..].
// Returns their number.
static int ic_extend_basis(Problem* P, double* V, int m, double* W, int nb, double* Cw, double* Gd,
                           double* Td, double thresh_rel) {
  const long nx = P->nx;
  std::vector<double> G0((size_t)nb * nb);
  P->dense->gemm(true, false, nb, nb, (int)nx, 1.0, W, (int)nx, W, (int)nx, 0.0, Gd, nb);
  P->to_host(G0.data(), Gd, G0.size());
  double scale = 0.0;
  for (int i = 0; i < nb; ++i) scale = std::max(scale, G0[(size_t)i * nb + i]);
  if (!(scale > 0.0)) return 0;
  for (int sweep = 0; sweep < 2 && m > 0; ++sweep) {
    P->dense->gemm(true, false, m, nb, (int)nx, 1.0, V, (int)nx, W, (int)nx, 0.0, Cw, m);
    P->dense->gemm(false, false, (int)nx, nb, m, -1.0, V, (int)nx, Cw, m, 1.0, W, (int)nx);
  }
  std::vector<double> G((size_t)nb * nb), w(nb), U((size_t)nb * nb);
  P->dense->gemm(true, false, nb, nb, (int)nx, 1.0, W, (int)nx, W, (int)nx, 0.0, Gd, nb);
  P->to_host(G.data(), Gd, G.size());
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < i; ++j) G[(size_t)j * nb + i] = G[(size_t)i * nb + j] = 0.5 * (G[(size_t)j * nb + i] + G[(size_t)i * nb + j]);
  if (!syev(nb, G.data(), nb, w.data(), U.data())) fail(LRPOST_EBREAKDOWN, "initial-condition basis Gram eigensolve");
  std::vector<double> T;
  int kn = 0;
  for (int i = nb - 1; i >= 0; --i) {
    if (!(w[i] > thresh_rel * scale)) continue;
    T.resize((size_t)(kn + 1) * nb);
    for (int r = 0; r < nb; ++r) T[(size_t)kn * nb + r] = U[(size_t)i * nb + r] / std::sqrt(w[i]);
    ++kn;
  }
  if (kn == 0) return 0;
  P->to_device(Td, T.data(), T.size());
  P->dense->gemm(false, false, (int)nx, kn, nb, 1.0, W, (int)nx, Td, nb, 0.0, V + (size_t)m * nx, (int)nx);
  // a second pass over the new columns against the basis and each other
  // (the normalization magnifies what the sweeps left of span(V))
  if (m > 0) {
    P->dense->gemm(true, false, m, kn, (int)nx, 1.0, V, (int)nx, V + (size_t)m * nx, (int)nx, 0.0, Cw, m);
    P->dense->gemm(false, false, (int)nx, kn, m, -1.0, V, (int)nx, Cw, m, 1.0, V + (size_t)m * nx, (int)nx);
  }
  std::vector<double> G2((size_t)kn * kn), w2(kn), U2((size_t)kn * kn);
  P->dense->gemm(true, false, kn, kn, (int)nx, 1.0, V + (size_t)m * nx, (int)nx, V + (size_t)m * nx, (int)nx, 0.0,
                 Gd, kn);
  P->to_host(G2.data(), Gd, G2.size());
  for (int i = 0; i < kn; ++i)
    for (int j = 0; j < i; ++j)
      G2[(size_t)j * kn + i] = G2[(size_t)i * kn + j] = 0.5 * (G2[(size_t)j * kn + i] + G2[(size_t)i * kn + j]);
  if (!syev(kn, G2.data(), kn, w2.data(), U2.data())) fail(LRPOST_EBREAKDOWN, "initial-condition basis Gram eigensolve");
  std::vector<double> T2;
  int k2 = 0;
  for (int i = kn - 1; i >= 0; --i) {
    if (!(w2[i] > 1e-8)) continue;
    T2.resize((size_t)(k2 + 1) * kn);
    for (int r = 0; r < kn; ++r) T2[(size_t)k2 * kn + r] = U2[(size_t)i * kn + r] / std::sqrt(w2[i]);
    ++k2;
  }
  if (k2 == 0) return 0;
  P->to_device(Td, T2.data(), T2.size());
  P->dense->gemm(false, false, (int)nx, k2, kn, 1.0, V + (size_t)m * nx, (int)nx, Td, kn, 0.0, W, (int)nx);
  LRP_HIP(hipMemcpyAsync(V + (size_t)m * nx, W, sizeof(double) * (size_t)nx * k2, hipMemcpyDeviceToDevice, P->st));
  return k2;
}

bool Problem::ic_eigensolve(double c, int k, int max_vectors, double rtol, double* values, double* vectors,
                            int* used) {
  // block size: 4 applies per step, 8 for many wanted pairs (each step's
  // space-time solves are batched, so a wider block costs little more time
  // than a narrow one on meshes too small to fill the device)
  const int kBlock = k >= 32 ? 8 : 4;
  int maxv = max_vectors > 0 ? max_vectors : std::max(8 * k, 40);
  maxv = (int)std::min<long>(maxv, nx);
  if (maxv < k) fail(LRPOST_EINVAL, "vector limit below the number of wanted eigenpairs");
  // (in mixed precision the float32 multigrid inside every apply leaves the
  // stored images G V slightly off a symmetric linear map, and the Ritz
  // residuals level off near 1e-7 of theta)
  if (!(rtol > 0.0)) rtol = desc.precision == LRPOST_MIXED ? std::max(1e-6, 0.1 * desc.trunc_tol)
                                                          : std::max(1e-8, 0.1 * desc.trunc_tol);
  DevMem V, GV, W, Cw, Gd, Td, Tm, Yd, X1, X2, th, nr;
  V.ensure(sizeof(double) * (size_t)nx * maxv);
  GV.ensure(sizeof(double) * (size_t)nx * maxv);
  W.ensure(sizeof(double) * (size_t)nx * kBlock);
  Cw.ensure(sizeof(double) * (size_t)maxv * kBlock);
  Gd.ensure(sizeof(double) * (size_t)kBlock * kBlock);
  Td.ensure(sizeof(double) * (size_t)kBlock * kBlock);
  Tm.ensure(sizeof(double) * (size_t)maxv * maxv);
  // start block: standard normal draws of the library's counter-based generator
  std::vector<double> w0((size_t)nx * kBlock);
  for (size_t i = 0; i < w0.size(); ++i) w0[i] = normal_draw(desc.seed, 11, i);
  to_device(W.as<double>(), w0.data(), w0.size());
  double* Vp = V.as<double>();
  double* GVp = GV.as<double>();
  int m = ic_extend_basis(this, Vp, 0, W.as<double>(), kBlock, Cw.as<double>(), Gd.as<double>(), Td.as<double>(),
                          1e-20);
  int last = 0;  // first column of the most recent block
  bool converged = false;
  std::vector<double> theta, Y;
  int kk = 0;
  while (m > 0) {
    ic_apply(m - last, Vp + (size_t)last * nx, GVp + (size_t)last * nx, c);
    // Rayleigh-Ritz on span(V): T = V^T G V (symmetrized), its eigenpairs
    std::vector<double> T((size_t)m * m), w(m), U((size_t)m * m);
    dense->gemm(true, false, m, m, (int)nx, 1.0, Vp, (int)nx, GVp, (int)nx, 0.0, Tm.as<double>(), m);
    to_host(T.data(), Tm.as<double>(), T.size());
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < i; ++j) T[(size_t)j * m + i] = T[(size_t)i * m + j] = 0.5 * (T[(size_t)j * m + i] + T[(size_t)i * m + j]);
    if (!syev(m, T.data(), m, w.data(), U.data())) fail(LRPOST_EBREAKDOWN, "initial-condition Ritz eigensolve");
    kk = std::min(k, m);
    theta.assign(kk, 0.0);
    Y.assign((size_t)m * kk, 0.0);
    for (int q = 0; q < kk; ++q) {
      theta[q] = w[m - 1 - q];
      std::copy(U.begin() + (size_t)(m - 1 - q) * m, U.begin() + (size_t)(m - q) * m, Y.begin() + (size_t)q * m);
    }
    // residuals ||G x - theta x|| of the wanted Ritz pairs: X1 = GV Y - (V Y) diag(theta)
    Yd.ensure(sizeof(double) * Y.size());
    X1.ensure(sizeof(double) * (size_t)nx * kk);
    X2.ensure(sizeof(double) * (size_t)nx * kk);
    th.ensure(sizeof(double) * kk);
    nr.ensure(sizeof(double) * kk);
    to_device(Yd.as<double>(), Y.data(), Y.size());
    to_device(th.as<double>(), theta.data(), theta.size());
    dense->gemm(false, false, (int)nx, kk, m, 1.0, GVp, (int)nx, Yd.as<double>(), m, 0.0, X1.as<double>(), (int)nx);
    dense->gemm(false, false, (int)nx, kk, m, 1.0, Vp, (int)nx, Yd.as<double>(), m, 0.0, X2.as<double>(), (int)nx);
    dense->dgmm_right((int)nx, kk, X2.as<double>(), (int)nx, th.as<double>(), X2.as<double>(), (int)nx);
    axpby<double>(st, nx, kk, X2.as<double>(), nx, X1.as<double>(), nx, -1.0, 1.0);
    ColGroup cg{X1.as<double>(), nr.as<double>(), nx, (int)nx, kk};
    col_sqnorms(st, 1, &cg);
    std::vector<double> rn(kk);
    to_host(rn.data(), nr.as<double>(), rn.size());
    // residuals relative to the largest Ritz value (the norm of G): every
    // apply carries the space-time solves' truncation error relative to the
    // whole operator, so a residual relative to a small theta cannot fall
    // below that error times theta_1 / theta
    double worst = 0.0;
    const double scale = std::max(std::abs(theta[0]), 1e-300);
    for (int q = 0; q < kk; ++q) worst = std::max(worst, std::sqrt(std::max(rn[q], 0.0)) / scale);
    stats.ritz_resid = worst;
    converged = kk == k && worst <= rtol;
    if (log_level > 0)
      std::fprintf(stderr,
                   "{\"ic_step\": %d, \"vectors\": %d, \"theta1\": %.10e, \"worst_rel_resid\": %.3e, "
                   "\"phase_s\": {\"prep\": %.4f, \"poles\": %.4f, \"project\": %.4f, \"projsolve\": %.4f, "
                   "\"trunc\": %.4f, \"check\": %.4f}}\n",
                   m / kBlock, m, theta.empty() ? 0.0 : theta[0], worst, phase_s[kPhPrep], phase_s[kPhPoles],
                   phase_s[kPhProject], phase_s[kPhProjSolve], phase_s[kPhTrunc], phase_s[kPhCheck]);
    if (converged || m + kBlock > maxv) break;
    // next block from G applied to the most recent one
    LRP_HIP(hipMemcpyAsync(W.as<double>(), GVp + (size_t)last * nx, sizeof(double) * (size_t)nx * (m - last),
                           hipMemcpyDeviceToDevice, st));
    const int kn = ic_extend_basis(this, Vp, m, W.as<double>(), m - last, Cw.as<double>(), Gd.as<double>(),
                                   Td.as<double>(), 1e-24);
    if (kn == 0) {  // invariant subspace: the Ritz pairs are exact
      converged = kk == k;
      break;
    }
    last = m;
    m += kn;
  }
  if (m == 0) fail(LRPOST_EBREAKDOWN, "initial-condition start block vanished");
  for (int q = 0; q < kk; ++q) values[q] = theta[q];
  for (int q = kk; q < k; ++q) values[q] = 0.0;
  LRP_HIP(hipMemsetAsync(vectors, 0, sizeof(double) * (size_t)nx * k, st));
  to_device(Yd.as<double>(), Y.data(), Y.size());
  dense->gemm(false, false, (int)nx, kk, m, 1.0, Vp, (int)nx, Yd.as<double>(), m, 0.0, vectors, (int)nx);
  stats.lanczos_steps = m / kBlock;
  if (used) *used = m;
  sync();
  return converged;
}

void Problem::ic_post_variance(double c, int k, const double* values, const double* vectors, double* out) {
  std::vector<double> w(std::max(k, 1), 0.0);
  for (int j = 0; j < k; ++j) w[j] = values[j] / (1.0 + values[j]);
  DevMem wd;
  wd.ensure(sizeof(double) * w.size());
  to_device(wd.as<double>(), w.data(), w.size());
  ic_post_var(st, nx, k, vectors, nx, wd.as<double>(), c, out);
  sync();
}

}  // namespace lrp
