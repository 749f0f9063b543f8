// Eigensolvers for the prior-preconditioned misfit Hessian G = P^{-1} H_mis.
//
// Block Lanczos with full re-orthogonalization in the P inner product: the
// low-rank Arnoldi process of Sec. 4 Algorithm 1 applied to a self-adjoint
// operator.  Every Krylov vector is a low-rank space-time vector; after each
// Hessian apply the new block is orthogonalized against all stored vectors
// (classical Gram-Schmidt, applied twice) and every linear combination is
// truncated back to low rank (Sec. 4 eq. lanczos2 and the truncation step
// that follows it).  Ritz pairs come from the symmetrized projected matrix.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace lrp {

// Counter-based normal draws: SplitMix64 (Steele, Lea, Flood 2014) for
// uniform bits, Box-Muller for the Gaussian pair.
static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
double normal_draw(uint64_t seed, uint64_t stream, uint64_t idx) {
  const uint64_t base = splitmix64(seed ^ splitmix64(stream * 0x632BE59BD9B4E019ull)) + 2 * (idx / 2);
  const double u1 = ((splitmix64(base) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((splitmix64(base + 1) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double r = std::sqrt(-2.0 * std::log(u1));
  return (idx & 1) ? r * std::sin(2.0 * M_PI * u2) : r * std::cos(2.0 * M_PI * u2);
}

// All basis vectors' spatial factors side by side on the device, so that the
// coefficients against every stored vector come from one Gram product.
struct Basis {
  Problem* P;
  DevMem A;
  long cap_cols = 0, used = 0;
  std::vector<long> off;
  std::vector<std::unique_ptr<LowRank>> vec;

  explicit Basis(Problem* p) : P(p) {}
  int size() const { return (int)vec.size(); }

  void append(std::unique_ptr<LowRank> v) {
    const long r = v->rank;
    if (used + r > cap_cols) {
      long nc = std::max<long>(2 * cap_cols, used + r + 64);
      DevMem na;
      na.ensure(sizeof(double) * (size_t)P->nx * nc);
      if (used > 0)
        LRP_HIP(hipMemcpyAsync(na.p, A.p, sizeof(double) * (size_t)P->nx * used, hipMemcpyDeviceToDevice, P->st));
      P->sync();
      A = std::move(na);
      cap_cols = nc;
    }
    if (r > 0)
      LRP_HIP(hipMemcpyAsync(A.as<double>() + (size_t)used * P->nx, v->a(), sizeof(double) * (size_t)P->nx * r,
                             hipMemcpyDeviceToDevice, P->st));
    off.push_back(used);
    used += r;
    vec.push_back(std::move(v));
  }

  // <v_k, w>_P for every stored vector k
  std::vector<double> coeffs(const LowRank& w) {
    std::vector<double> c(vec.size(), 0.0);
    if (w.rank == 0 || used == 0) return c;
    DevMem km;
    km.ensure(sizeof(double) * (size_t)P->nx * w.rank);
    P->apply_op(w.rank, w.a(), km.as<double>(), {{1.0, 1.0}});
    std::vector<double> G;
    P->gram((int)used, A.as<double>(), w.rank, km.as<double>(), G);
    const int nt = P->nt;
    for (size_t k = 0; k < vec.size(); ++k) {
      const LowRank& v = *vec[k];
      double s = 0.0;
      for (int j = 0; j < w.rank; ++j)
        for (int i = 0; i < v.rank; ++i) {
          double t = 0.0;
          for (int q = 0; q < nt; ++q) t += v.B[(size_t)i * nt + q] * w.B[(size_t)j * nt + q];
          s += G[(size_t)j * used + off[k] + i] * t;
        }
      c[k] = P->desc.alpha * P->tau * s;
    }
    return c;
  }
};

static std::unique_ptr<LowRank> copy_lr(Problem* P, const LowRank& x) {
  auto y = std::make_unique<LowRank>();
  y->resize(P->nx, P->nt, x.rank);
  if (x.rank > 0)
    LRP_HIP(hipMemcpyAsync(y->a(), x.a(), sizeof(double) * (size_t)P->nx * x.rank, hipMemcpyDeviceToDevice, P->st));
  y->B = x.B;
  return y;
}

// P-orthonormalize a block of vectors: returns the new vectors and the factor
// Rb (kout x b) with W_i = sum_l V_l Rb[l, i].
static std::vector<std::unique_ptr<LowRank>> orthonormalize_block(Problem* P, std::vector<std::unique_ptr<LowRank>>& W,
                                                                  std::vector<double>& Rb, int& kout, double tol,
                                                                  int cap) {
  const int b = (int)W.size();
  std::vector<double> Gb((size_t)b * b);
  for (int i = 0; i < b; ++i)
    for (int l = i; l < b; ++l) {
      const double g = P->p_inner(*W[i], *W[l]);
      Gb[(size_t)l * b + i] = g;
      Gb[(size_t)i * b + l] = g;
    }
  std::vector<double> w(b), U((size_t)b * b);
  if (!syev(b, Gb.data(), b, w.data(), U.data())) fail(LRPOST_EBREAKDOWN, "block Gram eigensolve failed");
  const double wmax = std::max(w[b - 1], 0.0);
  std::vector<int> keep;
  for (int j = b - 1; j >= 0; --j)
    if (wmax > 0 && w[j] > 1e-20 * wmax) keep.push_back(j);
  kout = (int)keep.size();
  Rb.assign((size_t)kout * b, 0.0);
  std::vector<std::unique_ptr<LowRank>> out;
  std::vector<const LowRank*> xs;
  for (auto& p : W) xs.push_back(p.get());
  for (int c = 0; c < kout; ++c) {
    const int j = keep[c];
    const double sw = std::sqrt(w[j]);
    std::vector<double> coef(b);
    for (int i = 0; i < b; ++i) {
      coef[i] = U[(size_t)j * b + i] / sw;
      Rb[(size_t)i * kout + c] = U[(size_t)j * b + i] * sw;
    }
    auto v = std::make_unique<LowRank>();
    P->lincomb(xs, coef, *v, tol, cap);
    // renormalize after truncation
    const double nv = std::sqrt(std::max(P->p_inner(*v, *v), 0.0));
    if (nv > 0)
      for (double& x : v->B) x /= nv;
    out.push_back(std::move(v));
  }
  return out;
}

EigResult block_lanczos(Problem* P, int k, int bsize, int max_vectors, double rtol) {
  const int nt = P->nt;
  const long nx = P->nx;
  const double tol = P->desc.trunc_tol;
  const int cap = P->desc.rank_cap;
  // seeded start block of rank-one vectors a_j (x) b_j
  std::vector<std::unique_ptr<LowRank>> W;
  {
    std::vector<double> ha((size_t)nx);
    for (int j = 0; j < bsize; ++j) {
      auto v = std::make_unique<LowRank>();
      v->resize(nx, nt, 1);
      for (long i = 0; i < nx; ++i) ha[i] = normal_draw(P->desc.seed, 2 * j, i);
      for (int t = 0; t < nt; ++t) v->B[t] = normal_draw(P->desc.seed, 2 * j + 1, t);
      P->to_device(v->a(), ha.data(), nx);
      P->sync();
      W.push_back(std::move(v));
    }
  }
  Basis basis(P);
  std::vector<double> Rb;
  int kb = 0;
  auto V = orthonormalize_block(P, W, Rb, kb, tol, cap);
  if (kb == 0) fail(LRPOST_EBREAKDOWN, "start block is zero");
  std::vector<int> block_start;  // basis index of each block's first vector
  std::vector<int> block_size;
  block_start.push_back(0);
  block_size.push_back(kb);
  for (auto& v : V) basis.append(std::move(v));
  const int mmax = max_vectors;
  std::vector<double> T((size_t)mmax * mmax, 0.0);
  EigResult res;
  std::vector<double> theta, Y;
  int m_conv = 0;
  for (int step = 0;; ++step) {
    const int j0 = block_start.back(), bj = block_size.back();
    // W = G V_j
    std::vector<std::unique_ptr<LowRank>> Wn;
    for (int i = 0; i < bj; ++i) {
      auto y = std::make_unique<LowRank>();
      P->hess_apply(*basis.vec[j0 + i], *y, true);
      Wn.push_back(std::move(y));
    }
    // full re-orthogonalization, classical Gram-Schmidt twice
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < bj; ++i) {
        std::vector<double> c = basis.coeffs(*Wn[i]);
        const int m = basis.size();
        for (int kk = 0; kk < m; ++kk) T[(size_t)(j0 + i) * mmax + kk] += c[kk];
        std::vector<const LowRank*> xs{Wn[i].get()};
        std::vector<double> cf{1.0};
        for (int kk = 0; kk < m; ++kk) {
          xs.push_back(basis.vec[kk].get());
          cf.push_back(-c[kk]);
        }
        auto out = std::make_unique<LowRank>();
        P->lincomb(xs, cf, *out, tol * 1e-1, cap);
        Wn[i] = std::move(out);
      }
    }
    const int m = basis.size();
    // Ritz values of the symmetrized projected matrix
    std::vector<double> Tm((size_t)m * m);
    for (int c = 0; c < m; ++c)
      for (int r = 0; r < m; ++r)
        Tm[(size_t)c * m + r] = 0.5 * (T[(size_t)c * mmax + r] + T[(size_t)r * mmax + c]);
    theta.assign(m, 0.0);
    Y.assign((size_t)m * m, 0.0);
    if (!syev(m, Tm.data(), m, theta.data(), Y.data())) fail(LRPOST_EBREAKDOWN, "projected eigensolve failed");
    // next block and its coupling factor
    std::vector<double> Rn;
    int kn = 0;
    auto Vn = orthonormalize_block(P, Wn, Rn, kn, tol, cap);
    // residual estimates ||G x - theta x||_P = ||Rn * Y[last block, s]||
    bool done = m >= k;
    for (int s = 0; s < std::min(k, m) && done; ++s) {
      const int col = m - 1 - s;  // descending order
      double r2 = 0.0;
      for (int l = 0; l < kn; ++l) {
        double t = 0.0;
        for (int i = 0; i < bj; ++i) t += Rn[(size_t)i * kn + l] * Y[(size_t)col * m + (j0 + i)];
        r2 += t * t;
      }
      if (std::sqrt(r2) > rtol * std::fabs(theta[col])) done = false;
    }
    res.steps = step + 1;
    m_conv = m;
    if (done || kn == 0 || m + kn > mmax) break;
    // store the coupling block below the diagonal: W_i = sum_l Vn_l Rn[l, i]
    for (int i = 0; i < bj; ++i)
      for (int l = 0; l < kn; ++l) T[(size_t)(j0 + i) * mmax + (m + l)] = Rn[(size_t)i * kn + l];
    block_start.push_back(m);
    block_size.push_back(kn);
    for (auto& v : Vn) basis.append(std::move(v));
  }
  P->stats.lanczos_steps = res.steps;
  // Ritz vectors of the k largest Ritz values
  const int m = m_conv;
  const int kk = std::min(k, m);
  std::vector<const LowRank*> xs;
  for (int i = 0; i < m; ++i) xs.push_back(basis.vec[i].get());
  for (int s = 0; s < kk; ++s) {
    const int col = m - 1 - s;
    res.lambda.push_back(theta[col]);
    std::vector<double> coef(m);
    for (int i = 0; i < m; ++i) coef[i] = Y[(size_t)col * m + i];
    auto v = std::make_unique<LowRank>();
    P->lincomb(xs, coef, *v, tol, cap);
    const double nv = std::sqrt(std::max(P->p_inner(*v, *v), 0.0));
    if (nv > 0)
      for (double& x : v->B) x /= nv;
    res.vecs.push_back(std::move(v));
  }
  return res;
}

}  // namespace lrp
