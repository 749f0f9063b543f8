// Eigensolvers for the prior-preconditioned misfit Hessian G = P^{-1} H_mis.
//
// Block Lanczos with full re-orthogonalization in the P inner product: the
// low-rank Arnoldi process of Sec. 4 Algorithm 1 applied to a self-adjoint
// operator (the truncated applies break exact symmetry; the projected matrix
// is symmetrized before its eigensolve).
//
// Storage: every Krylov vector is a low-rank space-time vector whose spatial
// factor lies in one shared spatial basis U (nx x s) with U^T (K+M) U = I,
// so that v_k = U C_k B_k^T with a small coefficient core C_k (s x r_k) and
// temporal factor B_k (nt x r_k).  A new apply output is absorbed by
// projecting its spatial factor on U (classical Gram-Schmidt, twice),
// truncating the remainder, sweeping its normalized directions against U
// once more and appending them to U.
// Inner products, Gram-Schmidt subtraction (the dot products and updates of
// Algorithm 1; the factor concatenation of eq. lanczos2) and Ritz
// combinations then act on the cores only: dense s x nt cores formed by
// GEMMs and truncated through a small SVD.  Only absorbing and materializing
// spatial factors touch nx-sized data.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <optional>

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

// A vector in coefficient form: v = U C B^T with C (s x r, leading
// dimension s) and B (nt x r), both on the device.
struct CVec {
  int s = 0, r = 0;
  DevMem C, B;
};

class SharedBasis {
 public:
  SharedBasis(Problem* p, int s_reserve, int rcap_total)
      : P(p), nx(p->nx), nt(p->nt), scale(p->desc.alpha * p->tau) {
    grow_U(std::max(std::min<long>(s_reserve, nx), (long)1));
    grow_all(std::max(rcap_total, 64));
  }

  Problem* P;
  long nx;
  int nt;
  double scale;  // alpha * tau: <X, Y>_P = scale * <X, (I kron (K+M)) Y>
  DevMem U;
  int s = 0, s_cap = 0;
  // basis vectors: cores padded to s_cap rows in C_all, temporal factors in B_all
  DevMem C_all, B_all;
  int used = 0, all_cap = 0;
  std::vector<int> off, rk;
  DevMem work1, work2, work3, wev, eye, eye_nt;
  DevMem ipw, ipo;  // inner products: Gram pairs, row-wise dot products

  int size() const { return (int)off.size(); }

  void grow_U(long need) {
    if (need <= s_cap) return;
    long nc = std::max<long>(need, 2L * s_cap);
    nc = std::min<long>(nc, nx);
    if (nc < need) fail(LRPOST_EINVAL, "shared spatial basis exceeds the number of nodes");
    DevMem nu;
    nu.ensure(sizeof(double) * (size_t)nx * nc);
    if (s > 0)
      LRP_HIP(hipMemcpyAsync(nu.p, U.p, sizeof(double) * (size_t)nx * s, hipMemcpyDeviceToDevice, P->st));
    if (all_cap > 0) {
      DevMem nC;
      nC.ensure(sizeof(double) * (size_t)nc * all_cap);
      LRP_HIP(hipMemsetAsync(nC.p, 0, sizeof(double) * (size_t)nc * all_cap, P->st));
      if (used > 0)
        LRP_HIP(hipMemcpy2DAsync(nC.p, sizeof(double) * nc, C_all.p, sizeof(double) * s_cap, sizeof(double) * s_cap,
                                 used, hipMemcpyDeviceToDevice, P->st));
      P->sync();
      C_all = std::move(nC);
    }
    P->sync();
    U = std::move(nu);
    s_cap = (int)nc;
  }

  void grow_all(int need) {
    if (need <= all_cap) return;
    const int nc = std::max(need, 2 * all_cap);
    DevMem nC, nB;
    nC.ensure(sizeof(double) * (size_t)s_cap * nc);
    nB.ensure(sizeof(double) * (size_t)nt * nc);
    LRP_HIP(hipMemsetAsync(nC.p, 0, sizeof(double) * (size_t)s_cap * nc, P->st));
    if (used > 0) {
      LRP_HIP(hipMemcpyAsync(nC.p, C_all.p, sizeof(double) * (size_t)s_cap * used, hipMemcpyDeviceToDevice, P->st));
      LRP_HIP(hipMemcpyAsync(nB.p, B_all.p, sizeof(double) * (size_t)nt * used, hipMemcpyDeviceToDevice, P->st));
    }
    P->sync();
    C_all = std::move(nC);
    B_all = std::move(nB);
    all_cap = nc;
  }

  // Express a low-rank vector in the basis, extending U by the directions of
  // its spatial factor outside span(U) (remainder truncated at a tenth of tol
  // relative to the vector's norm).  Returns the truncated core.
  CVec absorb(const LowRank& w, double tol, int cap, bool truncate_out = true) {
    CVec out;
    out.s = s;
    const int rw = w.rank;
    if (rw == 0) return out;
    DevMem R, KR;
    R.ensure(sizeof(double) * (size_t)nx * rw);
    KR.ensure(sizeof(double) * (size_t)nx * rw);
    LRP_HIP(hipMemcpyAsync(R.p, w.a(), sizeof(double) * (size_t)nx * rw, hipMemcpyDeviceToDevice, P->st));
    // ||w||^2 in the (K+M)-weighted Frobenius norm (without alpha tau)
    P->apply_op(rw, R.as<double>(), KR.as<double>(), {{1.0, 1.0}});
    std::vector<double> Gw;
    P->gram(rw, R.as<double>(), rw, KR.as<double>(), Gw);
    double wn2 = 0.0;
    for (int j = 0; j < rw; ++j)
      for (int i = 0; i < rw; ++i) {
        double t = 0.0;
        for (int k = 0; k < nt; ++k) t += w.B[(size_t)i * nt + k] * w.B[(size_t)j * nt + k];
        wn2 += Gw[(size_t)j * rw + i] * t;
      }
    const double wnorm = std::sqrt(std::max(wn2, 0.0));
    // coefficients on U, classical Gram-Schmidt twice: G = U^T (K+M) R
    const int s0 = s;
    // G, G2 (s0 x rw each), then Cq and its second-pass term (s0 x rq each, rq <= rw)
    work1.ensure(sizeof(double) * (size_t)std::max(s0, 1) * rw * 4);
    double* G = work1.as<double>();
    double* G2 = G + (size_t)std::max(s0, 1) * rw;
    for (int pass = 0; pass < 2 && s0 > 0; ++pass) {
      if (pass > 0) P->apply_op(rw, R.as<double>(), KR.as<double>(), {{1.0, 1.0}});
      double* dst = pass == 0 ? G : G2;
      P->gram_dev(s0, U.as<double>(), rw, KR.as<double>(), dst);
      P->proj_dev(s0, U.as<double>(), dst, s0, rw, R.as<double>(), 1.0, -1.0);
      if (pass > 0) axpby<double>(P->st, (long)s0 * rw, 1, G2, (long)s0 * rw, G, (long)s0 * rw, 1.0, 1.0);
    }
    // remainder R w.B^T: truncated relative to ||w||, (K+M)-orthonormal spatial factor
    LowRank rem;
    rem.nx = nx;
    rem.nt = nt;
    rem.rank = rw;
    rem.A = std::move(R);
    rem.B = w.B;
    P->truncate(rem, 0.1 * tol, cap, 2, wnorm, true);
    const int rq = rem.rank;  // truncated remainder = Q Bq^T, Q (K+M)-orthonormal
    std::vector<double> Bq = rem.B;
    // The remainder can lie many orders of magnitude below ||w||, and the
    // rounding left by the sweeps above is of order u ||w||: normalizing it
    // would amplify that leak by ||w|| / ||remainder|| and U would lose its
    // orthonormality step by step.  So the normalized directions are swept
    // against U once more (twice), the removed components Cq go to the core
    // (Q = U Cq + Q'), and Q' is re-orthonormalized through the eigenpairs
    // of its Gram matrix (directions that were mostly inside span(U) drop).
    double* Cq = nullptr;
    if (rq > 0 && s0 > 0) {
      Cq = G + (size_t)s0 * rw * 2;
      double* C2 = Cq + (size_t)s0 * rq;
      for (int pass = 0; pass < 2; ++pass) {
        P->apply_op(rq, rem.a(), KR.as<double>(), {{1.0, 1.0}});
        double* dst = pass == 0 ? Cq : C2;
        P->gram_dev(s0, U.as<double>(), rq, KR.as<double>(), dst);
        P->proj_dev(s0, U.as<double>(), dst, s0, rq, rem.a(), 1.0, -1.0);
        if (pass > 0) axpby<double>(P->st, (long)s0 * rq, 1, C2, (long)s0 * rq, Cq, (long)s0 * rq, 1.0, 1.0);
      }
      P->apply_op(rq, rem.a(), KR.as<double>(), {{1.0, 1.0}});
      std::vector<double> Gq;
      P->gram(rq, rem.a(), rq, KR.as<double>(), Gq);
      std::vector<double> e(rq), V((size_t)rq * rq);
      if (!syev(rq, Gq.data(), rq, e.data(), V.data())) fail(LRPOST_EBREAKDOWN, "basis extension eigensolve failed");
      std::vector<int> keep;
      for (int j = rq - 1; j >= 0; --j)
        if (e[j] > 0.1) keep.push_back(j);
      const int rk2 = (int)keep.size();
      std::vector<double> Tq((size_t)rq * std::max(rk2, 1)), Bn((size_t)nt * std::max(rk2, 1), 0.0);
      for (int c = 0; c < rk2; ++c) {
        const double se = std::sqrt(e[keep[c]]);
        const double* v = V.data() + (size_t)keep[c] * rq;
        for (int i = 0; i < rq; ++i) Tq[(size_t)c * rq + i] = v[i] / se;
        for (int i = 0; i < rq; ++i)
          for (int t = 0; t < nt; ++t) Bn[(size_t)c * nt + t] += Bq[(size_t)i * nt + t] * v[i] * se;
      }
      LowRank q2;
      q2.resize(nx, nt, rk2);
      if (rk2 > 0) P->proj(rq, rem.a(), Tq, rk2, q2.a(), 0.0);
      rem.A = std::move(q2.A);
      rem.B.assign(Bn.begin(), Bn.begin() + (size_t)nt * rk2);
      rem.rank = rk2;
    }
    const int rn = rem.rank;
    grow_U((long)s0 + rn);
    if (rn > 0)
      LRP_HIP(hipMemcpyAsync(U.as<double>() + (size_t)s0 * nx, rem.a(), sizeof(double) * (size_t)nx * rn,
                             hipMemcpyDeviceToDevice, P->st));
    s = s0 + rn;
    // core S (s x nt) = [G w.B^T + Cq Bq^T ; rem.B^T]
    work2.ensure(sizeof(double) * ((size_t)s * nt + (size_t)nt * (rw + rq + rn) + 64));
    double* S = work2.as<double>();
    double* Bd = S + (size_t)s * nt;  // nt x rw, then nt x rq, then nt x rn
    double* Bqd = Bd + (size_t)nt * rw;
    double* Bnd = Bqd + (size_t)nt * rq;
    P->to_device(Bd, w.B.data(), (size_t)nt * rw);
    if (Cq) P->to_device(Bqd, Bq.data(), (size_t)nt * rq);
    if (rn > 0) P->to_device(Bnd, rem.B.data(), (size_t)nt * rn);
    if (s0 > 0) P->dense->gemm(false, true, s0, nt, rw, 1.0, G, s0, Bd, nt, 0.0, S, s);
    if (Cq) P->dense->gemm(false, true, s0, nt, rq, 1.0, Cq, s0, Bqd, nt, 1.0, S, s);
    if (rn > 0) {
      // bottom rn rows: rem.B^T, written as I * rem.B^T
      eye.ensure(sizeof(double) * (size_t)rn * rn);
      std::vector<double> id((size_t)rn * rn, 0.0);
      for (int i = 0; i < rn; ++i) id[(size_t)i * rn + i] = 1.0;
      P->to_device(eye.as<double>(), id.data(), id.size());
      P->dense->gemm(false, true, rn, nt, rn, 1.0, eye.as<double>(), rn, Bnd, nt, 0.0, S + s0, s);
    }
    return truncate_out ? truncate_core(S, s, s, tol, cap) : dense_core(S, s);
  }

  // A dense core S (rows x nt, leading dimension rows) as a vector in
  // coefficient form without truncation: C = S, B = I.
  CVec dense_core(const double* S, int rows) {
    CVec out;
    out.s = rows;
    out.r = nt;
    out.C.ensure(sizeof(double) * (size_t)std::max(rows, 1) * nt);
    out.B.ensure(sizeof(double) * (size_t)nt * nt);
    if (!eye_nt.p) {
      std::vector<double> id((size_t)nt * nt, 0.0);
      for (int i = 0; i < nt; ++i) id[(size_t)i * nt + i] = 1.0;
      eye_nt.ensure(sizeof(double) * id.size());
      P->to_device(eye_nt.as<double>(), id.data(), id.size());
    }
    if (rows > 0)
      LRP_HIP(hipMemcpyAsync(out.C.p, S, sizeof(double) * (size_t)rows * nt, hipMemcpyDeviceToDevice, P->st));
    LRP_HIP(hipMemcpyAsync(out.B.p, eye_nt.p, sizeof(double) * (size_t)nt * nt, hipMemcpyDeviceToDevice, P->st));
    return out;
  }

  // Truncate a dense core S (rows x nt, leading dimension lds) to rank <= cap
  // at relative Frobenius tolerance tol.  Below 1e-7 the SVD runs on the host
  // by one-sided Jacobi (relative accuracy of small singular values);
  // otherwise through the eigenpairs of the smaller of S S^T and S^T S on
  // the device.
  CVec truncate_core(const double* S, int rows, int lds, double tol, int cap) {
    return std::move(truncate_cores(S, 1, 0, rows, lds, tol, cap)[0]);
  }

  // The same for `count` cores S + b stride of one shape, with the
  // eigenproblems of their Gram matrices solved as one batch.
  std::vector<CVec> truncate_cores(const double* S, int count, long stride, int rows, int lds, double tol, int cap) {
    std::vector<CVec> outs(count);
    for (auto& o : outs) o.s = rows;
    if (rows == 0 || count == 0) return outs;
    std::vector<double> sv;
    double tail = 0.0;
    if (tol < 1e-7) {
      for (int b = 0; b < count; ++b) {
        CVec& out = outs[b];
        std::vector<double> Sh((size_t)rows * nt);
        P->to_host_block(Sh.data(), S + b * stride, rows, nt, lds);
        std::vector<double> Us, Vs;
        svd(rows, nt, Sh.data(), rows, sv, Us, Vs);
        const int r = truncation_rank(sv, tol, cap, &tail);
        out.r = r;
        out.C.ensure(sizeof(double) * (size_t)rows * std::max(r, 1));
        out.B.ensure(sizeof(double) * (size_t)nt * std::max(r, 1));
        if (r > 0) {
          std::vector<double> Cm((size_t)rows * r);
          for (int j = 0; j < r; ++j)
            for (int i = 0; i < rows; ++i) Cm[(size_t)j * rows + i] = Us[(size_t)j * rows + i] * sv[j];
          P->to_device(out.C.as<double>(), Cm.data(), Cm.size());
          P->to_device(out.B.as<double>(), Vs.data(), (size_t)nt * r);
        }
      }
      P->sync();
      return outs;
    }
    // Gram matrix of the smaller side: S S^T (rows x rows) when rows < nt,
    // else S^T S (nt x nt)
    const bool left = rows < nt;
    const int g = left ? rows : nt;
    const size_t gsz = (size_t)g * g;
    work3.ensure(sizeof(double) * (gsz * count + (size_t)g * count + 64));
    double* Gt = work3.as<double>();
    double* w = Gt + gsz * count;
    if (left)
      P->dense->gemm_strided_batched(false, true, rows, rows, nt, 1.0, S, lds, stride, S, lds, stride, 0.0, Gt, g,
                                     (long)gsz, count);
    else
      P->dense->gemm_strided_batched(true, false, nt, nt, rows, 1.0, S, lds, stride, S, lds, stride, 0.0, Gt, g,
                                     (long)gsz, count);
    P->dense->syevd_batched(g, Gt, g, (long)gsz, w, g, count, wev);
    std::vector<double> wh((size_t)g * count);
    P->to_host(wh.data(), w, wh.size());
    for (int b = 0; b < count; ++b) {
      CVec& out = outs[b];
      sv.assign(g, 0.0);
      for (int c = 0; c < g; ++c) sv[c] = std::sqrt(std::max(wh[(size_t)b * g + g - 1 - c], 0.0));
      const int r = truncation_rank(sv, tol, cap, &tail);
      out.r = r;
      out.C.ensure(sizeof(double) * (size_t)rows * std::max(r, 1));
      out.B.ensure(sizeof(double) * (size_t)nt * std::max(r, 1));
      if (r == 0) continue;
      // eigenvectors of the r largest eigenvalues
      const double* Er = Gt + gsz * b + (size_t)(g - r) * g;
      if (left) {
        // S ~ U_r U_r^T S: C = U_r, B = S^T U_r
        LRP_HIP(hipMemcpyAsync(out.C.p, Er, sizeof(double) * (size_t)rows * r, hipMemcpyDeviceToDevice, P->st));
        P->dense->gemm(true, false, nt, r, rows, 1.0, S + b * stride, lds, Er, g, 0.0, out.B.as<double>(), nt);
      } else {
        // S ~ S V_r V_r^T: C = S V_r, B = V_r
        P->dense->gemm(false, false, rows, r, nt, 1.0, S + b * stride, lds, Er, g, 0.0, out.C.as<double>(), rows);
        LRP_HIP(hipMemcpyAsync(out.B.p, Er, sizeof(double) * (size_t)nt * r, hipMemcpyDeviceToDevice, P->st));
      }
    }
    P->sync();
    return outs;
  }

  // Dense core S (s x nt) = sum_t tc[t] C_t B_t^T over temporaries plus
  // sum_k coef[k] C_k B_k^T over stored vectors.
  void combine(const std::vector<const CVec*>& tv, const std::vector<double>& tc, const std::vector<double>& coef,
               double* S) {
    LRP_HIP(hipMemsetAsync(S, 0, sizeof(double) * (size_t)s * nt, P->st));
    for (size_t t = 0; t < tv.size(); ++t) {
      const CVec& v = *tv[t];
      if (v.r == 0 || tc[t] == 0.0) continue;
      P->dense->gemm(false, true, v.s, nt, v.r, tc[t], v.C.as<double>(), v.s, v.B.as<double>(), nt, 1.0, S, s);
    }
    if (!coef.empty() && used > 0) {
      std::vector<double> ce((size_t)used, 0.0);
      bool any = false;
      for (int k = 0; k < size(); ++k)
        for (int c = 0; c < rk[k]; ++c) {
          ce[(size_t)off[k] + c] = coef[k];
          any = any || coef[k] != 0.0;
        }
      if (any) {
        work1.ensure(sizeof(double) * ((size_t)s_cap * used + used + 64));
        double* Cs = work1.as<double>();
        double* cd = Cs + (size_t)s_cap * used;
        P->to_device(cd, ce.data(), ce.size());
        P->dense->dgmm_right(s, used, C_all.as<double>(), s_cap, cd, Cs, s_cap);
        P->dense->gemm(false, true, s, nt, used, 1.0, Cs, s_cap, B_all.as<double>(), nt, 1.0, S, s);
      }
    }
  }

  // <v_k, x>_P for every stored vector k, for each x in xs, with one
  // read-back.  With U (K+M)-orthonormal, <U C_k B_k^T, U C_x B_x^T>_P =
  // scale * sum (C_k^T C_x) .* (B_k^T B_x): per x the products G1 = C_all^T C_x
  // and G2 = B_all^T B_x (used x r) and their row-wise dot products (one value
  // per stored column) on the device; on the host the sums over each stored
  // vector's columns.
  std::vector<std::vector<double>> inner_all_many(const std::vector<const CVec*>& xs) {
    const int nxs = (int)xs.size();
    std::vector<std::vector<double>> cs(nxs, std::vector<double>(size(), 0.0));
    if (used == 0 || nxs == 0) return cs;
    int rmax = 0;
    for (const CVec* x : xs) rmax = std::max(rmax, x->r);
    if (rmax == 0) return cs;
    ipw.ensure(sizeof(double) * (size_t)used * rmax * 2);
    ipo.ensure(sizeof(double) * (size_t)used * nxs);
    double* G1 = ipw.as<double>();
    double* G2 = G1 + (size_t)used * rmax;
    double* h = ipo.as<double>();
    for (int a = 0; a < nxs; ++a) {
      const CVec& x = *xs[a];
      if (x.r == 0) {
        LRP_HIP(hipMemsetAsync(h + (size_t)a * used, 0, sizeof(double) * used, P->st));
        continue;
      }
      const int sm = std::min(x.s, s);
      P->dense->gemm(true, false, used, x.r, sm, 1.0, C_all.as<double>(), s_cap, x.C.as<double>(), x.s, 0.0, G1, used);
      P->dense->gemm(true, false, used, x.r, nt, 1.0, B_all.as<double>(), nt, x.B.as<double>(), nt, 0.0, G2, used);
      row_dot(P->st, used, x.r, G1, used, G2, used, h + (size_t)a * used);
    }
    std::vector<double> hh((size_t)used * nxs);
    P->to_host(hh.data(), h, hh.size());
    for (int a = 0; a < nxs; ++a)
      for (int k = 0; k < size(); ++k) {
        double acc = 0.0;
        for (int c2 = 0; c2 < rk[k]; ++c2) acc += hh[(size_t)a * used + off[k] + c2];
        cs[a][k] = scale * acc;
      }
    return cs;
  }
  std::vector<double> inner_all(const CVec& x) { return std::move(inner_all_many({&x})[0]); }

  // <x, y>_P for each pair, with one read-back (row-wise dot products of
  // x.C^T y.C and x.B^T y.B on the device, their sum on the host).
  std::vector<double> inner_pairs(const std::vector<std::pair<const CVec*, const CVec*>>& pr) {
    const int np = (int)pr.size();
    std::vector<double> out(np, 0.0);
    std::vector<size_t> ho(np + 1, 0);
    size_t wmax = 0;
    for (int a = 0; a < np; ++a) {
      const CVec &x = *pr[a].first, &y = *pr[a].second;
      const bool live = x.r > 0 && y.r > 0;
      ho[a + 1] = ho[a] + (live ? x.r : 0);
      if (live) wmax = std::max(wmax, (size_t)x.r * y.r);
    }
    if (ho[np] == 0) return out;
    ipw.ensure(sizeof(double) * wmax * 2);
    ipo.ensure(sizeof(double) * ho[np]);
    double* G1 = ipw.as<double>();
    double* G2 = G1 + wmax;
    double* h = ipo.as<double>();
    for (int a = 0; a < np; ++a) {
      const CVec &x = *pr[a].first, &y = *pr[a].second;
      if (ho[a + 1] == ho[a]) continue;
      const int sm = std::min(x.s, y.s);
      P->dense->gemm(true, false, x.r, y.r, sm, 1.0, x.C.as<double>(), x.s, y.C.as<double>(), y.s, 0.0, G1, x.r);
      P->dense->gemm(true, false, x.r, y.r, nt, 1.0, x.B.as<double>(), nt, y.B.as<double>(), nt, 0.0, G2, x.r);
      row_dot(P->st, x.r, y.r, G1, x.r, G2, x.r, h + ho[a]);
    }
    std::vector<double> hh(ho[np]);
    P->to_host(hh.data(), h, hh.size());
    for (int a = 0; a < np; ++a) {
      double acc = 0.0;
      for (size_t i = ho[a]; i < ho[a + 1]; ++i) acc += hh[i];
      out[a] = scale * acc;
    }
    return out;
  }
  double inner(const CVec& x, const CVec& y) { return inner_pairs({{&x, &y}})[0]; }

  // each core of vs scaled to unit P-norm (one read-back for all)
  void normalize(std::vector<CVec>& vs) {
    std::vector<std::pair<const CVec*, const CVec*>> pr;
    for (auto& v : vs) pr.push_back({&v, &v});
    const std::vector<double> n2 = inner_pairs(pr);
    for (size_t i = 0; i < vs.size(); ++i) {
      const double nv = std::sqrt(std::max(n2[i], 0.0));
      if (nv > 0) P->dense->scal(nt * vs[i].r, 1.0 / nv, vs[i].B.as<double>());
    }
  }

  void append(const CVec& v) {
    grow_all(used + v.r);
    if (v.r > 0) {
      LRP_HIP(hipMemcpy2DAsync(C_all.as<double>() + (size_t)used * s_cap, sizeof(double) * s_cap, v.C.p,
                               sizeof(double) * v.s, sizeof(double) * v.s, v.r, hipMemcpyDeviceToDevice, P->st));
      LRP_HIP(hipMemcpyAsync(B_all.as<double>() + (size_t)used * nt, v.B.p, sizeof(double) * (size_t)nt * v.r,
                             hipMemcpyDeviceToDevice, P->st));
    }
    off.push_back(used);
    rk.push_back(v.r);
    used += v.r;
  }

  // Spatial factor U C (nx x r) and host temporal factor.
  void materialize(const CVec& v, LowRank& out) {
    out.resize(nx, nt, v.r);
    if (v.r == 0) return;
    P->proj_dev(v.s, U.as<double>(), v.C.as<double>(), v.s, v.r, out.a(), 0.0);
    P->to_host(out.B.data(), v.B.as<double>(), (size_t)nt * v.r);
  }

  // The stored vectors k0 .. k0 + count - 1 as low-rank vectors: spatial
  // factors U C_k in one grouped projection, temporal factors (adjacent in
  // B_all) in one read-back.
  void materialize_block(int k0, int count, std::vector<LowRank>& outs) {
    std::vector<ProjGroup> pg;
    int cols = 0;
    for (int i = 0; i < count; ++i) {
      const int k = k0 + i;
      outs[i].resize(nx, nt, rk[k]);
      cols += rk[k];
      if (rk[k] > 0)
        pg.push_back(ProjGroup{U.as<double>(), C_all.as<double>() + (size_t)off[k] * s_cap, outs[i].a(), outs[i].a(),
                               nx, nx, nx, s_cap, s, rk[k]});
    }
    if (cols == 0) return;
    if (s > 0) P->proj_dev_grouped(pg, 1.0, 0.0);
    std::vector<double> Bh((size_t)nt * cols);
    P->to_host(Bh.data(), B_all.as<double>() + (size_t)off[k0] * nt, Bh.size());
    size_t o = 0;
    for (int i = 0; i < count; ++i) {
      const size_t len = (size_t)nt * rk[k0 + i];
      std::copy(Bh.begin() + o, Bh.begin() + o + len, outs[i].B.begin());
      o += len;
    }
  }

  CVec stored(int k) {
    CVec v;
    v.s = s;
    v.r = rk[k];
    v.C.ensure(sizeof(double) * (size_t)s * std::max(v.r, 1));
    v.B.ensure(sizeof(double) * (size_t)nt * std::max(v.r, 1));
    if (v.r > 0) {
      LRP_HIP(hipMemcpy2DAsync(v.C.p, sizeof(double) * s, C_all.as<double>() + (size_t)off[k] * s_cap,
                               sizeof(double) * s_cap, sizeof(double) * s, v.r, hipMemcpyDeviceToDevice, P->st));
      LRP_HIP(hipMemcpyAsync(v.B.p, B_all.as<double>() + (size_t)off[k] * nt, sizeof(double) * (size_t)nt * v.r,
                             hipMemcpyDeviceToDevice, P->st));
    }
    return v;
  }
};

// P-orthonormalize a block of temporaries: returns the new cores and the
// factor Rb (kout x b) with W_i = sum_l V_l Rb[l, i].  Directions whose
// P-norm is at most abs_drop are deflated: after the truncated applies and
// the Gram-Schmidt sweep they carry only truncation noise (a block direction
// of a converged invariant subspace).
static std::vector<CVec> orthonormalize_block(SharedBasis& sb, std::vector<CVec>& W, std::vector<double>& Rb,
                                              int& kout, double tol, int cap, double abs_drop) {
  Problem* P = sb.P;
  const int b = (int)W.size();
  std::vector<double> Gb((size_t)b * b);
  {
    std::vector<std::pair<const CVec*, const CVec*>> pr;
    for (int i = 0; i < b; ++i)
      for (int l = i; l < b; ++l) pr.push_back({&W[i], &W[l]});
    const std::vector<double> g = sb.inner_pairs(pr);
    size_t a = 0;
    for (int i = 0; i < b; ++i)
      for (int l = i; l < b; ++l, ++a) {
        Gb[(size_t)l * b + i] = g[a];
        Gb[(size_t)i * b + l] = g[a];
      }
  }
  std::vector<double> w(b), U((size_t)b * b);
  if (!syev(b, Gb.data(), b, w.data(), U.data())) fail(LRPOST_EBREAKDOWN, "block Gram eigensolve failed");
  const double wmax = std::max(w[b - 1], 0.0);
  std::vector<int> keep;
  for (int j = b - 1; j >= 0; --j)
    if (wmax > 0 && w[j] > 1e-20 * wmax && w[j] > abs_drop * abs_drop) keep.push_back(j);
  kout = (int)keep.size();
  if (P->log_level > 1) {
    std::fprintf(stderr, "{\"block_norms\": [");
    for (int j = b - 1; j >= 0; --j) std::fprintf(stderr, "%s%.4e", j == b - 1 ? "" : ", ", std::sqrt(std::max(w[j], 0.0)));
    std::fprintf(stderr, "], \"abs_drop\": %.3e, \"kept\": %d}\n", abs_drop, kout);
  }
  Rb.assign((size_t)kout * b, 0.0);
  std::vector<CVec> out;
  std::vector<const CVec*> tv;
  for (auto& x : W) tv.push_back(&x);
  // the kout new directions' cores are formed side by side and truncated as one batch
  DevMem Sbuf;
  const size_t slot = (size_t)std::max(sb.s, 1) * sb.nt;
  Sbuf.ensure(sizeof(double) * slot * std::max(kout, 1));
  for (int c = 0; c < kout; ++c) {
    const int j = keep[c];
    const double sw = std::sqrt(w[j]);
    std::vector<double> coef(b);
    for (int i = 0; i < b; ++i) {
      coef[i] = U[(size_t)j * b + i] / sw;
      Rb[(size_t)i * kout + c] = U[(size_t)j * b + i] * sw;
    }
    sb.combine(tv, coef, {}, Sbuf.as<double>() + c * slot);
  }
  auto vs = sb.truncate_cores(Sbuf.as<double>(), kout, (long)slot, sb.s, sb.s, tol, cap);
  sb.normalize(vs);
  for (auto& v : vs) out.push_back(std::move(v));
  return out;
}

EigResult block_lanczos(Problem* P, int k, int bsize, int max_vectors, double rtol, LanczosSolve* lin) {
  const int nt = P->nt;
  const long nx = P->nx;
  const double tol = P->desc.trunc_tol;
  const int cap = P->desc.rank_cap;
  const long s_reserve = std::min<long>(nx, (long)std::min(max_vectors, lin ? max_vectors : 4 * k + 16) * 16 + 64);
  SharedBasis sb(P, (int)s_reserve, std::max(max_vectors * cap / 2, 64));
  using clk = std::chrono::steady_clock;
  const auto t_start = clk::now();
  P->phase_s.fill(0.0);
  double t_apply = 0.0, t_orth = 0.0;
  // seeded start block of rank-one vectors a_j (x) b_j (in the linear-solve
  // mode the right-hand side first, then bsize - 1 of them)
  std::vector<CVec> W;
  if (lin) {
    if (!lin->rhs || lin->rhs->rank == 0) fail(LRPOST_EINVAL, "zero right-hand side");
    W.push_back(sb.absorb(*lin->rhs, tol, cap));
  }
  {
    std::vector<double> ha((size_t)nx);
    for (int j = lin ? 1 : 0; j < bsize; ++j) {
      LowRank v;
      v.resize(nx, nt, 1);
      for (long i = 0; i < nx; ++i) ha[i] = normal_draw(P->desc.seed, 2 * j, i);
      for (int t = 0; t < nt; ++t) v.B[t] = normal_draw(P->desc.seed, 2 * j + 1, t);
      P->to_device(v.a(), ha.data(), nx);
      P->sync();
      W.push_back(sb.absorb(v, tol, cap));
    }
  }
  std::vector<double> Rb;
  int kb = 0;
  auto V = orthonormalize_block(sb, W, Rb, kb, tol, cap, 0.0);
  if (kb == 0) fail(LRPOST_EBREAKDOWN, "start block is zero");
  // linear-solve mode: the right-hand side in the P-orthonormal basis (its
  // coefficients on the first block; zero on every later vector)
  std::vector<double> g0;
  double gnorm = 0.0;
  if (lin) {
    g0.assign(kb, 0.0);
    for (int c = 0; c < kb; ++c) {
      g0[c] = Rb[c];  // W_0 = sum_c V_c Rb[c, 0]
      gnorm += g0[c] * g0[c];
    }
    gnorm = std::sqrt(gnorm);
  }
  std::vector<double> zsol;
  std::vector<int> block_start{0}, block_size{kb};
  for (auto& v : V) sb.append(v);
  const int mmax = max_vectors;
  std::vector<double> T((size_t)mmax * mmax, 0.0);
  EigResult res;
  std::vector<double> theta, Y;
  int m_conv = 0;
  double last_worst = -1.0;
  DevMem Sbuf;
  for (int step = 0;; ++step) {
    const int j0 = block_start.back(), bj = block_size.back();
    // W = G V_j
    auto t0 = clk::now();
    std::vector<LowRank> outs(bj), xin(bj);
    std::vector<const LowRank*> px;
    std::vector<LowRank*> po;
    {
      Problem::PhaseTimer pt(P, Problem::kPhMaterialize);
      sb.materialize_block(j0, bj, xin);
      for (int i = 0; i < bj; ++i) {
        px.push_back(&xin[i]);
        po.push_back(&outs[i]);
      }
    }
    P->hess_apply_batch(px, po, true);
    xin.clear();
    auto t1 = clk::now();
    t_apply += std::chrono::duration<double>(t1 - t0).count();
    std::vector<CVec> Wn;
    // the apply outputs and both sweeps' results stay dense cores (no
    // truncation): the block orthonormalization below truncates the new
    // directions once
    {
      Problem::PhaseTimer pt(P, Problem::kPhAbsorb);
      for (int i = 0; i < bj; ++i) Wn.push_back(sb.absorb(outs[i], tol, cap, false));
    }
    outs.clear();
    std::optional<Problem::PhaseTimer> ptr(std::in_place, P, Problem::kPhReorth);
    // full re-orthogonalization, classical Gram-Schmidt twice, on the cores
    const size_t slot = (size_t)std::max(sb.s, 1) * nt;
    for (int pass = 0; pass < 2; ++pass) {
      Sbuf.ensure(sizeof(double) * slot);
      std::vector<const CVec*> pw;
      for (int i = 0; i < bj; ++i) pw.push_back(&Wn[i]);
      std::vector<std::vector<double>> cs = sb.inner_all_many(pw);
      for (int i = 0; i < bj; ++i) {
        std::vector<double>& c = cs[i];
        const int m = sb.size();
        for (int kk = 0; kk < m; ++kk) T[(size_t)(j0 + i) * mmax + kk] += c[kk];
        for (double& x : c) x = -x;
        sb.combine({&Wn[i]}, {1.0}, c, Sbuf.as<double>());
        Wn[i] = sb.dense_core(Sbuf.as<double>(), sb.s);
      }
    }
    ptr.reset();
    const int m = sb.size();
    // Ritz values of the symmetrized projected matrix
    std::vector<double> Tm((size_t)m * m);
    for (int c = 0; c < m; ++c)
      for (int r = 0; r < m; ++r) Tm[(size_t)c * m + r] = 0.5 * (T[(size_t)c * mmax + r] + T[(size_t)r * mmax + c]);
    if (!lin) {
      Problem::PhaseTimer pt(P, Problem::kPhRitz);
      P->sym_eig(m, Tm.data(), m, theta, Y);
    }
    // next block and its coupling factor
    std::vector<double> Rn;
    int kn = 0;
    double theta_max = 0.0;
    for (double t : theta) theta_max = std::max(theta_max, std::fabs(t));
    std::vector<CVec> Vn;
    {
      Problem::PhaseTimer pt(P, Problem::kPhOrthBlock);
      // new directions at the apply's truncation level are noise: for the
      // eigenproblem that level is tol times the largest Ritz value; for the
      // shifted linear system the components at the shift's scale matter
      const double drop = lin ? 10.0 * tol * lin->shift : 10.0 * tol * theta_max;
      Vn = orthonormalize_block(sb, Wn, Rn, kn, tol, cap, drop);
    }
    // residual estimates ||G x - theta x||_P = ||Rn * Y[last block, s]||
    bool done = m >= k;
    double worst = 0.0;
    // the linear solve is checked every kLinCheck block steps and at the end
    constexpr int kLinCheck = 4;
    const bool lin_check = lin && (step % kLinCheck == kLinCheck - 1 || kn == 0 || m + kn > mmax);
    if (lin && !lin_check) done = false;
    if (lin_check) {
      {
        Problem::PhaseTimer pt(P, Problem::kPhRitz);
        P->sym_eig(m, Tm.data(), m, theta, Y);
      }
      // Galerkin solution of (G + shift I) x = rhs on the basis:
      // z = Y diag(1 / (theta + shift)) Y^T g, with residual
      // ||(G + shift I) V z - rhs||_P = ||Rn z[last block]||
      zsol.assign(m, 0.0);
      for (int c = 0; c < m; ++c) {
        double t = 0.0;
        for (int i = 0; i < (int)g0.size(); ++i) t += Y[(size_t)c * m + i] * g0[i];
        t /= theta[c] + lin->shift;
        for (int i = 0; i < m; ++i) zsol[i] += Y[(size_t)c * m + i] * t;
      }
      double r2 = 0.0;
      for (int l = 0; l < kn; ++l) {
        double t = 0.0;
        for (int i = 0; i < bj; ++i) t += Rn[(size_t)i * kn + l] * zsol[j0 + i];
        r2 += t * t;
      }
      worst = std::sqrt(r2) / std::max(gnorm, 1e-300);
      done = worst <= lin->rtol;
    }
    for (int s = 0; s < (lin ? 0 : std::min(k, m)); ++s) {
      const int col = m - 1 - s;  // descending order
      double r2 = 0.0;
      for (int l = 0; l < kn; ++l) {
        double t = 0.0;
        for (int i = 0; i < bj; ++i) t += Rn[(size_t)i * kn + l] * Y[(size_t)col * m + (j0 + i)];
        r2 += t * t;
      }
      const double rel = std::sqrt(r2) / std::max(std::fabs(theta[col]), 1e-300);
      worst = std::max(worst, rel);
      if (rel > rtol) done = false;
    }
    res.steps = step + 1;
    m_conv = m;
    last_worst = worst;
    t_orth += std::chrono::duration<double>(clk::now() - t1).count();
    if (P->log_level > 1) {
      // orthonormality of the stored basis and symmetry of the projected matrix
      double orth = 0.0, asym = 0.0;
      int ar = -1, ac = -1;
      for (int a = 0; a < m; ++a) {
        CVec va = sb.stored(a);
        std::vector<double> ca = sb.inner_all(va);
        for (int b2 = 0; b2 < m; ++b2) orth = std::max(orth, std::fabs(ca[b2] - (a == b2 ? 1.0 : 0.0)));
        for (int b2 = 0; b2 < m; ++b2) {
          const double d = std::fabs(T[(size_t)a * mmax + b2] - T[(size_t)b2 * mmax + a]);
          if (d > asym) { asym = d; ar = b2; ac = a; }
        }
      }
      if (ar >= 0)
        std::fprintf(stderr, "{\"lanczos_asym_at\": [%d, %d], \"T_rc\": %.6e, \"T_cr\": %.6e}\n", ar, ac,
                     T[(size_t)ac * mmax + ar], T[(size_t)ar * mmax + ac]);
      std::vector<int> ranks;
      for (auto& v : Vn) ranks.push_back(v.r);
      std::fprintf(stderr, "{\"lanczos_check\": %d, \"next_block\": %d, \"orth_err\": %.3e, \"T_asym\": %.3e, "
                           "\"next_ranks\": [%d, %d, %d, %d]}\n",
                   step, kn, orth, asym, ranks.size() > 0 ? ranks[0] : -1, ranks.size() > 1 ? ranks[1] : -1,
                   ranks.size() > 2 ? ranks[2] : -1, ranks.size() > 3 ? ranks[3] : -1);
    }
    if (P->log_level > 0) {
      size_t fr = 0, tot = 0;
      (void)hipMemGetInfo(&fr, &tot);
      std::fprintf(stderr,
                   "{\"lanczos_step\": %d, \"vectors\": %d, \"basis_s\": %d, \"applies\": %lld, \"t_apply_s\": %.3f, "
                   "\"t_orth_s\": %.3f, \"t_total_s\": %.3f, \"worst_rel_resid\": %.3e, \"theta1\": %.10e, "
                   "\"pool_in_use_mb\": %.1f, \"device_free_mb\": %.1f, \"phases_s\": {\"prep\": %.3f, "
                   "\"poles\": %.3f, \"project\": %.3f, \"proj_solve\": %.3f, \"trunc\": %.3f, \"prior\": %.3f, "
                   "\"materialize\": %.3f, \"absorb\": %.3f, \"reorth\": %.3f, \"ritz\": %.3f, \"orth_block\": %.3f}}\n",
                   step, m, sb.s, (long long)P->stats.applies, t_apply, t_orth,
                   std::chrono::duration<double>(clk::now() - t_start).count(), worst, theta.empty() ? 0.0 : theta.back(),
                   P->pool->bytes_in_use() / 1048576.0, fr / 1048576.0, P->phase_s[0], P->phase_s[1], P->phase_s[2],
                   P->phase_s[3], P->phase_s[4], P->phase_s[5], P->phase_s[6], P->phase_s[7], P->phase_s[8],
                   P->phase_s[9], P->phase_s[10]);
      std::fflush(stderr);
    }
    // an empty next block means the Krylov space is invariant: its Ritz pairs are exact
    res.converged = done || kn == 0;
    if (done || kn == 0 || m + kn > mmax) break;
    // coupling block below the diagonal: W_i = sum_l Vn_l Rn[l, i]
    for (int i = 0; i < bj; ++i)
      for (int l = 0; l < kn; ++l) T[(size_t)(j0 + i) * mmax + (m + l)] = Rn[(size_t)i * kn + l];
    block_start.push_back(m);
    block_size.push_back(kn);
    for (auto& v : Vn) sb.append(v);
  }
  P->stats.lanczos_steps = res.steps;
  res.max_resid = last_worst;
  if (lin) {
    // the solution V z, formed on the cores and truncated once
    lin->resid = last_worst;
    lin->steps = res.steps;
    lin->converged = res.converged;
    const size_t slot = (size_t)std::max(sb.s, 1) * nt;
    Sbuf.ensure(sizeof(double) * slot);
    std::vector<double> coef(sb.size(), 0.0);
    for (int i = 0; i < (int)zsol.size() && i < sb.size(); ++i) coef[i] = zsol[i];
    sb.combine({}, {}, coef, Sbuf.as<double>());
    auto vs = sb.truncate_cores(Sbuf.as<double>(), 1, (long)slot, sb.s, sb.s, tol, cap);
    lin->x = std::make_unique<LowRank>();
    sb.materialize(vs[0], *lin->x);
    return res;
  }
  // Ritz vectors of the k largest Ritz values
  const int m = m_conv;
  const int kk = std::min(k, m);
  // (formed kRitzBatch at a time and truncated as one batch)
  constexpr int kRitzBatch = 8;
  const size_t slot = (size_t)std::max(sb.s, 1) * nt;
  Sbuf.ensure(sizeof(double) * slot * kRitzBatch);
  for (int s0 = 0; s0 < kk; s0 += kRitzBatch) {
    const int nb = std::min(kRitzBatch, kk - s0);
    for (int s = s0; s < s0 + nb; ++s) {
      const int col = m - 1 - s;
      res.lambda.push_back(theta[col]);
      std::vector<double> coef(sb.size(), 0.0);
      for (int i = 0; i < m; ++i) coef[i] = Y[(size_t)col * m + i];
      sb.combine({}, {}, coef, Sbuf.as<double>() + (s - s0) * slot);
    }
    auto vs = sb.truncate_cores(Sbuf.as<double>(), nb, (long)slot, sb.s, sb.s, tol, cap);
    sb.normalize(vs);
    for (auto& v : vs) {
      auto out = std::make_unique<LowRank>();
      sb.materialize(v, *out);
      res.vecs.push_back(std::move(out));
    }
  }
  return res;
}

// ---------------------------------------------------------------------------
// Two-pass randomized eigensolver (range finder and Rayleigh-Ritz of Halko,
// Martinsson and Tropp 2011) in the P inner product, on the shared spatial
// basis: pass one absorbs Y_j = G Omega_j; the Gram [<Y_i, Y_j>_P] gives a
// P-orthonormal basis Q_c = sum_j Y_j U_jc / sqrt(mu_c) (directions with
// mu_c <= 1e-14 max(mu) dropped) formed on the cores; pass two absorbs
// W_c = G Q_c; with MQ = [<Q_a, Q_b>_P] (the identity up to truncation) and
// T = [<Q_a, W_b>_P] the Ritz pairs solve T v = theta MQ v.  Ritz residuals
// ||sum_a (W_a - theta Q_a) v_a||_P come from the Grams of Q and W.
// ---------------------------------------------------------------------------
EigResult randomized_eig(Problem* P, int k, const std::vector<const LowRank*>& probes) {
  const int l = (int)probes.size();
  const double tol = P->desc.trunc_tol;
  const int cap = P->desc.rank_cap;
  const long nx = P->nx;
  const int nt = P->nt;
  if (l < 1) fail(LRPOST_EINVAL, "no probes");
  const long s_reserve = std::min<long>(nx, (long)(3 * l) * std::min(cap, 32) + 64);
  SharedBasis sb(P, (int)s_reserve, std::max(3 * l * cap, 64));
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto logline = [&](const char* phase, int done) {
    if (P->log_level > 0) {
      std::fprintf(stderr, "{\"randomized\": \"%s\", \"done\": %d, \"applies\": %lld, \"basis_s\": %d, \"t_s\": %.3f}\n",
                   phase, done, (long long)P->stats.applies, sb.s,
                   std::chrono::duration<double>(clk::now() - t0).count());
      std::fflush(stderr);
    }
  };
  // pass one: the probes applied in batches as large as device memory
  // allows (one multigrid solve for the pole solves of a whole batch);
  // cores are formed and truncated kBatch at a time
  constexpr int kBatch = 8;
  int rmax = 1;
  for (auto* w : probes) rmax = std::max(rmax, w->rank);
  const int abatch = P->apply_batch_limit(rmax, l);
  std::vector<CVec> Y;
  // The probes' images only span the trial space: the second pass makes the
  // Ritz values Rayleigh quotients of that space, so the space-time solves
  // of pass one are measured but not enriched (Gaussian probes have
  // independent nodal values, which the default poles resolve to about 1e-3)
  struct CheckScope {
    Problem* P;
    int saved;
    explicit CheckScope(Problem* p) : P(p), saved(p->st_check) { P->st_check = std::min(saved, 1); }
    ~CheckScope() { P->st_check = saved; }
  };
  std::optional<CheckScope> pass_one_check(std::in_place, P);
  for (int j0 = 0; j0 < l; j0 += abatch) {
    const int nbt = std::min(abatch, l - j0);
    std::vector<LowRank> ys(nbt);
    std::vector<const LowRank*> px(probes.begin() + j0, probes.begin() + j0 + nbt);
    std::vector<LowRank*> py;
    for (auto& y : ys) py.push_back(&y);
    P->hess_apply_batch(px, py, true);
    for (auto& y : ys) Y.push_back(sb.absorb(y, tol, cap));
    logline("pass1", j0 + nbt);
  }
  pass_one_check.reset();
  for (auto& y : Y) sb.append(y);
  std::vector<double> Gy((size_t)l * l);
  {
    std::vector<const CVec*> py;
    for (auto& y : Y) py.push_back(&y);
    const auto cs = sb.inner_all_many(py);
    for (int j = 0; j < l; ++j)
      for (int i = 0; i < l; ++i) Gy[(size_t)j * l + i] = cs[j][i];
  }
  for (int j = 0; j < l; ++j)
    for (int i = 0; i < j; ++i) Gy[(size_t)j * l + i] = Gy[(size_t)i * l + j] = 0.5 * (Gy[(size_t)j * l + i] + Gy[(size_t)i * l + j]);
  std::vector<double> mu(l), U((size_t)l * l);
  if (!syev(l, Gy.data(), l, mu.data(), U.data())) fail(LRPOST_EBREAKDOWN, "probe Gram eigensolve failed");
  std::vector<int> keep;
  for (int c = l - 1; c >= 0; --c)
    if (mu[l - 1] > 0 && mu[c] > 1e-14 * mu[l - 1]) keep.push_back(c);
  const int m = (int)keep.size();
  if (m == 0) fail(LRPOST_EBREAKDOWN, "the probes' images are zero");
  // orthonormal basis vectors, kBatch cores at a time truncated as one batch
  DevMem Sbuf;
  const size_t slot = (size_t)std::max(sb.s, 1) * nt;
  Sbuf.ensure(sizeof(double) * slot * kBatch);
  std::vector<CVec> Q;
  for (int c0 = 0; c0 < m; c0 += kBatch) {
    const int nb = std::min(kBatch, m - c0);
    for (int q = 0; q < nb; ++q) {
      const int c = keep[c0 + q];
      std::vector<double> coef(sb.size(), 0.0);
      for (int j = 0; j < l; ++j) coef[j] = U[(size_t)c * l + j] / std::sqrt(mu[c]);
      sb.combine({}, {}, coef, Sbuf.as<double>() + q * slot);
    }
    auto vs = sb.truncate_cores(Sbuf.as<double>(), nb, (long)slot, sb.s, sb.s, tol, cap);
    for (auto& v : vs) Q.push_back(std::move(v));
  }
  // pass two
  std::vector<CVec> W;
  const int abatch2 = P->apply_batch_limit(cap, m);
  for (int a0 = 0; a0 < m; a0 += abatch2) {
    const int nbt = std::min(abatch2, m - a0);
    std::vector<LowRank> qs(nbt), ws(nbt);
    std::vector<const LowRank*> pq;
    std::vector<LowRank*> pw;
    for (int a = 0; a < nbt; ++a) {
      sb.materialize(Q[a0 + a], qs[a]);
      pq.push_back(&qs[a]);
      pw.push_back(&ws[a]);
    }
    P->hess_apply_batch(pq, pw, true);
    for (auto& w : ws) W.push_back(sb.absorb(w, tol, cap));
    logline("pass2", a0 + nbt);
  }
  // stored vectors: Y (0 .. l-1), Q (l .. l+m-1), W (l+m .. l+2m-1)
  for (auto& q : Q) sb.append(q);
  for (auto& w : W) sb.append(w);
  std::vector<double> MQ((size_t)m * m), T((size_t)m * m), GW((size_t)m * m);
  std::vector<const CVec*> pqw;
  for (auto& q : Q) pqw.push_back(&q);
  for (auto& w : W) pqw.push_back(&w);
  const auto cqw = sb.inner_all_many(pqw);
  for (int b = 0; b < m; ++b) {
    const std::vector<double>& cq = cqw[b];
    const std::vector<double>& cw = cqw[m + b];
    for (int a = 0; a < m; ++a) {
      MQ[(size_t)b * m + a] = cq[l + a];
      T[(size_t)b * m + a] = cw[l + a];
      GW[(size_t)b * m + a] = cw[l + m + a];
    }
  }
  // generalized Rayleigh-Ritz through the eigenpairs of MQ: B = V_Q e^{-1/2}
  std::vector<double> eq(m), VQ((size_t)m * m);
  {
    std::vector<double> Ms((size_t)m * m);
    for (int b = 0; b < m; ++b)
      for (int a = 0; a < m; ++a) Ms[(size_t)b * m + a] = 0.5 * (MQ[(size_t)b * m + a] + MQ[(size_t)a * m + b]);
    if (!syev(m, Ms.data(), m, eq.data(), VQ.data())) fail(LRPOST_EBREAKDOWN, "basis Gram eigensolve failed");
  }
  std::vector<int> kq;
  for (int c = m - 1; c >= 0; --c)
    if (eq[c] > 1e-10 * eq[m - 1]) kq.push_back(c);
  const int mq = (int)kq.size();
  std::vector<double> Bm((size_t)m * mq);
  for (int c = 0; c < mq; ++c)
    for (int a = 0; a < m; ++a) Bm[(size_t)c * m + a] = VQ[(size_t)kq[c] * m + a] / std::sqrt(eq[kq[c]]);
  // Ts = B^T sym(T) B
  std::vector<double> Tsym((size_t)m * m), TB((size_t)m * mq), Ts((size_t)mq * mq);
  for (int b = 0; b < m; ++b)
    for (int a = 0; a < m; ++a) Tsym[(size_t)b * m + a] = 0.5 * (T[(size_t)b * m + a] + T[(size_t)a * m + b]);
  matmul(m, mq, m, Tsym.data(), m, false, Bm.data(), m, false, TB.data(), m, 1.0, 0.0);
  matmul(mq, mq, m, Bm.data(), m, true, TB.data(), m, false, Ts.data(), mq, 1.0, 0.0);
  std::vector<double> theta, V;
  P->sym_eig(mq, Ts.data(), mq, theta, V);
  const int kk = std::min(k, mq);
  EigResult res;
  res.steps = 2;
  double worst = 0.0;
  // Ritz vectors, kBatch cores at a time truncated as one batch (the shared
  // basis may have grown since the buffer was sized)
  const size_t slot2 = (size_t)std::max(sb.s, 1) * nt;
  Sbuf.ensure(sizeof(double) * slot2 * kBatch);
  for (int i0 = 0; i0 < kk; i0 += kBatch) {
    const int nb = std::min(kBatch, kk - i0);
    for (int i = i0; i < i0 + nb; ++i) {
      const int col = mq - 1 - i;
      const double th = theta[col];
      // coefficients on Q: c = B V[:, col]
      std::vector<double> c(m, 0.0);
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < mq; ++b) c[a] += Bm[(size_t)b * m + a] * V[(size_t)col * mq + b];
      // residual ||sum c_a (W_a - theta Q_a)||_P^2 = c^T (GW - theta (T + T^T) + theta^2 MQ) c
      double r2 = 0.0;
      for (int b = 0; b < m; ++b)
        for (int a = 0; a < m; ++a)
          r2 += c[a] * c[b] * (GW[(size_t)b * m + a] - th * (T[(size_t)b * m + a] + T[(size_t)a * m + b]) +
                               th * th * MQ[(size_t)b * m + a]);
      worst = std::max(worst, std::sqrt(std::max(r2, 0.0)) / std::max(std::fabs(th), 1e-300));
      std::vector<double> coef(sb.size(), 0.0);
      for (int a = 0; a < m; ++a) coef[l + a] = c[a];
      sb.combine({}, {}, coef, Sbuf.as<double>() + (i - i0) * slot2);
      res.lambda.push_back(th);
    }
    auto vs = sb.truncate_cores(Sbuf.as<double>(), nb, (long)slot2, sb.s, sb.s, tol, cap);
    sb.normalize(vs);
    for (auto& v : vs) {
      auto out = std::make_unique<LowRank>();
      sb.materialize(v, *out);
      res.vecs.push_back(std::move(out));
    }
  }
  res.max_resid = worst;
  logline("done", kk);
  return res;
}

}  // namespace lrp
