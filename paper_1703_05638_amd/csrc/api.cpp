// C-ABI entry points (declared in include/lrpost.h).  Every function catches
// all exceptions and turns them into a return code plus a thread-local
// message.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.h"

using namespace lrp;

static thread_local std::string g_last_error;

namespace lrp {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace lrp

template <typename F>
static int guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return LRPOST_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return LRPOST_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LRPOST_EINVAL;
  } catch (...) {
    g_last_error = "unknown error";
    return LRPOST_EINVAL;
  }
}

static Problem* impl(lrpost_problem* p) {
  if (!p || !p->impl) fail(LRPOST_EINVAL, "null problem handle");
  return p->impl.get();
}

// The space-time source problem (prior P = alpha tau (I kron (K + M))) is
// built on the heat operator; with a convection operator set, only the
// space-time solve and the initial-condition problem are defined.
static void require_heat(const Problem* P) {
  if (P->cd_on)
    fail(LRPOST_EINVAL, "a convection operator is set: only the space-time solve and the initial-condition problem use it");
}

// The problem that created e, which must be p (when p is given) and still
// alive; every stored vector must have that problem's shape.
static Problem* owner_of(lrpost_problem* p, const lrpost_eigs* e) {
  if (!e) fail(LRPOST_EINVAL, "null eigenpair handle");
  if (e->owner_alive.expired() || !e->owner)
    fail(LRPOST_EINVAL, "the problem of this eigenpair handle was destroyed or re-targeted");
  if (p && e->owner != p) fail(LRPOST_EINVAL, "eigenpair handle belongs to another problem");
  Problem* P = e->owner->impl.get();
  if (!P) fail(LRPOST_EINVAL, "null problem handle");
  for (auto& v : e->vecs)
    if (v->rank > 0 && (v->nx != P->nx || v->nt != P->nt))
      fail(LRPOST_EINVAL, "eigenvector shape does not match the problem");
  return P;
}

static void check_lr(const Problem* P, const lrpost_lowrank* x, bool need_data) {
  if (!x) fail(LRPOST_EINVAL, "null low-rank vector");
  if (x->nx != P->nx || x->nt != P->nt) fail(LRPOST_EINVAL, "low-rank vector shape does not match the problem");
  if (x->rank < 0 || x->rank > x->cap) fail(LRPOST_EINVAL, "rank outside [0, cap]");
  if (need_data && x->rank > 0 && (!x->W1 || !x->W2)) fail(LRPOST_EINVAL, "null factor pointer");
}

static void load_lr(Problem* P, const lrpost_lowrank* x, LowRank& out) {
  out.resize(P->nx, P->nt, x->rank);
  if (x->rank == 0) return;
  LRP_HIP(hipMemcpyAsync(out.a(), x->W1, sizeof(double) * (size_t)P->nx * x->rank, hipMemcpyDeviceToDevice, P->st));
  std::memcpy(out.B.data(), x->W2, sizeof(double) * (size_t)P->nt * x->rank);
}

static void store_lr(Problem* P, const LowRank& in, lrpost_lowrank* y) {
  if (in.rank > y->cap) fail(LRPOST_EINVAL, "output capacity " + std::to_string(y->cap) + " below rank " +
                                                std::to_string(in.rank));
  if (in.rank > 0 && (!y->W1 || !y->W2)) fail(LRPOST_EINVAL, "null output factor pointer");
  if (in.rank > 0) {
    LRP_HIP(hipMemcpyAsync(y->W1, in.a(), sizeof(double) * (size_t)P->nx * in.rank, hipMemcpyDeviceToDevice, P->st));
    std::memcpy(y->W2, in.B.data(), sizeof(double) * (size_t)P->nt * in.rank);
  }
  y->rank = in.rank;
  P->sync();
}

extern "C" {

const char* lrpost_last_error(void) { return g_last_error.c_str(); }
const char* lrpost_version(void) { return "lrpost 0.1 (gfx950)"; }

int lrpost_measure_fp64_rates(int iters, double* out) {
  return guarded([&] {
    if (!out) fail(LRPOST_EINVAL, "rate probe: null output");
    measure_fp64_rates(iters, &out[0], &out[1]);
  });
}

int lrpost_create(const lrpost_problem_desc* desc, lrpost_problem** out) {
  return guarded([&] {
    if (!desc || !out) fail(LRPOST_EINVAL, "null argument");
    *out = nullptr;
    auto h = new lrpost_problem();
    try {
      h->impl = std::make_unique<Problem>(*desc);
      // resolve the static Gram scratch of this device (lrpost_gram_noalloc)
      if (!gram_scratch_setup()) fail(LRPOST_EHIP, "hipGetSymbolAddress of the Gram scratch failed");
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
  });
}

int lrpost_destroy(lrpost_problem* p) {
  return guarded([&] { delete p; });
}

int lrpost_retarget(lrpost_problem* p, double alpha, double sigma, const double* box, uint64_t seed) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!box) fail(LRPOST_EINVAL, "null box");
    P->sync();
    P->set_observation(alpha, sigma, box, seed);
    // eigenpair handles of the previous target no longer describe this problem
    p->alive = std::make_shared<int>(0);
  });
}

int lrpost_get_stats(const lrpost_problem* p, lrpost_stats* s) {
  return guarded([&] {
    if (!p || !p->impl || !s) fail(LRPOST_EINVAL, "null argument");
    *s = p->impl->stats;
    p->impl->pool->counters(&s->pool_mallocs, &s->pool_trims, &s->pool_malloc_s);
  });
}

int lrpost_hess_apply(lrpost_problem* p, const lrpost_lowrank* x, lrpost_lowrank* y, int which) {
  return guarded([&] {
    Problem* P = impl(p);
    require_heat(P);
    PoolScope pool_scope(P->pool);
    check_lr(P, x, true);
    if (!y || y->nx != P->nx || y->nt != P->nt) fail(LRPOST_EINVAL, "output shape does not match the problem");
    if (which != LRPOST_MISFIT && which != LRPOST_PRECOND) fail(LRPOST_EINVAL, "unknown apply kind");
    LowRank xi, yo;
    load_lr(P, x, xi);
    P->hess_apply(xi, yo, which == LRPOST_PRECOND);
    store_lr(P, yo, y);
  });
}

int lrpost_hess_apply_batch(lrpost_problem* p, int nvec, const lrpost_lowrank* x, lrpost_lowrank* y, int which) {
  return guarded([&] {
    if (nvec < 0 || (nvec > 0 && (!x || !y))) fail(LRPOST_EINVAL, "bad batch");
    if (which != LRPOST_MISFIT && which != LRPOST_PRECOND) fail(LRPOST_EINVAL, "which must be MISFIT or PRECOND");
    Problem* P = impl(p);
    require_heat(P);
    PoolScope pool_scope(P->pool);
    std::vector<LowRank> xs(nvec), ys(nvec);
    std::vector<const LowRank*> px;
    std::vector<LowRank*> py;
    for (int i = 0; i < nvec; ++i) {
      check_lr(P, x + i, true);
      if (y[i].nx != P->nx || y[i].nt != P->nt) fail(LRPOST_EINVAL, "output shape does not match the problem");
      load_lr(P, x + i, xs[i]);
      px.push_back(&xs[i]);
      py.push_back(&ys[i]);
    }
    P->hess_apply_batch(px, py, which == LRPOST_PRECOND);
    for (int i = 0; i < nvec; ++i) store_lr(P, ys[i], y + i);
  });
}

int lrpost_spacetime_solve(lrpost_problem* p, const lrpost_lowrank* f, lrpost_lowrank* y, int adjoint) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    check_lr(P, f, true);
    if (!y || y->nx != P->nx || y->nt != P->nt) fail(LRPOST_EINVAL, "output shape does not match the problem");
    LowRank fi, yo;
    load_lr(P, f, fi);
    P->spacetime_solve(fi, yo, adjoint != 0);
    store_lr(P, yo, y);
  });
}

static void finish_eigs(lrpost_problem* p, Problem* P, EigResult& r, lrpost_eigs** out) {
  P->stats.ritz_resid = r.max_resid;
  auto e = new lrpost_eigs();
  e->owner = p;
  e->owner_alive = p->alive;
  e->lambda = r.lambda;
  e->vecs = std::move(r.vecs);
  *out = e;
}

int lrpost_eigensolve(lrpost_problem* p, int k, int method, int oversample, lrpost_eigs** out) {
  return guarded([&] {
    Problem* P = impl(p);
    require_heat(P);
    PoolScope pool_scope(P->pool);
    if (!out) fail(LRPOST_EINVAL, "null output");
    *out = nullptr;
    if (k < 1) fail(LRPOST_EINVAL, "k must be >= 1");
    // Ritz residual target: the truncation tolerance bounds how far the
    // residual of the truncated process can go down
    const double rtol = P->eig_rtol > 0 ? P->eig_rtol
                                        : std::max(P->desc.precision == LRPOST_FP64 ? 1e-9 : 1e-7,
                                                   0.1 * P->desc.trunc_tol);
    if (method == LRPOST_BLOCK_LANCZOS) {
      const int bsize = 4;
      const int maxv = P->eig_max_vectors > 0 ? P->eig_max_vectors : std::min(std::max(8 * k, 64), 800);
      EigResult r = block_lanczos(P, k, bsize, std::max(maxv, bsize), rtol);
      finish_eigs(p, P, r, out);
      if (!r.converged)
        fail(LRPOST_ENOCONV, "block Lanczos reached its limit of " + std::to_string(maxv) +
                                 " vectors with a relative Ritz residual estimate of " +
                                 std::to_string(r.max_resid) + " (target " + std::to_string(rtol) + ")");
      return;
    }
    if (method != LRPOST_RANDOMIZED) fail(LRPOST_EINVAL, "unsupported eigensolver method");
    if (oversample < 0) fail(LRPOST_EINVAL, "oversample must be >= 0");
    // k + oversample Gaussian probes G1 G2^T / sqrt(rp) of rank rp = min(32, rank_cap),
    // drawn with the library's counter-based generator (streams 1000 + 2j, 1001 + 2j)
    const int l = k + oversample;
    const int rp = std::min(32, P->desc.rank_cap);
    const long nx = P->nx;
    const int nt = P->nt;
    std::vector<LowRank> probes(l);
    std::vector<double> ha((size_t)nx * rp);
    for (int j = 0; j < l; ++j) {
      LowRank& w = probes[j];
      w.resize(nx, nt, rp);
      for (size_t i = 0; i < ha.size(); ++i) ha[i] = normal_draw(P->desc.seed, 1000 + 2 * (uint64_t)j, i);
      for (size_t i = 0; i < (size_t)nt * rp; ++i)
        w.B[i] = normal_draw(P->desc.seed, 1001 + 2 * (uint64_t)j, i) / std::sqrt((double)rp);
      P->to_device(w.a(), ha.data(), ha.size());
      P->sync();
    }
    std::vector<const LowRank*> pp;
    for (auto& w : probes) pp.push_back(&w);
    EigResult r = randomized_eig(P, k, pp);
    finish_eigs(p, P, r, out);
    if (!(r.max_resid <= rtol))
      fail(LRPOST_ENOCONV, "randomized eigensolver: largest relative Ritz residual " + std::to_string(r.max_resid) +
                               " above the target " + std::to_string(rtol));
  });
}

int lrpost_eigensolve_probes(lrpost_problem* p, int k, int nprobe, const lrpost_lowrank* probes,
                             lrpost_eigs** out) {
  return guarded([&] {
    Problem* P = impl(p);
    require_heat(P);
    PoolScope pool_scope(P->pool);
    if (!out || !probes) fail(LRPOST_EINVAL, "null argument");
    *out = nullptr;
    if (k < 1 || nprobe < 1) fail(LRPOST_EINVAL, "k and nprobe must be >= 1");
    std::vector<LowRank> ws(nprobe);
    for (int j = 0; j < nprobe; ++j) {
      check_lr(P, &probes[j], true);
      load_lr(P, &probes[j], ws[j]);
    }
    P->sync();
    std::vector<const LowRank*> pp;
    for (auto& w : ws) pp.push_back(&w);
    EigResult r = randomized_eig(P, k, pp);
    finish_eigs(p, P, r, out);
    const double rtol = P->eig_rtol > 0 ? P->eig_rtol
                                        : std::max(P->desc.precision == LRPOST_FP64 ? 1e-9 : 1e-7,
                                                   0.1 * P->desc.trunc_tol);
    if (!(r.max_resid <= rtol))
      fail(LRPOST_ENOCONV, "randomized eigensolver: largest relative Ritz residual " + std::to_string(r.max_resid) +
                               " above the target " + std::to_string(rtol));
  });
}

int lrpost_obs_count(const lrpost_problem* p) { return (p && p->impl) ? p->impl->nobs : -1; }

// Posterior mean: the block-Lanczos (conjugate-gradient) solve of
// (G + I) u = P^{-1} sigma^{-2} F^T y in the P inner product, which is the
// normal-equation system (H_mis + P) u = sigma^{-2} F^T y divided by P.
int lrpost_posterior_mean(lrpost_problem* p, const double* y_obs, int max_vectors, double rtol, lrpost_lowrank* mean,
                          double* rel_resid) {
  return guarded([&] {
    Problem* P = impl(p);
    require_heat(P);
    PoolScope pool_scope(P->pool);
    if (!y_obs || !mean) fail(LRPOST_EINVAL, "null argument");
    if (max_vectors < 0 || !(rtol >= 0)) fail(LRPOST_EINVAL, "max_vectors and rtol must be >= 0");
    if (mean->nx != P->nx || mean->nt != P->nt) fail(LRPOST_EINVAL, "output shape does not match the problem");
    LowRank c;
    P->data_rhs(y_obs, c);
    if (c.rank == 0) {
      mean->rank = 0;
      if (rel_resid) *rel_resid = 0.0;
      return;
    }
    LanczosSolve lin;
    lin.rhs = &c;
    lin.shift = 1.0;
    lin.rtol = rtol > 0 ? rtol : std::max(1e-7, 1e3 * P->desc.trunc_tol);
    const int maxv = max_vectors > 0 ? max_vectors : 800;
    block_lanczos(P, 1, 4, std::max(maxv, 8), 0.0, &lin);
    store_lr(P, *lin.x, mean);
    if (rel_resid) *rel_resid = lin.resid;
    if (!lin.converged) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "posterior mean: relative residual estimate %.3e above %.3e after %d block steps",
                    lin.resid, lin.rtol, lin.steps);
      fail(LRPOST_ENOCONV, msg);
    }
  });
}

int lrpost_eig_count(const lrpost_eigs* e) { return e ? (int)e->lambda.size() : 0; }

int lrpost_eig_values(const lrpost_eigs* e, double* lambda) {
  return guarded([&] {
    if (!e || !lambda) fail(LRPOST_EINVAL, "null argument");
    std::memcpy(lambda, e->lambda.data(), sizeof(double) * e->lambda.size());
  });
}

int lrpost_eig_vector_rank(const lrpost_eigs* e, int i) {
  if (!e || i < 0 || i >= (int)e->vecs.size()) return -1;
  return e->vecs[i]->rank;
}

int lrpost_eig_vector(const lrpost_eigs* e, int i, lrpost_lowrank* v) {
  return guarded([&] {
    if (!e || !v || i < 0 || i >= (int)e->vecs.size()) fail(LRPOST_EINVAL, "bad eigenvector index");
    Problem* P = owner_of(nullptr, e);
    PoolScope pool_scope(P->pool);
    if (v->nx != P->nx || v->nt != P->nt) fail(LRPOST_EINVAL, "output shape does not match the problem");
    store_lr(P, *e->vecs[i], v);
  });
}

int lrpost_eigs_free(lrpost_eigs* e) {
  return guarded([&] { delete e; });
}

int lrpost_eigs_from_pairs(lrpost_problem* p, int k, const double* lambda, const lrpost_lowrank* v,
                           lrpost_eigs** out) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!out || k < 0 || (k > 0 && (!lambda || !v))) fail(LRPOST_EINVAL, "bad arguments");
    auto e = new lrpost_eigs();
    e->owner = p;
    e->owner_alive = p->alive;
    try {
      for (int i = 0; i < k; ++i) {
        check_lr(P, v + i, true);
        auto x = std::make_unique<LowRank>();
        load_lr(P, v + i, *x);
        e->vecs.push_back(std::move(x));
        e->lambda.push_back(lambda[i]);
      }
      P->sync();
    } catch (...) {
      delete e;
      throw;
    }
    *out = e;
  });
}

// diag(Gamma_post,k)[x, t] = dprior[x] - sum_i d_i (sum_c A_i[x, c] B_i[t, c])^2
int lrpost_post_variance(lrpost_problem* p, const lrpost_eigs* e, double* diag, int on_device) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!e || !diag) fail(LRPOST_EINVAL, "null argument");
    (void)owner_of(p, e);
    const int k = (int)e->vecs.size();
    int R = 0;
    std::vector<int> seg{0};
    for (auto& v : e->vecs) { R += v->rank; seg.push_back(R); }
    const int nt = P->nt;
    const long nx = P->nx;
    DevMem A, Bt, segd, dco, D;
    A.ensure(sizeof(double) * (size_t)nx * std::max(R, 1));
    std::vector<double> bt((size_t)std::max(R, 1) * nt, 0.0), dc(std::max(k, 1), 0.0);
    for (int i = 0; i < k; ++i) {
      const LowRank& v = *e->vecs[i];
      if (v.rank > 0)
        LRP_HIP(hipMemcpyAsync(A.as<double>() + (size_t)seg[i] * nx, v.a(), sizeof(double) * nx * v.rank,
                               hipMemcpyDeviceToDevice, P->st));
      for (int c = 0; c < v.rank; ++c)
        for (int t = 0; t < nt; ++t) bt[(size_t)t * R + seg[i] + c] = v.B[(size_t)c * nt + t];
      dc[i] = e->lambda[i] / (1.0 + e->lambda[i]);
    }
    Bt.ensure(sizeof(double) * bt.size());
    P->to_device(Bt.as<double>(), bt.data(), bt.size());
    segd.ensure(sizeof(int) * seg.size());
    P->to_device_bytes(segd.p, seg.data(), sizeof(int) * seg.size());
    dco.ensure(sizeof(double) * dc.size());
    P->to_device(dco.as<double>(), dc.data(), dc.size());
    double* out = diag;
    if (!on_device) {
      D.ensure(sizeof(double) * (size_t)nx * nt);
      out = D.as<double>();
    }
    post_variance(P->st, nx, nt, k, segd.as<int>(), dco.as<double>(), A.as<double>(), nx, Bt.as<double>(),
                  std::max(R, 1), P->dprior.as<double>(), out, nx);
    LRP_HIP(hipGetLastError());
    if (!on_device) P->to_host(diag, out, (size_t)nx * nt);
    P->sync();
  });
}

int lrpost_prior_variance(lrpost_problem* p, double* dprior) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!dprior) fail(LRPOST_EINVAL, "null argument");
    std::memcpy(dprior, P->dprior_h.data(), sizeof(double) * P->nx);
  });
}

// s = L xi - sum_i p_i <v_i, L xi>_P v_i with p_i = 1 - (1 + lambda_i)^{-1/2}:
// the prior draw L xi, then the low-rank correction of its covariance.
int lrpost_sample(lrpost_problem* p, const lrpost_eigs* e, int ns, const double* xi, double* out, int on_device) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!e || !xi || !out) fail(LRPOST_EINVAL, "null argument");
    (void)owner_of(p, e);
    if (ns < 0) fail(LRPOST_EINVAL, "ns must be >= 0");
    if (ns == 0) return;
    const int nt = P->nt;
    const long nx = P->nx;
    const long cols = (long)ns * nt;
    if (cols > 65535) fail(LRPOST_EINVAL, "ns * nt must be at most 65535");
    const int k = (int)e->vecs.size();
    int R = 0;
    std::vector<int> seg{0};
    for (auto& v : e->vecs) { R += v->rank; seg.push_back(R); }
    DevMem Xd, Ls, Y, A, Z, Cm;
    const double* X = xi;
    if (!on_device) {
      Xd.ensure(sizeof(double) * (size_t)nx * cols);
      P->to_device(Xd.as<double>(), xi, (size_t)nx * cols);
      X = Xd.as<double>();
    }
    double* Lx = out;
    if (!on_device) {
      Ls.ensure(sizeof(double) * (size_t)nx * cols);
      Lx = Ls.as<double>();
    }
    P->prior_sqrt((int)cols, X, Lx);
    if (R > 0) {
      // <v_i, L xi>_P = alpha tau sum(B_i^T .* (A_i^T (K+M) L xi)) per sample
      Y.ensure(sizeof(double) * (size_t)nx * cols);
      P->apply_op((int)cols, Lx, Y.as<double>(), {{1.0, 1.0}});
      A.ensure(sizeof(double) * (size_t)nx * R);
      for (int i = 0; i < k; ++i) {
        const LowRank& v = *e->vecs[i];
        if (v.rank > 0)
          LRP_HIP(hipMemcpyAsync(A.as<double>() + (size_t)seg[i] * nx, v.a(), sizeof(double) * nx * v.rank,
                                 hipMemcpyDeviceToDevice, P->st));
      }
      Z.ensure(sizeof(double) * (size_t)R * cols);
      P->dense->gemm(true, false, R, (int)cols, (int)nx, 1.0, A.as<double>(), (int)nx, Y.as<double>(), (int)nx, 0.0,
                     Z.as<double>(), R);
      std::vector<double> Zh((size_t)R * cols);
      P->to_host(Zh.data(), Z.as<double>(), Zh.size());
      const double at = P->desc.alpha * P->tau;
      std::vector<double> Ch((size_t)R * cols, 0.0);
      for (int s = 0; s < ns; ++s)
        for (int i = 0; i < k; ++i) {
          const LowRank& v = *e->vecs[i];
          double c = 0.0;
          for (int cc = 0; cc < v.rank; ++cc)
            for (int t = 0; t < nt; ++t)
              c += Zh[((size_t)s * nt + t) * R + seg[i] + cc] * v.B[(size_t)cc * nt + t];
          const double coef = -(1.0 - 1.0 / std::sqrt(1.0 + e->lambda[i])) * at * c;
          for (int cc = 0; cc < v.rank; ++cc)
            for (int t = 0; t < nt; ++t)
              Ch[((size_t)s * nt + t) * R + seg[i] + cc] = coef * v.B[(size_t)cc * nt + t];
        }
      Cm.ensure(sizeof(double) * Ch.size());
      P->to_device(Cm.as<double>(), Ch.data(), Ch.size());
      P->dense->gemm(false, false, (int)nx, (int)cols, R, 1.0, A.as<double>(), (int)nx, Cm.as<double>(), R, 1.0, Lx,
                     (int)nx);
    }
    if (!on_device) P->to_host(out, Lx, (size_t)nx * cols);
    P->sync();
  });
}

int lrpost_set_eig_limits(lrpost_problem* p, int max_vectors, double rtol) {
  return guarded([&] {
    Problem* P = impl(p);
    if (max_vectors < 0 || !(rtol >= 0)) fail(LRPOST_EINVAL, "max_vectors and rtol must be >= 0");
    P->eig_max_vectors = max_vectors;
    P->eig_rtol = rtol;
  });
}

// ||G v_i - lambda_i v_i||_P / |lambda_i| from applies of the library's G to
// the stored vectors (a batch of four at a time): the residual is the
// low-rank concatenation [A_g, A_v] [B_g, -lambda B_v]^T, its P-norm from one
// weighted Gram product.
int lrpost_eig_residuals(lrpost_problem* p, const lrpost_eigs* e, double* resid) {
  return guarded([&] {
    Problem* P = impl(p);
    require_heat(P);
    PoolScope pool_scope(P->pool);
    if (!e || !resid) fail(LRPOST_EINVAL, "null argument");
    (void)owner_of(p, e);
    const int k = (int)e->vecs.size();
    const long nx = P->nx;
    const int nt = P->nt;
    constexpr int kBatch = 4;
    for (int i0 = 0; i0 < k; i0 += kBatch) {
      const int nb = std::min(kBatch, k - i0);
      std::vector<LowRank> outs(nb);
      std::vector<const LowRank*> px;
      std::vector<LowRank*> po;
      for (int i = 0; i < nb; ++i) {
        px.push_back(e->vecs[i0 + i].get());
        po.push_back(&outs[i]);
      }
      P->hess_apply_batch(px, po, true);
      for (int i = 0; i < nb; ++i) {
        const LowRank& v = *e->vecs[i0 + i];
        const LowRank& g = outs[i];
        const double lam = e->lambda[i0 + i];
        LowRank r;
        r.resize(nx, nt, g.rank + v.rank);
        if (g.rank > 0)
          LRP_HIP(hipMemcpyAsync(r.a(), g.a(), sizeof(double) * nx * g.rank, hipMemcpyDeviceToDevice, P->st));
        if (v.rank > 0)
          LRP_HIP(hipMemcpyAsync(r.a() + (size_t)g.rank * nx, v.a(), sizeof(double) * nx * v.rank,
                                 hipMemcpyDeviceToDevice, P->st));
        std::copy(g.B.begin(), g.B.end(), r.B.begin());
        for (size_t t = 0; t < v.B.size(); ++t) r.B[(size_t)g.rank * nt + t] = -lam * v.B[t];
        const double r2 = r.rank > 0 ? P->p_inner(r, r) : 0.0;
        resid[i0 + i] = std::sqrt(std::max(r2, 0.0)) / std::max(std::fabs(lam), 1e-300);
      }
    }
    P->sync();
  });
}

int lrpost_set_st_check(lrpost_problem* p, int mode, double rtol) {
  return guarded([&] {
    Problem* P = impl(p);
    if (mode < 0 || mode > 3 || !(rtol >= 0)) fail(LRPOST_EINVAL, "mode must be 0..3 and rtol >= 0");
    P->st_check = mode;
    P->st_rtol = rtol;
    if (mode == 0) P->stats.last_st_resid = P->stats.last_st_presid = -1.0;
  });
}

int lrpost_set_log(lrpost_problem* p, int level) {
  return guarded([&] { impl(p)->log_level = level; });
}

int lrpost_profile(lrpost_problem* p, int enable) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    P->sync();
    P->prof_on = enable != 0;
    P->prof_reset();
  });
}

int lrpost_profile_read(lrpost_problem* p, int kernel, int64_t* launches, double* total_ms, double* bytes,
                        double* flops) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!launches || !total_ms || !bytes) fail(LRPOST_EINVAL, "null argument");
    if (kernel < 0 || kernel > LRPOST_KERNEL_TRIDIAG) fail(LRPOST_EINVAL, "unknown kernel kind");
    P->prof_read(kernel, launches, total_ms, bytes, flops);
  });
}

int lrpost_set_mg_fused(lrpost_problem* p, int on) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    P->sync();
    P->mg_fused = on != 0;
  });
}

int lrpost_set_autotune(int on) {
  return guarded([&] { set_stencil_autotune(on != 0); });
}

int lrpost_autotune_report(char* buf, size_t len) {
  const std::string rep = stencil_autotune_report();
  if (buf && len > 0) {
    const size_t n = std::min(len - 1, rep.size());
    std::memcpy(buf, rep.data(), n);
    buf[n] = 0;
  }
  return (int)rep.size();
}

int lrpost_set_apply_batch(lrpost_problem* p, int n) {
  return guarded([&] {
    Problem* P = impl(p);
    if (n < 0) fail(LRPOST_EINVAL, "n must be >= 0");
    P->apply_batch_max = n;
  });
}

int lrpost_set_graphs(lrpost_problem* p, int on) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    P->sync();
    P->use_graphs = on != 0;
    if (!P->use_graphs) P->drop_graphs();
  });
}

int lrpost_set_obs_mask(lrpost_problem* p, const uint8_t* mask) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!mask) fail(LRPOST_EINVAL, "null mask");
    P->sync();
    P->set_obs_mask(mask);
    p->alive = std::make_shared<int>(0);  // eigenpairs of the old operator are stale
  });
}

int lrpost_ic_apply(lrpost_problem* p, double prior_var, int nvec, const double* U, double* Y) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!(prior_var > 0.0)) fail(LRPOST_EINVAL, "prior variance must be positive");
    if (nvec < 0) fail(LRPOST_EINVAL, "negative vector count");
    if (nvec > 0 && (!U || !Y)) fail(LRPOST_EINVAL, "null vector buffer");
    P->ic_apply(nvec, U, Y, prior_var);
  });
}

int lrpost_ic_eigensolve(lrpost_problem* p, double prior_var, int k, int max_vectors, double rtol, double* values,
                         double* vectors, int* used_vectors) {
  int rc = LRPOST_OK;
  const int g = guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!(prior_var > 0.0)) fail(LRPOST_EINVAL, "prior variance must be positive");
    if (k < 1 || k > P->nx) fail(LRPOST_EINVAL, "k out of range");
    if (!values || !vectors) fail(LRPOST_EINVAL, "null output buffer");
    if (!P->ic_eigensolve(prior_var, k, max_vectors, rtol, values, vectors, used_vectors)) {
      rc = LRPOST_ENOCONV;
      char msg[160];
      std::snprintf(msg, sizeof msg, "initial-condition eigensolve stopped at its vector limit; worst relative Ritz residual %.3e",
                    P->stats.ritz_resid);
      fail(LRPOST_ENOCONV, msg);
    }
  });
  return g != LRPOST_OK ? g : rc;
}

int lrpost_ic_post_variance(lrpost_problem* p, double prior_var, int k, const double* values, const double* vectors,
                            double* out, int on_device) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!(prior_var > 0.0)) fail(LRPOST_EINVAL, "prior variance must be positive");
    if (k < 0 || (k > 0 && (!values || !vectors)) || !out) fail(LRPOST_EINVAL, "null or invalid argument");
    if (on_device) {
      P->ic_post_variance(prior_var, k, values, vectors, out);
    } else {
      DevMem d;
      d.ensure(sizeof(double) * P->nx);
      P->ic_post_variance(prior_var, k, values, vectors, d.as<double>());
      P->to_host(out, d.as<double>(), P->nx);
    }
  });
}

int lrpost_convdiff_params(int N, int nt, double T, double nu, double wind, double delta, double* out) {
  return guarded([&] {
    if (N < 2 || nt < 1 || !(T > 0.0) || !(nu > 0.0) || !std::isfinite(T) || !std::isfinite(nu) ||
        !std::isfinite(wind) || !std::isfinite(delta) || !out)
      fail(LRPOST_EINVAL, "bad arguments");
    const CdParams c = cd_params(N, nt, T, nu, wind, delta);
    const double v[7] = {c.delta, c.fov_re, c.fov_im, c.ns_alpha, c.ns_radius, (double)c.ns_iters, c.lam_min};
    std::copy(v, v + 7, out);
  });
}

int lrpost_set_convection(lrpost_problem* p, double nu, double wind, double delta) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    P->set_convection(nu, wind, delta);
  });
}

static void cd_coefs(const Problem* P, int ncols, const void* A, const void* B, const double* coef,
                     std::vector<ShiftCoef>& ab) {
  if (!P->cd_on) fail(LRPOST_EINVAL, "no convection operator set");
  if (ncols < 0 || (ncols > 0 && (!A || !B || !coef))) fail(LRPOST_EINVAL, "bad arguments");
  ab.resize(ncols);
  for (int c = 0; c < ncols; ++c) ab[c] = {coef[2 * c], coef[2 * c + 1]};
}

int lrpost_convdiff_apply(lrpost_problem* p, int ncols, const double* X, double* Y, const double* coef,
                          int transpose) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    std::vector<ShiftCoef> ab;
    cd_coefs(P, ncols, X, Y, coef, ab);
    P->cd_apply(ncols, X, Y, ab, transpose ? -1 : 1);
    P->sync();
  });
}

int lrpost_convdiff_solve(lrpost_problem* p, int ncols, const double* B, double* X, const double* coef,
                          int transpose) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    std::vector<ShiftCoef> ab;
    cd_coefs(P, ncols, B, X, coef, ab);
    P->cd_solve(ncols, B, X, ab, transpose ? -1 : 1);
    P->sync();
  });
}

int lrpost_release_cache(lrpost_problem* p, uint64_t* released_bytes) {
  return guarded([&] {
    Problem* P = impl(p);
    P->sync();
    P->fin_keep_.clear();  // the kept basis buffers go back to the pool first
    const size_t b = P->pool->trim();
    if (released_bytes) *released_bytes = (uint64_t)b;
  });
}

int lrpost_graph_info(const lrpost_problem* p, int64_t* captured, int64_t* launches) {
  return guarded([&] {
    if (!p || !p->impl || !captured || !launches) fail(LRPOST_EINVAL, "null argument");
    *captured = p->impl->stats_graphs_captured;
    *launches = p->impl->stats_graph_launches;
  });
}

int lrpost_stencil_apply(lrpost_problem* p, int ncols, const double* X, double* Y, const double* Z,
                         const double* coef) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (ncols < 0 || (ncols > 0 && (!X || !Y || !coef))) fail(LRPOST_EINVAL, "bad arguments");
    std::vector<ShiftCoef> ab(ncols);
    std::vector<double> zc(ncols);
    for (int c = 0; c < ncols; ++c) { ab[c] = {coef[3 * c], coef[3 * c + 1]}; zc[c] = coef[3 * c + 2]; }
    P->apply_op(ncols, X, Y, ab, Z, Z ? &zc : nullptr);
    P->sync();
  });
}

int lrpost_mg_solve(lrpost_problem* p, int ncols, const double* B, double* X, const double* coef, int cycles) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (ncols < 0 || (ncols > 0 && (!B || !X || !coef)) || cycles < 1) fail(LRPOST_EINVAL, "bad arguments");
    std::vector<ShiftCoef> ab(ncols);
    for (int c = 0; c < ncols; ++c) {
      ab[c] = {coef[2 * c], coef[2 * c + 1]};
      if (ab[c].a < 0 || ab[c].b < 0 || ab[c].a + ab[c].b <= 0) fail(LRPOST_EINVAL, "operator must be a K + b M, a, b >= 0");
    }
    P->mg_solve(ncols, B, X, ab, cycles);
    P->sync();
  });
}

int lrpost_gram(lrpost_problem* p, int m, const double* A, int q, const double* B, double* C_host) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (m < 0 || q < 0 || (m > 0 && q > 0 && (!A || !B || !C_host))) fail(LRPOST_EINVAL, "bad arguments");
    std::vector<double> C;
    P->gram(m, A, q, B, C);
    if (!C.empty()) std::memcpy(C_host, C.data(), sizeof(double) * C.size());
  });
}

int lrpost_set_sweep_precision(lrpost_problem* p, int fp32_first) {
  return guarded([&] {
    Problem* P = impl(p);
    P->sync();
    P->sweep_f32 = fp32_first != 0;
  });
}

// C = A^T B with A in float32 on the float32 matrix cores (the kernel of the
// first Gram-Schmidt sweep in mixed precision); C to host.
int lrpost_gram_f32(lrpost_problem* p, int m, const float* A, int q, const double* B, double* C_host) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (m < 0 || q < 0 || (m > 0 && q > 0 && (!A || !B || !C_host))) fail(LRPOST_EINVAL, "bad arguments");
    if (m == 0 || q == 0) return;
    DevMem Cd;
    Cd.ensure(sizeof(double) * (size_t)m * q);
    std::vector<GramGroup> g{GramGroup{nullptr, B, nullptr, Cd.as<double>(), P->nx, P->nx, m, 0, m, q, 0, A}};
    P->gram_dev_grouped(g);
    P->to_host(C_host, Cd.as<double>(), (size_t)m * q);
  });
}

// C = A^T B with the partial products in the static per-device scratch: no
// allocation, no synchronization (the result is complete when p's stream
// reaches it).  Same kernels and chunking as lrpost_gram.
int lrpost_gram_noalloc(lrpost_problem* p, int m, const double* A, int q, const double* B, double* C_dev) {
  return guarded([&] {
    Problem* P = impl(p);
    if (m < 0 || q < 0 || (m > 0 && q > 0 && (!A || !B || !C_dev))) fail(LRPOST_EINVAL, "bad arguments");
    if (m == 0 || q == 0) return;
    const long need = gram_part_doubles(P->nx, m, q);
    if (need > kGramScratchDoubles)
      fail(LRPOST_EINVAL, "Gram of " + std::to_string(m) + " x " + std::to_string(q) + " needs " +
                              std::to_string(need * 8) + " bytes of scratch, above the static " +
                              std::to_string(kGramScratchDoubles * 8));
    double* scratch = gram_scratch_device();
    if (!scratch) scratch = gram_scratch_setup();
    if (!scratch) fail(LRPOST_EHIP, "hipGetSymbolAddress of the Gram scratch failed");
    GramGroup g{A, B, scratch, C_dev, P->nx, P->nx, m, 0, m, q, 0};
    gram_mfma_partials(P->st, P->nx, 1, &g);
    sum_partials_grouped(P->st, 1, &g);
    LRP_HIP(hipGetLastError());
  });
}

int lrpost_truncate(lrpost_problem* p, lrpost_lowrank* x, double tol, int weighted) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    check_lr(P, x, true);
    LowRank t;
    load_lr(P, x, t);
    P->truncate(t, tol > 0 ? tol : P->desc.trunc_tol, P->desc.rank_cap, weighted ? 1 : 0);
    store_lr(P, t, x);
  });
}

}  // extern "C"
