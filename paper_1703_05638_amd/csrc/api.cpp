// C-ABI entry points (declared in include/lrpost.h).  Every function catches
// all exceptions and turns them into a return code plus a thread-local
// message.
#include <cmath>
#include <cstring>
#include <string>

#include "internal.h"

using namespace lrp;

static thread_local std::string g_last_error;

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

int lrpost_create(const lrpost_problem_desc* desc, lrpost_problem** out) {
  return guarded([&] {
    if (!desc || !out) fail(LRPOST_EINVAL, "null argument");
    *out = nullptr;
    auto h = new lrpost_problem();
    try {
      h->impl = std::make_unique<Problem>(*desc);
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

int lrpost_get_stats(const lrpost_problem* p, lrpost_stats* s) {
  return guarded([&] {
    if (!p || !p->impl || !s) fail(LRPOST_EINVAL, "null argument");
    *s = p->impl->stats;
  });
}

int lrpost_hess_apply(lrpost_problem* p, const lrpost_lowrank* x, lrpost_lowrank* y, int which) {
  return guarded([&] {
    Problem* P = impl(p);
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
    for (int i = 0; i < nvec; ++i) {
      const int rc = lrpost_hess_apply(p, x + i, y + i, which);
      if (rc != LRPOST_OK) fail(rc, g_last_error);
    }
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

int lrpost_eigensolve(lrpost_problem* p, int k, int method, int oversample, lrpost_eigs** out) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!out) fail(LRPOST_EINVAL, "null output");
    *out = nullptr;
    if (k < 1) fail(LRPOST_EINVAL, "k must be >= 1");
    if (method != LRPOST_BLOCK_LANCZOS) fail(LRPOST_EINVAL, "unsupported eigensolver method");
    (void)oversample;
    // Ritz residual target: the truncation tolerance bounds how far the
    // residual of the truncated process can go down
    const double rtol = std::max(P->desc.precision == LRPOST_FP64 ? 1e-9 : 1e-7, 0.1 * P->desc.trunc_tol);
    const int bsize = 4;
    const int maxv = std::max(8 * k, 64);
    EigResult r = block_lanczos(P, k, bsize, std::min(maxv, 800), rtol);
    auto e = new lrpost_eigs();
    e->owner = p;
    e->lambda = r.lambda;
    e->vecs = std::move(r.vecs);
    *out = e;
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
    Problem* P = impl(e->owner);
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
    LRP_HIP(hipMemcpyAsync(segd.p, seg.data(), sizeof(int) * seg.size(), hipMemcpyHostToDevice, P->st));
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
    if (!on_device) LRP_HIP(hipMemcpyAsync(diag, out, sizeof(double) * (size_t)nx * nt, hipMemcpyDeviceToHost, P->st));
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

int lrpost_sample(lrpost_problem* p, const lrpost_eigs* e, int ns, const double* xi, double* out) {
  return guarded([&] {
    (void)p; (void)e; (void)ns; (void)xi; (void)out;
    fail(LRPOST_EINVAL, "sampling is not available in this build");
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
    P->prof_used = 0;
    P->prof_bytes = 0.0;
  });
}

int lrpost_profile_read(lrpost_problem* p, int64_t* launches, double* total_ms, double* bytes) {
  return guarded([&] {
    Problem* P = impl(p);
    PoolScope pool_scope(P->pool);
    if (!launches || !total_ms || !bytes) fail(LRPOST_EINVAL, "null argument");
    P->prof_read(launches, total_ms, bytes);
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
