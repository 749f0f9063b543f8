// Problem setup, multigrid driver, the low-rank space-time solver and the
// Hessian apply.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <numeric>
#include <thread>

#include "internal.h"

namespace lrp {

void fail(int code, const std::string& msg) { throw Error(code, msg); }

std::shared_ptr<Pool>& current_pool() {
  static thread_local std::shared_ptr<Pool> pool;
  return pool;
}

void DevMem::release() {
  if (p) {
    if (pool) pool->release(p, bytes);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
}

void DevMem::ensure(size_t nbytes) {
  if (nbytes <= bytes) return;
  release();
  if (!pool) pool = current_pool();
  if (pool) {
    p = pool->alloc(std::max<size_t>(nbytes, 256), &bytes);
    return;
  }
  size_t want = std::max<size_t>(nbytes, 256);
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    fail(LRPOST_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
  }
  bytes = want;
}

void LowRank::resize(long nx_, int nt_, int r) {
  nx = nx_;
  nt = nt_;
  rank = r;
  A.ensure(sizeof(double) * (size_t)nx * std::max(r, 1));
  B.assign((size_t)nt * r, 0.0);
}

// Interval [l, u] of the symbol of D^{-1}(a K + b M) over the high
// frequencies, on a level with spacing h (bh2 = b h^2).  With c1 = cos(theta1),
// c2 = cos(theta2) the stencil symbols are K: (8 - 2 c1 - 2 c2 - 4 c1 c2)/3 and
// M/h^2: (2 + c1)(2 + c2)/9; both are bilinear in (c1, c2), so extremes over
// the rectangles that make up the high-frequency set {min(c1, c2) <= 0} sit at
// their corners.  The maximum over all frequencies is taken at the corners of
// [-1, 1]^2.
void smoother_interval(double a, double bh2, double* lo, double* hi) {
  auto sym = [&](double c1, double c2) {
    const double k = (8.0 - 2.0 * c1 - 2.0 * c2 - 4.0 * c1 * c2) / 3.0;
    const double m = (2.0 + c1) * (2.0 + c2) / 9.0;
    return (a * k + bh2 * m) / (a * 8.0 / 3.0 + bh2 * 4.0 / 9.0);
  };
  double smax = 0.0;
  for (double c1 : {-1.0, 1.0})
    for (double c2 : {-1.0, 1.0}) smax = std::max(smax, sym(c1, c2));
  double smin = 1e300;
  const double pts[7][2] = {{-1, -1}, {-1, 1}, {0, -1}, {0, 1}, {1, -1}, {1, 0}, {-1, 0}};
  for (auto& p : pts) smin = std::min(smin, sym(p[0], p[1]));
  *lo = smin;
  *hi = smax;
}

// Chebyshev semi-iteration on [lo, hi] (Golub-Varga / Saad's three-term form):
// x_1 = x_0 + r_0/theta; x_{k+1} = x_k + rho_k rho_{k-1} (x_k - x_{k-1}) + (2 rho_k/delta) r_k
// with theta = (hi+lo)/2, delta = (hi-lo)/2, rho_0 = delta/theta,
// rho_k = 1/(2 theta/delta - rho_{k-1}) and r = D^{-1}(b - A x).
void chebyshev_coefs(double lo, double hi, int nu, double* alpha, double* beta) {
  const double th = 0.5 * (hi + lo), de = 0.5 * (hi - lo), sg = th / de;
  double rho = 1.0 / sg;
  alpha[0] = 0.0;
  beta[0] = 1.0 / th;
  for (int k = 1; k < nu; ++k) {
    const double rn = 1.0 / (2.0 * sg - rho);
    alpha[k] = rn * rho;
    beta[k] = 2.0 * rn / de;
    rho = rn;
  }
}

static void stencil_weights(double a, double b, double h, double* w) {
  const double h2 = h * h;
  w[0] = a * 8.0 / 3.0 + b * 4.0 * h2 / 9.0;
  w[1] = -a / 3.0 + b * h2 / 9.0;
  w[2] = -a / 3.0 + b * h2 / 36.0;
}

// Newton-Schulz steps X <- X (2I - A X) from X_0 = 2 / (1 + L) I for an
// SPD A with spectrum in [1, L]: the error I - A X_k has spectral radius
// rho^(2^k), rho = (L - 1) / (L + 1); the count takes it below 1e-18 (plus
// one step).
static int ns_steps(double L) {
  const double rho = (L - 1.0) / (L + 1.0);
  if (!(rho > 0.0)) return 1;
  return std::max(1, (int)std::ceil(std::log2(std::log(1e-18) / std::log(rho))) + 1);
}

// f(0) .. f(n-1) on up to kHostThreads host threads (pure host work only:
// no HIP calls inside f).  An exception thrown by f (an allocation failure)
// is caught in its thread; once every thread has joined, the first one is
// rethrown in the caller.  Slices whose thread cannot be started run on the
// calling thread.
static constexpr int kHostThreads = 8;
template <class F>
static void host_parallel(int n, F&& f) {
  if (n <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  const int nt = std::min(n, kHostThreads);
  std::vector<std::exception_ptr> err(nt);
  auto slice = [&](int t) {
    try {
      for (int i = t; i < n; i += nt) f(i);
    } catch (...) {
      err[t] = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  int t = 1;
  try {
    for (; t < nt; ++t) th.emplace_back(slice, t);
  } catch (...) {
  }
  for (int u = t; u < nt; ++u) slice(u);
  slice(0);
  for (auto& x : th) x.join();
  for (const auto& e : err)
    if (e) std::rethrow_exception(e);
}

Problem::Problem(const lrpost_problem_desc& d) : desc(d) {
  if (d.N < 4 || d.N > 4096 || (d.N & (d.N - 1)) != 0) fail(LRPOST_EINVAL, "N must be a power of two in [4, 4096]");
  if (d.nt < 1) fail(LRPOST_EINVAL, "nt must be >= 1");
  if (!(d.T > 0) || !(d.alpha > 0) || !(d.sigma > 0)) fail(LRPOST_EINVAL, "T, alpha and sigma must be positive");
  if (!(d.trunc_tol > 0) || !(d.trunc_tol < 1)) fail(LRPOST_EINVAL, "trunc_tol must lie in (0, 1)");
  if (d.rank_cap < 1) fail(LRPOST_EINVAL, "rank_cap must be >= 1");
  if (d.precision != LRPOST_FP64 && d.precision != LRPOST_MIXED) fail(LRPOST_EINVAL, "unknown precision");
  if (d.mg_levels != 0)
    fail(LRPOST_EINVAL, "mg_levels must be 0: the multigrid hierarchy always coarsens to the LDS-resident levels");
  pool = std::make_shared<Pool>();
  PoolScope scope(pool);
  N = d.N;
  n = N - 1;
  nt = d.nt;
  nx = (long)n * n;
  h = 1.0 / N;
  tau = d.T / nt;
  st = (hipStream_t)d.hip_stream;
  if (!st) {
    // a blocking stream of the problem's own: ordered with the null stream
    // like every blocking stream, and one that graphs can be captured on
    LRP_HIP(hipStreamCreate(&own_stream_));
    st = own_stream_;
  }
  dense = std::make_unique<GpuDense>(st);
  // multigrid hierarchy: n, (n-1)/2, ..., 1
  for (int m = n; m >= 1; m = (m - 1) / 2) {
    lv.push_back({m, (long)m * m, 1.0 / (m + 1)});
    if (m == 1) break;
  }
  lds_level = 0;
  while (lv[lds_level].n > kCoarseLdsMaxN) ++lds_level;
  // diag((K+M)^{-1}) from the sine eigenpairs of K and M:
  // (K+M)^{-1} = sum_p phi_p phi_p^T / (kappa_p + mu_p), phi_p = s_i (x) s_j,
  // s_j(ii) = sqrt(2h) sin(ii j pi h), kappa = k_i m_j + m_i k_j, mu = m_i m_j.
  {
    std::vector<double> k1(n), m1(n), Sq((size_t)n * n);
    for (int j = 0; j < n; ++j) {
      const double th = (j + 1) * M_PI * h;
      k1[j] = (4.0 / h) * std::sin(th / 2) * std::sin(th / 2);
      m1[j] = (h / 3.0) * (2.0 + std::cos(th));
    }
    for (int mode = 0; mode < n; ++mode)
      for (int node = 0; node < n; ++node) {
        const double s = std::sqrt(2.0 * h) * std::sin((double)(node + 1) * (mode + 1) * M_PI * h);
        Sq[(size_t)mode * n + node] = s * s;  // Sq[node, mode]
      }
    std::vector<double> W((size_t)n * n), T1((size_t)n * n);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        W[(size_t)j * n + i] = 1.0 / (k1[i] * m1[j] + m1[i] * k1[j] + m1[i] * m1[j]);
    // D = Sq W Sq^T, D[ii, jj]
    matmul(n, n, n, Sq.data(), n, false, W.data(), n, false, T1.data(), n, 1.0, 0.0);
    kmdiag_h_.assign((size_t)n * n, 0.0);
    matmul(n, n, n, T1.data(), n, false, Sq.data(), n, true, kmdiag_h_.data(), n, 1.0, 0.0);
  }
  set_observation(d.alpha, d.sigma, d.box, d.seed);
  const double lt = -std::log10(d.trunc_tol);
  // the Chebyshev-smoothed V-cycle contracts the error by about 0.05 per cycle
  st_cycles = std::max(3, (int)std::ceil((lt + 2.0) / 1.25));
  prior_cycles = std::max(4, (int)std::ceil((lt + 3.0) / 1.25));
  // the spectrum of M^{-1} K lies in [2 pi^2, 24 / h^2) (element bound 2 x 12 / h^2)
  init_st_poles(2.0 * M_PI * M_PI, 24.0 / (h * h));
  stats.last_st_resid = -1.0;
  stats.last_st_presid = -1.0;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) == hipSuccess) free_at_create = fr;
  else (void)hipGetLastError();
}

// Inner-solver settings of the space-time solves from the truncation
// tolerance and the spectrum [lam_min, lam_max] of the symmetric part of
// M^{-1} times the spatial operator: poles of the spatial rational Krylov
// basis log-spaced over the time-step scaled spectrum, and the Newton-Schulz
// bound of the projected I + tau K.  For tolerances down to 1e-7 the poles
// cover [0.3 tau lambda_min, 10]: modes with tau lambda beyond about 10
// respond to the source within one step and need no poles of their own, and
// this placement reaches the tolerance with fewer poles than spreading them
// over the whole spectrum (measured on rough random sources at 64^2 and
// 128^2 meshes with nt = 200).  count_scale multiplies the pole count.
void Problem::init_st_poles(double lam_min, double lam_max, double count_scale) {
  const double lt = -std::log10(desc.trunc_tol);
  st_poles = std::max(4, (int)std::lround(count_scale * std::min(24, (int)std::lround(1.5 * lt) + 1)));
  pole_lam_max_ = lam_max;
  // Newton-Schulz inverse of the projected I + tau K (space-time finish):
  // spectrum bound (with a margin for the rounding of the basis) and the
  // number of steps that takes the error factor below 1e-18
  ns_bound_ = 1.0 + 1.05 * tau * lam_max;
  ns_iters_ = ns_steps(ns_bound_);
  const double plo = std::min(1e-2, 0.5 * tau * lam_min);
  const double phi = std::max(10.0 * plo, std::min(tau * lam_max, 1e4));
  if (lt <= 7.0) {
    st_poles = std::max(4, (int)std::lround(count_scale * ((int)std::lround(1.2 * lt) + 1)));
    const double lo = 0.3 * tau * lam_min;
    const double hi = std::max(10.0 * lo, std::min(tau * lam_max, 10.0));
    poles.resize(st_poles);
    for (int i = 0; i < st_poles; ++i) poles[i] = lo * std::pow(hi / lo, (double)i / (st_poles - 1));
  } else {
    poles.resize(st_poles);
    for (int i = 0; i < st_poles; ++i)
      poles[i] = plo * std::pow(phi / plo, st_poles == 1 ? 0.0 : (double)i / (st_poles - 1));
  }
}

int Problem::apply_batch_limit(int r, int want) const {
  if (want <= 1) return std::max(want, 1);
  if (apply_batch_max > 0) return std::min(apply_batch_max, want);
  // bytes per pole-solve column: solution and right-hand side (float64), the
  // multigrid levels' x, t and b (4/3 of the finest level) in the working
  // precision, the float32 copies of a mixed solve, the basis and the
  // residual-check buffers (float64)
  const double elem = desc.precision == LRPOST_MIXED ? 4.0 : 8.0;
  const double per_col = 8.0 * 2 + elem * 3.0 * 4.0 / 3.0 + (desc.precision == LRPOST_MIXED ? 8.0 : 0.0) + 8.0 * 2;
  const double per_input = per_col * (double)std::max(r, 1) * (double)poles.size() * (double)nx;
  const double budget = 0.5 * (double)free_at_create;
  const int fit = per_input > 0 ? (int)(budget / per_input) : want;
  return std::max(1, std::min(want, fit));
}

// The parts of a problem that depend on the prior scale, the noise level,
// the observation box and the start-block seed: the observation mask (closed
// box, 1e-12 slack) and diag(P^{-1}) = (alpha tau)^{-1} diag((K+M)^{-1}).
// Everything else (mesh, multigrid hierarchy, poles, device pool, graphs)
// depends only on the mesh, the time steps and the tolerances.
void Problem::set_observation(double alpha, double sigma, const double* box, uint64_t seed) {
  if (!(alpha > 0) || !(sigma > 0)) fail(LRPOST_EINVAL, "alpha and sigma must be positive");
  std::vector<uint8_t> mh(nx, 0);
  int cnt = 0;
  const double eps = 1e-12;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const double x1 = (i + 1) * h, x2 = (j + 1) * h;
      const bool in = x1 >= box[0] - eps && x1 <= box[1] + eps && x2 >= box[2] - eps && x2 <= box[3] + eps;
      mh[(size_t)j * n + i] = in ? 1 : 0;
      cnt += in ? 1 : 0;
    }
  if (cnt == 0) fail(LRPOST_EINVAL, "observation box holds no mesh node");
  desc.alpha = alpha;
  desc.sigma = sigma;
  for (int i = 0; i < 4; ++i) desc.box[i] = box[i];
  desc.seed = seed;
  mask_h.swap(mh);
  nobs = cnt;
  mask.ensure(nx);
  to_device_bytes(mask.p, mask_h.data(), nx);
  dprior_h.resize(nx);
  const double sc = 1.0 / (alpha * tau);
  for (long i = 0; i < nx; ++i) dprior_h[i] = sc * kmdiag_h_[i];
  dprior.ensure(sizeof(double) * nx);
  to_device(dprior.as<double>(), dprior_h.data(), nx);
  sync();
}

Problem::~Problem() {
  if (st) (void)hipStreamSynchronize(st);
  else (void)hipDeviceSynchronize();
  for (auto& ps : prof_)
    for (auto& ev : ps.ev) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
  drop_graphs();
  if (staging_) (void)hipHostFree(staging_);
  if (readback_) (void)hipHostFree(readback_);
  if (own_stream_) {
    dense.reset();
    (void)hipStreamDestroy(own_stream_);
  }
}

void Problem::drop_graphs() {
  for (auto& g : graphs_) (void)hipGraphExecDestroy(g.second.exec);
  graphs_.clear();
}

void Problem::sync() {
  LRP_HIP(hipStreamSynchronize(st));
  staging_used_ = 0;
}

// Host-to-device copies go through a pinned staging arena so that the host
// source may be reused at once; the arena is recycled at every stream sync.
void Problem::to_device_bytes(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  if (!staging_) LRP_HIP(hipHostMalloc(&staging_, kStagingBytes, hipHostMallocDefault));
  const char* s = static_cast<const char*>(src);
  char* d = static_cast<char*>(dst);
  while (bytes > 0) {
    const size_t chunk = std::min(bytes, kStagingBytes);
    if (staging_used_ + chunk > kStagingBytes) sync();
    char* slot = static_cast<char*>(staging_) + staging_used_;
    std::memcpy(slot, s, chunk);
    staging_used_ += (chunk + 255) & ~size_t(255);
    LRP_HIP(hipMemcpyAsync(d, slot, chunk, hipMemcpyHostToDevice, st));
    s += chunk;
    d += chunk;
    bytes -= chunk;
  }
}

void Problem::to_device(double* dst, const double* src, size_t count) {
  to_device_bytes(dst, src, sizeof(double) * count);
}

void Problem::to_host_bytes(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) {
    sync();
    return;
  }
  if (!readback_) LRP_HIP(hipHostMalloc(&readback_, kReadbackBytes, hipHostMallocDefault));
  const char* s = static_cast<const char*>(src);
  char* d = static_cast<char*>(dst);
  while (bytes > 0) {  // each chunk's sync also drains the stream
    const size_t chunk = std::min(bytes, kReadbackBytes);
    LRP_HIP(hipMemcpyAsync(readback_, s, chunk, hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(d, readback_, chunk);
    s += chunk;
    d += chunk;
    bytes -= chunk;
  }
}

void Problem::to_host_block(double* dst, const double* src, int rows, int cols, long ld) {
  if (rows <= 0 || cols <= 0) {
    sync();
    return;
  }
  if (ld == rows) return to_host(dst, src, (size_t)rows * cols);
  if (!readback_) LRP_HIP(hipHostMalloc(&readback_, kReadbackBytes, hipHostMallocDefault));
  const int per = (int)std::max<size_t>(1, kReadbackBytes / (sizeof(double) * rows));
  for (int c0 = 0; c0 < cols; c0 += per) {
    const int nc = std::min(per, cols - c0);
    LRP_HIP(hipMemcpy2DAsync(readback_, sizeof(double) * rows, src + (size_t)c0 * ld, sizeof(double) * ld,
                             sizeof(double) * rows, nc, hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(dst + (size_t)c0 * rows, readback_, sizeof(double) * rows * nc);
  }
}

void Problem::to_host(double* dst, const double* src, size_t count) {
  to_host_bytes(dst, src, sizeof(double) * count);
}


void Problem::apply_op(int ncols, const double* X, double* Y, const std::vector<ShiftCoef>& ab, const double* Z,
                       const std::vector<double>* zc) {
  if (ncols <= 0) return;
  if (ab.size() == 1 && (!zc || zc->size() == 1)) {
    // one operator for all columns: its weights are uploaded once per problem
    const double c = zc ? (*zc)[0] : 0.0;
    const std::array<double, 3> key{ab[0].a, ab[0].b, c};
    auto it = op_w_cache_.find(key);
    if (it == op_w_cache_.end()) {
      double w[4];
      stencil_weights(ab[0].a, ab[0].b, h, w);
      w[3] = c;
      DevMem d;
      d.ensure(sizeof(double) * 4);
      to_device(d.as<double>(), w, 4);
      it = op_w_cache_.emplace(key, std::move(d)).first;
    }
    const double* w = it->second.as<double>();
    timed(LRPOST_KERNEL_STENCIL, sizeof(double) * (Z ? 3.0 : 2.0) * (double)nx * ncols,
          [&] { stencil<double>(st, n, ncols, X, nx, Y, nx, Z, nx, w, 0); });
    LRP_HIP(hipGetLastError());
    return;
  }
  op_w_h_.assign((size_t)4 * ncols, 0.0);
  for (int c = 0; c < ncols; ++c) {
    const ShiftCoef& s = ab.size() == 1 ? ab[0] : ab[c];
    stencil_weights(s.a, s.b, h, &op_w_h_[(size_t)4 * c]);
    op_w_h_[(size_t)4 * c + 3] = zc ? (zc->size() == 1 ? (*zc)[0] : (*zc)[c]) : 0.0;
  }
  op_w_.ensure(sizeof(double) * op_w_h_.size());
  to_device(op_w_.as<double>(), op_w_h_.data(), op_w_h_.size());
  timed(LRPOST_KERNEL_STENCIL, sizeof(double) * (Z ? 3.0 : 2.0) * (double)nx * ncols,
        [&] { stencil<double>(st, n, ncols, X, nx, Y, nx, Z, nx, op_w_.as<double>(), 4); });
  LRP_HIP(hipGetLastError());
}

void Problem::upload_mg_params(const std::vector<ShiftCoef>& ab) {
  const int L = (int)lv.size();
  const int ncols = (int)ab.size();
  mg_param_h_.assign((size_t)L * ncols * kMgStride, 0.0);
  double al[kMgMaxSteps], be[kMgMaxSteps];
  for (int l = 0; l < L; ++l)
    for (int c = 0; c < ncols; ++c) {
      double* w = &mg_param_h_[((size_t)l * ncols + c) * kMgStride];
      stencil_weights(ab[c].a, ab[c].b, lv[l].h, w);
      double lo, hi;
      smoother_interval(ab[c].a, ab[c].b * lv[l].h * lv[l].h, &lo, &hi);
      chebyshev_coefs(lo, hi, kMgNu, al, be);
      for (int s = 0; s < kMgNu; ++s) {
        w[4 + 2 * s] = al[s];
        w[5 + 2 * s] = be[s] / w[0];
      }
    }
  mg_param_.ensure(sizeof(double) * mg_param_h_.size());
  to_device(mg_param_.as<double>(), mg_param_h_.data(), mg_param_h_.size());
}

bool Problem::GraphKey::operator<(const GraphKey& o) const {
  return std::tie(elem, ncols, B, X, work, prm, acc, fused) <
         std::tie(o.elem, o.ncols, o.B, o.X, o.work, o.prm, o.acc, o.fused);
}

template <class Launch>
void Problem::run_graph(const GraphKey& key, Launch&& launch) {
  if (!use_graphs || prof_on || !st) {
    launch();
    return;
  }
  auto it = graphs_.find(key);
  if (it == graphs_.end()) {
    if (graphs_.size() >= kMaxGraphs) {
      // drop the oldest-created graph (the work queued before keeps its own copy)
      auto old = graphs_.begin();
      for (auto g = graphs_.begin(); g != graphs_.end(); ++g)
        if (g->second.serial < old->second.serial) old = g;
      LRP_HIP(hipGraphExecDestroy(old->second.exec));
      graphs_.erase(old);
    }
    hipGraph_t graph = nullptr;
    LRP_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      launch();
    } catch (...) {
      // leave the stream out of capture mode before the error propagates
      if (hipStreamEndCapture(st, &graph) == hipSuccess && graph) (void)hipGraphDestroy(graph);
      throw;
    }
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (e != hipSuccess || !graph) fail(LRPOST_EHIP, std::string("V-cycle graph capture failed: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) fail(LRPOST_EHIP, std::string("V-cycle graph instantiation failed: ") + hipGetErrorString(e2));
    it = graphs_.emplace(key, GraphEntry{exec, graph_serial_++}).first;
    ++stats_graphs_captured;
  }
  LRP_HIP(hipGraphLaunch(it->second.exec, st));
  ++stats_graph_launches;
}

// One V-cycle with zero initial guess and kMgNu Chebyshev smoothing steps
// before and after each coarse-grid correction; levels at or below lds_level
// run inside a single kernel with all data in LDS.  Smoothing alternates
// between the level's x and t buffers, writing each iterate over the one two
// steps back, so that with an odd step count the result lands in x.
template <typename T>
void Problem::vcycle_zero(int ncols, const T* B, T* X, bool accumulate) {
  const int L = (int)lv.size();
  // workspace: per level l >= 1: x, b, t (nx_l * ncols each); level 0: t
  std::vector<size_t> off(L + 1, 0);
  size_t tot = (size_t)lv[0].nx * ncols;
  for (int l = 1; l <= lds_level; ++l) {
    off[l] = tot;
    tot += 3 * (size_t)lv[l].nx * ncols;
  }
  DevMem& work = sizeof(T) == sizeof(double) ? mg_work_ : mg_work_f_;
  if (lds_level > 0) work.ensure(sizeof(T) * tot);
  // The launch sequence of one V-cycle depends only on the shape and the
  // buffers, so it is captured once into a HIP graph per (precision, shape,
  // buffers) and replayed: one graph launch instead of 2 L + 1 kernel
  // launches.  The sequence holds kernels only (no memset, copy or host
  // work), and everything it reads -- right-hand side, parameters, workspace
  // -- is read at replay time.  Timed runs launch the kernels one by one.
  const GraphKey key{sizeof(T), ncols, (const void*)B, (const void*)X, work.p, mg_param_.p, accumulate ? 1 : 0,
                     vcycle_fused() ? 1 : 0};
  run_graph(key, [&] { vcycle_launch<T>(ncols, B, X, accumulate, off); });
}

template <typename T>
void Problem::vcycle_launch(int ncols, const T* B, T* X, bool accumulate, const std::vector<size_t>& off) {
  const int L = (int)lv.size();
  const double* P = mg_param_.as<double>();
  auto prm = [&](int l) { return P + (size_t)l * ncols * kMgStride; };
  if (lds_level == 0) {
    mg_coarse_lds<T>(st, lv[0].n, L, ncols, B, nx, X, nx, prm(0), kMgNu, kMgNu);
    return;
  }
  DevMem& work = sizeof(T) == sizeof(double) ? mg_work_ : mg_work_f_;
  T* base = work.as<T>();
  auto xw = [&](int l) { return base + off[l]; };
  auto bw = [&](int l) { return base + off[l] + (size_t)lv[l].nx * ncols; };
  auto tw = [&](int l) { return base + off[l] + 2 * (size_t)lv[l].nx * ncols; };
  if (vcycle_fused()) {
    static_assert(kMgNu == kMgFusedNu, "fused kernels take the smoother's step count");
    // down: level l pre-smoothes into its t buffer and writes the coarse
    // right-hand side; up: x_l = smoothing from t_l + P x_{l+1}
    for (int l = 0; l < lds_level; ++l) {
      const int nl = lv[l].n, nc = lv[l + 1].n;
      const T* b = l == 0 ? B : bw(l);
      T* t = l == 0 ? base : tw(l);
      timed(LRPOST_KERNEL_MG_DOWN, sizeof(T) * ((double)nl * nl * 2 + (double)nc * nc) * ncols,
            [&] { mg_down<T>(st, nl, ncols, b, lv[l].nx, t, bw(l + 1), lv[l + 1].nx, prm(l)); });
    }
    mg_coarse_lds<T>(st, lv[lds_level].n, L - lds_level, ncols, bw(lds_level), lv[lds_level].nx, xw(lds_level),
                     lv[lds_level].nx, prm(lds_level), kMgNu, kMgNu);
    for (int l = lds_level - 1; l >= 0; --l) {
      const int nl = lv[l].n, nc = lv[l + 1].n;
      const T* b = l == 0 ? B : bw(l);
      const T* t = l == 0 ? base : tw(l);
      T* x = l == 0 ? X : xw(l);
      const bool acc = accumulate && l == 0;
      timed(LRPOST_KERNEL_MG_UP, sizeof(T) * ((double)nl * nl * (acc ? 4 : 3) + (double)nc * nc) * ncols,
            [&] { mg_up<T>(st, nl, ncols, t, xw(l + 1), lv[l + 1].nx, b, lv[l].nx, x, prm(l), acc); });
    }
    return;
  }
  // down: pre-smoothing from zero, x_s in (s odd ? x : t)
  for (int l = 0; l < lds_level; ++l) {
    const int nl = lv[l].n;
    const long ldl = lv[l].nx;
    T* x = l == 0 ? X : xw(l);
    const T* b = l == 0 ? B : bw(l);
    T* t = l == 0 ? base : tw(l);
    for (int s = 0; s < kMgNu; ++s) {
      const T* xc = s == 0 ? nullptr : ((s % 2) ? x : t);
      T* xo = (s % 2 == 0) ? x : t;
      const T* xp = s <= 1 ? nullptr : xo;
      smooth_step<T>(nl, ncols, xc, xp, xo, b, ldl, prm(l), s);
    }
    mg_resid_restrict<T>(st, nl, ncols, x, b, ldl, bw(l + 1), lv[l + 1].nx, prm(l));
  }
  // coarse levels in LDS
  mg_coarse_lds<T>(st, lv[lds_level].n, L - lds_level, ncols, bw(lds_level), lv[lds_level].nx, xw(lds_level),
                        lv[lds_level].nx, prm(lds_level), kMgNu, kMgNu);
  // up: t = x + P e, then post-smoothing from t, x_s in (s even ? t : x)
  for (int l = lds_level - 1; l >= 0; --l) {
    const int nl = lv[l].n;
    const long ldl = lv[l].nx;
    T* x = l == 0 ? X : xw(l);
    const T* b = l == 0 ? B : bw(l);
    T* t = l == 0 ? base : tw(l);
    mg_prolong_add<T>(st, nl, ncols, xw(l + 1), lv[l + 1].nx, x, t, ldl);
    for (int s = 0; s < kMgNu; ++s) {
      const T* xc = (s % 2 == 0) ? t : x;
      T* xo = (s % 2 == 0) ? x : t;
      const T* xp = s == 0 ? nullptr : xo;
      smooth_step<T>(nl, ncols, xc, xp, xo, b, ldl, prm(l), s);
    }
  }
}


// One Chebyshev smoother step, credited with its algorithmic traffic: read
// xc, xp and b once, write xo once (neighbour reads of xc are cache hits).
template <typename T>
void Problem::smooth_step(int nl, int ncols, const T* xc, const T* xp, T* xo, const T* b, long ld, const double* prm,
                          int s) {
  const int streams = 2 + (xc ? 1 : 0) + (xp ? 1 : 0);
  timed(LRPOST_KERNEL_SMOOTHER_STEP, (double)streams * sizeof(T) * (double)nl * nl * ncols,
        [&] { mg_smooth_step<T>(st, nl, ncols, xc, xp, xo, b, ld, prm, s); });
}

void Problem::prof_reset() {
  for (auto& ps : prof_) {
    ps.used = 0;
    ps.bytes = 0.0;
    ps.flops = 0.0;
  }
}

void Problem::prof_read(int kind, int64_t* launches, double* ms, double* bytes, double* flops) {
  sync();
  ProfSlot& ps = prof_[kind];
  double tot = 0.0;
  for (size_t i = 0; i < ps.used; ++i) {
    float t = 0.0f;
    LRP_HIP(hipEventElapsedTime(&t, ps.ev[i].first, ps.ev[i].second));
    tot += t;
  }
  *launches = (int64_t)ps.used;
  *ms = tot;
  *bytes = ps.bytes;
  if (flops) *flops = ps.flops;
  ps.used = 0;
  ps.bytes = 0.0;
  ps.flops = 0.0;
}

void Problem::mg_cycles_f32(int ncols, const float* B, float* X, const std::vector<ShiftCoef>& neg, int cycles) {
  vcycle_zero<float>(ncols, B, X);
  if (cycles <= 1) return;
  const size_t blk = (size_t)nx * ncols;
  float* R = mg_f_.as<float>() + 2 * blk;
  float* E = R + blk;
  op_w_h_.assign((size_t)4 * ncols, 0.0);
  for (int c = 0; c < ncols; ++c) {
    stencil_weights(neg[c].a, neg[c].b, h, &op_w_h_[(size_t)4 * c]);
    op_w_h_[(size_t)4 * c + 3] = 1.0;
  }
  op_w_.ensure(sizeof(double) * op_w_h_.size());
  to_device(op_w_.as<double>(), op_w_h_.data(), op_w_h_.size());
  for (int cyc = 1; cyc < cycles; ++cyc) {
    timed(LRPOST_KERNEL_STENCIL, sizeof(float) * 3.0 * (double)nx * ncols,
          [&] { stencil<float>(st, n, ncols, X, nx, R, nx, B, nx, op_w_.as<double>()); });  // R = B - A X
    if (vcycle_fused()) {
      vcycle_zero<float>(ncols, R, X, true);  // X += V(R) in the finest up kernel
    } else {
      vcycle_zero<float>(ncols, R, E);
      axpby<float>(st, nx, ncols, E, nx, X, nx, 1.0, 1.0);
    }
  }
}

void Problem::mg_solve(int ncols, const double* B, double* X, const std::vector<ShiftCoef>& ab_in, int cycles,
                       int refine) {
  if (ncols <= 0) return;
  std::vector<ShiftCoef> ab(ncols);
  for (int c = 0; c < ncols; ++c) ab[c] = ab_in.size() == 1 ? ab_in[0] : ab_in[c];
  upload_mg_params(ab);
  std::vector<ShiftCoef> neg(ncols);
  for (int c = 0; c < ncols; ++c) neg[c] = {-ab[c].a, -ab[c].b};
  std::vector<double> one(1, 1.0);
  const size_t blk = (size_t)nx * ncols;
  if (desc.precision == LRPOST_MIXED) {
    // float32 V-cycles; each refinement round solves for the correction of
    // the float64 residual and adds it in float64
    mg_f_.ensure(sizeof(float) * 4 * blk);
    float* Bf = mg_f_.as<float>();
    float* Xf = Bf + blk;
    d2f(st, (long)blk, B, Bf);
    mg_cycles_f32(ncols, Bf, Xf, neg, cycles);
    f2d(st, (long)blk, Xf, X);
    if (refine > 0) {
      mg_res_.ensure(sizeof(double) * blk);
      double* R = mg_res_.as<double>();
      for (int r = 0; r < refine; ++r) {
        apply_op(ncols, X, R, neg, B, &one);  // R = B - A X in float64
        d2f(st, (long)blk, R, Bf);
        mg_cycles_f32(ncols, Bf, Xf, neg, cycles);
        f2d(st, (long)blk, Xf, R);
        axpby<double>(st, nx, ncols, R, nx, X, nx, 1.0, 1.0);
      }
    }
    LRP_HIP(hipGetLastError());
    return;
  }
  vcycle_zero<double>(ncols, B, X);
  if (cycles <= 1) {
    LRP_HIP(hipGetLastError());
    return;
  }
  // residual correction: X += V(B - A X)
  mg_res_.ensure(sizeof(double) * 2 * blk);
  double* R = mg_res_.as<double>();
  double* E = R + blk;
  for (int cyc = 1; cyc < cycles; ++cyc) {
    apply_op(ncols, X, R, neg, B, &one);
    if (vcycle_fused()) {
      vcycle_zero<double>(ncols, R, X, true);  // X += V(R) in the finest up kernel
    } else {
      vcycle_zero<double>(ncols, R, E);
      axpby<double>(st, nx, ncols, E, nx, X, nx, 1.0, 1.0);
    }
  }
  LRP_HIP(hipGetLastError());
}

void Problem::gram(int m, const double* A, int q, const double* B, std::vector<double>& C) {
  C.assign((size_t)m * q, 0.0);
  if (m <= 0 || q <= 0) return;
  gram_out_.ensure(sizeof(double) * (size_t)m * q);
  gram_dev(m, A, q, B, gram_out_.as<double>());
  to_host(C.data(), gram_out_.as<double>(), (size_t)m * q);
}

void Problem::proj(int m, const double* A, const std::vector<double>& Q, int p, double* C, double beta) {
  if (p <= 0) return;
  proj_q_.ensure(sizeof(double) * std::max<size_t>(1, (size_t)m * p));
  if (m > 0) to_device(proj_q_.as<double>(), Q.data(), (size_t)m * p);
  timed(LRPOST_KERNEL_PROJ, sizeof(double) * (double)(m + (beta != 0.0 ? 2 : 1) * p) * nx,
        [&] { ::lrp::proj<double>(st, nx, m, A, nx, proj_q_.as<double>(), m, p, C, nx, beta); },
        2.0 * m * p * (double)nx);
  LRP_HIP(hipGetLastError());
}

// Stage 1 (the matrix-core kernel) is credited with reading A and B once and
// with 2 m q nx flops.
void Problem::gram_dev(int m, const double* A, int q, const double* B, double* C) {
  if (m <= 0 || q <= 0) return;
  std::vector<GramGroup> g{GramGroup{A, B, nullptr, C, nx, nx, m, 0, m, q, 0}};
  gram_dev_grouped(g);
}

// Several Gram products A_g^T B_g (nx rows) with one launch per stage for up
// to kProjGroupMax of them; each result is the one gram_dev gives.  Products
// of different tile shapes (64, 128 or 192 rows from m; 64 or 128 columns
// from q) go to separate launches, so that each runs with its own tile.
void Problem::gram_dev_grouped(std::vector<GramGroup>& gs) {
  std::vector<size_t> off(gs.size() + 1, 0);
  for (size_t i = 0; i < gs.size(); ++i) off[i + 1] = off[i] + (size_t)gram_part_doubles(nx, gs[i].m, gs[i].q);
  if (off.back() == 0) return;
  gram_part_.ensure(sizeof(double) * off.back());
  for (size_t i = 0; i < gs.size(); ++i) gs[i].part = gram_part_.as<double>() + off[i];
  for (int cls = 1; cls <= 12; ++cls) {
    // tile class: height from m (1..3), width from q (64 or 128), float64 or
    // float32 operands (one kernel per launch)
    std::vector<GramGroup> gc;
    for (const GramGroup& g : gs)
      if (g.m > 0 && g.q > 0 && gram_bm(g.m) + 3 * (gram_bq(g.q) - 1) + 6 * (g.A32 ? 1 : 0) == cls) gc.push_back(g);
    for (size_t g0 = 0; g0 < gc.size(); g0 += kProjGroupMax) {
      const int n = (int)std::min<size_t>(kProjGroupMax, gc.size() - g0);
      double bytes = 0.0, flops = 0.0;
      for (int i = 0; i < n; ++i) {
        const GramGroup& g = gc[g0 + i];
        bytes += ((g.A32 ? sizeof(float) : sizeof(double)) * (double)g.m + sizeof(double) * (double)g.q) * nx;
        flops += 2.0 * g.m * g.q * (double)nx;
      }
      timed(gc[g0].A32 ? LRPOST_KERNEL_GRAM32 : LRPOST_KERNEL_GRAM, bytes,
            [&] { gram_mfma_partials(st, nx, n, gc.data() + g0); }, flops);
      sum_partials_grouped(st, n, gc.data() + g0);
    }
  }
  LRP_HIP(hipGetLastError());
}

void Problem::proj_dev(int m, const double* A, const double* Q, int ldq, int p, double* C, double beta,
                       double alpha) {
  if (p <= 0) return;
  timed(LRPOST_KERNEL_PROJ, sizeof(double) * (double)(m + (beta != 0.0 ? 2 : 1) * p) * nx, [&] {
    if (alpha == 1.0 || m <= 0) {
      ::lrp::proj<double>(st, nx, m, A, nx, Q, ldq, p, C, nx, beta);
    } else {
      const ProjGroup g{A, Q, C, C, nx, nx, nx, ldq, m, p};
      proj_grouped(st, 1, &g, alpha, beta);
    }
  }, 2.0 * m * p * (double)nx);
  LRP_HIP(hipGetLastError());
}

// Several projections C_g = beta C_g + alpha A_g Q_g (nx rows), grouped
// launches credited like proj_dev.
void Problem::proj_dev_grouped(const std::vector<ProjGroup>& pg_all, double alpha, double beta) {
  // float64 and float32-operand products in separate launches
  for (int f32 = 0; f32 < 2; ++f32) {
    std::vector<ProjGroup> pg;
    for (const ProjGroup& g : pg_all)
      if ((g.A32 != nullptr) == (f32 == 1)) pg.push_back(g);
    for (size_t g0 = 0; g0 < pg.size(); g0 += kProjGroupMax) {
      const int n = (int)std::min<size_t>(kProjGroupMax, pg.size() - g0);
      double bytes = 0.0, flops = 0.0;
      for (int i = 0; i < n; ++i) {
        const ProjGroup& g = pg[g0 + i];
        bytes += ((g.A32 ? sizeof(float) : sizeof(double)) * (double)g.m +
                  sizeof(double) * (double)((beta != 0.0 ? 2 : 1) * g.p)) * g.nrows;
        flops += 2.0 * g.m * g.p * (double)g.nrows;
      }
      timed(f32 ? LRPOST_KERNEL_PROJ32 : LRPOST_KERNEL_PROJ, bytes,
            [&] { proj_grouped(st, n, pg.data() + g0, alpha, beta); }, flops);
    }
  }
  LRP_HIP(hipGetLastError());
}

// K and M are diagonalized by the two-dimensional discrete sine transform
// S kron S with the orthonormal, symmetric DST-I matrix
// S[i][p] = sqrt(2/(n+1)) sin((i+1)(p+1) pi/(n+1)).  With the 1D eigenvalues
// k_p = (2/h)(1 - cos t_p) of K1 = tridiag(-1, 2, -1)/h and
// m_p = (h/3)(2 + cos t_p) of M1 = (h/6) tridiag(1, 4, 1), t_p = (p+1) pi h,
// mode (p, q) of K + M = K1 kron M1 + M1 kron K1 + M1 kron M1 has eigenvalue
// k_p m_q + m_p k_q + m_p m_q.  The prior covariance's symmetric root
// (alpha tau)^{-1/2} (K+M)^{-1/2} is then S2 diag(w) S2 with w the scaled
// inverse square roots; on a nodal vector viewed as the n x n matrix
// X[i, j] (x1 index i fastest) it is S (w .* (S X S)) S.
void Problem::prior_sqrt(int ncols, const double* X, double* Y) {
  if (ncols <= 0) return;
  if (!sine_.p) {
    std::vector<double> S((size_t)n * n), w(nx), k1(n), m1(n);
    const double sc = std::sqrt(2.0 / (n + 1));
    for (int p = 0; p < n; ++p) {
      for (int i = 0; i < n; ++i) S[(size_t)p * n + i] = sc * std::sin(M_PI * (double)(i + 1) * (p + 1) / (n + 1));
      const double c = std::cos(M_PI * (p + 1) * h);
      k1[p] = 2.0 / h * (1.0 - c);
      m1[p] = h / 3.0 * (2.0 + c);
    }
    const double s = 1.0 / std::sqrt(desc.alpha * tau);
    for (int q = 0; q < n; ++q)
      for (int p = 0; p < n; ++p) w[(size_t)q * n + p] = s / std::sqrt(k1[p] * m1[q] + m1[p] * k1[q] + m1[p] * m1[q]);
    sine_.ensure(sizeof(double) * S.size());
    root_w_.ensure(sizeof(double) * w.size());
    to_device(sine_.as<double>(), S.data(), S.size());
    to_device(root_w_.as<double>(), w.data(), w.size());
  }
  const double* S = sine_.as<double>();
  sqrt_tmp_.ensure(sizeof(double) * (size_t)nx * ncols);
  double* T = sqrt_tmp_.as<double>();
  const long nn = (long)n * n;
  // along x1: T = S X over all n * ncols lines; along x2: Y_c = T_c S per vector
  dense->gemm(false, false, n, n * ncols, n, 1.0, S, n, X, n, 0.0, T, n);
  dense->gemm_strided_batched(false, false, n, n, n, 1.0, T, n, nn, S, n, 0, 0.0, Y, n, nn, ncols);
  scale_nodes(st, nx, ncols, Y, nx, root_w_.as<double>());
  LRP_HIP(hipGetLastError());
  dense->gemm_strided_batched(false, false, n, n, n, 1.0, Y, n, nn, S, n, 0, 0.0, T, n, nn, ncols);
  dense->gemm(false, false, n, n * ncols, n, 1.0, S, n, T, n, 0.0, Y, n);
}

void Problem::sym_eig(int nn, const double* A, int lda, std::vector<double>& w, std::vector<double>& V) {
  w.assign(nn, 0.0);
  V.assign((size_t)nn * nn, 0.0);
  if (nn == 0) return;
  if (nn <= 64) {
    if (!syev(nn, A, lda, w.data(), V.data())) fail(LRPOST_EBREAKDOWN, "symmetric eigensolve failed");
    return;
  }
  std::vector<double> tmp((size_t)nn * nn);
  for (int j = 0; j < nn; ++j)
    for (int i = 0; i < nn; ++i) tmp[(size_t)j * nn + i] = 0.5 * (A[(size_t)j * lda + i] + A[(size_t)i * lda + j]);
  st_small_.ensure(sizeof(double) * ((size_t)nn * nn + nn));
  double* dA = st_small_.as<double>();
  double* dw = dA + (size_t)nn * nn;
  to_device(dA, tmp.data(), tmp.size());
  dense->syevd(nn, dA, nn, dw, eig_work_);
  // eigenvectors and eigenvalues are adjacent on the device: one read-back
  tmp.resize((size_t)nn * nn + nn);
  to_host(tmp.data(), dA, tmp.size());
  std::copy(tmp.begin(), tmp.begin() + (size_t)nn * nn, V.begin());
  std::copy(tmp.begin() + (size_t)nn * nn, tmp.end(), w.begin());
}

void Problem::small_svd(int m, int nn, const double* A, int lda, bool accurate, std::vector<double>& s,
                        std::vector<double>& U, std::vector<double>& V) {
  const int k = std::min(m, nn);
  if (accurate || k <= 48) {
    svd(m, nn, A, lda, s, U, V);
    return;
  }
  // eigenpairs of the smaller Gram matrix
  const bool right = nn <= m;  // A^T A (nn x nn) when nn <= m
  const int g = right ? nn : m;
  std::vector<double> G((size_t)g * g);
  if (right) matmul(g, g, m, A, lda, true, A, lda, false, G.data(), g, 1.0, 0.0);
  else matmul(g, g, nn, A, lda, false, A, lda, true, G.data(), g, 1.0, 0.0);
  std::vector<double> w, E;
  sym_eig(g, G.data(), g, w, E);
  s.assign(k, 0.0);
  U.assign((size_t)m * k, 0.0);
  V.assign((size_t)nn * k, 0.0);
  for (int c = 0; c < k; ++c) {
    const int j = g - 1 - c;  // descending
    const double sv = std::sqrt(std::max(w[j], 0.0));
    s[c] = sv;
    if (right) {
      for (int i = 0; i < nn; ++i) V[(size_t)c * nn + i] = E[(size_t)j * g + i];
      if (sv > 0)
        for (int i = 0; i < m; ++i) {
          double t = 0.0;
          for (int l = 0; l < nn; ++l) t += A[(size_t)l * lda + i] * E[(size_t)j * g + l];
          U[(size_t)c * m + i] = t / sv;
        }
    } else {
      for (int i = 0; i < m; ++i) U[(size_t)c * m + i] = E[(size_t)j * g + i];
      if (sv > 0)
        for (int i = 0; i < nn; ++i) {
          double t = 0.0;
          for (int l = 0; l < m; ++l) t += A[(size_t)i * lda + l] * E[(size_t)j * g + l];
          V[(size_t)c * nn + i] = t / sv;
        }
    }
  }
}

// ---------------------------------------------------------------------------
// Low-rank space-time solve of tau K Y + M Y C^T = F1 F2^T (Sec. 6.1 eq.
// st_pde with L = tau K; implicit Euler C = I - S).
//
// The spatial factor is sought in a block rational Krylov space
// span{(tau K + p_i M)^{-1} F1}, built with multigrid solves and kept
// M-orthonormal.  On that space the projected problem (Sec. 6.1 eq. amen_2,
// the small system in time) is solved exactly: with Q^T M Q = I and
// Q^T tau K Q = E diag(theta) E^T, each projected mode obeys
// (1 + theta_i) z_k = z_{k-1} + g_k.  The result Q E Z is truncated through an
// SVD of the small coefficient matrix (M-weighted Frobenius norm).
// The adjoint equation tau K Y + M Y C = F is the same problem with time
// reversed on both sides.
// ---------------------------------------------------------------------------
void Problem::st_prepare(const std::vector<const LowRank*>& F, bool adjoint, std::vector<StPrep>& prs) {
  // 1. orthonormalize each source's spatial factor (eigen-based, drops null
  // directions); the Gram matrices of all sources are one grouped launch and
  // one read-back, the transforms one grouped projection
  const int nb = (int)F.size();
  std::vector<size_t> goff(nb + 1, 0);
  for (int j = 0; j < nb; ++j) {
    prs[j].r1 = 0;
    goff[j + 1] = goff[j] + (size_t)F[j]->rank * F[j]->rank;
  }
  if (goff[nb] == 0) return;
  st_prep_g_.ensure(sizeof(double) * goff[nb]);
  double* Gd = st_prep_g_.as<double>();
  std::vector<GramGroup> gg;
  for (int j = 0; j < nb; ++j) {
    const int rf0 = F[j]->rank;
    if (rf0 > 0) gg.push_back(GramGroup{F[j]->a(), F[j]->a(), nullptr, Gd + goff[j], nx, nx, rf0, 0, rf0, rf0, 0});
  }
  gram_dev_grouped(gg);
  std::vector<double> Gh(goff[nb]);
  to_host(Gh.data(), Gd, Gh.size());
  std::vector<std::vector<double>> T1(nb);
  std::vector<int> ok(nb, 1);
  host_parallel(nb, [&](int j) {
    const LowRank& f = *F[j];
    const int rf0 = f.rank;
    StPrep& pr = prs[j];
    if (rf0 == 0) return;
    std::vector<double> w(rf0), U((size_t)rf0 * rf0);
    if (!syev(rf0, Gh.data() + goff[j], rf0, w.data(), U.data())) {
      ok[j] = 0;
      return;
    }
    const double wmax = std::max(w[rf0 - 1], 0.0);
    std::vector<int> keep;
    for (int c = rf0 - 1; c >= 0; --c)
      if (w[c] > 1e-26 * wmax && wmax > 0) keep.push_back(c);
    const int r1 = (int)keep.size();
    if (r1 == 0) return;
    T1[j].assign((size_t)rf0 * r1, 0.0);
    std::vector<double>& F2p = pr.F2p;
    F2p.assign((size_t)nt * r1, 0.0);
    for (int c = 0; c < r1; ++c) {
      const int e = keep[c];
      const double sw = std::sqrt(w[e]);
      for (int i = 0; i < rf0; ++i) T1[j][(size_t)c * rf0 + i] = U[(size_t)e * rf0 + i] / sw;
      for (int k = 0; k < nt; ++k) {
        const int kk = adjoint ? nt - 1 - k : k;
        double acc = 0.0;
        for (int i = 0; i < rf0; ++i) acc += f.B[(size_t)i * nt + kk] * U[(size_t)e * rf0 + i];
        F2p[(size_t)c * nt + k] = acc * sw;
      }
    }
    pr.r1 = r1;
  });
  for (int j = 0; j < nb; ++j)
    if (!ok[j]) fail(LRPOST_EBREAKDOWN, "source Gram eigensolve failed");
  std::vector<double> Th(goff[nb], 0.0);
  std::vector<ProjGroup> pg;
  for (int j = 0; j < nb; ++j)
    if (prs[j].r1 > 0) std::copy(T1[j].begin(), T1[j].end(), Th.begin() + goff[j]);
  st_prep_t_.ensure(sizeof(double) * goff[nb]);
  to_device(st_prep_t_.as<double>(), Th.data(), Th.size());
  for (int j = 0; j < nb; ++j) {
    StPrep& pr = prs[j];
    if (pr.r1 == 0) continue;
    const int rf0 = F[j]->rank;
    pr.Fb.ensure(sizeof(double) * (size_t)nx * pr.r1);
    pg.push_back(ProjGroup{F[j]->a(), st_prep_t_.as<double>() + goff[j], pr.Fb.as<double>(), pr.Fb.as<double>(), nx, nx,
                           nx, rf0, rf0, pr.r1});
  }
  proj_dev_grouped(pg, 1.0, 0.0);
}


// Pole solves of a batch of prepared sources in one multigrid solve with
// per-column shifts: Wall (nx x sum_j r1_j npol) holds, pole after pole and
// source after source, (tau K + p_i M)^{-1} Fb_j.
double* Problem::st_pole_solves(const std::vector<const StPrep*>& prs) {
  const int npol = (int)poles.size();
  long cols = 0;
  for (auto* pr : prs) cols += (long)pr->r1 * npol;
  if (cols == 0) return nullptr;
  st_wall_.ensure(sizeof(double) * (size_t)nx * cols);
  st_brep_.ensure(sizeof(double) * (size_t)nx * cols);
  double* Wall = st_wall_.as<double>();
  double* Brep = st_brep_.as<double>();
  // pole-major: the sources' columns for pole i are adjacent (block i of
  // width sum r1), the first block assembled from the sources and copied on
  std::vector<ShiftCoef> ab((size_t)cols);
  const long R1 = cols / npol;
  long off = 0;
  for (auto* pr : prs) {
    if (pr->r1 == 0) continue;
    LRP_HIP(hipMemcpyAsync(Brep + (size_t)off * nx, pr->Fb.p, sizeof(double) * (size_t)nx * pr->r1,
                           hipMemcpyDeviceToDevice, st));
    off += pr->r1;
  }
  for (int i = 1; i < npol; ++i)
    LRP_HIP(hipMemcpyAsync(Brep + (size_t)i * R1 * nx, Brep, sizeof(double) * (size_t)nx * R1,
                           hipMemcpyDeviceToDevice, st));
  for (int i = 0; i < npol; ++i)
    for (long c = 0; c < R1; ++c) ab[(size_t)i * R1 + c] = {tau, poles[i]};
  st_spatial_solve((int)cols, Brep, Wall, ab, st_cycles);
  return Wall;
}

void Problem::spacetime_solve(const LowRank& F, LowRank& Y, bool adjoint) {
  spacetime_solve_batch({&F}, {&Y}, adjoint);
}

// Space-time solves of a batch with the residual monitor of the AMEn solver
// (Sec. 6.1): the relative residual of eq. st_pde is measured for every
// truncated solution, as is the residual preconditioned by two V-cycles of
// M + tau K per time step (the block-diagonal part of eq. pre_1), whose
// relative size tracks the relative error of the solution.  Where the
// preconditioned residual exceeds the threshold the spatial basis of that
// source is enriched -- the pole set refined by the geometric midpoints of
// neighbouring poles and extended at the original spacing up to the top of
// the time-step-scaled spectrum, which resolves sources with much fine-scale
// content -- and the solve repeated.  A residual still above the threshold
// is counted (st_unresolved), and in the strict mode ends in LRPOST_ENOCONV.
// The default threshold is 50 trunc_tol; in mixed precision at least 1e-4,
// since the float32 multigrid solves that build the basis bound the
// attainable preconditioned residual (measured up to about 1e-4 on 256^2
// meshes and 7e-4 on 1024^2 meshes for sources with independent nodal
// values).
void Problem::spacetime_solve_batch(const std::vector<const LowRank*>& F, const std::vector<LowRank*>& Y,
                                    bool adjoint) {
  cd_sign = adjoint ? -1 : 1;  // the adjoint solves carry the transposed spatial operator
  if (poles_low_.empty()) {
    st_solve_group(F, Y, adjoint);
    return;
  }
  // sources of rank at most 2 (one basis column per pole and source column)
  // are solved with the larger pole set of low-rank sources, the others with
  // the base set; each source's result depends on its own rank only
  std::vector<const LowRank*> Fl, Fh;
  std::vector<LowRank*> Yl, Yh;
  for (size_t j = 0; j < F.size(); ++j) {
    if (F[j]->rank <= 2) {
      Fl.push_back(F[j]);
      Yl.push_back(Y[j]);
    } else {
      Fh.push_back(F[j]);
      Yh.push_back(Y[j]);
    }
  }
  if (!Fl.empty()) {
    const std::vector<double> base = poles;
    poles = poles_low_;
    try {
      st_solve_group(Fl, Yl, adjoint);
    } catch (...) {
      poles = base;
      throw;
    }
    poles = base;
  }
  if (!Fh.empty()) st_solve_group(Fh, Yh, adjoint);
}

// One group of sources with the current pole set: a pass, then the residual
// check and at most one enrichment (see spacetime_solve_batch).
void Problem::st_solve_group(const std::vector<const LowRank*>& F, const std::vector<LowRank*>& Y, bool adjoint) {
  st_solve_pass(F, Y, adjoint);
  if (st_check == 0) return;
  const int nb = (int)F.size();
  std::vector<const LowRank*> cy(Y.begin(), Y.end());
  std::vector<double> rel, prel;
  {
    PhaseTimer pt(this, kPhCheck);
    st_residuals(F, cy, adjoint, rel, prel);
  }
  auto record = [&]() {
    double w = 0.0, wp = 0.0;
    for (size_t j = 0; j < rel.size(); ++j) {
      w = std::max(w, rel[j]);
      wp = std::max(wp, prel[j]);
    }
    stats.last_st_resid = w;
    stats.last_st_presid = wp;
    return wp;
  };
  record();
  if (st_check < 2) return;
  const double thr = st_rtol > 0 ? st_rtol
                                 : std::max(50.0 * desc.trunc_tol, desc.precision == LRPOST_MIXED ? 1e-4 : 0.0);
  std::vector<int> bad;
  for (int j = 0; j < nb; ++j)
    if (!(prel[j] <= thr)) bad.push_back(j);
  if (bad.empty()) return;
  ++stats.st_enrichments;
  const std::vector<double> base = poles;
  const double ratio = base.size() > 1 ? std::sqrt(base[1] / base[0]) : 3.0;
  std::vector<double> fine;
  fine.push_back(base.front() / ratio);
  for (size_t i = 0; i < base.size(); ++i) {
    fine.push_back(base[i]);
    if (i + 1 < base.size()) fine.push_back(std::sqrt(base[i] * base[i + 1]));
  }
  const double top = std::min(tau * pole_lam_max_, 1e4);
  for (double p = base.back() * ratio; p < top * ratio && fine.size() < 48; p *= ratio * ratio) fine.push_back(p);
  // the enriched solves in chunks whose pole-solve columns stay within those
  // of the first pass, so that enrichment needs no more device memory
  long budget_cols = 0;
  for (int j = 0; j < nb; ++j) budget_cols += (long)F[j]->rank * (long)base.size();
  std::vector<const LowRank*> Fb;
  std::vector<LowRank*> Yb;
  for (int j : bad) {
    Fb.push_back(F[j]);
    Yb.push_back(Y[j]);
  }
  poles = fine;
  try {
    size_t i0 = 0;
    while (i0 < Fb.size()) {
      size_t i1 = i0;
      long cols = 0;
      while (i1 < Fb.size() && (i1 == i0 || cols + (long)Fb[i1]->rank * (long)fine.size() <= budget_cols)) {
        cols += (long)Fb[i1]->rank * (long)fine.size();
        ++i1;
      }
      st_solve_pass(std::vector<const LowRank*>(Fb.begin() + i0, Fb.begin() + i1),
                    std::vector<LowRank*>(Yb.begin() + i0, Yb.begin() + i1), adjoint);
      i0 = i1;
    }
  } catch (...) {
    poles = base;
    throw;
  }
  poles = base;
  std::vector<const LowRank*> cyb(Yb.begin(), Yb.end());
  {
    PhaseTimer pt(this, kPhCheck);
    st_residuals(Fb, cyb, adjoint, rel, prel);
  }
  const double worst = record();
  if (worst <= thr) return;
  ++stats.st_unresolved;
  if (st_check >= 3) {
    char msg[160];
    std::snprintf(msg, sizeof msg,
                  "space-time solve: preconditioned relative residual %.3e above %.3e after enrichment", worst, thr);
    fail(LRPOST_ENOCONV, msg);
  }
}

// Relative residuals ||tau K Y + M Y D^T - F||_F / ||F||_F of the solutions
// Y_j = Y1 Y2^T of sources F_j = F1 F2^T, with D = C (forward: y_k - y_{k-1})
// or C^T (adjoint: y_k - y_{k+1}).  The residual is A B^T with
// A = [tau K Y1, M Y1, F1] and B = [Y2, D Y2, -F2]; with the host QR
// B = Q_B R_B its norm is ||A R_B^T||_F, formed on the device and summed
// through a Gram product, so that the cancellation between the three terms
// happens in the explicit sum and not between squared norms.
void Problem::st_residuals(const std::vector<const LowRank*>& F, const std::vector<const LowRank*>& Y, bool adjoint,
                           std::vector<double>& rel, std::vector<double>& prel) {
  const int nb = (int)F.size();
  rel.assign(nb, 0.0);
  prel.assign(nb, 0.0);
  std::vector<int> w(nb), c(nb), f(nb);
  std::vector<size_t> aoff(nb + 1, 0), coff(nb + 1, 0), qoff(nb + 1, 0), goff(nb + 1, 0);
  for (int j = 0; j < nb; ++j) {
    f[j] = F[j]->rank;
    w[j] = 2 * Y[j]->rank + f[j];
    c[j] = std::min(nt, w[j]);
    aoff[j + 1] = aoff[j] + (size_t)w[j];
    coff[j + 1] = coff[j] + (size_t)c[j];
    qoff[j + 1] = qoff[j] + (size_t)w[j] * c[j];
    goff[j + 1] = goff[j] + (size_t)c[j] * c[j] + (size_t)f[j] * f[j];
  }
  if (aoff[nb] == 0) return;
  st_res_a_.ensure(sizeof(double) * (size_t)nx * aoff[nb]);
  st_res_b_.ensure(sizeof(double) * (size_t)nx * std::max<size_t>(coff[nb], 1));
  st_res_q_.ensure(sizeof(double) * std::max<size_t>(qoff[nb], 1));
  st_res_g_.ensure(sizeof(double) * std::max<size_t>(goff[nb], 1));
  double* A = st_res_a_.as<double>();
  double* Bd = st_res_b_.as<double>();
  std::vector<double> Qh(std::max<size_t>(qoff[nb], 1), 0.0);
  std::vector<std::vector<double>> F2g(nb);
  std::vector<ProjGroup> pg;
  std::vector<GramGroup> gg;
  for (int j = 0; j < nb; ++j) {
    const LowRank& y = *Y[j];
    const LowRank& fs = *F[j];
    const int r = y.rank;
    double* Aj = A + aoff[j] * nx;
    if (r > 0) {
      st_apply(r, y.a(), Aj, {{tau, 0.0}});
      apply_op(r, y.a(), Aj + (size_t)r * nx, {{0.0, 1.0}});
    }
    if (f[j] > 0)
      LRP_HIP(hipMemcpyAsync(Aj + (size_t)2 * r * nx, fs.a(), sizeof(double) * nx * f[j], hipMemcpyDeviceToDevice, st));
  }
  // host side of every source on parallel threads (no HIP calls inside)
  host_parallel(nb, [&](int j) {
    const LowRank& y = *Y[j];
    const LowRank& fs = *F[j];
    const int r = y.rank;
    // B = [Y2, D Y2, -F2] (nt x w) and its triangular factor
    std::vector<double> B((size_t)nt * std::max(w[j], 1), 0.0);
    for (int cc = 0; cc < r; ++cc)
      for (int k = 0; k < nt; ++k) {
        const double v = y.B[(size_t)cc * nt + k];
        const int kn = adjoint ? k + 1 : k - 1;
        const double prev = (kn >= 0 && kn < nt) ? y.B[(size_t)cc * nt + kn] : 0.0;
        B[(size_t)cc * nt + k] = v;
        B[(size_t)(r + cc) * nt + k] = v - prev;
      }
    for (int cc = 0; cc < f[j]; ++cc)
      for (int k = 0; k < nt; ++k) B[(size_t)(2 * r + cc) * nt + k] = -fs.B[(size_t)cc * nt + k];
    if (w[j] == 0) return;
    std::vector<double> RB;
    householder_r(nt, w[j], B.data(), nt, RB);
    // R_B^T (w x c)
    double* Rt = Qh.data() + qoff[j];
    for (int jj = 0; jj < c[j]; ++jj)
      for (int i = 0; i < w[j]; ++i) Rt[(size_t)jj * w[j] + i] = RB[(size_t)i * c[j] + jj];
    // Gram of the source's temporal factor (host)
    F2g[j].assign((size_t)f[j] * f[j], 0.0);
    for (int a = 0; a < f[j]; ++a)
      for (int b = 0; b < f[j]; ++b) {
        double t = 0.0;
        for (int k = 0; k < nt; ++k) t += fs.B[(size_t)a * nt + k] * fs.B[(size_t)b * nt + k];
        F2g[j][(size_t)b * f[j] + a] = t;
      }
  });
  to_device(st_res_q_.as<double>(), Qh.data(), Qh.size());
  double* Gd = st_res_g_.as<double>();
  for (int j = 0; j < nb; ++j) {
    if (w[j] == 0) continue;
    double* Cj = Bd + coff[j] * nx;
    pg.push_back(ProjGroup{A + aoff[j] * nx, st_res_q_.as<double>() + qoff[j], Cj, Cj, nx, nx, nx, w[j], w[j], c[j]});
    gg.push_back(GramGroup{Cj, Cj, nullptr, Gd + goff[j], nx, nx, c[j], 0, c[j], c[j], 0});
    if (f[j] > 0) {
      const double* F1 = A + (aoff[j] + (size_t)2 * Y[j]->rank) * nx;
      gg.push_back(GramGroup{F1, F1, nullptr, Gd + goff[j] + (size_t)c[j] * c[j], nx, nx, f[j], 0, f[j], f[j], 0});
    }
  }
  proj_dev_grouped(pg, 1.0, 0.0);
  // the preconditioned residual (I kron (M + tau K))^{-1} R = (P A R_B^T) Q_B^T
  // and source P F1 F2^T, P two V-cycles for M + tau K: the residual columns
  // of all sources and their source columns in one multigrid solve
  std::vector<size_t> poff(nb + 1, 0);
  for (int j = 0; j < nb; ++j) poff[j + 1] = poff[j] + (size_t)c[j] + f[j];
  st_res_p_.ensure(sizeof(double) * (size_t)nx * std::max<size_t>(poff[nb], 1) * 2);
  double* Pin = st_res_p_.as<double>();
  double* Pout = Pin + (size_t)nx * poff[nb];
  for (int j = 0; j < nb; ++j) {
    if (c[j] > 0)
      LRP_HIP(hipMemcpyAsync(Pin + poff[j] * nx, Bd + coff[j] * nx, sizeof(double) * nx * c[j],
                             hipMemcpyDeviceToDevice, st));
    if (f[j] > 0)
      LRP_HIP(hipMemcpyAsync(Pin + (poff[j] + c[j]) * nx, A + (aoff[j] + (size_t)2 * Y[j]->rank) * nx,
                             sizeof(double) * nx * f[j], hipMemcpyDeviceToDevice, st));
  }
  if (poff[nb] > 0) st_spatial_solve((int)poff[nb], Pin, Pout, {{tau, 1.0}}, 2);
  std::vector<size_t> hoff(nb + 1, 0);
  for (int j = 0; j < nb; ++j) hoff[j + 1] = hoff[j] + (size_t)c[j] * c[j] + (size_t)f[j] * f[j];
  st_res_h_.ensure(sizeof(double) * std::max<size_t>(hoff[nb], 1));
  double* Hd = st_res_h_.as<double>();
  for (int j = 0; j < nb; ++j) {
    if (c[j] > 0) {
      const double* Pc = Pout + poff[j] * nx;
      gg.push_back(GramGroup{Pc, Pc, nullptr, Hd + hoff[j], nx, nx, c[j], 0, c[j], c[j], 0});
    }
    if (f[j] > 0) {
      const double* Pf = Pout + (poff[j] + c[j]) * nx;
      gg.push_back(GramGroup{Pf, Pf, nullptr, Hd + hoff[j] + (size_t)c[j] * c[j], nx, nx, f[j], 0, f[j], f[j], 0});
    }
  }
  gram_dev_grouped(gg);
  std::vector<double> Gh(goff[nb]), Hh(hoff[nb]);
  to_host(Gh.data(), Gd, Gh.size());
  to_host(Hh.data(), Hd, Hh.size());
  auto ratio = [&](const double* G, const double* G1, int j) {
    double r2 = 0.0, f2 = 0.0;
    for (int i = 0; i < c[j]; ++i) r2 += G[(size_t)i * c[j] + i];
    for (size_t i = 0; i < (size_t)f[j] * f[j]; ++i) f2 += G1[i] * F2g[j][i];
    return f2 > 0 ? std::sqrt(std::max(r2, 0.0) / f2) : (r2 > 0 ? INFINITY : 0.0);
  };
  for (int j = 0; j < nb; ++j) {
    if (w[j] == 0) continue;
    rel[j] = ratio(Gh.data() + goff[j], Gh.data() + goff[j] + (size_t)c[j] * c[j], j);
    prel[j] = ratio(Hh.data() + hoff[j], Hh.data() + hoff[j] + (size_t)c[j] * c[j], j);
  }
}

void Problem::st_solve_pass(const std::vector<const LowRank*>& F, const std::vector<LowRank*>& Y, bool adjoint) {
  const int nb = (int)F.size();
  std::vector<StPrep> prs(nb);
  std::vector<const StPrep*> pp;
  {
    PhaseTimer pt(this, kPhPrep);
    st_prepare(F, adjoint, prs);
    for (int j = 0; j < nb; ++j) pp.push_back(&prs[j]);
  }
  double* Wall;
  {
    PhaseTimer pt(this, kPhPoles);
    Wall = st_pole_solves(pp);
  }
  // the bases of the batch's sources reuse the buffers of the previous batch
  // (grown as needed): their sizes follow the sources' ranks, and allocating
  // them per batch left the caching pool with blocks of many sizes
  std::vector<StFin> fins(nb);
  for (int j = 0; j < nb && j < (int)fin_keep_.size(); ++j) fins[j] = std::move(fin_keep_[j]);
  {
    PhaseTimer pt(this, kPhProject);
    st_project_batch(prs, Wall, fins);
  }
  {
    PhaseTimer pt(this, kPhTrunc);
    st_truncate(fins, Y, adjoint);
  }
  if ((int)fin_keep_.size() < nb) fin_keep_.resize(nb);
  for (int j = 0; j < nb; ++j) fin_keep_[j] = std::move(fins[j]);
}

// Bases and projected problems of a batch of prepared sources whose pole
// solves are in Wall (pole-major, overwritten): per source fin.Q (nx x q,
// M-orthonormal) and fin.Zp (q x nt) with the space-time solution Q Zp.
void Problem::st_project_batch(const std::vector<StPrep>& prs, double* Wall, std::vector<StFin>& fins) {
  // 2. block-by-block M-orthonormalization of the pole solutions.  Block
  // Gram-Schmidt against Q in the M inner product, twice, with the block
  // normalized between the two sweeps: (1) project the raw block out of
  // span(Q); (2) orthonormalize it by its Gram eigenpairs (SVQB, Stathopoulos
  // and Wu 2002), dropping directions whose M-norm fell below 1e-11 of the
  // block's original scale; (3) project the normalized block out of span(Q)
  // again: a direction that kept little of its norm in (1) carries the
  // rounding of that sweep magnified by the normalization, and this sweep
  // removes it; (4) orthonormalize again, dropping directions that now keep
  // less than 1e-4 of their norm (they were inside span(Q)).  A Gram-based
  // Cholesky cannot tell nearly dependent directions from rounding noise, so
  // it is not used here.  The sources of the batch go through the pole blocks
  // in lockstep: their small Gram matrices reach the host together (two round
  // trips per pole block for the whole batch), the stencil products of their
  // blocks are one launch (the blocks of one pole are adjacent columns), and
  // their Gram products and projections are grouped launches.  Each source's
  // arithmetic is the same as on its own.
  const int nb = (int)prs.size();
  const int npol = (int)poles.size();
  const std::vector<ShiftCoef> Mop{{0.0, 1.0}};
  const std::vector<ShiftCoef> Kop{{tau, 0.0}};
  std::vector<int> q(nb, 0), pre(nb + 1, 0);
  std::vector<size_t> coff(nb + 1, 0), toff(nb + 1, 0);
  int rmax = 0;
  for (int j = 0; j < nb; ++j) {
    fins[j].q = 0;
    const int r1 = prs[j].r1;
    pre[j + 1] = pre[j] + r1;
    coff[j + 1] = coff[j] + (size_t)r1 * npol * r1;  // sweep coefficients, at most qmax x r1
    toff[j + 1] = toff[j] + (size_t)r1 * r1;         // orthonormalizing transforms
    rmax = std::max(rmax, r1);
    if (r1 == 0) continue;
    const int qmax = r1 * npol;
    fins[j].Q.ensure(sizeof(double) * (size_t)nx * qmax);
    if (desc.precision == LRPOST_MIXED && sweep_f32) fins[j].Q32.ensure(sizeof(float) * (size_t)nx * qmax);
    fins[j].Kt.ensure(sizeof(double) * (size_t)qmax * qmax);  // q x q projected tau K, leading dimension qmax
  }
  if (rmax == 0 || !Wall) return;
  const int R1 = pre[nb];
  // pole block ip of source j: Wall columns ip R1 + pre[j] ...
  auto Wj = [&](int ip, int j) { return Wall + ((size_t)ip * R1 + pre[j]) * nx; };
  st_mw_.ensure(sizeof(double) * (size_t)nx * R1);
  st_w2_.ensure(sizeof(double) * (size_t)nx * R1);
  st_c_.ensure(sizeof(double) * coff[nb]);
  st_tm_.ensure(sizeof(double) * toff[nb]);
  double* MW = st_mw_.as<double>();  // M (or tau K) times the blocks of all sources
  double* W2 = st_w2_.as<double>();  // the normalized blocks, source after source
  double* Cd = st_c_.as<double>();
  double* Td = st_tm_.as<double>();
  const size_t gs = (size_t)rmax * rmax;  // one Gram slot; two per source
  st_g_.ensure(sizeof(double) * gs * 2 * nb);
  double* Gd = st_g_.as<double>();
  std::vector<double> Gh(gs * 2 * nb), Th(toff[nb]);
  auto slot = [&](int j, int k) { return (size_t)(2 * j + k) * gs; };
  auto gram_g = [&](const double* A, const double* B, double* C, int m, int qq, long ldc) {
    return GramGroup{A, B, nullptr, C, nx, nx, ldc, 0, m, qq, 0};
  };
  auto proj_g = [&](const double* A, const double* Qm, int ldq, double* C, int m, int p) {
    return ProjGroup{A, Qm, C, C, nx, nx, nx, ldq, m, p};
  };
  // the sweep X_j -= Q_j (Q_j^T M X_j) of every source with a basis (M X_j
  // in MW at column mwc[j]); extra Gram products ride along in the launch
  // (in mixed precision the first sweep reads the float32 copy of Q and runs
  // on the float32 matrix cores: its coefficients are accurate to about 1e-6
  // of the block, and the second, float64 sweep removes what it leaves)
  const bool f32_sweep = desc.precision == LRPOST_MIXED && sweep_f32;
  auto sweep = [&](const std::vector<int>& kc, const std::vector<double*>& X, const std::vector<int>& mwc,
                   std::vector<GramGroup> gg, bool first) {
    std::vector<ProjGroup> pg;
    for (int j = 0; j < nb; ++j) {
      if (q[j] == 0 || kc[j] == 0) continue;
      const double* Q = fins[j].Q.as<double>();
      GramGroup g = gram_g(Q, MW + (size_t)mwc[j] * nx, Cd + coff[j], q[j], kc[j], q[j]);
      ProjGroup pj = proj_g(Q, Cd + coff[j], q[j], X[j], q[j], kc[j]);
      if (first && f32_sweep) g.A32 = pj.A32 = fins[j].Q32.as<float>();
      gg.push_back(g);
      pg.push_back(pj);
    }
    gram_dev_grouped(gg);
    proj_dev_grouped(pg, -1.0, 1.0);
  };
  // the host transforms Tm[j] (rows x cols[j]) to the device, one upload
  auto upload = [&](const std::vector<std::vector<double>>& Tm, const std::vector<int>& cols) {
    for (int j = 0; j < nb; ++j)
      if (cols[j] > 0) std::copy(Tm[j].begin(), Tm[j].end(), Th.begin() + toff[j]);
    to_device(Td, Th.data(), Th.size());
  };
  // eigenpairs of a block's Gram G (kc x kc, host) above thresh -> the
  // orthonormalizing transform Tm (kc x kn); -1 if the eigensolve failed.
  // Pure host arithmetic: the sources' solves run on parallel host threads.
  auto svqb_host = [](int kc, const double* G, double thresh, std::vector<double>& Tm) -> int {
    // Fast path, Tm = R^{-1} from the Cholesky factor G = R^T R, taken when
    // the block is safely full-rank and well conditioned: lambda_min(G) =
    // 1 / ||R^{-1}||_2^2 >= 1 / ||R^{-1}||_F^2 = 1 / f, so f < 1 / (100 thresh)
    // means every eigenvalue exceeds 100 thresh (the eigen-based transform
    // would keep every column; W R^{-1} is an M-orthonormal basis of the same
    // span), and f max_i G_ii < 1e12 bounds the condition number.  Otherwise
    // the eigen-based transform below.
    {
      std::vector<double> R((size_t)kc * kc);
      double gmax = 0.0;
      for (int i = 0; i < kc; ++i) gmax = std::max(gmax, G[(size_t)i * kc + i]);
      if (cholesky_upper(kc, G, kc, R.data())) {
        Tm.assign((size_t)kc * kc, 0.0);
        upper_inverse(kc, R.data(), Tm.data());
        double f = 0.0;
        for (double x : Tm) f += x * x;
        if (std::isfinite(f) && 100.0 * thresh * f < 1.0 && f * gmax < 1e12) return kc;
      }
    }
    std::vector<double> Gw(G, G + (size_t)kc * kc), wv(kc, 0.0), Uv((size_t)kc * kc, 0.0);
    if (!syev(kc, Gw.data(), kc, wv.data(), Uv.data())) return -1;
    std::vector<int> kk;
    for (int i = kc - 1; i >= 0; --i)
      if (wv[i] > thresh) kk.push_back(i);
    const int kn = (int)kk.size();
    Tm.assign((size_t)kc * std::max(kn, 1), 0.0);
    for (int c = 0; c < kn; ++c)
      for (int i = 0; i < kc; ++i) Tm[(size_t)c * kc + i] = Uv[(size_t)kk[c] * kc + i] / std::sqrt(wv[kk[c]]);
    return kn;
  };
  // Tm = R^{-1} from the Cholesky factor G = R^T R when every eigenvalue of G
  // is above min_eig (lambda_min >= 1 / ||R^{-1}||_F^2); false otherwise
  auto chol_transform = [](int kc, const double* G, double min_eig, std::vector<double>& Tm) -> bool {
    std::vector<double> R((size_t)kc * kc);
    if (!cholesky_upper(kc, G, kc, R.data())) return false;
    Tm.assign((size_t)kc * kc, 0.0);
    upper_inverse(kc, R.data(), Tm.data());
    double f = 0.0;
    for (double x : Tm) f += x * x;
    return std::isfinite(f) && f * min_eig < 1.0;
  };
  std::vector<int> k1(nb, 0), k2(nb, 0), pre2(nb + 1, 0), mw1(nb), mw2(nb);
  std::vector<double> ref(nb, 0.0);
  std::vector<std::vector<double>> Tm(nb);
  std::vector<double*> X1(nb), X2(nb);
  for (int j = 0; j < nb; ++j) mw1[j] = pre[j];
  for (int ip = 0; ip < npol; ++ip) {
    // stage 1: first sweep, Gram of the swept block; the reference scale of
    // the raw block is its largest squared M-norm, ||X_c||_M^2 = ||C_c||^2 +
    // ||X'_c||_M^2 with C the sweep's coefficients (Q is M-orthonormal), so it
    // needs no Gram of the raw block
    std::vector<int> r1s(nb);
    std::vector<GramGroup> g1;
    std::vector<ColGroup> cn;
    for (int j = 0; j < nb; ++j) {
      r1s[j] = prs[j].r1;
      X1[j] = Wj(ip, j);
      if (r1s[j] == 0) continue;
      g1.push_back(gram_g(X1[j], MW + (size_t)pre[j] * nx, Gd + slot(j, 1), r1s[j], r1s[j], r1s[j]));
      if (q[j] > 0) cn.push_back(ColGroup{Cd + coff[j], Gd + slot(j, 0), q[j], q[j], r1s[j]});
    }
    apply_op(R1, Wj(ip, 0), MW, Mop);
    sweep(r1s, X1, mw1, {}, true);
    col_sqnorms(st, (int)cn.size(), cn.data());
    apply_op(R1, Wj(ip, 0), MW, Mop);
    gram_dev_grouped(g1);
    to_host(Gh.data(), Gd, Gh.size());
    for (int j = 0; j < nb; ++j) {
      const int r1 = prs[j].r1;
      ref[j] = 0.0;
      for (int c = 0; c < r1; ++c)
        ref[j] = std::max(ref[j], (q[j] > 0 ? Gh[slot(j, 0) + c] : 0.0) + Gh[slot(j, 1) + (size_t)c * r1 + c]);
    }
    host_parallel(nb, [&](int j) {
      k1[j] = (prs[j].r1 > 0 && ref[j] > 0) ? svqb_host(prs[j].r1, Gh.data() + slot(j, 1), 1e-22 * ref[j], Tm[j]) : 0;
    });
    for (int j = 0; j < nb; ++j) {
      if (k1[j] < 0) fail(LRPOST_EBREAKDOWN, "basis Gram eigensolve");
      pre2[j + 1] = pre2[j] + k1[j];
    }
    const int K1 = pre2[nb];
    if (K1 == 0) continue;
    upload(Tm, k1);
    {
      std::vector<ProjGroup> pg;
      for (int j = 0; j < nb; ++j) {
        X2[j] = W2 + (size_t)pre2[j] * nx;
        mw2[j] = pre2[j];
        if (k1[j] > 0) pg.push_back(proj_g(X1[j], Td + toff[j], prs[j].r1, X2[j], prs[j].r1, k1[j]));
      }
      proj_dev_grouped(pg, 1.0, 0.0);
    }
    // stage 2: second sweep of the normalized block X.  Its Gram rides along
    // with the sweep's product, [Q | X]^T M X = [C; G], and the Gram of the
    // swept block is G - C^T C (Pythagoras; C is small after the first
    // sweep).  That form is used when its Cholesky factor shows every
    // eigenvalue above 1e-4, where its absolute rounding (1e-16 of ||G||) is
    // at most 1e-12 relative; otherwise the source's swept block gets its own
    // M product and Gram, as computed directly they round relative to the
    // small directions.  Each source decides on its own numbers.  In mixed
    // precision the projection X -= Q C of this sweep reads the float32 copy
    // of Q when every column of C is below 1e-5 (its rounding, 1e-7 of
    // ||Q C||, is then below 1e-12 of the normalized block).
    apply_op(K1, W2, MW, Mop);
    {
      std::vector<GramGroup> gg;
      for (int j = 0; j < nb; ++j) {
        if (k1[j] == 0) continue;
        const int mq = q[j] + k1[j];
        GramGroup g = gram_g(fins[j].Q.as<double>(), MW + (size_t)pre2[j] * nx, Cd + coff[j], mq, k1[j], mq);
        if (q[j] > 0) {
          g.A2 = X2[j];
          g.m2 = k1[j];
        } else {
          g.A = X2[j];
        }
        gg.push_back(g);
      }
      gram_dev_grouped(gg);
    }
    for (int j = 0; j < nb; ++j) {
      if (k1[j] == 0) continue;
      const int mq = q[j] + k1[j];
      LRP_HIP(hipMemcpy2DAsync(Gd + slot(j, 0), sizeof(double) * k1[j], Cd + coff[j] + q[j], sizeof(double) * mq,
                               sizeof(double) * k1[j], k1[j], hipMemcpyDeviceToDevice, st));
      if (q[j] > 0)
        dense->gemm(true, false, k1[j], k1[j], q[j], 1.0, Cd + coff[j], mq, Cd + coff[j], mq, 0.0, Gd + slot(j, 1),
                    k1[j]);
    }
    to_host(Gh.data(), Gd, Gh.size());
    {
      std::vector<ProjGroup> pg;
      for (int j = 0; j < nb; ++j) {
        if (k1[j] == 0 || q[j] == 0) continue;
        const int mq = q[j] + k1[j];
        ProjGroup pj = proj_g(fins[j].Q.as<double>(), Cd + coff[j], mq, X2[j], q[j], k1[j]);
        if (f32_sweep) {
          const double* CC = Gh.data() + slot(j, 1);
          double cmax = 0.0;
          for (int c = 0; c < k1[j]; ++c) cmax = std::max(cmax, CC[(size_t)c * k1[j] + c]);
          if (cmax < 1e-10) pj.A32 = fins[j].Q32.as<float>();
        }
        pg.push_back(pj);
      }
      proj_dev_grouped(pg, -1.0, 1.0);
    }
    std::vector<int> direct(nb, 0);
    host_parallel(nb, [&](int j) {
      k2[j] = 0;
      if (k1[j] == 0) return;
      const int kc = k1[j];
      double* G = Gh.data() + slot(j, 0);
      if (q[j] > 0) {
        const double* CC = Gh.data() + slot(j, 1);
        for (size_t e = 0; e < (size_t)kc * kc; ++e) G[e] -= CC[e];
      }
      k2[j] = chol_transform(kc, G, 1e-4, Tm[j]) ? kc : -1;
      if (k2[j] < 0) direct[j] = 1;
    });
    stats.st_direct_grams += (int32_t)std::count(direct.begin(), direct.end(), 1);
    if (std::count(direct.begin(), direct.end(), 1) > 0) {
      std::vector<GramGroup> g2;
      for (int j = 0; j < nb; ++j) {
        if (!direct[j]) continue;
        double* MX = MW + (size_t)pre2[j] * nx;
        apply_op(k1[j], X2[j], MX, Mop);
        g2.push_back(gram_g(X2[j], MX, Gd + slot(j, 0), k1[j], k1[j], k1[j]));
      }
      gram_dev_grouped(g2);
      to_host(Gh.data(), Gd, Gh.size());
      host_parallel(nb, [&](int j) {
        if (direct[j]) k2[j] = svqb_host(k1[j], Gh.data() + slot(j, 0), 1e-8, Tm[j]);
      });
    }
    for (int j = 0; j < nb; ++j)
      if (k2[j] < 0) fail(LRPOST_EBREAKDOWN, "basis Gram eigensolve");
    upload(Tm, k2);
    std::vector<ProjGroup> pg;
    std::vector<GramGroup> gk;
    for (int j = 0; j < nb; ++j) {
      if (k2[j] == 0) continue;
      double* Qn = fins[j].Q.as<double>() + (size_t)q[j] * nx;
      pg.push_back(proj_g(X2[j], Td + toff[j], k1[j], Qn, k1[j], k2[j]));
      // the float32 copy of the new columns for the next first sweeps
      if (f32_sweep) pg.back().C32 = fins[j].Q32.as<float>() + (size_t)q[j] * nx;
    }
    proj_dev_grouped(pg, 1.0, 0.0);
    // extend Kt = Q^T tau K Q by the new columns (upper triangle suffices;
    // the convection-diffusion operator forms its full Kt after the loop)
    for (int j = 0; j < nb && !cd_on; ++j) {
      const int kcols = k2[j];
      if (kcols == 0) continue;
      double* Q = fins[j].Q.as<double>();
      double* KQn = MW + (size_t)pre[j] * nx;
      apply_op(kcols, Q + (size_t)q[j] * nx, KQn, Kop);
      const int qmax = prs[j].r1 * npol;
      gk.push_back(gram_g(Q, KQn, fins[j].Kt.as<double>() + (size_t)q[j] * qmax, q[j] + kcols, kcols, qmax));
    }
    gram_dev_grouped(gk);
    for (int j = 0; j < nb; ++j) q[j] += k2[j];
  }
  if (cd_on) {
    // a projected operator that is not symmetric: Kt = Q^T (tau L) Q in full
    // (L^T in adjoint solves), one source after another through one buffer
    for (int j = 0; j < nb; ++j) {
      if (q[j] == 0) continue;
      st_lq_.ensure(sizeof(double) * (size_t)nx * q[j]);
      const double* Q = fins[j].Q.as<double>();
      st_apply(q[j], Q, st_lq_.as<double>(), Kop);
      std::vector<GramGroup> gk{gram_g(Q, st_lq_.as<double>(), fins[j].Kt.as<double>(), q[j], q[j],
                                       prs[j].r1 * npol)};
      gram_dev_grouped(gk);
    }
  }
  PhaseTimer pt(this, kPhProjSolve);
  for (int j = 0; j < nb; ++j) stats.last_basis = q[j];
  st_solve_projected(prs, q, fins);
}

// 3. Projected problems of the sources of a batch on the device, given their
// bases (fin.Q, q[j] columns) and projected tau K (fin.Kt, leading dimension
// r1 npol): fin.Zp (q[j] x nt).  The small dense products of all sources run
// as grouped matrix-core launches; each source's arithmetic is the same as
// on its own.
void Problem::st_solve_projected(const std::vector<StPrep>& prs, const std::vector<int>& q, std::vector<StFin>& fins) {
  const int npol = (int)poles.size();
  std::vector<int> act;
  for (int j = 0; j < (int)prs.size(); ++j)
    if (q[j] > 0) act.push_back(j);
  const int na = (int)act.size();
  if (na == 0) return;
  // per source: S (q x r1) = Q^T Fb, F2t (r1 x nt) = F2p^T, X1 and X2 (q x nt),
  // and four q x q matrices
  std::vector<size_t> off(na + 1, 0);
  for (int a = 0; a < na; ++a) {
    const size_t qa = q[act[a]], r1 = prs[act[a]].r1;
    off[a + 1] = off[a] + qa * r1 + r1 * nt + 2 * qa * nt + 4 * qa * qa;
  }
  st_small_.ensure(sizeof(double) * (off[na] + 64));
  struct Bufs {
    double *S, *F2t, *X1, *X2, *M[4];
  };
  std::vector<Bufs> bf(na);
  for (int a = 0; a < na; ++a) {
    const size_t qa = q[act[a]], r1 = prs[act[a]].r1;
    double* p = st_small_.as<double>() + off[a];
    bf[a].S = p;
    bf[a].F2t = bf[a].S + qa * r1;
    bf[a].X1 = bf[a].F2t + r1 * nt;
    bf[a].X2 = bf[a].X1 + qa * nt;
    for (int k = 0; k < 4; ++k) bf[a].M[k] = bf[a].X2 + qa * nt + (size_t)k * qa * qa;
  }
  auto grouped = [&](double alpha, double beta, auto&& set) {
    std::vector<ProjGroup> g(na);
    for (int a = 0; a < na; ++a) set(a, q[act[a]], g[a]);
    proj_dev_grouped(g, alpha, beta);  // timed as LRPOST_KERNEL_PROJ
  };
  auto diag = [&](std::vector<double*> A, double v) {
    for (int a0 = 0; a0 < na; a0 += kProjGroupMax) {
      DiagGroups dg{};
      const int n = std::min(kProjGroupMax, na - a0);
      for (int i = 0; i < n; ++i) {
        dg.A[i] = A[a0 + i];
        dg.lda[i] = q[act[a0 + i]];
        dg.n[i] = q[act[a0 + i]];
      }
      add_diag_grouped(st, dg, n, v);
    }
  };
  // A = (I + Kt)^{-1} by the Newton-Schulz iteration X <- X (2I - (I + Kt) X)
  // from X_0 = 2 / (1 + L) I: with Q M-orthonormal the eigenvalues of
  // I + Kt lie in [1, L], L = 1 + tau lambda_max(M^{-1} K), so the error
  // I - (I + Kt) X_j has spectral radius ((L - 1) / (L + 1))^(2^j) and the
  // iteration count follows from L alone.  Only matrix products are used,
  // which round identically on every run (a library Cholesky inverse did
  // not when other work shared the device).
  // M[0] = I + Kt (full symmetric), M[1] and M[2] the iterates, M[3] = T.
  std::vector<double*> Apd(na), Xa(na), Xn(na), T(na);
  for (int a = 0; a < na; ++a) {
    const int j = act[a], qa = q[j];
    const int qmax = prs[j].r1 * npol;
    Apd[a] = bf[a].M[0];
    Xa[a] = bf[a].M[1];
    Xn[a] = bf[a].M[2];
    T[a] = bf[a].M[3];
    LRP_HIP(hipMemcpy2DAsync(Apd[a], sizeof(double) * qa, fins[j].Kt.as<double>(), sizeof(double) * qmax,
                             sizeof(double) * qa, qa, hipMemcpyDeviceToDevice, st));
    if (!cd_on) symmetrize_upper(st, qa, Apd[a], qa);
    LRP_HIP(hipMemsetAsync(Xa[a], 0, sizeof(double) * (size_t)qa * qa, st));
  }
  diag(Apd, 1.0);
  // the convection-diffusion operator: X_0 = cd_ns_alpha_ I and a step count
  // from the field of values of I + Kt (set_convection)
  diag(Xa, cd_on ? cd_ns_alpha_ : 2.0 / (1.0 + ns_bound_));
  const int ns_steps_now = cd_on ? cd_ns_iters_ : ns_iters_;
  for (int it = 0; it < ns_steps_now; ++it) {
    grouped(-1.0, 0.0, [&](int a, int qa, ProjGroup& g) {  // T = -(I + Kt) X
      g = ProjGroup{Apd[a], Xa[a], T[a], T[a], qa, qa, qa, qa, qa, qa};
    });
    diag(T, 2.0);  // T = 2I - (I + Kt) X
    grouped(1.0, 0.0, [&](int a, int qa, ProjGroup& g) {  // Xn = X T
      g = ProjGroup{Xa[a], T[a], Xn[a], Xn[a], qa, qa, qa, qa, qa, qa};
    });
    std::swap(Xa, Xn);
  }
  // Xa = A; the other two q x q buffers hold its powers
  std::vector<double*> P1(na), P2(na);
  for (int a = 0; a < na; ++a) {
    P1[a] = Apd[a];
    P2[a] = T[a];
  }
  // With Q^T M Q = I each column obeys (I + Kt) z_k = z_{k-1} + g_k,
  // g_k = S F2p^T e_k: a linear recurrence z_k = A z_{k-1} + A g_k with the
  // constant matrix A, evaluated by recursive doubling over time: after the
  // level with stride d, X[:, k] = sum_{j < 2d, j <= k} A^j (A G)[:, k-j]; the
  // next level adds A^{2d} X[:, k - 2d].  The eigenvalues of A lie in (0, 1],
  // so the powers stay bounded.
  for (int a = 0; a < na; ++a) {
    const int j = act[a], r1 = prs[j].r1;
    gram_dev(q[j], fins[j].Q.as<double>(), r1, prs[j].Fb.as<double>(), bf[a].S);
    std::vector<double>& ft = tmp_h_;
    ft.resize((size_t)r1 * nt);
    for (int t = 0; t < nt; ++t)
      for (int i = 0; i < r1; ++i) ft[(size_t)t * r1 + i] = prs[j].F2p[(size_t)i * nt + t];
    to_device(bf[a].F2t, ft.data(), ft.size());
  }
  grouped(1.0, 0.0, [&](int a, int qa, ProjGroup& g) {  // G = S F2p^T (in X2)
    const int r1 = prs[act[a]].r1;
    g = ProjGroup{bf[a].S, bf[a].F2t, bf[a].X2, bf[a].X2, qa, qa, qa, r1, r1, nt};
  });
  grouped(1.0, 0.0, [&](int a, int qa, ProjGroup& g) {  // X1 = A G
    g = ProjGroup{Xa[a], bf[a].X2, bf[a].X1, bf[a].X1, qa, qa, qa, qa, qa, nt};
  });
  std::vector<double*> Apow = Xa, cur(na), nxt(na), pw = P1;
  for (int a = 0; a < na; ++a) {
    cur[a] = bf[a].X1;
    nxt[a] = bf[a].X2;
  }
  for (int d = 1; d < nt; d *= 2) {
    for (int a0 = 0; a0 < na; a0 += kProjGroupMax) {
      CopyGroups cg{};
      const int n = std::min(kProjGroupMax, na - a0);
      for (int i = 0; i < n; ++i) {
        cg.src[i] = cur[a0 + i];
        cg.dst[i] = nxt[a0 + i];
        cg.len[i] = (long)q[act[a0 + i]] * nt;
      }
      copy_grouped(st, cg, n);
    }
    grouped(1.0, 1.0, [&](int a, int qa, ProjGroup& g) {  // nxt[:, d:] += A^d cur[:, :nt-d]
      g = ProjGroup{Apow[a], cur[a], nxt[a] + (size_t)d * qa, nxt[a] + (size_t)d * qa, qa, qa, qa, qa, qa, nt - d};
    });
    std::swap(cur, nxt);
    if (2 * d < nt) {
      grouped(1.0, 0.0, [&](int a, int qa, ProjGroup& g) {  // A^{2d} = A^d A^d
        g = ProjGroup{Apow[a], Apow[a], pw[a], pw[a], qa, qa, qa, qa, qa, qa};
      });
      Apow = pw;
      pw = pw[0] == P1[0] ? P2 : P1;
    }
  }
  for (int a = 0; a < na; ++a) {
    const int j = act[a];
    fins[j].q = q[j];
    fins[j].Zp.ensure(sizeof(double) * (size_t)q[j] * nt);
    LRP_HIP(hipMemcpyAsync(fins[j].Zp.p, cur[a], sizeof(double) * (size_t)q[j] * nt, hipMemcpyDeviceToDevice, st));
  }
}

// Truncation of the projected solutions Y_j = Q_j Zp_j (Q_j M-orthonormal:
// M-weighted Frobenius norm).  Below 1e-7 each Zp runs through the host
// Jacobi SVD; otherwise the eigenpairs of the Gram matrices of the smaller
// side are solved as one batch: Zp^T Zp (nt x nt) when nt is at most the
// batch's largest q, else Zp Zp^T zero-padded to that q.
void Problem::st_truncate(std::vector<StFin>& fins, const std::vector<LowRank*>& Y, bool adjoint) {
  const int nb = (int)fins.size();
  double tail = 0.0;
  auto store_B = [&](LowRank& y, const std::vector<double>& B2, int ry) {
    for (int c = 0; c < ry; ++c)
      for (int k = 0; k < nt; ++k) y.B[(size_t)c * nt + (adjoint ? nt - 1 - k : k)] = B2[(size_t)c * nt + k];
  };
  for (int j = 0; j < nb; ++j) {
    Y[j]->nx = nx;
    Y[j]->nt = nt;
    if (fins[j].q == 0) Y[j]->resize(nx, nt, 0);
  }
  if (desc.trunc_tol < 1e-7) {
    // every source's Zp to the host, their SVDs on parallel host threads
    // (pure host arithmetic), then the truncated products source by source
    std::vector<std::vector<double>> Zhs(nb), svs(nb), Uzs(nb), Vzs(nb);
    for (int j = 0; j < nb; ++j) {
      const int q = fins[j].q;
      if (q == 0) continue;
      Zhs[j].resize((size_t)q * nt);
      to_host(Zhs[j].data(), fins[j].Zp.as<double>(), Zhs[j].size());
    }
    host_parallel(nb, [&](int j) {
      // only the kept singular vectors are formed
      if (fins[j].q > 0)
        svd(fins[j].q, nt, Zhs[j].data(), fins[j].q, svs[j], Uzs[j], Vzs[j], [&](const std::vector<double>& sv) {
          double t = 0.0;
          return truncation_rank(sv, desc.trunc_tol, desc.rank_cap, &t);
        });
    });
    for (int j = 0; j < nb; ++j) {
      const int q = fins[j].q;
      if (q == 0) continue;
      const std::vector<double>& sv = svs[j];
      const std::vector<double>& Uz = Uzs[j];
      const std::vector<double>& Vz = Vzs[j];
      const int ry = truncation_rank(sv, desc.trunc_tol, desc.rank_cap, &tail);
      Y[j]->resize(nx, nt, ry);
      if (ry > 0) {
        std::vector<double> Cm((size_t)q * ry);
        for (int c = 0; c < ry; ++c)
          for (int i = 0; i < q; ++i) Cm[(size_t)c * q + i] = Uz[(size_t)c * q + i] * sv[c];
        proj(q, fins[j].Q.as<double>(), Cm, ry, Y[j]->a(), 0.0);
        store_B(*Y[j], Vz, ry);
      }
    }
    stats.last_tail = tail;
    sync();
    return;
  }
  std::vector<int> act;
  int qb = 0;
  for (int j = 0; j < nb; ++j)
    if (fins[j].q > 0) {
      act.push_back(j);
      qb = std::max(qb, fins[j].q);
    }
  const int na = (int)act.size();
  if (na == 0) {
    sync();
    return;
  }
  const bool right = nt <= qb;
  const int g = right ? nt : qb;
  const size_t gsz = (size_t)g * g;
  st_gram_.ensure(sizeof(double) * (gsz * na + (size_t)g * na + 64));
  double* G = st_gram_.as<double>();
  double* wg = G + gsz * na;
  if (!right) LRP_HIP(hipMemsetAsync(G, 0, sizeof(double) * gsz * na, st));
  for (int a = 0; a < na; ++a) {
    const StFin& f = fins[act[a]];
    const double* Zp = f.Zp.as<double>();
    if (right) dense->gemm(true, false, nt, nt, f.q, 1.0, Zp, f.q, Zp, f.q, 0.0, G + gsz * a, g);
    else dense->gemm(false, true, f.q, f.q, nt, 1.0, Zp, f.q, Zp, f.q, 0.0, G + gsz * a, g);
  }
  dense->syevd_batched(g, G, g, (long)gsz, wg, g, na, eig_work_);
  // One read-back for the eigenvalues and, per source, the temporal factors
  // of the rc = min(cap, g) leading directions (the kept ones are the last r
  // of them once the ranks are known): the eigenvectors themselves when nt is
  // the small side, else Zp^T U.
  const int rc = desc.rank_cap > 0 ? std::min(desc.rank_cap, g) : g;
  const size_t wlen = (size_t)g * na, clen = (size_t)nt * rc;
  st_c_.ensure(sizeof(double) * (wlen + clen * na + (size_t)qb * rc + 64));
  double* Rd = st_c_.as<double>();               // eigenvalues, then the candidate temporal factors
  double* Cm = Rd + wlen + clen * na;            // q x r scratch
  LRP_HIP(hipMemcpyAsync(Rd, wg, sizeof(double) * wlen, hipMemcpyDeviceToDevice, st));
  for (int a = 0; a < na; ++a) {
    const StFin& f = fins[act[a]];
    const double* Ec = G + gsz * a + (size_t)(g - rc) * g;  // eigenvectors of the rc largest eigenvalues
    double* Ba = Rd + wlen + clen * a;
    if (right) LRP_HIP(hipMemcpyAsync(Ba, Ec, sizeof(double) * clen, hipMemcpyDeviceToDevice, st));
    else dense->gemm(true, false, nt, rc, f.q, 1.0, f.Zp.as<double>(), f.q, Ec, g, 0.0, Ba, nt);
  }
  std::vector<double> Rh(wlen + clen * na);
  to_host(Rh.data(), Rd, Rh.size());
  std::vector<int> ry(na);
  for (int a = 0; a < na; ++a) {
    std::vector<double> sv(g);
    for (int c = 0; c < g; ++c) sv[c] = std::sqrt(std::max(Rh[(size_t)a * g + g - 1 - c], 0.0));
    ry[a] = truncation_rank(sv, desc.trunc_tol, desc.rank_cap, &tail);
  }
  for (int a = 0; a < na; ++a) {
    const StFin& f = fins[act[a]];
    LowRank& y = *Y[act[a]];
    const int q = f.q, r = ry[a];
    const double* Zp = f.Zp.as<double>();
    y.resize(nx, nt, r);
    if (r == 0) continue;
    // eigenvectors of the kept directions are the last r columns
    const double* Ek = G + gsz * a + (size_t)(g - r) * g;
    if (right) {
      // Y = Q (Zp V_r) V_r^T
      dense->gemm(false, false, q, r, nt, 1.0, Zp, q, Ek, nt, 0.0, Cm, q);
      proj_dev(q, f.Q.as<double>(), Cm, q, r, y.a(), 0.0);
    } else {
      // Y = Q U_r (Zp^T U_r)^T, U_r the first q rows of the padded eigenvectors
      proj_dev(q, f.Q.as<double>(), Ek, g, r, y.a(), 0.0);
    }
    const auto b0 = Rh.begin() + wlen + clen * a + (size_t)nt * (rc - r);
    std::vector<double> B2(b0, b0 + (size_t)nt * r);
    store_B(y, B2, r);
  }
  stats.last_tail = tail;
}

// G x = alpha^{-1} (K+M)^{-1} M P1 P2^T (precond) or H_mis x = tau M P1 P2^T (misfit),
// with Y = forward solve of the source tau M X1 X2^T, Z = sigma^{-2} mask .* Y and
// P the adjoint solve of Z (Sec. 6.1 eq. misfit).
void Problem::hess_apply(const LowRank& x, LowRank& y, bool precond) { hess_apply_batch({&x}, {&y}, precond); }

// Several applies with the multigrid work fused: the forward solves' pole
// solves in one multigrid solve, the adjoint solves' in another, and the
// prior solves of all outputs in a third.
void Problem::hess_apply_batch(const std::vector<const LowRank*>& x, const std::vector<LowRank*>& y, bool precond) {
  const int nb = (int)x.size();
  stats.applies += nb;
  std::vector<LowRank> F(nb), Yf(nb), Zs(nb), Pa(nb);
  std::vector<const LowRank*> pF, pZ;
  std::vector<LowRank*> pY, pP;
  for (int j = 0; j < nb; ++j) {
    F[j].resize(nx, nt, x[j]->rank);
    if (x[j]->rank > 0) apply_op(x[j]->rank, x[j]->a(), F[j].a(), {{0.0, tau}});
    F[j].B = x[j]->B;
    pF.push_back(&F[j]);
    pY.push_back(&Yf[j]);
  }
  spacetime_solve_batch(pF, pY, false);
  for (int j = 0; j < nb; ++j) {
    stats.last_rank_y = Yf[j].rank;
    Zs[j].resize(nx, nt, Yf[j].rank);
    if (Yf[j].rank > 0)
      mask_scale<double>(st, nx, Yf[j].rank, Yf[j].a(), nx, Zs[j].a(), nx, mask.as<uint8_t>(),
                         1.0 / (desc.sigma * desc.sigma));
    Zs[j].B = Yf[j].B;
    pZ.push_back(&Zs[j]);
    pP.push_back(&Pa[j]);
  }
  spacetime_solve_batch(pZ, pP, true);
  int R = 0;
  for (int j = 0; j < nb; ++j) R += Pa[j].rank;
  PhaseTimer pt(this, kPhPrior);
  DevMem mp, out;
  if (R > 0 && precond) {
    mp.ensure(sizeof(double) * (size_t)nx * R);
    out.ensure(sizeof(double) * (size_t)nx * R);
    int off = 0;
    for (int j = 0; j < nb; ++j) {
      if (Pa[j].rank > 0) apply_op(Pa[j].rank, Pa[j].a(), mp.as<double>() + (size_t)off * nx, {{0.0, 1.0}});
      off += Pa[j].rank;
    }
    if (desc.precision == LRPOST_MIXED)  // float32 cycles, float64 refinement rounds
      mg_solve(R, mp.as<double>(), out.as<double>(), {{1.0, 1.0}}, (prior_cycles + 1) / 2,
               desc.trunc_tol < 1e-7 ? 2 : 1);
    else
      mg_solve(R, mp.as<double>(), out.as<double>(), {{1.0, 1.0}}, prior_cycles);
  }
  int off = 0;
  for (int j = 0; j < nb; ++j) {
    LowRank& yj = *y[j];
    const int r = Pa[j].rank;
    stats.last_rank_p = r;
    yj.nx = nx;
    yj.nt = nt;
    yj.resize(nx, nt, r);
    if (r > 0) {
      if (precond)
        axpby<double>(st, nx, r, out.as<double>() + (size_t)off * nx, nx, yj.a(), nx, 1.0 / desc.alpha, 0.0);
      else
        apply_op(r, Pa[j].a(), yj.a(), {{0.0, tau}});
      yj.B = Pa[j].B;
    }
    off += r;
    stats.last_rank_out = r;
  }
  sync();
}

// c = P^{-1} sigma^{-2} F^T y = alpha^{-1} (K+M)^{-1} M Z with Z the adjoint
// space-time solve of the data scattered to the observed nodes (the tail of
// the Hessian apply, with the data in place of the observed state).  The
// data matrix enters exactly as (y V) V^T, V the eigenvectors of y^T y
// (nt x nt), so its rank is at most nt.
void Problem::data_rhs(const double* y, LowRank& c) {
  std::vector<int> obs;
  for (long i = 0; i < nx; ++i)
    if (mask_h[i]) obs.push_back((int)i);
  const int m = (int)obs.size();
  std::vector<double> G((size_t)nt * nt, 0.0), w(nt), V((size_t)nt * nt);
  for (int a = 0; a < nt; ++a)
    for (int b = a; b < nt; ++b) {
      double t = 0.0;
      for (int i = 0; i < m; ++i) t += y[(size_t)a * m + i] * y[(size_t)b * m + i];
      G[(size_t)b * nt + a] = G[(size_t)a * nt + b] = t;
    }
  if (!syev(nt, G.data(), nt, w.data(), V.data())) fail(LRPOST_EBREAKDOWN, "data Gram eigensolve failed");
  const double wmax = std::max(w[nt - 1], 0.0);
  std::vector<int> keep;
  for (int j = nt - 1; j >= 0; --j)
    if (wmax > 0 && w[j] > 1e-28 * wmax) keep.push_back(j);
  const int r = (int)keep.size();
  LowRank Z;
  Z.resize(nx, nt, r);
  if (r == 0) {
    c.resize(nx, nt, 0);
    return;
  }
  std::vector<double> Zh((size_t)nx * r, 0.0);
  const double s2 = 1.0 / (desc.sigma * desc.sigma);
  for (int cc = 0; cc < r; ++cc) {
    const double* v = V.data() + (size_t)keep[cc] * nt;
    for (int i = 0; i < m; ++i) {
      double t = 0.0;
      for (int k = 0; k < nt; ++k) t += y[(size_t)k * m + i] * v[k];
      Zh[(size_t)cc * nx + obs[i]] = s2 * t;
    }
    for (int k = 0; k < nt; ++k) Z.B[(size_t)cc * nt + k] = v[k];
  }
  to_device(Z.a(), Zh.data(), Zh.size());
  LowRank Pa;
  spacetime_solve_batch({&Z}, {&Pa}, true);
  c.resize(nx, nt, Pa.rank);
  if (Pa.rank == 0) return;
  DevMem mp, out;
  mp.ensure(sizeof(double) * (size_t)nx * Pa.rank);
  out.ensure(sizeof(double) * (size_t)nx * Pa.rank);
  apply_op(Pa.rank, Pa.a(), mp.as<double>(), {{0.0, 1.0}});
  if (desc.precision == LRPOST_MIXED)
    mg_solve(Pa.rank, mp.as<double>(), out.as<double>(), {{1.0, 1.0}}, (prior_cycles + 1) / 2,
             desc.trunc_tol < 1e-7 ? 2 : 1);
  else
    mg_solve(Pa.rank, mp.as<double>(), out.as<double>(), {{1.0, 1.0}}, prior_cycles);
  axpby<double>(st, nx, Pa.rank, out.as<double>(), nx, c.a(), nx, 1.0 / desc.alpha, 0.0);
  c.B = Pa.B;
  sync();
}

// ---------------------------------------------------------------------------
// Truncation (Sec. 4, after eq. lanczos2) of X = A B^T.
//  1. Householder QR of the small temporal factor, B = Q_B R_B (host), and
//     A' = A R_B^T on the device, so that X = A' Q_B^T with c = min(nt, rank)
//     spatial columns.
//  2. Orthonormalization of A' in the chosen weight by Gram products on the
//     device and small factorizations on the host.  Well-conditioned input:
//     CholeskyQR2.  Otherwise (the usual case for sums of many Krylov
//     vectors): a shifted Cholesky pass (Fukaya, Kannan, Nakatsukasa,
//     Yamamoto, Yanagisawa 2020), which maps A' to a basis of norm at most
//     one whose numerically null directions become tiny; an eigen-based pass
//     that drops directions of Gram eigenvalue below 1e-15 of the largest
//     (their contribution to X is at rounding level); then CholeskyQR2.
//  3. SVD of the small factor R_A (X = Q R_A Q_B^T); the smallest rank whose
//     discarded tail is within tol (relative Frobenius) is kept and one
//     projection forms the new spatial factor.
// ---------------------------------------------------------------------------
void Problem::truncate(LowRank& x, double tol, int cap, int weight, double ref_norm, bool orth_spatial) {
  const int R = x.rank;
  if (R == 0) return;
  const std::vector<ShiftCoef> Wop = weight == 1 ? std::vector<ShiftCoef>{{0.0, 1.0}}
                                                 : std::vector<ShiftCoef>{{1.0, 1.0}};
  const double u = 1.1102230246251565e-16;
  // 1. temporal QR and reduction
  std::vector<double> QB, RB;
  householder_qr(nt, R, x.B.data(), nt, QB, RB);
  const int c = std::min(nt, R);
  std::vector<double> RBt((size_t)R * c);  // R x c = RB^T
  for (int j = 0; j < c; ++j)
    for (int i = 0; i < R; ++i) RBt[(size_t)j * R + i] = RB[(size_t)i * c + j];
  DevMem qa, qb, wa;
  qa.ensure(sizeof(double) * (size_t)nx * c);
  qb.ensure(sizeof(double) * (size_t)nx * c);
  if (weight != 0) wa.ensure(sizeof(double) * (size_t)nx * c);
  proj(R, x.a(), RBt, c, qa.as<double>(), 0.0);
  double* src = qa.as<double>();
  double* dst = qb.as<double>();
  int kcur = c;
  auto gram_w = [&](const double* s, int k, std::vector<double>& G) {
    const double* ws = s;
    if (weight != 0) {
      apply_op(k, s, wa.as<double>(), Wop);
      ws = wa.as<double>();
    }
    gram(k, s, k, ws, G);
  };
  // RA (kcur x c): X = src RA Q_B^T holds throughout
  std::vector<double> RA((size_t)c * c, 0.0);
  for (int i = 0; i < c; ++i) RA[(size_t)i * c + i] = 1.0;
  // Each step computes (T, Rf) with src = (src T) Rf, kout columns; the last
  // step's T is folded into the final projection instead of being applied.
  std::vector<double> T, Rf;
  int kout = 0;
  auto chol_step = [&](const std::vector<double>& G, double shift) -> bool {
    std::vector<double> Gs = G, Rk((size_t)kcur * kcur);
    for (int i = 0; i < kcur; ++i) Gs[(size_t)i * kcur + i] += shift;
    if (!cholesky_upper(kcur, Gs.data(), kcur, Rk.data())) return false;
    T.assign((size_t)kcur * kcur, 0.0);
    upper_inverse(kcur, Rk.data(), T.data());
    Rf = Rk;
    kout = kcur;
    return true;
  };
  auto eig_step = [&](const std::vector<double>& G) {
    std::vector<double> w(kcur), U((size_t)kcur * kcur);
    if (!syev(kcur, G.data(), kcur, w.data(), U.data())) fail(LRPOST_EBREAKDOWN, "Gram eigensolve in truncation");
    const double wmax = std::max(w[kcur - 1], 0.0);
    std::vector<int> keep;
    for (int j = kcur - 1; j >= 0; --j)
      if (wmax > 0 && w[j] > 1e-15 * wmax) keep.push_back(j);
    kout = (int)keep.size();
    T.assign((size_t)kcur * std::max(kout, 1), 0.0);
    Rf.assign((size_t)std::max(kout, 1) * kcur, 0.0);
    for (int cc = 0; cc < kout; ++cc) {
      const double sw = std::sqrt(w[keep[cc]]);
      for (int i = 0; i < kcur; ++i) {
        T[(size_t)cc * kcur + i] = U[(size_t)keep[cc] * kcur + i] / sw;
        Rf[(size_t)i * kout + cc] = U[(size_t)keep[cc] * kcur + i] * sw;
      }
    }
  };
  auto accept = [&](bool apply_T) {
    // RA <- Rf RA ; src <- src T (when apply_T)
    std::vector<double> nra((size_t)std::max(kout, 1) * c, 0.0);
    if (kout > 0) matmul(kout, c, kcur, Rf.data(), kout, false, RA.data(), kcur, false, nra.data(), kout, 1.0, 0.0);
    RA.swap(nra);
    if (apply_T && kout > 0) {
      proj(kcur, src, T, kout, dst, 0.0);
      std::swap(src, dst);
    }
  };
  std::vector<double> G;
  gram_w(src, kcur, G);
  double tr = 0.0;
  for (int i = 0; i < kcur; ++i) tr += G[(size_t)i * kcur + i];
  if (!(tr > 0)) {
    x.resize(nx, nt, 0);
    return;
  }
  // Plain CholeskyQR2 when the first factor certifies the conditioning:
  // ||R||_F ||R^{-1}||_F bounds cond_2(A') from above, and below 1e5 the
  // second pass restores orthonormality to rounding level.  If a later
  // Cholesky of the plain path still fails, the shifted path starts over
  // from A' (still intact in qa: the plain path's first projection writes qb).
  const std::vector<double> G0 = G;
  auto cond_ok = [&]() {
    double fr = 0.0, fi = 0.0;
    for (int j = 0; j < kcur; ++j)
      for (int i = 0; i <= j; ++i) {
        fr += Rf[(size_t)j * kcur + i] * Rf[(size_t)j * kcur + i];
        fi += T[(size_t)j * kcur + i] * T[(size_t)j * kcur + i];
      }
    return std::sqrt(fr * fi) < 1e5;
  };
  bool plain = chol_step(G, 0.0) && cond_ok();
  if (plain) {
    accept(true);
    kcur = kout;
    gram_w(src, kcur, G);
    if (!chol_step(G, 0.0)) {
      plain = false;
      src = qa.as<double>();
      dst = qb.as<double>();
      kcur = c;
      G = G0;
      RA.assign((size_t)c * c, 0.0);
      for (int i = 0; i < c; ++i) RA[(size_t)i * c + i] = 1.0;
    }
  }
  if (!plain) {
    double shift = 11.0 * ((double)nx * kcur + (double)kcur * (kcur + 1)) * u * tr;
    int attempt = 0;
    while (!chol_step(G, shift)) {
      if (++attempt > 20) fail(LRPOST_EBREAKDOWN, "shifted Cholesky failed in truncation");
      shift *= 10.0;
    }
    accept(true);
    kcur = kout;
    gram_w(src, kcur, G);
    eig_step(G);
    if (kout == 0) { x.resize(nx, nt, 0); return; }
    // the eigen step is applied now; CholeskyQR2 follows
    accept(true);
    kcur = kout;
    gram_w(src, kcur, G);
    if (!chol_step(G, 0.0)) fail(LRPOST_EBREAKDOWN, "Cholesky failed after the eigen pass in truncation");
    accept(true);
    kcur = kout;
    gram_w(src, kcur, G);
    if (!chol_step(G, 0.0)) fail(LRPOST_EBREAKDOWN, "Cholesky failed in truncation");
  }
  // last step: Q = src T (not applied), RA <- Rf RA
  accept(false);
  const int k = kout;
  // 3. SVD of RA (k x c)
  std::vector<double> s, Us, Vs;
  small_svd(k, c, RA.data(), k, tol < 1e-7, s, Us, Vs);
  double tail = 0.0;
  double tol_eff = tol;
  if (ref_norm > 0) {
    double tot = 0.0;
    for (double x2 : s) tot += x2 * x2;
    tot = std::sqrt(tot);
    tol_eff = tot > 0 ? tol * ref_norm / tot : 1.0;
  }
  const int r = truncation_rank(s, tol_eff, cap, &tail);
  stats.last_tail = tail;
  const int mn = (int)s.size();
  std::vector<double> Cm((size_t)kcur * std::max(r, 1), 0.0);  // T (kcur x k) * Us_r diag(s_r)
  for (int j = 0; j < r; ++j)
    for (int i = 0; i < kcur; ++i) {
      double t = 0.0;
      for (int l = 0; l < k; ++l) t += T[(size_t)l * kcur + i] * Us[(size_t)j * k + l];
      Cm[(size_t)j * kcur + i] = orth_spatial ? t : t * s[j];
    }
  std::vector<double> newB((size_t)nt * r, 0.0);
  if (r > 0) matmul(nt, r, c, QB.data(), nt, false, Vs.data(), c, false, newB.data(), nt, 1.0, 0.0);
  if (orth_spatial)
    for (int j = 0; j < r; ++j)
      for (int t = 0; t < nt; ++t) newB[(size_t)j * nt + t] *= s[j];
  (void)mn;
  LowRank out;
  out.resize(nx, nt, r);
  if (r > 0) proj(kcur, src, Cm, r, out.a(), 0.0);
  sync();
  x.A = std::move(out.A);
  x.B = std::move(newB);
  x.rank = r;
}

double Problem::p_inner(const LowRank& x, const LowRank& y) {
  if (x.rank == 0 || y.rank == 0) return 0.0;
  DevMem km;
  km.ensure(sizeof(double) * (size_t)nx * y.rank);
  apply_op(y.rank, y.a(), km.as<double>(), {{1.0, 1.0}});
  std::vector<double> G;
  gram(x.rank, x.a(), y.rank, km.as<double>(), G);
  double s = 0.0;
  for (int j = 0; j < y.rank; ++j)
    for (int i = 0; i < x.rank; ++i) {
      double t = 0.0;
      for (int k = 0; k < nt; ++k) t += x.B[(size_t)i * nt + k] * y.B[(size_t)j * nt + k];
      s += G[(size_t)j * x.rank + i] * t;
    }
  return desc.alpha * tau * s;
}

void Problem::lincomb(const std::vector<const LowRank*>& xs, const std::vector<double>& c, LowRank& out, double tol,
                      int cap) {
  constexpr int kRmax = 256;
  std::vector<const LowRank*> items;
  std::vector<double> coef;
  for (size_t i = 0; i < xs.size(); ++i)
    if (xs[i]->rank > 0 && c[i] != 0.0) { items.push_back(xs[i]); coef.push_back(c[i]); }
  if (items.empty()) { out.resize(nx, nt, 0); return; }
  // group so that each concatenation stays within kRmax columns
  std::vector<std::unique_ptr<LowRank>> partial;
  size_t i = 0;
  while (i < items.size()) {
    int R = 0;
    size_t j = i;
    while (j < items.size() && (R + items[j]->rank <= kRmax || j == i)) { R += items[j]->rank; ++j; }
    auto acc = std::make_unique<LowRank>();
    acc->resize(nx, nt, R);
    int off = 0;
    for (size_t t = i; t < j; ++t) {
      const LowRank* v = items[t];
      LRP_HIP(hipMemcpyAsync(acc->a() + (size_t)off * nx, v->a(), sizeof(double) * nx * v->rank,
                             hipMemcpyDeviceToDevice, st));
      for (int cc = 0; cc < v->rank; ++cc)
        for (int k = 0; k < nt; ++k) acc->B[(size_t)(off + cc) * nt + k] = coef[t] * v->B[(size_t)cc * nt + k];
      off += v->rank;
    }
    partial.push_back(std::move(acc));
    i = j;
  }
  if (partial.size() == 1) {
    truncate(*partial[0], tol, cap, 2);
    out.A = std::move(partial[0]->A);
    out.B = std::move(partial[0]->B);
    out.rank = partial[0]->rank;
    out.nx = nx;
    out.nt = nt;
    return;
  }
  // truncate the partial sums more tightly, then combine them
  std::vector<const LowRank*> ps;
  for (auto& p : partial) {
    truncate(*p, tol * 1e-2, -1, 2);
    ps.push_back(p.get());
  }
  lincomb(ps, std::vector<double>(ps.size(), 1.0), out, tol, cap);
}

}  // namespace lrp
