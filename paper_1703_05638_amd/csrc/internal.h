// Internal declarations of the lrpost library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <array>
#include <chrono>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lrpost.h"
#include "dense.h"
#include "kernels.h"

namespace lrp {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] void fail(int code, const std::string& msg);

// matrix-core and vector-FMA float64 TFLOP/s of the current device (rates.hip)
void measure_fp64_rates(int iters, double* mfma_tflops, double* valu_tflops);

#define LRP_HIP(call)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      ::lrp::fail(LRPOST_EHIP, std::string(#call) + " failed: " + hipGetErrorString(e_));          \
  } while (0)

// Caching device allocator of one problem (see gpu_dense.cpp).
class Pool {
 public:
  Pool();
  ~Pool();
  void* alloc(size_t bytes, size_t* got);
  void release(void* p, size_t bytes);
  size_t trim();  // frees the cached blocks, returns their bytes
  size_t bytes_in_use() const;
  size_t peak_bytes() const;
  // device allocations made, cache releases forced by a failed allocation,
  // and the host seconds spent in both
  void counters(int64_t* mallocs, int64_t* trims, double* seconds) const;

 private:
  struct Impl;
  Impl* impl_;
};

// Pool that DevMem allocations on this thread draw from (set per API call).
std::shared_ptr<Pool>& current_pool();
struct PoolScope {
  std::shared_ptr<Pool> prev;
  explicit PoolScope(const std::shared_ptr<Pool>& p) : prev(current_pool()) { current_pool() = p; }
  ~PoolScope() { current_pool() = prev; }
};

// Device allocation owned by the holder; grows on demand, never shrinks.
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  std::shared_ptr<Pool> pool;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : p(o.p), bytes(o.bytes), pool(std::move(o.pool)) { o.p = nullptr; o.bytes = 0; }
  DevMem& operator=(DevMem&& o) noexcept {
    release();
    p = o.p; bytes = o.bytes; pool = std::move(o.pool); o.p = nullptr; o.bytes = 0;
    return *this;
  }
  ~DevMem() { release(); }
  void release();
  void ensure(size_t nbytes);
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// rocBLAS GEMM and rocSOLVER symmetric eigensolver on the problem's stream.
class GpuDense {
 public:
  explicit GpuDense(hipStream_t st);
  ~GpuDense();
  void gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
            double beta, double* C, int ldc);
  // batch of C_b = alpha op(A_b) op(B_b) + beta C_b with constant strides (stride 0: shared operand)
  void gemm_strided_batched(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda, long sa,
                            const double* B, int ldb, long sb, double beta, double* C, int ldc, long sc, int batch);
  // A (n x n, upper triangle) -> eigenvectors in place, eigenvalues ascending in w (all device)
  void syevd(int n, double* A, int lda, double* w, DevMem& work);
  // the same for `batch` matrices A + b strideA (eigenvalues at w + b strideW);
  // one batched solve costs about as much as one single solve
  void syevd_batched(int n, double* A, int lda, long strideA, double* w, long strideW, int batch, DevMem& work);
  // C = A diag(x) (A, C: m x n device; x: n device)
  void dgmm_right(int m, int n, const double* A, int lda, const double* x, double* C, int ldc);
  void scal(int n, double alpha, double* x);

 private:
  void* handle = nullptr;
  hipStream_t st_ = nullptr;
};

// A low-rank space-time vector X = A B^T with A on the device (nx x rank,
// leading dimension nx) and B on the host (nt x rank, leading dimension nt).
struct LowRank {
  int rank = 0;
  DevMem A;
  std::vector<double> B;
  long nx = 0;
  int nt = 0;
  void resize(long nx_, int nt_, int r);
  double* a() const { return A.as<double>(); }
};

struct MgLevel {
  int n;      // interior nodes per side
  long nx;    // n*n
  double h;   // mesh spacing
};

// Spatial operator a K + b M on the finest mesh, per column.
struct ShiftCoef {
  double a, b;
};

// Host settings of the convection-diffusion operator (convdiff.cpp): delta
// (from the Peclet rule when given < 0), the symmetric part's spectrum bounds
// of M^{-1} L and the skew part's bound, the rectangle [1, fov_re] x
// i[-fov_im, fov_im] holding the field of values of the projected I + tau K~,
// and the Newton-Schulz start, its radius bound and step count.
struct CdParams {
  double delta, lam_min, lam_sym, skew, fov_re, fov_im, ns_alpha, ns_radius;
  int ns_iters;
};
CdParams cd_params(int N, int nt, double T, double nu, double w, double delta);

class Problem {
 public:
  explicit Problem(const lrpost_problem_desc& d);
  ~Problem();

  lrpost_problem_desc desc;
  int N, n, nt;
  long nx;
  double h, tau;
  hipStream_t st;
  std::vector<MgLevel> lv;
  int lds_level;  // first level solved inside one LDS workgroup
  std::vector<uint8_t> mask_h;
  std::vector<double> kmdiag_h_;  // diag((K+M)^{-1}), n x n nodes
  // re-target to another prior scale, noise level, box and seed
  void set_observation(double alpha, double sigma, const double* box, uint64_t seed);
  DevMem mask;
  int nobs = 0;
  std::vector<double> dprior_h;  // diag(P^{-1}) per node
  DevMem dprior;
  lrpost_stats stats{};

  // ---- small host/device transfers -------------------------------------
  // Every host transfer goes through pinned buffers of the problem's own:
  // the runtime stages pageable copies through buffers that all threads
  // share, and problems served concurrently read back corrupted values
  // through them.  to_host* return after the data has arrived.
  void sync();
  void to_host(double* dst, const double* src, size_t count);
  void to_device(double* dst, const double* src, size_t count);
  void to_host_bytes(void* dst, const void* src, size_t bytes);
  void to_device_bytes(void* dst, const void* src, size_t bytes);
  // rows x cols block of doubles with leading dimension ld (device) into a
  // contiguous host array (leading dimension rows)
  void to_host_block(double* dst, const double* src, int rows, int cols, long ld);

  // ---- spatial building blocks (double) --------------------------------
  // Y = (a_j K + b_j M) X + c_j Z on the finest level
  void apply_op(int ncols, const double* X, double* Y, const std::vector<ShiftCoef>& ab,
                const double* Z = nullptr, const std::vector<double>* zc = nullptr);
  // X ~ (a_j K + b_j M)^{-1} B by `cycles` V-cycles from zero
  // In LRPOST_MIXED mode the V-cycles run in float32: `cycles` of them per
  // round, and `refine` further rounds each start from the float64 residual
  // B - A X (iterative refinement); in float64 mode `refine` is ignored.
  void mg_solve(int ncols, const double* B, double* X, const std::vector<ShiftCoef>& ab, int cycles,
                int refine = 0);
  // C (host, m x q) = A^T B
  void gram(int m, const double* A, int q, const double* B, std::vector<double>& C);
  // C (device, m x q, leading dimension m) = A^T B
  void gram_dev(int m, const double* A, int q, const double* B, double* C);
  // several device Gram products (nx rows; part is set here) in grouped launches
  void gram_dev_grouped(std::vector<GramGroup>& gs);
  // several device projections C_g = beta C_g + alpha A_g Q_g in grouped launches
  void proj_dev_grouped(const std::vector<ProjGroup>& pg, double alpha, double beta);
  // C = beta C + A Q (Q host m x p)
  void proj(int m, const double* A, const std::vector<double>& Q, int p, double* C, double beta);
  // C = beta C + alpha A Q (Q device m x p, leading dimension ldq)
  void proj_dev(int m, const double* A, const double* Q, int ldq, int p, double* C, double beta, double alpha = 1.0);
  // Y = L X for ncols nodal vectors, L = (alpha tau)^{-1/2} (K+M)^{-1/2} (symmetric root)
  void prior_sqrt(int ncols, const double* X, double* Y);
  // symmetric eigenproblem of a host matrix (ascending), on the GPU above a small size
  void sym_eig(int n, const double* A, int lda, std::vector<double>& w, std::vector<double>& V);
  // thin SVD of a small host matrix; `accurate` asks for relative accuracy of
  // small singular values (one-sided Jacobi), otherwise the smaller Gram's
  // eigenpairs are used (resolves singular values down to about 1e-8 of the largest)
  void small_svd(int m, int n, const double* A, int lda, bool accurate, std::vector<double>& s,
                 std::vector<double>& U, std::vector<double>& V);

  std::shared_ptr<Pool> pool;
  std::unique_ptr<GpuDense> dense;

  // progress lines (JSON, stderr) of the eigensolvers when > 0
  int log_level = 0;
  // eigensolver limits (0: the defaults of lrpost_eigensolve)
  int eig_max_vectors = 0;
  double eig_rtol = 0.0;

  // host wall time per phase of a Hessian apply and of the Lanczos step,
  // reported in the progress lines (a phase that ends in a read-back also
  // carries the device time of the work it queued)
  enum Phase {
    kPhPrep, kPhPoles, kPhProject, kPhProjSolve, kPhTrunc, kPhPrior,
    kPhMaterialize, kPhAbsorb, kPhReorth, kPhRitz, kPhOrthBlock, kPhCheck, kPhCount
  };
  std::array<double, kPhCount> phase_s{};
  // (log_level > 2 drains the stream at the end of every phase, so that each
  // phase carries exactly its own device time)
  struct PhaseTimer {
    Problem* p;
    double& acc;
    std::chrono::steady_clock::time_point t0;
    PhaseTimer(Problem* pr, Phase ph) : p(pr), acc(pr->phase_s[ph]), t0(std::chrono::steady_clock::now()) {}
    ~PhaseTimer() {
      if (p->log_level > 2) (void)hipStreamSynchronize(p->st);
      acc += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  };

  // opt-in timing of the multigrid kernels with HIP events, per kernel kind
  // (LRPOST_KERNEL_*): every launch is bracketed by an event pair on the
  // problem's stream and credited with its algorithmic bytes
  struct ProfSlot {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    double bytes = 0.0, flops = 0.0;
  };
  bool prof_on = false;
  std::array<ProfSlot, 10> prof_;
  template <class Launch>
  void timed(int kind, double bytes, Launch&& launch, double flops = 0.0);
  template <typename T>
  void smooth_step(int nl, int ncols, const T* xc, const T* xp, T* xo, const T* b, long ld, const double* prm, int s);
  void prof_reset();
  void prof_read(int kind, int64_t* launches, double* ms, double* bytes, double* flops);
  // level-fused multigrid kernels on meshes with up to kMgFusedMaxN nodes per
  // side (on by default; off selects the per-step kernels)
  bool mg_fused = true;
  // V-cycles replayed from captured HIP graphs (on by default; needs a
  // non-null stream)
  bool use_graphs = true;
  hipStream_t own_stream_ = nullptr;  // created when the description names no stream
  int64_t stats_graphs_captured = 0, stats_graph_launches = 0;
  void drop_graphs();

  // ---- low-rank operations ---------------------------------------------
  // Solve tau K Y + M Y C^T = F (forward) or tau K Y + M Y C = F (adjoint).
  void spacetime_solve(const LowRank& F, LowRank& Y, bool adjoint);
  // The same for several sources, with all pole solves in one multigrid solve.
  void spacetime_solve_batch(const std::vector<const LowRank*>& F, const std::vector<LowRank*>& Y, bool adjoint);
  void st_solve_group(const std::vector<const LowRank*>& F, const std::vector<LowRank*>& Y, bool adjoint);
  // the initial-condition problem (ic.cpp): observed nodes from a mask, the
  // prior-preconditioned misfit Hessian G = c sigma^-2 C^T K^-T B^T B K^-1 C
  // on initial states (C = e_1 kron M), its leading eigenpairs and the
  // posterior variance c (I + G)^-1
  void set_obs_mask(const uint8_t* m);
  // ---- convection-diffusion operator (convdiff.cpp) ----------------------
  // With cd_on the space-time solves use the SUPG operator
  // L = nu K + w N + delta w^2 S (wind (0, w) along x2, Sec. 6.3) in place of
  // K: L in forward solves, L^T in adjoint ones (cd_sign -1).  Its shifted
  // solves are exact (sine transform along x1, tridiagonal systems along x2).
  bool cd_on = false;
  double cd_nu = 0.0, cd_w = 0.0, cd_delta = 0.0;
  int cd_sign = 1;
  // nu <= 0: back to the heat operator K
  void set_convection(double nu, double w, double delta);
  // Y = (a_j L + b_j M) X (sign -1: a_j L^T + b_j M)
  void cd_apply(int ncols, const double* X, double* Y, const std::vector<ShiftCoef>& ab, int sign);
  // X = (a_j L + b_j M)^{-1} B (sign -1: transposed), a_j, b_j >= 0, a_j + b_j > 0
  void cd_solve(int ncols, const double* B, double* X, const std::vector<ShiftCoef>& ab, int sign);
  // the space-time solver's spatial operator (tau L, tau L^T or tau K) and
  // its shifted solves (exact, or `cycles` V-cycles for K)
  void st_apply(int ncols, const double* X, double* Y, const std::vector<ShiftCoef>& ab);
  void st_spatial_solve(int ncols, const double* B, double* X, const std::vector<ShiftCoef>& ab, int cycles);
  // poles and Newton-Schulz bound from the spectrum of the operator's
  // symmetric part; count_scale multiplies the number of poles
  void init_st_poles(double lam_min, double lam_max, double count_scale = 1.0);
  void ic_apply(int nvec, const double* U, double* Y, double c);
  bool ic_eigensolve(double c, int k, int max_vectors, double rtol, double* values, double* vectors, int* used);
  void ic_post_variance(double c, int k, const double* values, const double* vectors, double* out);
  // Hessian applies of several vectors with fused multigrid solves.
  void hess_apply_batch(const std::vector<const LowRank*>& x, const std::vector<LowRank*>& y, bool precond);
  struct StPrep {
    int r1 = 0;
    DevMem Fb;               // orthonormal spatial factor of the source (nx x r1)
    std::vector<double> F2p; // its temporal factor (nt x r1), time-reversed for the adjoint
  };
  void st_prepare(const std::vector<const LowRank*>& F, bool adjoint, std::vector<StPrep>& prs);
  double* st_pole_solves(const std::vector<const StPrep*>& prs);
  // per source: M-orthonormal basis Q (nx x q) and projected solution Zp
  // (q x nt); Kt (projected tau K) is built with the basis
  struct StFin {
    int q = 0;
    DevMem Q, Zp, Kt;
    DevMem Q32;  // float32 copy of Q for the first Gram-Schmidt sweep (mixed precision)
  };
  // mixed precision: the first Gram-Schmidt sweep of the basis building on
  // the float32 matrix cores (the second stays float64)
  bool sweep_f32 = true;
  std::vector<StFin> fin_keep_;  // basis buffers kept between batches (st_solve_pass)
  void st_project_batch(const std::vector<StPrep>& prs, double* Wall, std::vector<StFin>& fins);
  void st_solve_projected(const std::vector<StPrep>& prs, const std::vector<int>& q, std::vector<StFin>& fins);
  void st_truncate(std::vector<StFin>& fins, const std::vector<LowRank*>& Y, bool adjoint);
  // prepare, pole solves, projection and truncation with the current poles
  void st_solve_pass(const std::vector<const LowRank*>& F, const std::vector<LowRank*>& Y, bool adjoint);
  // relative Frobenius residuals of eq. st_pde for the solutions Y_j of F_j
  // and of the same residuals preconditioned by two V-cycles of M + tau K
  void st_residuals(const std::vector<const LowRank*>& F, const std::vector<const LowRank*>& Y, bool adjoint,
                    std::vector<double>& rel, std::vector<double>& prel);
  // residual check of every space-time solve: 0 off, 1 measure (last_st_resid,
  // last_st_presid), 2 measure and, with the preconditioned residual above
  // the threshold, enrich the basis once (st_unresolved counts solves still
  // above it), 3 as 2 but fail with LRPOST_ENOCONV when still above it
  int st_check = 2;
  double st_rtol = 0.0;
  // G x (precond) or H_mis x (misfit).
  void hess_apply(const LowRank& x, LowRank& y, bool precond);
  // Truncate in place; weight 0: Euclidean, 1: M, 2: K+M.  With ref_norm > 0
  // the discarded tail is bounded by tol * ref_norm instead of tol * ||x||;
  // with orth_spatial the new spatial factor is W-orthonormal and the
  // singular values go to the temporal factor.
  void truncate(LowRank& x, double tol, int cap, int weight, double ref_norm = 0.0, bool orth_spatial = false);
  // P inner product alpha tau <X, (I kron (K+M)) Y>.
  double p_inner(const LowRank& x, const LowRank& y);
  // how many applies of inputs of rank <= r fit in one batch (at most want):
  // per input, the pole solves and spatial basis of its forward solve take
  // about r * (poles) nx doubles several times over; batches use at most
  // half of the device memory free when the problem was created, or the
  // limit set by lrpost_set_apply_batch
  int apply_batch_limit(int r, int want) const;
  int apply_batch_max = 0;
  size_t free_at_create = 0;
  // P^{-1} sigma^{-2} F^T y for observations y (nobs x nt, host, column-major;
  // the observed nodes in increasing node order): the right-hand side of the
  // normal equations of the posterior mean, divided by P.
  void data_rhs(const double* y, LowRank& c);
  // sum_i c_i x_i as a truncated low-rank vector (P-weighted truncation).
  void lincomb(const std::vector<const LowRank*>& xs, const std::vector<double>& c, LowRank& out, double tol,
               int cap);

  // ---- configuration of the inner solvers --------------------------------
  int st_poles = 0;
  int st_cycles = 0;
  int prior_cycles = 0;
  std::vector<double> poles;
  // sine basis of K and M (device, n x n) and the per-mode weights of L (device, nx)
  DevMem sine_, root_w_, sqrt_tmp_;

 private:
  DevMem mg_param_, mg_work_, mg_res_, gram_part_, gram_out_, proj_q_, op_w_;
  std::map<std::array<double, 3>, DevMem> op_w_cache_;  // weights of column-uniform operators
  static constexpr size_t kStagingBytes = size_t(32) << 20;
  static constexpr size_t kReadbackBytes = size_t(8) << 20;
  void* staging_ = nullptr;   // pinned, host -> device, recycled at every sync
  size_t staging_used_ = 0;
  void* readback_ = nullptr;  // pinned, device -> host
  double ns_bound_ = 1.0;     // upper bound of the eigenvalues of the projected I + tau K
  int ns_iters_ = 1;          // Newton-Schulz steps for its inverse
  double pole_lam_max_ = 0.0; // top of the spatial spectrum (enrichment poles)
  // convection-diffusion: Newton-Schulz start X_0 = cd_ns_alpha_ I and steps;
  // sine matrix (n x n), sine-mode mass and stiffness eigenvalues (n), the
  // per-column shifts and stencil weights, the transform buffer, and the
  // buffer of tau L Q for the projected operator
  // a larger pole set for sources of rank <= 2 (empty: the base set for all)
  std::vector<double> poles_low_;
  double cd_ns_alpha_ = 1.0;
  int cd_ns_iters_ = 1;
  DevMem cd_S_, cd_mu_, cd_kap_, cd_ab_, cd_wt_, cd_tmp_, st_lq_;
  std::vector<double> cd_mu_h_, cd_kap_h_;
  std::vector<double> mg_param_h_, op_w_h_;
  std::vector<double> tmp_h_;
  template <typename T>
  void vcycle_zero(int ncols, const T* B, T* X, bool accumulate = false);  // accumulate: X += V(B), fused path only
  template <typename T>
  void vcycle_launch(int ncols, const T* B, T* X, bool accumulate, const std::vector<size_t>& off);
  // HIP graphs of V-cycle launch sequences, one per precision, shape and buffers
  struct GraphKey {
    size_t elem;
    int ncols;
    const void *B, *X, *work, *prm;
    int acc, fused;
    bool operator<(const GraphKey& o) const;
  };
  struct GraphEntry {
    hipGraphExec_t exec;
    uint64_t serial;
  };
  static constexpr size_t kMaxGraphs = 64;
  std::map<GraphKey, GraphEntry> graphs_;
  uint64_t graph_serial_ = 0;
  template <class Launch>
  void run_graph(const GraphKey& key, Launch&& launch);
  // the V-cycle runs through the level-fused kernels (which can accumulate)
  bool vcycle_fused() const { return mg_fused && lds_level > 0 && lv[0].n <= kMgFusedMaxN; }
  // cycles V-cycles in float32 on nx x ncols float data (residual correction between cycles)
  void mg_cycles_f32(int ncols, const float* B, float* X, const std::vector<ShiftCoef>& neg, int cycles);
  DevMem mg_work_f_, mg_f_;
  void upload_mg_params(const std::vector<ShiftCoef>& ab);
  // space-time solver workspaces
  DevMem st_res_a_, st_res_b_, st_res_q_, st_res_g_, st_res_p_, st_res_h_;
  DevMem st_gram_, st_g_, st_mw_, st_w2_, st_tm_, st_prep_g_, st_prep_t_, st_wall_, st_brep_, st_small_, st_c_, eig_work_;
};

// kernel launches bracketed by event pairs while timing is on (LRPOST_KERNEL_*)
template <class Launch>
inline void Problem::timed(int kind, double bytes, Launch&& launch, double flops) {
  if (!prof_on) {
    launch();
    return;
  }
  ProfSlot& ps = prof_[kind];
  if (ps.used == ps.ev.size()) {
    hipEvent_t a, e;
    LRP_HIP(hipEventCreate(&a));
    LRP_HIP(hipEventCreate(&e));
    ps.ev.push_back({a, e});
  }
  auto& ev = ps.ev[ps.used++];
  LRP_HIP(hipEventRecord(ev.first, st));
  launch();
  LRP_HIP(hipEventRecord(ev.second, st));
  ps.bytes += bytes;
  ps.flops += flops;
}

void smoother_interval(double a, double bh2, double* lo, double* hi);
void chebyshev_coefs(double lo, double hi, int nu, double* alpha, double* beta);
constexpr int kMgNu = 3;  // Chebyshev steps before and after each coarse correction (odd)
double normal_draw(uint64_t seed, uint64_t stream, uint64_t idx);

struct EigResult {
  std::vector<double> lambda;
  std::vector<std::unique_ptr<LowRank>> vecs;
  int steps = 0;
  double max_resid = -1.0;  // largest relative Ritz residual estimate of the returned pairs
  bool converged = true;    // every wanted pair met the residual target within the vector limit
};
// Linear-solve mode of the block Lanczos process: (G + shift I) x = rhs in
// the P inner product (G is P-self-adjoint), solved by the Galerkin condition
// on the block Krylov space started from rhs (the Lanczos form of conjugate
// gradients, with full re-orthogonalization).
struct LanczosSolve {
  const LowRank* rhs = nullptr;
  double shift = 1.0;
  double rtol = 1e-8;           // stop at ||residual||_P <= rtol ||rhs||_P (recurrence estimate)
  std::unique_ptr<LowRank> x;   // the solution
  double resid = -1.0;
  int steps = 0;
  bool converged = false;
};
EigResult block_lanczos(Problem* P, int k, int bsize, int max_vectors, double rtol, LanczosSolve* lin = nullptr);
// Two-pass randomized eigensolver on the given probes (space-time vectors).
EigResult randomized_eig(Problem* P, int k, const std::vector<const LowRank*>& probes);

}  // namespace lrp

struct lrpost_problem {
  std::unique_ptr<lrp::Problem> impl;
  // expires when the handle is destroyed; eigs handles keep a weak reference
  std::shared_ptr<int> alive = std::make_shared<int>(0);
};

struct lrpost_eigs {
  lrpost_problem* owner = nullptr;
  std::weak_ptr<int> owner_alive;
  std::vector<double> lambda;
  std::vector<std::unique_ptr<lrp::LowRank>> vecs;
};
