// Dense helpers on the device through rocBLAS (plain GEMMs) and rocSOLVER
// (symmetric eigensolver), used for the projected problems whose sizes are
// the spatial basis size q or the number of Lanczos vectors (tens to about a
// thousand).  Also the caching device allocator.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace lrp {

// ---- caching allocator ---------------------------------------------------
// Blocks up to 256 MiB are rounded up to a power of two (at least 4 KiB);
// larger ones to a multiple of 256 MiB, so that the multi-GB pole-solve
// blocks of the finest meshes waste at most 256 MiB each.  Free blocks wait
// in per-size lists.  A pool belongs to one problem, whose work is ordered
// on one stream, so a block freed by one operation can be handed to the next
// without waiting: any reuse is ordered after the earlier use on that stream.
struct Pool::Impl {
  std::mutex mu;
  std::map<size_t, std::vector<void*>> free_lists;
  size_t cached = 0, in_use = 0, peak = 0;
  int64_t mallocs = 0, trims = 0;
  double malloc_s = 0.0;
};

Pool::Pool() : impl_(new Impl) {}
Pool::~Pool() {
  (void)hipDeviceSynchronize();
  for (auto& fl : impl_->free_lists)
    for (void* p : fl.second) (void)hipFree(p);
  delete impl_;
}

static size_t rounded_size(size_t bytes) {
  constexpr size_t kLarge = size_t(256) << 20;
  if (bytes > kLarge) return (bytes + kLarge - 1) / kLarge * kLarge;
  size_t s = 4096;
  while (s < bytes) s <<= 1;
  return s;
}

void* Pool::alloc(size_t bytes, size_t* got) {
  const size_t r = rounded_size(bytes);
  {
    std::lock_guard<std::mutex> lk(impl_->mu);
    auto it = impl_->free_lists.find(r);
    if (it != impl_->free_lists.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      impl_->cached -= r;
      impl_->in_use += r;
      impl_->peak = std::max(impl_->peak, impl_->in_use);
      *got = r;
      return p;
    }
  }
  void* p = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  bool trimmed = false;
  hipError_t e = hipMalloc(&p, r);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // release cached blocks and retry once
    trim();
    trimmed = true;
    e = hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(LRPOST_ENOMEM, "device allocation of " + std::to_string(r) + " bytes failed");
    }
  }
  const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  std::lock_guard<std::mutex> lk(impl_->mu);
  // allocation trace for tuning the pool: LRPOST_POOL_LOG=1 prints every
  // device allocation (bytes, cached and in-use bytes, whether the cache was
  // released first, host seconds)
  static const bool log = [] {
    const char* e = std::getenv("LRPOST_POOL_LOG");
    return e && e[0] == '1';
  }();
  if (log)
    std::fprintf(stderr, "pool malloc %zu cached %zu in_use %zu trim %d s %.4f\n", r, impl_->cached, impl_->in_use,
                 trimmed ? 1 : 0, dt);
  ++impl_->mallocs;
  impl_->trims += trimmed ? 1 : 0;
  impl_->malloc_s += dt;
  impl_->in_use += r;
  impl_->peak = std::max(impl_->peak, impl_->in_use);
  *got = r;
  return p;
}

void Pool::release(void* p, size_t bytes) {
  if (!p) return;
  const size_t r = rounded_size(bytes);
  std::lock_guard<std::mutex> lk(impl_->mu);
  impl_->free_lists[r].push_back(p);
  impl_->cached += r;
  impl_->in_use -= r;
}

size_t Pool::trim() {
  std::vector<void*> drop;
  size_t bytes = 0;
  {
    std::lock_guard<std::mutex> lk(impl_->mu);
    for (auto& fl : impl_->free_lists) {
      drop.insert(drop.end(), fl.second.begin(), fl.second.end());
      fl.second.clear();
    }
    bytes = impl_->cached;
    impl_->cached = 0;
  }
  if (!drop.empty()) {
    (void)hipDeviceSynchronize();
    for (void* p : drop) (void)hipFree(p);
  }
  return bytes;
}

size_t Pool::bytes_in_use() const { return impl_->in_use; }
void Pool::counters(int64_t* mallocs, int64_t* trims, double* seconds) const {
  std::lock_guard<std::mutex> lk(impl_->mu);
  *mallocs = impl_->mallocs;
  *trims = impl_->trims;
  *seconds = impl_->malloc_s;
}
size_t Pool::peak_bytes() const { return impl_->peak; }

// ---- rocBLAS / rocSOLVER ---------------------------------------------------
// Calls of different problems (different handles and streams, from the
// serving loop's worker threads) interfered here: rocSOLVER factorizations
// that overlapped on the device came out wrong, and rocBLAS calls that were
// enqueued, or ran on the device, at the same time as another stream's
// changed results far beyond rounding.  So every rocBLAS and rocSOLVER call
// is issued under one process-wide lock and, on the device, waits for the
// previous such call if that was issued on another stream (an event chain:
// the host does not block, and calls on one stream only keep their stream
// order).  A rocSOLVER call in addition holds a second lock until its stream
// has drained, so at most one runs at a time.
static std::mutex g_solver_mu;
static std::mutex g_blas_mu;
constexpr int kMaxDevices = 64;
static hipEvent_t g_blas_done[kMaxDevices] = {};     // end of the last call per device, any stream
static hipStream_t g_blas_stream[kMaxDevices] = {};  // the stream that call was issued on

struct BlasSection {
  std::lock_guard<std::mutex> lk;
  hipStream_t st;
  int dev = 0;
  explicit BlasSection(hipStream_t s) : lk(g_blas_mu), st(s) {
    LRP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(LRPOST_EINVAL, "device ordinal out of range");
    if (!g_blas_done[dev]) LRP_HIP(hipEventCreateWithFlags(&g_blas_done[dev], hipEventDisableTiming));
    else if (g_blas_stream[dev] != st) LRP_HIP(hipStreamWaitEvent(st, g_blas_done[dev], 0));
  }
  ~BlasSection() {
    (void)hipEventRecord(g_blas_done[dev], st);
    g_blas_stream[dev] = st;
  }
};
struct SolverSection {
  std::lock_guard<std::mutex> lk;
  BlasSection blas;
  explicit SolverSection(hipStream_t s) : lk(g_solver_mu), blas(s) {}
  ~SolverSection() { (void)hipStreamSynchronize(blas.st); }
};
static void rb_check(rocblas_status s, const char* what) {
  if (s != rocblas_status_success) fail(LRPOST_EHIP, std::string(what) + " failed (rocblas status " + std::to_string((int)s) + ")");
}

GpuDense::GpuDense(hipStream_t st) {
  rocblas_handle h;
  std::lock_guard<std::mutex> lk(g_blas_mu);
  rb_check(rocblas_create_handle(&h), "rocblas_create_handle");
  rb_check(rocblas_set_stream(h, st), "rocblas_set_stream");
  // no split-K GEMM solutions with atomic accumulation: reproducible results
  rb_check(rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed), "rocblas_set_atomics_mode");
  handle = h;
  st_ = st;
}

GpuDense::~GpuDense() {
  if (!handle) return;
  std::lock_guard<std::mutex> lk(g_blas_mu);
  rocblas_destroy_handle((rocblas_handle)handle);
  // the stream may be destroyed next and its handle value reused: make the
  // next call on any stream wait for the chain again
  for (auto& s : g_blas_stream)
    if (s == st_) s = nullptr;
}

void GpuDense::gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B,
                    int ldb, double beta, double* C, int ldc) {
  if (m <= 0 || n <= 0) return;
  BlasSection blas(st_);
  rb_check(rocblas_dgemm((rocblas_handle)handle, ta ? rocblas_operation_transpose : rocblas_operation_none,
                         tb ? rocblas_operation_transpose : rocblas_operation_none, m, n, k, &alpha, A, lda, B, ldb,
                         &beta, C, ldc),
           "rocblas_dgemm");
}

void GpuDense::gemm_strided_batched(bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda,
                                    long sa, const double* B, int ldb, long sb, double beta, double* C, int ldc,
                                    long sc, int batch) {
  if (m <= 0 || n <= 0 || batch <= 0) return;
  BlasSection blas(st_);
  rb_check(rocblas_dgemm_strided_batched((rocblas_handle)handle, ta ? rocblas_operation_transpose : rocblas_operation_none,
                                         tb ? rocblas_operation_transpose : rocblas_operation_none, m, n, k, &alpha, A,
                                         lda, sa, B, ldb, sb, &beta, C, ldc, sc, batch),
           "rocblas_dgemm_strided_batched");
}

void GpuDense::syevd(int n, double* A, int lda, double* w, DevMem& work) {
  if (n <= 0) return;
  work.ensure(sizeof(double) * (size_t)n + 64);
  int* info = reinterpret_cast<int*>(work.as<char>() + sizeof(double) * (size_t)n);
  SolverSection section(st_);
  rb_check(rocsolver_dsyevd((rocblas_handle)handle, rocblas_evect_original, rocblas_fill_upper, n, A, lda, w,
                            work.as<double>(), info),
           "rocsolver_dsyevd");
}

void GpuDense::syevd_batched(int n, double* A, int lda, long strideA, double* w, long strideW, int batch,
                             DevMem& work) {
  if (n <= 0 || batch <= 0) return;
  if (batch == 1) return syevd(n, A, lda, w, work);
  work.ensure(sizeof(double) * (size_t)n * batch + sizeof(int) * (size_t)batch + 64);
  int* info = reinterpret_cast<int*>(work.as<char>() + sizeof(double) * (size_t)n * batch);
  SolverSection section(st_);
  rb_check(rocsolver_dsyevd_strided_batched((rocblas_handle)handle, rocblas_evect_original, rocblas_fill_upper, n, A,
                                            lda, strideA, w, strideW, work.as<double>(), n, info, batch),
           "rocsolver_dsyevd_strided_batched");
}

void GpuDense::dgmm_right(int m, int n, const double* A, int lda, const double* x, double* C, int ldc) {
  if (m <= 0 || n <= 0) return;
  BlasSection blas(st_);
  rb_check(rocblas_ddgmm((rocblas_handle)handle, rocblas_side_right, m, n, A, lda, x, 1, C, ldc), "rocblas_ddgmm");
}

void GpuDense::scal(int n, double alpha, double* x) {
  if (n <= 0) return;
  BlasSection blas(st_);
  rb_check(rocblas_dscal((rocblas_handle)handle, n, &alpha, x, 1), "rocblas_dscal");
}

}  // namespace lrp
