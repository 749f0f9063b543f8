// Device kernels for gfx950: Q1 stencil SpMM, geometric-multigrid passes,
// tall-skinny Gram and projection products, elementwise helpers and the
// posterior-variance product.
//
// Layout: a spatial block holds ncols columns of nx = n*n nodes, column-major
// with leading dimension ld; node (i, j) (0-based, i along x1) sits at j*n + i.
// Homogeneous Dirichlet conditions: nodes outside 0..n-1 read as zero.
//
// Q1 stencils on the uniform mesh of spacing h (interior node, 3x3 block):
//   stiffness K: centre 8/3, the eight neighbours -1/3 (independent of h);
//   mass      M: centre 4h^2/9, edge neighbours h^2/9, corners h^2/36.
// The operator a K + b M is therefore a 9-point stencil with three weights
// (centre, edge, corner); they are precomputed per column on the host.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <type_traits>

#include "kernels.h"

namespace lrp {

// Fused multiply-add with one rounding, written out where the per-step and
// the level-fused multigrid kernels must round identically (the compiler's
// own contraction of a*b + c*d may pick either product).
__device__ inline float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Workgroup w of a launch over strips of columns -> (strip, column): the
// hardware hands workgroups to the 8 XCDs round robin, so consecutive strips
// of a column are given to workgroups 8 apart, which share an XCD and its L2
// (neighbouring strips read each other's edge rows).
__device__ inline void strip_of(int nstrip, int& strip, int& col) {
  const int w = blockIdx.x, g = gridDim.x;
  const int full = g & ~7;
  const int lw = w < full ? (w & 7) * (full >> 3) + (w >> 3) : w;
  strip = lw % nstrip;
  col = lw / nstrip;
}

// ---------------------------------------------------------------------------
// Stencil: Y[:,c] = wc*x + we*(edges) + wk*(corners) + zc * Z[:,c]
// Each thread owns one x1 index and walks S consecutive rows, keeping the
// three rows it needs in registers; the x1 neighbours come from the
// neighbouring lanes' loads through the L1 cache.  Column c's weights are
// W[wstride * c .. + 3] (wstride 0: one set for all columns).
// ---------------------------------------------------------------------------
template <typename T, int S>
__global__ __launch_bounds__(256) void k_stencil(int n, const T* __restrict__ X, long ldx, T* __restrict__ Y, long ldy,
                                                 const T* __restrict__ Z, long ldz, const double* __restrict__ W,
                                                 int wstride) {
  const int col = blockIdx.z;
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j0 = (blockIdx.y * 4 + threadIdx.y) * S;
  if (i >= n || j0 >= n) return;
  const double* w = W + (long)wstride * col;
  const T wc = (T)w[0], we = (T)w[1], wk = (T)w[2], zc = (T)w[3];
  const T* x = X + (long)col * ldx;
  T* y = Y + (long)col * ldy;
  const T* z = Z ? Z + (long)col * ldz : nullptr;
  const bool hl = i > 0, hr = i + 1 < n;
  auto row = [&](int j, T& l, T& m, T& r) {
    if (j < 0 || j >= n) { l = m = r = T(0); return; }
    const T* p = x + (long)j * n + i;
    m = p[0];
    l = hl ? p[-1] : T(0);
    r = hr ? p[1] : T(0);
  };
  T l0, m0, r0, l1, m1, r1, l2, m2, r2;
  row(j0 - 1, l0, m0, r0);
  row(j0, l1, m1, r1);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = j0 + s;
    if (j >= n) break;
    row(j + 1, l2, m2, r2);
    T v = wc * m1 + we * ((l1 + r1) + (m0 + m2)) + wk * ((l0 + r0) + (l2 + r2));
    if (z) v += zc * z[(long)j * n + i];
    y[(long)j * n + i] = v;
    l0 = l1; m0 = m1; r0 = r1;
    l1 = l2; m1 = m2; r1 = r2;
  }
}

// Strip form for meshes of up to 1024 nodes per side: a workgroup of TW >= n
// threads owns S consecutive full mesh rows of one column (one contiguous
// stretch of memory), thread i walks mesh column i down the strip with the
// three rows it needs in registers, and its left and right neighbours come
// from the same rows' cache lines.  Loads are unconditional (indices clamped
// into the mesh, out-of-mesh values scaled to zero) so that they overlap;
// strips that lie inside the mesh skip the row checks.  Consecutive strips of
// a column share an XCD (see strip_of).
template <typename T, int TW, int S, bool HASZ, bool INNER>
__device__ inline void stencil_strip_body(int n, int strip, int col, const T* __restrict__ X, long ldx,
                                          T* __restrict__ Y, long ldy, const T* __restrict__ Z, long ldz,
                                          const double* __restrict__ W, int wstride) {
  const int i = threadIdx.x;
  const int j0 = strip * S;
  const double* w = W + (long)wstride * col;
  const T wc = (T)w[0], we = (T)w[1], wk = (T)w[2], zc = (T)w[3];
  const T* x = X + (long)col * ldx;
  T* y = Y + (long)col * ldy;
  const unsigned ic = i < n ? i : n - 1, il = i > 0 ? (i < n ? i - 1 : n - 1) : 0, ir = i + 1 < n ? i + 1 : n - 1;
  const T kl = i > 0 ? T(1) : T(0), kr = i + 1 < n ? T(1) : T(0);
  auto row = [&](int j, T& l, T& m, T& r) {
    const int jc = INNER ? j : (j < 0 ? 0 : (j >= n ? n - 1 : j));
    const T* p = x + (unsigned)(jc * n);
    const T kj = (INNER || (j >= 0 && j < n)) ? T(1) : T(0);
    m = p[ic] * kj;
    l = p[il] * (kl * kj);
    r = p[ir] * (kr * kj);
  };
  T zv[S];
  if (HASZ) {
    const T* z = Z + (long)col * ldz;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = j0 + s;
      const int jc = INNER ? j : (j >= n ? n - 1 : j);
      zv[s] = (z + (unsigned)(jc * n))[ic];
    }
  }
  T l0, m0, r0, l1, m1, r1, l2, m2, r2;
  row(j0 - 1, l0, m0, r0);
  row(j0, l1, m1, r1);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = j0 + s;
    row(j + 1, l2, m2, r2);
    T v = wc * m1 + we * ((l1 + r1) + (m0 + m2)) + wk * ((l0 + r0) + (l2 + r2));
    if (HASZ) v += zc * zv[s];
    if (i < n && (INNER || j < n)) (y + (unsigned)(j * n))[(unsigned)i] = v;
    l0 = l1; m0 = m1; r0 = r1;
    l1 = l2; m1 = m2; r1 = r2;
  }
}

template <typename T, int TW, int S, bool HASZ>
__global__ __launch_bounds__(TW) void k_stencil_strip(int n, int nstrip, const T* __restrict__ X, long ldx,
                                                      T* __restrict__ Y, long ldy, const T* __restrict__ Z,
                                                      long ldz, const double* __restrict__ W, int wstride) {
  int strip, col;
  strip_of(nstrip, strip, col);
  const int j0 = strip * S;
  if (j0 >= 1 && j0 + S + 1 <= n)
    stencil_strip_body<T, TW, S, HASZ, true>(n, strip, col, X, ldx, Y, ldy, Z, ldz, W, wstride);
  else
    stencil_strip_body<T, TW, S, HASZ, false>(n, strip, col, X, ldx, Y, ldy, Z, ldz, W, wstride);
}

template <typename T, int TW, int S>
static void launch_stencil_strip(hipStream_t st, int n, int ncols, const T* X, long ldx, T* Y, long ldy, const T* Z,
                                 long ldz, const double* W, int wstride) {
  const int nstrip = (n + S - 1) / S;
  if (Z)
    hipLaunchKernelGGL((k_stencil_strip<T, TW, S, true>), dim3(nstrip * ncols), dim3(TW), 0, st, n, nstrip, X, ldx,
                       Y, ldy, Z, ldz, W, wstride);
  else
    hipLaunchKernelGGL((k_stencil_strip<T, TW, S, false>), dim3(nstrip * ncols), dim3(TW), 0, st, n, nstrip, X,
                       ldx, Y, ldy, Z, ldz, W, wstride);
}

// ---------------------------------------------------------------------------
// Autotuner of the stencil strip height S (8, 16 or 32 mesh rows per
// workgroup).  Every node is computed by the same operations whatever S is,
// so the choice changes timing only, never results.  The first launch of a
// shape class -- precision, thread count, mesh side, column count rounded to
// a power of two, with or without the added term -- times each height over
// three launches (events on the caller's stream, after one untimed launch)
// and keeps the fastest for the process; later launches of the class use it.
// Launches whose output aliases an input, or that are being captured into a
// graph, use the rule below without timing: tall strips (less halo
// re-reading) when there are enough columns for a few thousand workgroups.
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
  int elem, tw, n, cls, hasz;
  bool operator<(const TuneKey& o) const {
    return std::tie(elem, tw, n, cls, hasz) < std::tie(o.elem, o.tw, o.n, o.cls, o.hasz);
  }
};
struct TuneEntry {
  int S;
  float us[3];  // per launch, S = 8, 16, 32
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;
bool g_tune_on = true;
constexpr int kTuneS[3] = {8, 16, 32};
}  // namespace

void set_stencil_autotune(bool on) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_on = on;
}

std::string stencil_autotune_report() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::string out;
  char line[256];
  for (const auto& kv : g_tune) {
    const TuneKey& k = kv.first;
    const TuneEntry& e = kv.second;
    std::snprintf(line, sizeof line,
                  "stencil %s threads=%d n=%d cols<=%d %s: S=%d (us per launch: S8 %.1f, S16 %.1f, S32 %.1f)\n",
                  k.elem == 8 ? "float64" : "float32", k.tw, k.n, 1 << k.cls, k.hasz ? "with z" : "no z", e.S,
                  e.us[0], e.us[1], e.us[2]);
    out += line;
  }
  return out;
}

template <typename T, int TW>
static void launch_stencil_s(int S, hipStream_t st, int n, int ncols, const T* X, long ldx, T* Y, long ldy,
                             const T* Z, long ldz, const double* W, int wstride) {
  if (S == 32) launch_stencil_strip<T, TW, 32>(st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
  else if (S == 16) launch_stencil_strip<T, TW, 16>(st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
  else launch_stencil_strip<T, TW, 8>(st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
}

template <typename T, int TW>
static void stencil_strips(hipStream_t st, int n, int ncols, const T* X, long ldx, T* Y, long ldy, const T* Z,
                           long ldz, const double* W, int wstride) {
  const long want = 2048;
  const int rule = (long)((n + 31) / 32) * ncols >= want ? 32 : (long)((n + 15) / 16) * ncols >= want ? 16 : 8;
  int cls = 0;
  while ((1 << cls) < ncols) ++cls;
  const TuneKey key{(int)sizeof(T), TW, n, cls, Z ? 1 : 0};
  int S = rule;
  bool tune = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) S = it->second.S;
    else tune = g_tune_on;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (tune && (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)) tune = false;
  if (tune && ((const void*)Y == (const void*)X || (Z && (const void*)Y == (const void*)Z))) tune = false;
  if (!tune) {
    launch_stencil_s<T, TW>(S, st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
    return;
  }
  TuneEntry e{rule, {0.f, 0.f, 0.f}};
  hipEvent_t a = nullptr, b = nullptr;
  bool ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
  float best = 0.f;
  for (int v = 0; v < 3 && ok; ++v) {
    launch_stencil_s<T, TW>(kTuneS[v], st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
    ok = hipEventRecord(a, st) == hipSuccess;
    for (int r = 0; r < 3; ++r) launch_stencil_s<T, TW>(kTuneS[v], st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
    float ms = 0.f;
    ok = ok && hipEventRecord(b, st) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
         hipEventElapsedTime(&ms, a, b) == hipSuccess;
    e.us[v] = 1000.f * ms / 3.f;
    if (ok && (v == 0 || e.us[v] < best)) {
      best = e.us[v];
      e.S = kTuneS[v];
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (!ok) e.S = rule;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.emplace(key, e);
  }
  // the output of the last timed launch is already the result
}

template <typename T>
void stencil(hipStream_t st, int n, int ncols, const T* X, long ldx, T* Y, long ldy, const T* Z, long ldz,
             const double* W, int wstride) {
  if (ncols <= 0 || n <= 0) return;
  if (n <= 64) return stencil_strips<T, 64>(st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
  if (n <= 128) return stencil_strips<T, 128>(st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
  if (n <= 256) return stencil_strips<T, 256>(st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
  if (n <= 512) return stencil_strips<T, 512>(st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
  if (n <= 1024) return stencil_strips<T, 1024>(st, n, ncols, X, ldx, Y, ldy, Z, ldz, W, wstride);
  constexpr int S = 8;
  dim3 blk(64, 4);
  dim3 grd((n + 63) / 64, (n + 4 * S - 1) / (4 * S), ncols);
  hipLaunchKernelGGL((k_stencil<T, S>), grd, blk, 0, st, n, X, ldx, Y, ldy, Z, ldz, W, wstride);
}
template void stencil<double>(hipStream_t, int, int, const double*, long, double*, long, const double*, long,
                              const double*, int);
template void stencil<float>(hipStream_t, int, int, const float*, long, float*, long, const float*, long,
                             const double*, int);

// ---------------------------------------------------------------------------
// Multigrid passes.  Per level and column the host provides kMgStride doubles
//   {wc, we, wk, 0, alpha_0, beta_0, alpha_1, beta_1, ...}
// with the stencil weights and the Chebyshev-smoother coefficients of each
// step (beta already divided by the diagonal wc).  One smoother step:
//   xo = xc + alpha_s (xc - xp) + beta_s (b - A xc),
// where a null xc or xp stands for zero.  xo may alias xp (each node reads
// its own xp value before writing it; neighbours are read from xc only).
// ---------------------------------------------------------------------------
template <typename T, int S>
__global__ __launch_bounds__(256) void k_cheb(int n, const T* Xc, const T* Xp, T* Xo, const T* __restrict__ B,
                                              long ld, const double* __restrict__ P, int step) {
  // only the explicit fmad() calls fuse: the per-step and level-fused
  // kernels then round every node identically
#pragma clang fp contract(off)
  const int col = blockIdx.z;
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j0 = (blockIdx.y * 4 + threadIdx.y) * S;
  if (i >= n || j0 >= n) return;
  const double* pc = P + (long)col * kMgStride;
  const T wc = (T)pc[0], we = (T)pc[1], wk = (T)pc[2];
  const T al = (T)pc[4 + 2 * step], be = (T)pc[5 + 2 * step];
  const T* b = B + (long)col * ld;
  T* xo = Xo + (long)col * ld;
  const T* xp = Xp ? Xp + (long)col * ld : nullptr;
  if (!Xc) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = j0 + s;
      if (j >= n) break;
      const long idx = (long)j * n + i;
      const T prev = xp ? xp[idx] : T(0);
      xo[idx] = fmad(be, b[idx], -al * prev);
    }
    return;
  }
  const T* x = Xc + (long)col * ld;
  const bool hl = i > 0, hr = i + 1 < n;
  auto row = [&](int j, T& l, T& m, T& r) {
    if (j < 0 || j >= n) { l = m = r = T(0); return; }
    const T* p = x + (long)j * n + i;
    m = p[0];
    l = hl ? p[-1] : T(0);
    r = hr ? p[1] : T(0);
  };
  T l0, m0, r0, l1, m1, r1, l2, m2, r2;
  row(j0 - 1, l0, m0, r0);
  row(j0, l1, m1, r1);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = j0 + s;
    if (j >= n) break;
    row(j + 1, l2, m2, r2);
    const long idx = (long)j * n + i;
    const T ax = fmad(wk, (l0 + r0) + (l2 + r2), fmad(we, (l1 + r1) + (m0 + m2), wc * m1));
    const T prev = xp ? xp[idx] : T(0);
    xo[idx] = fmad(be, b[idx] - ax, fmad(al, m1 - prev, m1));
    l0 = l1; m0 = m1; r0 = r1;
    l1 = l2; m1 = m2; r1 = r2;
  }
}

template <typename T>
void mg_smooth_step(hipStream_t st, int n, int ncols, const T* Xc, const T* Xp, T* Xo, const T* B, long ld,
                    const double* P, int step) {
  constexpr int S = 4;
  dim3 blk(64, 4);
  dim3 grd((n + 63) / 64, (n + 4 * S - 1) / (4 * S), ncols);
  hipLaunchKernelGGL((k_cheb<T, S>), grd, blk, 0, st, n, Xc, Xp, Xo, B, ld, P, step);
}
template void mg_smooth_step<double>(hipStream_t, int, int, const double*, const double*, double*, const double*,
                                     long, const double*, int);
template void mg_smooth_step<float>(hipStream_t, int, int, const float*, const float*, float*, const float*, long,
                                    const double*, int);

// Coarse right-hand side bc = P^T (b - A x): coarse node (I, J) sits on fine
// node (2I+1, 2J+1) (0-based); bilinear-interpolation transpose weights
// 1 (centre), 1/2 (edges), 1/4 (corners).  A workgroup covers 64 x 4 coarse
// nodes: it stages the fine iterate of the 129 x 9 fine nodes they touch
// (plus a one-node halo) in LDS with coalesced row loads, forms each fine
// residual once, and restricts from LDS.
constexpr int RCI = 64, RCJ = 4;                       // coarse tile
constexpr int RFI = 2 * RCI + 1, RFJ = 2 * RCJ + 1;    // fine residual tile (129 x 9)

template <typename T>
__global__ __launch_bounds__(256) void k_resid_restrict(int n, int nc, const T* __restrict__ X,
                                                        const T* __restrict__ B, long ld, T* __restrict__ Bc,
                                                        long ldc, const double* __restrict__ P) {
  // only the explicit fmad() calls fuse: the per-step and level-fused
  // kernels then round every node identically
#pragma clang fp contract(off)
  __shared__ T xs[RFJ + 2][RFI + 3];
  __shared__ T rs[RFJ][RFI + 1];
  const int col = blockIdx.z;
  const int I0 = blockIdx.x * RCI, J0 = blockIdx.y * RCJ;
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const T wc = (T)P[kMgStride * col + 0], we = (T)P[kMgStride * col + 1], wk = (T)P[kMgStride * col + 2];
  const T* x = X ? X + (long)col * ld : nullptr;
  const T* b = B + (long)col * ld;
  const int fi0 = 2 * I0, fj0 = 2 * J0;  // fine origin of the residual tile
  if (x) {
    for (int p = tid; p < (RFJ + 2) * (RFI + 2); p += 256) {
      const int r = p / (RFI + 2), c = p % (RFI + 2);
      const int fj = fj0 - 1 + r, fi = fi0 - 1 + c;
      xs[r][c] = (fi >= 0 && fj >= 0 && fi < n && fj < n) ? x[(long)fj * n + fi] : T(0);
    }
    __syncthreads();
  }
  for (int p = tid; p < RFJ * RFI; p += 256) {
    const int r = p / RFI, c = p % RFI;
    const int fj = fj0 + r, fi = fi0 + c;
    T v = T(0);
    if (fi < n && fj < n) {
      v = b[(long)fj * n + fi];
      if (x)
        v -= fmad(wk, (xs[r][c] + xs[r][c + 2]) + (xs[r + 2][c] + xs[r + 2][c + 2]),
                  fmad(we, (xs[r + 1][c] + xs[r + 1][c + 2]) + (xs[r][c + 1] + xs[r + 2][c + 1]),
                       wc * xs[r + 1][c + 1]));
    }
    rs[r][c] = v;
  }
  __syncthreads();
  const int I = I0 + threadIdx.x, J = J0 + threadIdx.y;
  if (I >= nc || J >= nc) return;
  const int r = 2 * threadIdx.y + 1, c = 2 * threadIdx.x + 1;
  const T acc = rs[r][c] + T(0.5) * ((rs[r][c - 1] + rs[r][c + 1]) + (rs[r - 1][c] + rs[r + 1][c])) +
                T(0.25) * ((rs[r - 1][c - 1] + rs[r - 1][c + 1]) + (rs[r + 1][c - 1] + rs[r + 1][c + 1]));
  Bc[(long)col * ldc + (long)J * nc + I] = acc;
}

template <typename T>
void mg_resid_restrict(hipStream_t st, int n, int ncols, const T* X, const T* B, long ld, T* Bc, long ldc,
                       const double* P) {
  const int nc = (n - 1) / 2;
  dim3 blk(64, 4);
  dim3 grd((nc + 63) / 64, (nc + 3) / 4, ncols);
  hipLaunchKernelGGL((k_resid_restrict<T>), grd, blk, 0, st, n, nc, X, B, ld, Bc, ldc, P);
}
template void mg_resid_restrict<double>(hipStream_t, int, int, const double*, const double*, long, double*, long,
                                        const double*);
template void mg_resid_restrict<float>(hipStream_t, int, int, const float*, const float*, long, float*, long,
                                       const double*);

// Xo = Xi + P e (bilinear interpolation of the coarse correction).
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(int n, int nc, const T* __restrict__ E, long ldc,
                                                     const T* __restrict__ Xi, T* __restrict__ Xo, long ld) {
  // only the explicit fmad() calls fuse: the per-step and level-fused
  // kernels then round every node identically
#pragma clang fp contract(off)
  const int col = blockIdx.z;
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  if (i >= n || j >= n) return;
  const T* e = E + (long)col * ldc;
  auto at = [&](int I, int J) -> T { return (I < 0 || J < 0 || I >= nc || J >= nc) ? T(0) : e[(long)J * nc + I]; };
  // fine index f: odd (f = 2I+1) coincides with coarse I; even f = 2I lies between I-1 and I
  T v;
  const bool io = (i & 1), jo = (j & 1);
  const int Ii = (i - 1) >> 1, Jj = (j - 1) >> 1;  // valid when odd
  if (io && jo) v = at(Ii, Jj);
  else if (io) v = T(0.5) * (at(Ii, j / 2 - 1) + at(Ii, j / 2));
  else if (jo) v = T(0.5) * (at(i / 2 - 1, Jj) + at(i / 2, Jj));
  else v = T(0.25) * (at(i / 2 - 1, j / 2 - 1) + at(i / 2, j / 2 - 1) + at(i / 2 - 1, j / 2) + at(i / 2, j / 2));
  const long idx = (long)col * ld + (long)j * n + i;
  Xo[idx] = Xi[idx] + v;
}

template <typename T>
void mg_prolong_add(hipStream_t st, int n, int ncols, const T* E, long ldc, const T* Xi, T* Xo, long ld) {
  const int nc = (n - 1) / 2;
  dim3 blk(64, 4);
  dim3 grd((n + 63) / 64, (n + 3) / 4, ncols);
  hipLaunchKernelGGL((k_prolong_add<T>), grd, blk, 0, st, n, nc, E, ldc, Xi, Xo, ld);
}
template void mg_prolong_add<double>(hipStream_t, int, int, const double*, long, const double*, double*, long);
template void mg_prolong_add<float>(hipStream_t, int, int, const float*, long, const float*, float*, long);

// ---------------------------------------------------------------------------
// Level-fused multigrid passes for meshes of up to 1023 nodes per side.
//
// A workgroup owns a strip of S consecutive mesh rows of one column, over the
// full row width (TW >= n + 1 threads, thread i holding mesh column i) or over
// a tile of TW - 2H columns plus H halo columns on each side (thread i holding
// mesh column c0 + i).  Each thread keeps its mesh column of the strip plus a
// halo of rows above and below in registers, so vertical neighbours are
// register reads and only the left and right neighbours pass through LDS (one
// exchange per smoother step).  Each Chebyshev step of the smoother is
// recomputed on a halo one row (and, in tiles, one column) narrower than the
// step before, so that the strip needs no data from other workgroups between
// steps.  Per node and step the arithmetic is the per-step kernels' (same
// operands, same order), so tiles and whole rows give the same bits.
//
//   down:  x = NU smoother steps from zero for A x = b, and the coarse
//          right-hand side bc = P^T (b - A x); reads b, writes x and bc.
//   up:    t = xi + P e (bilinear prolongation of the coarse correction e),
//          then NU smoother steps from t; reads xi, e, b, writes x.
//
// Workgroups are numbered so that consecutive tiles and strips of a column
// share an XCD (hardware dispatch goes round robin over the 8 XCDs), keeping
// the halo rows and columns that neighbouring workgroups both read in one L2.
// ---------------------------------------------------------------------------

// One smoother step on rows [lo, hi] of the register column:
//   out = cur + al (cur - prv) + be (b - A cur),
// with cur's rows [lo - 1, hi + 1] exchanged through LDS first.  Rows outside
// the mesh (jb + r outside [0, n)) are kept at zero (INNER strips have every
// row inside the mesh); so are the lanes whose mesh column lies outside it
// (inm false), whose cur and prv are zero and whose coefficients are taken as
// zero.  Lane i sits at LDS column i + 1; columns 0 and TW + 1 hold zeros.
template <typename T, int TW, int R, int lo, int hi, bool INNER>
__device__ __forceinline__ void strip_step(const T (&cur)[R], const T (&prv)[R], T (&out)[R], const T (&b)[R], T* xs, int i,
                                  bool inm, int n, int jb, T wc, T we, T wk, T al, T be) {
  // only the explicit fmad() calls fuse: the per-step and level-fused
  // kernels then round every node identically
#pragma clang fp contract(off)
  constexpr int LP = TW + 2;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r >= lo - 1 && r <= hi + 1) xs[r * LP + i + 1] = cur[r];
  __syncthreads();
  T hs[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r >= lo - 1 && r <= hi + 1) hs[r] = xs[r * LP + i] + xs[r * LP + i + 2];
  const T alm = inm ? al : T(0), bem = inm ? be : T(0);
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r >= lo && r <= hi) {
      const T m = cur[r];
      const T ax = fmad(wk, hs[r - 1] + hs[r + 1], fmad(we, hs[r] + (cur[r - 1] + cur[r + 1]), wc * m));
      const T v = fmad(bem, b[r] - ax, fmad(alm, m - prv[r], m));
      const int j = jb + r;
      out[r] = (INNER || (j >= 0 && j < n)) ? v : T(0);
    }
}

// Row r of a strip's register column (mesh row jb + r, mesh column c) of a
// column-major n x n block: every load is unconditional, with the row and
// column indices clamped into the mesh, so that all of them are in flight at
// once; values outside the mesh are zeroed after (in columns outside 0..n-1
// only when LANES).
template <typename T, int R, bool INNER, bool LANES>
__device__ __forceinline__ void load_rows(const T* __restrict__ a, int n, int c, int jb, T (&v)[R], int r0 = 0,
                                 int r1 = R) {
#pragma clang fp contract(off)
  const unsigned ic = c < 0 ? 0 : (c < n ? c : n - 1);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < r0 || r >= r1) continue;
    const int j = jb + r;
    const int jc = INNER ? j : (j < 0 ? 0 : (j >= n ? n - 1 : j));
    const T x = (a + (unsigned)(jc * n))[ic];
    if (!LANES && INNER) {
      v[r] = x;
    } else {
      // scaled by 1 or 0 rather than selected: a select of a loaded value is
      // compiled into a branch around the load, which serializes the loads
      const bool keep = (!LANES || (c >= 0 && c < n)) && (INNER || (j >= 0 && j < n));
      v[r] = x * (keep ? T(1) : T(0));
    }
  }
}

template <typename T, int TW, int S, int NU, bool INNER>
__device__ __forceinline__ void mg_down_body(T* xs, int n, int col, int strip, int c0, int own_lo, int own_hi, int I0, int ncw,
                                    const T* __restrict__ B, long ld, T* __restrict__ Xo, T* __restrict__ Bc,
                                    long ldc, const double* __restrict__ P) {
  // only the explicit fmad() calls fuse: the per-step and level-fused
  // kernels then round every node identically
#pragma clang fp contract(off)
  constexpr int R = S + 2 * NU + 1;  // rows j0 - NU .. j0 + S + NU
  constexpr int LP = TW + 2;
  const int i = threadIdx.x, c = c0 + i;
  const bool inm = c >= 0 && c < n;
  const int j0 = strip * S, jb = j0 - NU;
  const double* pc = P + (long)col * kMgStride;
  const T wc = (T)pc[0], we = (T)pc[1], wk = (T)pc[2];
  T bv[R], x0[R], x1[R];
  load_rows<T, R, INNER, false>(B + (long)col * ld, n, c, jb, bv);
  // step 0 from zero: x_1 = be_0 b (zero outside the mesh)
  const T be0 = inm ? (T)pc[5] : T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    x1[r] = be0 * bv[r];
    x0[r] = T(0);
  }
  // step s (1, 2) computes rows [s, R-1-s]
  strip_step<T, TW, R, 1, R - 2, INNER>(x1, x0, x0, bv, xs, i, inm, n, jb, wc, we, wk, (T)pc[6], (T)pc[7]);
  strip_step<T, TW, R, 2, R - 3, INNER>(x0, x1, x1, bv, xs, i, inm, n, jb, wc, we, wk, (T)pc[8], (T)pc[9]);
  const T(&x)[R] = x1;
  // owned rows of the owned mesh columns
  T* xo = Xo + (long)col * ld;
  const bool own = i >= own_lo && i < own_hi && c < n;
#pragma unroll
  for (int r = NU; r < NU + S; ++r) {
    const int j = jb + r;
    if (own && (INNER || j < n)) (xo + (unsigned)(j * n))[(unsigned)c] = x[r];
  }
  // residual on rows j0 .. j0 + S (local r = NU .. NU + S), then restriction
  const int nc = (n - 1) / 2;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r >= NU - 1 && r <= NU + S + 1) xs[r * LP + i + 1] = x[r];
  __syncthreads();
  T res[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r >= NU && r <= NU + S) {
      const T hm = xs[r * LP + i] + xs[r * LP + i + 2];
      const T hu = xs[(r - 1) * LP + i] + xs[(r - 1) * LP + i + 2];
      const T hd = xs[(r + 1) * LP + i] + xs[(r + 1) * LP + i + 2];
      T v = bv[r];
      v -= fmad(wk, hu + hd, fmad(we, hm + (x[r - 1] + x[r + 1]), wc * x[r]));
      res[r] = v;
    }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r >= NU && r <= NU + S) xs[(r - NU) * LP + i + 1] = res[r];
  __syncthreads();
  // coarse nodes I0 .. I0 + ncw - 1 of coarse rows J0 .. J0 + S/2 - 1: the
  // fine centre 2I + 1 and its neighbours are mesh columns inside
  // [c0 + own_lo, c0 + own_hi], where the residual is exact
  const int J0 = j0 / 2;
  T* bc = Bc + (long)col * ldc;
  for (int p = i; p < (S / 2) * ncw; p += TW) {
    const int Jl = p / ncw, I = I0 + (p - Jl * ncw);
    if (J0 + Jl >= nc) break;
    if (I >= nc) continue;
    const T* rs = xs + (2 * Jl + 1) * LP + (2 * I + 1 - c0) + 1;  // fine node (2I+1, 2J+1)
    const T acc = rs[0] + T(0.5) * ((rs[-1] + rs[1]) + (rs[-LP] + rs[LP])) +
                  T(0.25) * ((rs[-LP - 1] + rs[-LP + 1]) + (rs[LP - 1] + rs[LP + 1]));
    bc[(long)(J0 + Jl) * nc + I] = acc;
  }
}

// Halo columns of the tiled passes: the down pass needs its smoothed iterate
// one column beyond the residual it restricts, which needs one column beyond
// the owned coarse nodes' fine neighbours (2 steps + 1 + 1); the up pass its
// three smoother steps.
constexpr int kDownHalo = 4, kUpHalo = 3;

// Workgroup -> (strip, tile, column): the tiles of a strip, then the strips,
// then the columns, in XCD-grouped order (strip_of).
__device__ inline void tile_of(int nstrip, int ntile, int& strip, int& tile, int& col) {
  int st;
  strip_of(nstrip * ntile, st, col);
  strip = st / ntile;
  tile = st - strip * ntile;
}

// TILED false: one workgroup covers a whole mesh row (TW >= n + 1); true:
// tiles of TW - 2 H owned mesh columns with H halo columns each side.
// at least four waves per SIMD in float32 (at most 128 registers per lane;
// three in float64, whose strips need more): several workgroups per compute
// unit overlap one's loads with another's smoothing
template <typename T>
constexpr int mg_min_waves() {
  return sizeof(T) == 4 ? 4 : 3;
}

template <typename T, int TW, int S, int NU, bool TILED>
__global__ __launch_bounds__(TW, mg_min_waves<T>()) void k_mg_down(int n, int nstrip, int ntile, const T* __restrict__ B, long ld,
                                                T* __restrict__ Xo, T* __restrict__ Bc, long ldc,
                                                const double* __restrict__ P) {
  static_assert(NU == 3, "three smoother steps");
  constexpr int R = S + 2 * NU + 1;
  constexpr int LP = TW + 2;
  constexpr int H = TILED ? kDownHalo : 0, W = TW - 2 * H;
  static_assert(W % 2 == 0, "owned tile width must be even (coarse nodes align with tiles)");
  __shared__ T xs[R * LP];
  int strip, tile, col;
  tile_of(nstrip, ntile, strip, tile, col);
  for (int r = threadIdx.x; r < R; r += TW) {
    xs[r * LP] = T(0);
    xs[r * LP + TW + 1] = T(0);
  }
  const int c0 = tile * W - H;
  const int I0 = TILED ? tile * (W / 2) : 0, ncw = TILED ? W / 2 : (n - 1) / 2;
  const int jb = strip * S - NU;
  if (jb >= 0 && jb + R <= n)
    mg_down_body<T, TW, S, NU, true>(xs, n, col, strip, c0, H, H + W, I0, ncw, B, ld, Xo, Bc, ldc, P);
  else
    mg_down_body<T, TW, S, NU, false>(xs, n, col, strip, c0, H, H + W, I0, ncw, B, ld, Xo, Bc, ldc, P);
}

template <typename T, int TW, int S, int NU, bool INNER, bool ACC>
__device__ __forceinline__ void mg_up_body(T* xs, int n, int col, int strip, int c0, int own_lo, int own_hi,
                                  const T* __restrict__ Xi, const T* __restrict__ E, long ldc,
                                  const T* __restrict__ B, long ld, T* __restrict__ Xo,
                                  const double* __restrict__ P) {
  // only the explicit fmad() calls fuse: the per-step and level-fused
  // kernels then round every node identically
#pragma clang fp contract(off)
  constexpr int R = S + 2 * NU;  // rows j0 - NU .. j0 + S + NU - 1
  constexpr int NCR = R / 2 + 1;  // coarse rows j0/2 - 2 + q, q < NCR
  const int i = threadIdx.x, c = c0 + i;
  const bool inm = c >= 0 && c < n;
  const int j0 = strip * S, jb = j0 - NU;
  const int nc = (n - 1) / 2;
  const double* pc = P + (long)col * kMgStride;
  const T wc = (T)pc[0], we = (T)pc[1], wk = (T)pc[2];
  const T* e = E + (long)col * ldc;
  // coarse columns feeding fine column c: odd c sits on coarse (c-1)/2; even c
  // lies between c/2 - 1 and c/2 (lanes outside the mesh read clamped
  // addresses and are zeroed below)
  const bool io = c & 1;
  const int ca = io ? (c - 1) >> 1 : (c >> 1) - 1, cb = c >> 1;
  const int J0 = j0 / 2 - 2;  // j0 even, jb = j0 - 3 odd: row r is odd when r is even
  const bool oka = ca >= 0 && ca < nc, okb = !io && cb >= 0 && cb < nc;
  const unsigned cac = ca < 0 ? 0 : (ca >= nc ? nc - 1 : ca), cbc = cb < 0 ? 0 : (cb >= nc ? nc - 1 : cb);
  T ea[NCR], eb[NCR];
#pragma unroll
  for (int q = 0; q < NCR; ++q) {
    const int J = J0 + q;
    const bool okj = J >= 0 && J < nc;
    const int Jc = J < 0 ? 0 : (J >= nc ? nc - 1 : J);
    const T* er = e + (unsigned)(Jc * nc);  // uniform row base
    const T va = er[cac], vb = er[cbc];
    ea[q] = va * ((okj && oka) ? T(1) : T(0));  // scaled, not selected (see load_rows)
    eb[q] = vb * ((okj && okb) ? T(1) : T(0));
  }
  T bv[R], x0[R], x1[R];
  load_rows<T, R, INNER, true>(Xi + (long)col * ld, n, c, jb, x0);
  load_rows<T, R, INNER, false>(B + (long)col * ld, n, c, jb, bv, 1, R - 1);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T v;
    if ((r & 1) == 0) {  // odd fine row j = 2J+1, J = J0 + r/2
      const int q = r / 2;
      v = io ? ea[q] : T(0.5) * (ea[q] + eb[q]);
    } else {  // even fine row between coarse J0 + (r-1)/2 and the next
      const int q = (r - 1) / 2;
      v = io ? T(0.5) * (ea[q] + ea[q + 1]) : T(0.25) * (ea[q] + eb[q] + ea[q + 1] + eb[q + 1]);
    }
    const int j = jb + r;
    x0[r] = (inm && (INNER || (j >= 0 && j < n))) ? x0[r] + v : T(0);
    x1[r] = T(0);
  }
  // step s (0, 1, 2) computes rows [s + 1, R - 2 - s]; step 0 has no previous iterate
  strip_step<T, TW, R, 1, R - 2, INNER>(x0, x1, x1, bv, xs, i, inm, n, jb, wc, we, wk, (T)pc[4], (T)pc[5]);
  strip_step<T, TW, R, 2, R - 3, INNER>(x1, x0, x0, bv, xs, i, inm, n, jb, wc, we, wk, (T)pc[6], (T)pc[7]);
  strip_step<T, TW, R, 3, R - 4, INNER>(x0, x1, x1, bv, xs, i, inm, n, jb, wc, we, wk, (T)pc[8], (T)pc[9]);
  const T(&x)[R] = x1;
  T* xo = Xo + (long)col * ld;
  const bool own = i >= own_lo && i < own_hi && c < n;
  if (ACC) {
    // Xo += x: all old values are read (clamped rows and columns) before any store
    T old[S];
    const unsigned ic = c < 0 ? 0 : (c < n ? c : n - 1);
#pragma unroll
    for (int r = NU; r < NU + S; ++r) {
      const int j = jb + r;
      const int jc = INNER ? j : (j >= n ? n - 1 : j);
      old[r - NU] = (xo + (unsigned)(jc * n))[ic];
    }
#pragma unroll
    for (int r = NU; r < NU + S; ++r) {
      const int j = jb + r;
      if (own && (INNER || j < n)) (xo + (unsigned)(j * n))[(unsigned)c] = old[r - NU] + x[r];
    }
    return;
  }
#pragma unroll
  for (int r = NU; r < NU + S; ++r) {
    const int j = jb + r;
    if (own && (INNER || j < n)) (xo + (unsigned)(j * n))[(unsigned)c] = x[r];
  }
}

template <typename T, int TW, int S, int NU, bool ACC, bool TILED>
__global__ __launch_bounds__(TW, mg_min_waves<T>()) void k_mg_up(int n, int nstrip, int ntile, const T* __restrict__ Xi,
                                              const T* __restrict__ E, long ldc, const T* __restrict__ B, long ld,
                                              T* __restrict__ Xo, const double* __restrict__ P) {
  static_assert(NU == 3, "three smoother steps; the coarse-row bookkeeping assumes a halo of three rows");
  constexpr int R = S + 2 * NU;
  constexpr int LP = TW + 2;
  constexpr int H = TILED ? kUpHalo : 0, W = TW - 2 * H;
  __shared__ T xs[R * LP];
  int strip, tile, col;
  tile_of(nstrip, ntile, strip, tile, col);
  for (int r = threadIdx.x; r < R; r += TW) {
    xs[r * LP] = T(0);
    xs[r * LP + TW + 1] = T(0);
  }
  const int c0 = tile * W - H;
  const int jb = strip * S - NU;
  if (jb >= 0 && jb + R <= n)
    mg_up_body<T, TW, S, NU, true, ACC>(xs, n, col, strip, c0, H, H + W, Xi, E, ldc, B, ld, Xo, P);
  else
    mg_up_body<T, TW, S, NU, false, ACC>(xs, n, col, strip, c0, H, H + W, Xi, E, ldc, B, ld, Xo, P);
}

// Strip height per precision and row width: as tall as the register budget
// of TW threads allows (the halo overhead is (2 NU + 1) / S).
template <typename T, int TW>
constexpr int strip_rows() {
  return sizeof(T) == 4 ? 16 : (TW <= 512 ? 8 : 4);
}

// Meshes of at least kMgTileMinN nodes per side run the tiled passes with
// workgroups of kMgTileTW threads: a whole-row workgroup of 512 or 1024
// threads holds its strip in LDS and registers alone on its compute unit, so
// its loads and its smoother steps alternate instead of overlapping; tiles of
// kMgTileTW columns let several workgroups share a compute unit.  192 threads
// cover the 1023- and 511-node rows with the least recomputed halo (6 and 3
// tiles, 1.13 times the row), against 1.25 and 1.5 times for 256.
constexpr int kMgTileMinN = 256, kMgTileTW = 192;

template <typename T, int TW, bool TILED>
static void launch_down(hipStream_t st, int n, int ncols, const T* B, long ld, T* X, T* Bc, long ldc,
                        const double* P) {
  constexpr int S = strip_rows<T, TILED ? 512 : TW>();
  constexpr int W = TW - 2 * (TILED ? kDownHalo : 0);
  const int nstrip = (n + S - 1) / S, ntile = TILED ? (n + W - 1) / W : 1;
  hipLaunchKernelGGL((k_mg_down<T, TW, S, kMgFusedNu, TILED>), dim3(nstrip * ntile * ncols), dim3(TW), 0, st, n,
                     nstrip, ntile, B, ld, X, Bc, ldc, P);
}

template <typename T, int TW, bool TILED>
static void launch_up(hipStream_t st, int n, int ncols, const T* Xi, const T* E, long ldc, const T* B, long ld,
                      T* Xo, const double* P, bool acc) {
  constexpr int S = strip_rows<T, TILED ? 512 : TW>();
  constexpr int W = TW - 2 * (TILED ? kUpHalo : 0);
  const int nstrip = (n + S - 1) / S, ntile = TILED ? (n + W - 1) / W : 1;
  if (acc)
    hipLaunchKernelGGL((k_mg_up<T, TW, S, kMgFusedNu, true, TILED>), dim3(nstrip * ntile * ncols), dim3(TW), 0, st,
                       n, nstrip, ntile, Xi, E, ldc, B, ld, Xo, P);
  else
    hipLaunchKernelGGL((k_mg_up<T, TW, S, kMgFusedNu, false, TILED>), dim3(nstrip * ntile * ncols), dim3(TW), 0, st,
                       n, nstrip, ntile, Xi, E, ldc, B, ld, Xo, P);
}

template <typename T>
void mg_down(hipStream_t st, int n, int ncols, const T* B, long ld, T* X, T* Bc, long ldc, const double* P) {
  if (n < 64) launch_down<T, 64, false>(st, n, ncols, B, ld, X, Bc, ldc, P);
  else if (n < 128) launch_down<T, 128, false>(st, n, ncols, B, ld, X, Bc, ldc, P);
  else if (n < kMgTileMinN) launch_down<T, 256, false>(st, n, ncols, B, ld, X, Bc, ldc, P);
  else launch_down<T, kMgTileTW, true>(st, n, ncols, B, ld, X, Bc, ldc, P);
}

template <typename T>
void mg_up(hipStream_t st, int n, int ncols, const T* Xi, const T* E, long ldc, const T* B, long ld, T* Xo,
           const double* P, bool acc) {
  if (n < 64) launch_up<T, 64, false>(st, n, ncols, Xi, E, ldc, B, ld, Xo, P, acc);
  else if (n < 128) launch_up<T, 128, false>(st, n, ncols, Xi, E, ldc, B, ld, Xo, P, acc);
  else if (n < kMgTileMinN) launch_up<T, 256, false>(st, n, ncols, Xi, E, ldc, B, ld, Xo, P, acc);
  else launch_up<T, kMgTileTW, true>(st, n, ncols, Xi, E, ldc, B, ld, Xo, P, acc);
}
template void mg_down<double>(hipStream_t, int, int, const double*, long, double*, double*, long, const double*);
template void mg_down<float>(hipStream_t, int, int, const float*, long, float*, float*, long, const double*);
template void mg_up<double>(hipStream_t, int, int, const double*, const double*, long, const double*, long, double*,
                            const double*, bool);
template void mg_up<float>(hipStream_t, int, int, const float*, const float*, long, const float*, long, float*,
                           const double*, bool);

// ---------------------------------------------------------------------------
// Coarse levels in LDS: one workgroup per column runs a full V-cycle from the
// level with n0 = nlds (<= 31) nodes per side down to a single node, entirely
// in shared memory.  Pc holds per level (0 = the level entering LDS) and
// column the kMgStride smoother parameters: Pc[(lvl * ncols + col) * kMgStride].
// Output: X = V-cycle(B) with zero initial guess, nu1 / nu2 Chebyshev steps.
// ---------------------------------------------------------------------------
constexpr int kLdsMaxN = 31;
constexpr int kLdsTotal = 961 + 225 + 49 + 9 + 1;  // 31^2 + 15^2 + 7^2 + 3^2 + 1^2

template <typename T>
__device__ inline T lds_at(const T* a, int n, int i, int j) {
  return (i < 0 || j < 0 || i >= n || j >= n) ? T(0) : a[j * n + i];
}

// nu Chebyshev steps on one level held in LDS: x holds x_0 (or is treated as
// zero), t is scratch; the result is left in x.
template <typename T>
__device__ void lds_smooth(int n, T* x, T* t, const T* b, const double* pc, int nu, bool zero) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const T wc = (T)pc[0], we = (T)pc[1], wk = (T)pc[2];
  // step s reads xc and xp and writes into the buffer holding xp:
  // s = 0: xc = x (or 0), writes t;  s = 1: xc = t, xp = x, writes x; ...
  for (int s = 0; s < nu; ++s) {
    const T al = (T)pc[4 + 2 * s], be = (T)pc[5 + 2 * s];
    T* xc = (s % 2 == 0) ? x : t;
    T* xo = (s % 2 == 0) ? t : x;
    const bool cz = zero && s == 0;        // xc is zero
    const bool pz = s == 0 || (zero && s == 1);  // xp is zero
    for (int p = tid; p < n * n; p += nth) {
      const int i = p % n, j = p / n;
      T ax = T(0), xcv = T(0);
      if (!cz) {
        xcv = xc[p];
        ax = wc * xcv + we * (lds_at(xc, n, i - 1, j) + lds_at(xc, n, i + 1, j) + lds_at(xc, n, i, j - 1) +
                              lds_at(xc, n, i, j + 1)) +
             wk * (lds_at(xc, n, i - 1, j - 1) + lds_at(xc, n, i + 1, j - 1) + lds_at(xc, n, i - 1, j + 1) +
                   lds_at(xc, n, i + 1, j + 1));
      }
      const T prev = pz ? T(0) : xo[p];
      xo[p] = xcv + al * (xcv - prev) + be * (b[p] - ax);
    }
    __syncthreads();
  }
  if (nu % 2 == 1) {
    for (int p = tid; p < n * n; p += nth) x[p] = t[p];
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_lds(int n0, int nlev, const T* __restrict__ B, long ldb,
                                                    T* __restrict__ X, long ldx, const double* __restrict__ Pc,
                                                    int ncols, int nu1, int nu2) {
  __shared__ T xs[kLdsTotal];
  __shared__ T bs[kLdsTotal];
  __shared__ T ts[kLdsMaxN * kLdsMaxN];
  const int col = blockIdx.x;
  const int tid = threadIdx.x, nth = blockDim.x;
  int off[6], nn[6];
  {
    int o = 0, m = n0;
    for (int l = 0; l < nlev; ++l) { off[l] = o; nn[l] = m; o += m * m; m = (m - 1) / 2; }
  }
  for (int p = tid; p < n0 * n0; p += nth) bs[p] = B[(long)col * ldb + p];
  __syncthreads();
  auto prm = [&](int l, int k) -> T { return (T)Pc[((long)l * ncols + col) * kMgStride + k]; };
  auto pcl = [&](int l) -> const double* { return Pc + ((long)l * ncols + col) * kMgStride; };
  // down
  for (int l = 0; l < nlev; ++l) {
    const int n = nn[l];
    T* x = xs + off[l];
    T* b = bs + off[l];
    const T wc = prm(l, 0), we = prm(l, 1), wk = prm(l, 2);
    if (n == 1) {  // exact solve of the 1x1 system
      if (tid == 0) x[0] = b[0] / wc;
      __syncthreads();
      break;
    }
    lds_smooth(n, x, ts, b, pcl(l), nu1, true);
    // restrict residual
    const int nc = (n - 1) / 2;
    T* bc = bs + off[l + 1];
    for (int p = tid; p < nc * nc; p += nth) {
      const int I = p % nc, J = p / nc;
      T acc = T(0);
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          const int i = 2 * I + 1 + di, j = 2 * J + 1 + dj;
          const T ax = wc * lds_at(x, n, i, j) +
                       we * (lds_at(x, n, i - 1, j) + lds_at(x, n, i + 1, j) + lds_at(x, n, i, j - 1) +
                             lds_at(x, n, i, j + 1)) +
                       wk * (lds_at(x, n, i - 1, j - 1) + lds_at(x, n, i + 1, j - 1) +
                             lds_at(x, n, i - 1, j + 1) + lds_at(x, n, i + 1, j + 1));
          const T w = (di == 0 ? T(1) : T(0.5)) * (dj == 0 ? T(1) : T(0.5));
          acc += w * (b[j * n + i] - ax);
        }
      bc[p] = acc;
    }
    __syncthreads();
  }
  // up
  for (int l = nlev - 2; l >= 0; --l) {
    const int n = nn[l], nc = nn[l + 1];
    T* x = xs + off[l];
    const T* e = xs + off[l + 1];
    for (int p = tid; p < n * n; p += nth) {
      const int i = p % n, j = p / n;
      T v;
      const bool io = (i & 1), jo = (j & 1);
      const int Ii = (i - 1) >> 1, Jj = (j - 1) >> 1;
      if (io && jo) v = lds_at(e, nc, Ii, Jj);
      else if (io) v = T(0.5) * (lds_at(e, nc, Ii, j / 2 - 1) + lds_at(e, nc, Ii, j / 2));
      else if (jo) v = T(0.5) * (lds_at(e, nc, i / 2 - 1, Jj) + lds_at(e, nc, i / 2, Jj));
      else
        v = T(0.25) * (lds_at(e, nc, i / 2 - 1, j / 2 - 1) + lds_at(e, nc, i / 2, j / 2 - 1) +
                       lds_at(e, nc, i / 2 - 1, j / 2) + lds_at(e, nc, i / 2, j / 2));
      x[p] += v;
    }
    __syncthreads();
    lds_smooth(n, x, ts, bs + off[l], pcl(l), nu2, false);
  }
  for (int p = tid; p < n0 * n0; p += nth) X[(long)col * ldx + p] = xs[p];
}

template <typename T>
void mg_coarse_lds(hipStream_t st, int n0, int nlev, int ncols, const T* B, long ldb, T* X, long ldx,
                   const double* Pc, int nu1, int nu2) {
  hipLaunchKernelGGL((k_coarse_lds<T>), dim3(ncols), dim3(256), 0, st, n0, nlev, B, ldb, X, ldx, Pc, ncols, nu1,
                     nu2);
}
template void mg_coarse_lds<double>(hipStream_t, int, int, int, const double*, long, double*, long, const double*,
                                    int, int);
template void mg_coarse_lds<float>(hipStream_t, int, int, int, const float*, long, float*, long, const double*, int,
                                   int);

// ---------------------------------------------------------------------------
// Gram C = A^T B (A: nrows x m, B: nrows x q).  Stage 1: each workgroup takes
// a chunk of rows and a 32 x 32 output tile, stages A and B rows through LDS
// and writes a partial tile; stage 2 sums the partials in a fixed order
// (deterministic, no atomics).  Accumulation in double.
// ---------------------------------------------------------------------------
constexpr int GT = 32;     // output tile edge
constexpr int GR = 64;     // rows staged per LDS step

template <typename T>
__global__ __launch_bounds__(256) void k_gram_partial(long nrows, long rows_per_chunk, int m, const T* __restrict__ A,
                                                      long lda, int q, const T* __restrict__ B, long ldb,
                                                      double* __restrict__ part) {
  __shared__ double As[GR][GT + 1];
  __shared__ double Bs[GR][GT + 1];
  const int tm = blockIdx.x, tq = blockIdx.y, chunk = blockIdx.z;
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;  // each thread: 2 x 2 outputs
  const long r0 = (long)chunk * rows_per_chunk;
  const long r1 = min(nrows, r0 + rows_per_chunk);
  double acc[2][2] = {{0, 0}, {0, 0}};
  for (long rb = r0; rb < r1; rb += GR) {
    // load GR x GT of A (columns tm*GT ..) and B
    for (int p = tid; p < GR * GT; p += 256) {
      const int rr = p % GR, cc = p / GR;
      const long r = rb + rr;
      const int ca = tm * GT + cc, cb = tq * GT + cc;
      As[rr][cc] = (r < r1 && ca < m) ? (double)A[(long)ca * lda + r] : 0.0;
      Bs[rr][cc] = (r < r1 && cb < q) ? (double)B[(long)cb * ldb + r] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < GR; ++rr) {
      const double a0 = As[rr][tx], a1 = As[rr][tx + 16];
      const double b0 = Bs[rr][ty], b1 = Bs[rr][ty + 16];
      acc[0][0] += a0 * b0; acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0; acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
  // partial layout: [chunk][q][m] column-major m x q per chunk
  double* P = part + (long)chunk * m * q;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int i = tm * GT + tx + 16 * a, j = tq * GT + ty + 16 * b;
      if (i < m && j < q) P[(long)j * m + i] = acc[a][b];
    }
}

// C[idx] = sum over chunks of part[chunk][idx].  A workgroup takes 64
// consecutive outputs (coalesced reads) and spreads the chunks over 16 lanes
// (chunk c to lane c % 16, each lane's loads independent of one another);
// the 16 lane sums are combined through LDS in a fixed order, so the result
// does not depend on scheduling.
constexpr int SP_X = 64, SP_Y = 16;
__global__ __launch_bounds__(SP_X * SP_Y) void k_sum_partials(int nchunk, long count, const double* __restrict__ part,
                                                             double* __restrict__ C) {
  __shared__ double red[SP_Y][SP_X + 1];
  const int tx = threadIdx.x % SP_X, ty = threadIdx.x / SP_X;
  const long idx = (long)blockIdx.x * SP_X + tx;
  const long idc = idx < count ? idx : count - 1;
  double s = 0.0;
  int c = ty;
  for (; c + 3 * SP_Y < nchunk; c += 4 * SP_Y) {
    const double a0 = part[(long)c * count + idc], a1 = part[(long)(c + SP_Y) * count + idc];
    const double a2 = part[(long)(c + 2 * SP_Y) * count + idc], a3 = part[(long)(c + 3 * SP_Y) * count + idc];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; c < nchunk; c += SP_Y) s += part[(long)c * count + idc];
  red[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && idx < count) {
    double t = red[0][tx];
#pragma unroll
    for (int y = 1; y < SP_Y; ++y) t += red[y][tx];
    C[idx] = t;
  }
}

int gram_chunks(long nrows, int m, int q) {
  // aim for about 2048 workgroups in stage 1, at least 1024 rows per chunk
  const long tiles = (long)((m + GT - 1) / GT) * ((q + GT - 1) / GT);
  long c = 2048 / (tiles > 0 ? tiles : 1);
  const long cmax = (nrows + 1023) / 1024;
  if (c > cmax) c = cmax;
  if (c > 256) c = 256;
  if (c < 1) c = 1;
  return (int)c;
}

// ---------------------------------------------------------------------------
// FP64 Gram on the matrix cores.  Workgroup (tm, tq, chunk) accumulates a
// (64 BM) x (64 BQ) output tile over its chunk of rows; with BM = 3 the tile
// covers m <= 192, so each operand of the usual tall-skinny products is read
// from memory once.  Rows are staged through LDS GK at a time (coalesced:
// consecutive lanes read consecutive rows of one column), stored
// [column][row] so that each MFMA operand is one LDS read per lane; the next
// stages are fetched into registers while the matrix cores work on the
// current one, and stored to the second LDS buffer.  The waves form a 4 x WQ
// grid (8 or 16 waves); each owns (16 BM) x (64 BQ / WQ) of the tile as
// blocks of v_mfma_f64_16x16x4f64: for the 16 x 4 operand lane l holds
// element (l % 16, l / 16), for the 4 x 16 operand element (l / 16, l % 16),
// and the 16 x 16 result element (l / 16 + 4 v, l % 16) in slot v.  The row
// blocks of the m waves interleave (block a of m-wave wm starts at row
// 64 a + 16 wm), and on a tile that the product covers only in part each
// wave skips the products of its blocks that lie wholly outside it: the
// waves of one m index share a SIMD, so a ragged tile's remaining work stays
// spread over the four matrix units (the products of 64 rows and fewer than
// 64 columns, and the last tile of a wide one, are most of the launches).
// ---------------------------------------------------------------------------
typedef double gram_d4 __attribute__((ext_vector_type(4)));
constexpr int GTH = 512;  // threads per workgroup of the 64-wide and float32 tiles
// Tile width 64 BQ in the q direction: BQ = 2 when q > 64, so that the wide
// operand of products with more than 64 columns on both sides is read half
// as often.  Stages of GK rows go through two LDS buffers; AHEAD stages are in
// flight in registers (NC / (TH / GK) values per thread and set) while the
// matrix cores work on the buffered one.  GK = 32, or 16 for the 192-row
// tiles and the 128 x 128 tile (their two 32-row buffers would crowd or
// overflow the 160 KiB of LDS, and shorter stages keep two register sets
// within 128 registers per lane).
template <int BM, int BQ>
struct GramShape {
  static constexpr int GM = 64 * BM, GQ = 64 * BQ;
  static constexpr int GK = ((BQ == 2 && BM >= 2) || BM == 3) ? 16 : 32;
  // waves in the q direction (4 in m): all tiles but the 64 x 64 one run 16
  // waves of 16 BM x 16 BQ output each, whose small accumulator sets leave
  // room for four waves per SIMD (128 registers per lane) and, except in the
  // 192 x 128 tile, for two register sets in flight
  static constexpr int AHEAD = (BM == 3 && BQ == 2) ? 1 : 2;
  static constexpr int WQ = (BQ == 2 || BM >= 2) ? 4 : 2;
  static constexpr int TH = 256 * WQ;  // threads per workgroup
};

template <int BM, int BQ>
__device__ __forceinline__ void gram_tile(long nrows, long rows_per_chunk, int m, const double* __restrict__ A,
                                          long lda, int q, const double* __restrict__ B, long ldb,
                                          double* __restrict__ part, int tm, int tq, int chunk, int row0,
                                          int ldp) {
  // (m columns of A starting at output row row0 of the ldp x q partials)
  constexpr int GM = GramShape<BM, BQ>::GM;   // output tile height (m direction)
  constexpr int GQ = GramShape<BM, BQ>::GQ;   // output tile width (q direction)
  constexpr int GK = GramShape<BM, BQ>::GK;   // rows per LDS stage
  constexpr int TH = GramShape<BM, BQ>::TH;   // threads
  constexpr int WQ = GramShape<BM, BQ>::WQ;   // waves in the q direction
  constexpr int BW = 4 * BQ / WQ;             // 16-wide output blocks per wave in q
  constexpr int NC = GM + GQ;                 // staged columns per row
  constexpr int NU = NC / (TH / GK);          // columns per loading thread
  static_assert(NC % (TH / GK) == 0 && GM % (TH / GK) == 0, "loader layout");
  __shared__ double S[2][NC][GK + 1];         // two stages of [column][row]: A columns, then B columns
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 3, wq = wave >> 2;
  const long r0 = (long)chunk * rows_per_chunk;
  const long r1 = min(nrows, r0 + rows_per_chunk);
  gram_d4 acc[BM][BW];
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BW; ++b) acc[a][b] = gram_d4{0.0, 0.0, 0.0, 0.0};
  const int lr = tid & (GK - 1), lc = tid / GK;  // loader: row lr of columns lc, lc + TH / GK, ...
  const long nst = (r1 > r0) ? (r1 - r0 + GK - 1) / GK : 0;
  // this thread's staged columns: u < NA are columns of A, the rest of B,
  // each as an element offset from the tile's first column (clamped into
  // range: a clamped column only feeds output rows or columns that are never
  // written, so only rows outside the chunk need zeroing)
  constexpr int NA = GM / (TH / GK);
  const double* __restrict__ At = A + (long)tm * GM * lda;
  const double* __restrict__ Bt = B + (long)tq * GQ * ldb;
  const int ma = m - 1 - tm * GM, qb = q - 1 - tq * GQ;
  // (32-bit: at most 191 x 16.8e6 for the largest mesh, 4095^2 nodes)
  unsigned co[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int c = lc + (TH / GK) * u;
    co[u] = u < NA ? (unsigned)min(c, ma) * (unsigned)lda : (unsigned)min(c - GM, qb) * (unsigned)ldb;
  }
  // loads are unconditional (row clamped into the chunk) so that a stage's
  // loads are in flight together; rows outside the chunk are scaled to zero
  // as they are stored to LDS (a select of a loaded value is compiled into a
  // branch around the load)
  auto fetch = [&](long it, double (&rv)[NU]) {
    const long r = r0 + it * GK + lr;
    const long rc = r < r1 ? r : r1 - 1;
#pragma unroll
    for (int u = 0; u < NU; ++u) rv[u] = (u < NA ? At : Bt)[(long)co[u] + rc];
  };
  auto stage = [&](long it, const double (&rv)[NU], int buf) {
    const double keep = r0 + it * GK + lr < r1 ? 1.0 : 0.0;
#pragma unroll
    for (int u = 0; u < NU; ++u) S[buf][lc + (TH / GK) * u][lr] = rv[u] * keep;
  };
  const int ci = lane & 15, ck = lane >> 4;
  // blocks of this wave inside the product (wave-uniform)
  bool va[BM], vb[BW];
  bool whole = true;
#pragma unroll
  for (int a = 0; a < BM; ++a) {
    va[a] = 64 * a + 16 * wm <= ma;
    whole = whole && va[a];
  }
#pragma unroll
  for (int b = 0; b < BW; ++b) {
    vb[b] = wq * 16 * BW + 16 * b <= qb;
    whole = whole && vb[b];
  }
  // MASKED: skip the blocks outside the product (the operands are read
  // either way: LDS holds every staged column)
  auto mma_step = [&](int cb, auto masked) {
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      double bf[BW], af[BM];
#pragma unroll
      for (int b = 0; b < BW; ++b) bf[b] = S[cb][GM + wq * 16 * BW + 16 * b + ci][kk + ck];
#pragma unroll
      for (int a = 0; a < BM; ++a) af[a] = S[cb][64 * a + 16 * wm + ci][kk + ck];
#pragma unroll
      for (int a = 0; a < BM; ++a)
#pragma unroll
        for (int b = 0; b < BW; ++b)
          if (!decltype(masked)::value || (va[a] && vb[b]))
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  };
  // the pipeline over the chunk, with the products of every block or of the
  // blocks inside the product only
  auto run = [&](auto masked) {
    auto mma = [&](int cb) { mma_step(cb, masked); };
    // AHEAD = 2: while stage it is multiplied out of LDS buffer
    // it % 2, stage it + 1 is arriving in one register set (issued one stage
    // earlier) and stage it + 2 is issued into the other; after the products,
    // stage it + 1 goes to the other LDS buffer (its readers, stage it - 1,
    // passed the previous barrier): one barrier per stage
    if constexpr (GramShape<BM, BQ>::AHEAD == 2) {
      double ra[NU], rb[NU];
      if (nst > 0) {
        fetch(0, ra);
        stage(0, ra, 0);
      }
      if (nst > 1) fetch(1, rb);
      __syncthreads();
      for (long it = 0; it < nst; it += 2) {
        if (it + 2 < nst) fetch(it + 2, ra);
        mma(0);
        if (it + 1 < nst) stage(it + 1, rb, 1);
        __syncthreads();
        if (it + 1 >= nst) break;
        if (it + 3 < nst) fetch(it + 3, rb);
        mma(1);
        if (it + 2 < nst) stage(it + 2, ra, 0);
        __syncthreads();
      }
    } else {
      // one stage in flight: stage it + 1 arrives in registers while stage it
      // is multiplied, then goes to the other LDS buffer
      double rv[NU];
      if (nst > 0) {
        fetch(0, rv);
        stage(0, rv, 0);
      }
      __syncthreads();
      for (long it = 0; it < nst; ++it) {
        const int cb = (int)(it & 1);
        if (it + 1 < nst) fetch(it + 1, rv);
        mma(cb);
        if (it + 1 < nst) stage(it + 1, rv, cb ^ 1);
        __syncthreads();
      }
    }
  };
  if (whole)
    run(std::false_type{});
  else
    run(std::true_type{});
  // partial layout: [chunk] column-major ldp x q
  double* P = part + (long)chunk * ldp * q + row0;
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BW; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tm * GM + 64 * a + 16 * wm + (lane >> 4) + 4 * v;
        const int j = tq * GQ + wq * 16 * BW + 16 * b + (lane & 15);
        if (i < m && j < q) P[(long)j * ldp + i] = acc[a][b][v];
      }
}

// Several Gram products in one launch: blockIdx.z = group * nchunk_max +
// chunk; each product keeps its own chunking (rows per chunk from its own
// shape), so its partial sums are exactly those of a launch of its own.
//
// A product with a second segment (m2 > 0) takes ceil((m - m2) / 64 BM) row
// tiles over A, then ceil(m2 / 64 BM) over A2, each tile in one segment.
template <int BM, int BQ>
__global__ __launch_bounds__((GramShape<BM, BQ>::TH)) void k_gram_mfma(long nrows, GramGroups gs) {
  const int gi = blockIdx.z / gs.nchunk_max, chunk = blockIdx.z % gs.nchunk_max;
  const GramGroup& g = gs.g[gi];
  constexpr int GM = 64 * BM;
  const int m1 = g.m - g.m2, t1 = (m1 + GM - 1) / GM;
  int tm = blockIdx.x, mseg = m1, row0 = 0;
  const double* A = g.A;
  if (tm >= t1) {
    tm -= t1;
    mseg = g.m2;
    row0 = m1;
    A = g.A2;
  }
  if (chunk >= g.nchunk || tm * GM >= mseg || (int)blockIdx.y * 64 * BQ >= g.q) return;
  gram_tile<BM, BQ>(nrows, g.rpc, mseg, A, g.lda, g.q, g.B, g.ldb, g.part, tm, blockIdx.y, chunk, row0, g.m);
}

// ---------------------------------------------------------------------------
// The same tiles on the float32 matrix cores (v_mfma_f32_16x16x4f32) for the
// first Gram-Schmidt sweep of the mixed-precision basis building: A is a
// float32 copy of the basis, B is float64 and rounded to float32 as it is
// staged, a chunk accumulates in float32 (the partial products of the chunks
// are summed in float64).  LDS holds float32, so 32-row stages fit for every
// tile shape.  Operand lane layout as for the float64 instruction; result
// element (kF32Row(l, v), l % 16) in slot v.
// ---------------------------------------------------------------------------
typedef float gram_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int kF32Row(int lane, int v) { return 4 * (lane >> 4) + v; }

template <int BM, int BQ>
__device__ __forceinline__ void gram_tile_f32(long nrows, long rows_per_chunk, int m, const float* __restrict__ A,
                                              long lda, int q, const double* __restrict__ B, long ldb,
                                              double* __restrict__ part, int tm, int tq, int chunk) {
  constexpr int GM = 64 * BM, GQ = 64 * BQ, GK = 32;
  constexpr int NC = GM + GQ;
  constexpr int NU = NC / (GTH / GK);
  constexpr int NA = GM / (GTH / GK);
  __shared__ float S[2][NC][GK + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 3, wq = wave >> 2;
  const long r0 = (long)chunk * rows_per_chunk;
  const long r1 = min(nrows, r0 + rows_per_chunk);
  gram_f4 acc[BM][2 * BQ];
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < 2 * BQ; ++b) acc[a][b] = gram_f4{0.f, 0.f, 0.f, 0.f};
  const int lr = tid & (GK - 1), lc = tid / GK;
  const long nst = (r1 > r0) ? (r1 - r0 + GK - 1) / GK : 0;
  const float* __restrict__ At = A + (long)tm * GM * lda;
  const double* __restrict__ Bt = B + (long)tq * GQ * ldb;
  const int ma = m - 1 - tm * GM, qb = q - 1 - tq * GQ;
  unsigned co[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int c = lc + (GTH / GK) * u;
    co[u] = u < NA ? (unsigned)min(c, ma) * (unsigned)lda : (unsigned)min(c - GM, qb) * (unsigned)ldb;
  }
  // loads as in gram_tile (rows outside the chunk zeroed as they are staged)
  auto fetch = [&](long it, float (&rv)[NU]) {
    const long r = r0 + it * GK + lr;
    const long rc = r < r1 ? r : r1 - 1;
#pragma unroll
    for (int u = 0; u < NU; ++u) rv[u] = u < NA ? At[(long)co[u] + rc] : (float)Bt[(long)co[u] + rc];
  };
  auto stage = [&](long it, const float (&rv)[NU], int buf) {
    const float keep = r0 + it * GK + lr < r1 ? 1.f : 0.f;
#pragma unroll
    for (int u = 0; u < NU; ++u) S[buf][lc + (GTH / GK) * u][lr] = rv[u] * keep;
  };
  const int ci = lane & 15, ck = lane >> 4;
  auto mma = [&](int cb) {
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      float bf[2 * BQ];
#pragma unroll
      for (int b = 0; b < 2 * BQ; ++b) bf[b] = S[cb][GM + wq * 32 * BQ + 16 * b + ci][kk + ck];
#pragma unroll
      for (int a = 0; a < BM; ++a) {
        const float af = S[cb][wm * 16 * BM + 16 * a + ci][kk + ck];
#pragma unroll
        for (int b = 0; b < 2 * BQ; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf[b], acc[a][b], 0, 0, 0);
      }
    }
  };
  // one stage in flight (a second register set costs more in occupancy
  // than it gains for these tiles)
  float rv[NU];
  if (nst > 0) {
    fetch(0, rv);
    stage(0, rv, 0);
  }
  __syncthreads();
  for (long it = 0; it < nst; ++it) {
    const int cb = (int)(it & 1);
    if (it + 1 < nst) fetch(it + 1, rv);
    mma(cb);
    if (it + 1 < nst) stage(it + 1, rv, cb ^ 1);
    __syncthreads();
  }
  double* P = part + (long)chunk * m * q;
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < 2 * BQ; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tm * GM + wm * 16 * BM + 16 * a + kF32Row(lane, v);
        const int j = tq * GQ + wq * 32 * BQ + 16 * b + (lane & 15);
        if (i < m && j < q) P[(long)j * m + i] = (double)acc[a][b][v];
      }
}

template <int BM, int BQ>
__global__ __launch_bounds__(GTH) void k_gram_f32(long nrows, GramGroups gs) {
  const int gi = blockIdx.z / gs.nchunk_max, chunk = blockIdx.z % gs.nchunk_max;
  const GramGroup& g = gs.g[gi];
  if (chunk >= g.nchunk || (int)blockIdx.x * 64 * BM >= g.m || (int)blockIdx.y * 64 * BQ >= g.q) return;
  gram_tile_f32<BM, BQ>(nrows, g.rpc, g.m, g.A32, g.lda, g.q, g.B, g.ldb, g.part, blockIdx.x, blockIdx.y, chunk);
}

// tile height 64 BM: the smallest that covers m, at most 192 (the 256-row
// tile needs 146 registers per lane, which leaves one workgroup per CU; wider
// products take several tiles); tile width 64 BQ
int gram_bm(int m) { return m <= 64 ? 1 : m <= 128 ? 2 : 3; }
int gram_bq(int q) { return q <= 64 ? 1 : 2; }

int gram_chunks_mfma(long nrows, int m, int q) {
  // about one workgroup per CU (longer chunks beat more, shorter ones: a
  // chunk's stages are dependent round trips to memory), at least 128 rows
  // per chunk, and per-chunk partial products of at most about 35% of the
  // operand bytes
  const int gm = 64 * gram_bm(m), gq = 64 * gram_bq(q);
  const long tiles = (long)((m + gm - 1) / gm) * ((q + gq - 1) / gq);
  long c = 256 / (tiles > 0 ? tiles : 1);
  const long cmax = (nrows + 127) / 128;
  const long cpart = (long)(0.35 * (double)(m + q) * (double)nrows / ((double)m * q)) + 1;
  c = std::min(c, std::min(cmax, cpart));
  if (c > 1024) c = 1024;
  if (c < 1) c = 1;
  return (int)c;
}

template <typename T>
void gram(hipStream_t st, long nrows, int m, const T* A, long lda, int q, const T* B, long ldb, double* C,
          double* part) {
  if (m <= 0 || q <= 0) return;
  const int nchunk = gram_chunks(nrows, m, q);
  long rpc = (nrows + nchunk - 1) / nchunk;
  rpc = ((rpc + GR - 1) / GR) * GR;
  dim3 grd((m + GT - 1) / GT, (q + GT - 1) / GT, nchunk);
  hipLaunchKernelGGL((k_gram_partial<T>), grd, dim3(256), 0, st, nrows, rpc, m, A, lda, q, B, ldb, part);
  const long count = (long)m * q;
  hipLaunchKernelGGL(k_sum_partials, dim3((count + SP_X - 1) / SP_X), dim3(SP_X * SP_Y), 0, st, nchunk, count, part, C);
}

void gram_mfma_partials(hipStream_t st, long nrows, int count, GramGroup* groups) {
  for (int g0 = 0; g0 < count; g0 += kProjGroupMax) {
    GramGroups gs{};
    const int n = std::min(kProjGroupMax, count - g0);
    int mmax = 0, qmax = 0, cmax = 1;
    for (int i = 0; i < n; ++i) {
      GramGroup& g = groups[g0 + i];
      if (g.m2 < 0 || g.m2 > g.m || (g.m2 > 0 && (!g.A2 || g.A32)))
        throw std::invalid_argument("gram: invalid second segment");
      g.nchunk = (g.m > 0 && g.q > 0) ? gram_chunks_mfma(nrows, g.m, g.q) : 0;
      long rpc = g.nchunk > 0 ? (nrows + g.nchunk - 1) / g.nchunk : 0;
      g.rpc = ((rpc + 31) / 32) * 32;  // a multiple of every stage height
      gs.g[i] = g;
      mmax = std::max(mmax, g.m);
      qmax = std::max(qmax, g.q);
      cmax = std::max(cmax, g.nchunk);
    }
    if (mmax <= 0 || qmax <= 0) continue;
    gs.nchunk_max = cmax;
    const int bm = gram_bm(mmax), gm = 64 * bm;
    int qmin = qmax;
    for (int i = 0; i < n; ++i)
      if (gs.g[i].q > 0) qmin = std::min(qmin, gs.g[i].q);
    // the wide tile only when every product of the launch is wider than 64
    const int bq = gram_bq(qmin), gq = 64 * bq;
    int tmax = 0;  // row tiles: each segment of a product starts a tile
    for (int i = 0; i < n; ++i) {
      const GramGroup& g = gs.g[i];
      tmax = std::max(tmax, (g.m - g.m2 + gm - 1) / gm + (g.m2 + gm - 1) / gm);
    }
    dim3 grd(tmax, (qmax + gq - 1) / gq, n * cmax);
    if (gs.g[0].A32) {  // a launch is all float32 or all float64 (the caller groups them)
      if (bq == 1) {
        switch (bm) {
          case 1: hipLaunchKernelGGL((k_gram_f32<1, 1>), grd, dim3(GTH), 0, st, nrows, gs); break;
          case 2: hipLaunchKernelGGL((k_gram_f32<2, 1>), grd, dim3(GTH), 0, st, nrows, gs); break;
          default: hipLaunchKernelGGL((k_gram_f32<3, 1>), grd, dim3(GTH), 0, st, nrows, gs);
        }
      } else {
        switch (bm) {
          case 1: hipLaunchKernelGGL((k_gram_f32<1, 2>), grd, dim3(GTH), 0, st, nrows, gs); break;
          case 2: hipLaunchKernelGGL((k_gram_f32<2, 2>), grd, dim3(GTH), 0, st, nrows, gs); break;
          default: hipLaunchKernelGGL((k_gram_f32<3, 2>), grd, dim3(GTH), 0, st, nrows, gs);
        }
      }
      continue;
    }
    if (bq == 1) {
      switch (bm) {
        case 1: hipLaunchKernelGGL((k_gram_mfma<1, 1>), grd, dim3(GramShape<1, 1>::TH), 0, st, nrows, gs); break;
        case 2: hipLaunchKernelGGL((k_gram_mfma<2, 1>), grd, dim3(GramShape<2, 1>::TH), 0, st, nrows, gs); break;
        default: hipLaunchKernelGGL((k_gram_mfma<3, 1>), grd, dim3(GramShape<3, 1>::TH), 0, st, nrows, gs);
      }
    } else {
      switch (bm) {
        case 1: hipLaunchKernelGGL((k_gram_mfma<1, 2>), grd, dim3(GramShape<1, 2>::TH), 0, st, nrows, gs); break;
        case 2: hipLaunchKernelGGL((k_gram_mfma<2, 2>), grd, dim3(GramShape<2, 2>::TH), 0, st, nrows, gs); break;
        default: hipLaunchKernelGGL((k_gram_mfma<3, 2>), grd, dim3(GramShape<3, 2>::TH), 0, st, nrows, gs);
      }
    }
  }
}

void sum_partials(hipStream_t st, int nchunk, long count, const double* part, double* C) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_sum_partials, dim3((count + SP_X - 1) / SP_X), dim3(SP_X * SP_Y), 0, st, nchunk, count, part, C);
}

// C_g (m x q, leading dimension ldc) = the sum of the nchunk partial products,
// for several products in one launch (blockIdx.y = g)
__global__ __launch_bounds__(SP_X * SP_Y) void k_sum_partials_grouped(SumGroups gs) {
  const SumGroup& g = gs.g[blockIdx.y];
  const long count = (long)g.m * g.q;
  if ((long)blockIdx.x * SP_X >= count) return;
  __shared__ double red[SP_Y][SP_X + 1];
  const int tx = threadIdx.x % SP_X, ty = threadIdx.x / SP_X;
  const long idx = (long)blockIdx.x * SP_X + tx;
  const long idc = idx < count ? idx : count - 1;
  const double* __restrict__ part = g.part;
  double s = 0.0;
  int c = ty;
  for (; c + 3 * SP_Y < g.nchunk; c += 4 * SP_Y) {
    const double a0 = part[(long)c * count + idc], a1 = part[(long)(c + SP_Y) * count + idc];
    const double a2 = part[(long)(c + 2 * SP_Y) * count + idc], a3 = part[(long)(c + 3 * SP_Y) * count + idc];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; c < g.nchunk; c += SP_Y) s += part[(long)c * count + idc];
  red[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && idx < count) {
    double t = red[0][tx];
#pragma unroll
    for (int y = 1; y < SP_Y; ++y) t += red[y][tx];
    g.C[(idx % g.m) + (idx / g.m) * g.ldc] = t;
  }
}

void sum_partials_grouped(hipStream_t st, int count, const GramGroup* groups) {
  for (int g0 = 0; g0 < count; g0 += kProjGroupMax) {
    SumGroups gs{};
    const int n = std::min(kProjGroupMax, count - g0);
    long cmax = 0;
    for (int i = 0; i < n; ++i) {
      const GramGroup& g = groups[g0 + i];
      gs.g[i] = SumGroup{g.part, g.C, g.ldc, g.m, g.q, g.nchunk};
      if (g.nchunk > 0) cmax = std::max(cmax, (long)g.m * g.q);
    }
    if (cmax <= 0) continue;
    hipLaunchKernelGGL(k_sum_partials_grouped, dim3((cmax + SP_X - 1) / SP_X, n), dim3(SP_X * SP_Y), 0, st, gs);
  }
}

// Column sums of squares of small matrices: one workgroup per column and
// matrix (blockIdx.y), strided partial sums and a fixed-order tree.
struct ColGroups {
  ColGroup g[kProjGroupMax];
};
__global__ __launch_bounds__(256) void k_col_sqnorms(ColGroups gs) {
  const ColGroup& g = gs.g[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= g.cols) return;
  __shared__ double red[256];
  const double* col = g.C + (long)c * g.ld;
  double acc = 0.0;
  for (int i = threadIdx.x; i < g.rows; i += 256) acc = fma(col[i], col[i], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) g.out[c] = red[0];
}

void col_sqnorms(hipStream_t st, int count, const ColGroup* groups) {
  for (int g0 = 0; g0 < count; g0 += kProjGroupMax) {
    ColGroups gs{};
    const int n = std::min(kProjGroupMax, count - g0);
    int cmax = 0;
    for (int i = 0; i < n; ++i) {
      gs.g[i] = groups[g0 + i];
      cmax = std::max(cmax, gs.g[i].cols);
    }
    if (cmax <= 0) continue;
    hipLaunchKernelGGL(k_col_sqnorms, dim3(cmax, n), dim3(256), 0, st, gs);
  }
}

// Posterior variance of the initial-condition problem, one thread per node
// (columns of V read coalesced, the k terms summed in order).
__global__ __launch_bounds__(256) void k_ic_post_var(long nx, int k, const double* __restrict__ V, long ldv,
                                                     const double* __restrict__ w, double c, double* __restrict__ out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= nx) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) {
    const double v = V[i + (long)j * ldv];
    acc = fma(w[j] * v, v, acc);
  }
  out[i] = c - c * acc;
}

void ic_post_var(hipStream_t st, long nx, int k, const double* V, long ldv, const double* w, double c, double* out) {
  if (nx <= 0) return;
  hipLaunchKernelGGL(k_ic_post_var, dim3((nx + 255) / 256), dim3(256), 0, st, nx, k, V, ldv, w, c, out);
}

// The scratch array itself.  Host code never passes its name to a kernel:
// the name is a host-side stand-in, and only the address from
// hipGetSymbolAddress (one per device) is device memory.
static __device__ __align__(256) double scratch[kGramScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

double* gram_scratch_setup() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

double* gram_scratch_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

long gram_part_doubles(long nrows, int m, int q) {
  return (m > 0 && q > 0) ? (long)gram_chunks_mfma(nrows, m, q) * m * q : 0;
}

template <>
void gram<double>(hipStream_t st, long nrows, int m, const double* A, long lda, int q, const double* B, long ldb,
                  double* C, double* part) {
  if (m <= 0 || q <= 0) return;
  GramGroup g{A, B, part, C, lda, ldb, m, 0, m, q, 0};
  gram_mfma_partials(st, nrows, 1, &g);
  sum_partials_grouped(st, 1, &g);
}
template void gram<float>(hipStream_t, long, int, const float*, long, int, const float*, long, double*, double*);

// ---------------------------------------------------------------------------
// Projection C = beta*C + A Q (A: nrows x m, Q: m x p small (double, device),
// C: nrows x p).  Each thread owns one row and up to PT output columns;
// Q is staged through LDS in slabs of 32 rows.
// ---------------------------------------------------------------------------
constexpr int PT = 16;

template <typename T>
void axpby(hipStream_t st, long nx, int ncols, const T* X, long ldx, T* Y, long ldy, double a, double b);

template <typename T>
__global__ __launch_bounds__(256) void k_proj(long nrows, int m, const T* __restrict__ A, long lda,
                                              const double* __restrict__ Q, int ldq, int p, T* __restrict__ C,
                                              long ldc, double beta) {
  __shared__ double Qs[32][PT];
  const long r = (long)blockIdx.x * 256 + threadIdx.x;
  const int c0 = blockIdx.y * PT;
  double acc[PT];
#pragma unroll
  for (int c = 0; c < PT; ++c) acc[c] = 0.0;
  for (int k0 = 0; k0 < m; k0 += 32) {
    for (int t = threadIdx.x; t < 32 * PT; t += 256) {
      const int kk = t % 32, cc = t / 32;
      Qs[kk][cc] = (k0 + kk < m && c0 + cc < p) ? Q[(long)(c0 + cc) * ldq + k0 + kk] : 0.0;
    }
    __syncthreads();
    if (r < nrows) {
      const int kmax = min(32, m - k0);
      for (int kk = 0; kk < kmax; ++kk) {
        const double a = (double)A[(long)(k0 + kk) * lda + r];
#pragma unroll
        for (int c = 0; c < PT; ++c) acc[c] += a * Qs[kk][c];
      }
    }
    __syncthreads();
  }
  if (r < nrows) {
#pragma unroll
    for (int c = 0; c < PT; ++c) {
      if (c0 + c < p) {
        T* dst = C + (long)(c0 + c) * ldc + r;
        *dst = (T)(beta == 0.0 ? acc[c] : beta * (double)(*dst) + acc[c]);
      }
    }
  }
}

template <typename T>
void proj(hipStream_t st, long nrows, int m, const T* A, long lda, const double* Q, int ldq, int p, T* C, long ldc,
          double beta) {
  if (p <= 0) return;
  if (m <= 0) {
    if (beta == 0.0) axpby<T>(st, nrows, p, C, ldc, C, ldc, 0.0, 0.0);
    return;
  }
  dim3 grd((nrows + 255) / 256, (p + PT - 1) / PT);
  hipLaunchKernelGGL((k_proj<T>), grd, dim3(256), 0, st, nrows, m, A, lda, Q, ldq, p, C, ldc, beta);
}

// FP64 projection on the matrix cores, computed as C^T = Q^T A^T so that the
// 16 lanes of one result row of an MFMA block hold 16 consecutive rows of C
// (coalesced stores).  Workgroup: 64 rows x 64 output columns; the inner
// dimension m is staged through two LDS buffers 16 at a time, A as [k][row]
// and Q as [k][column]; each wave owns 32 rows x 32 columns as 2 x 2 MFMA
// blocks.
constexpr int PR = 64, PC = 64, PK = 32;

// One 64 x 64 tile (rows row0.., columns col0..) of C = beta Cin + alpha A Q,
// for the whole workgroup (Cin may be C).
__device__ __forceinline__ void proj_tile(long nrows, int m, const double* __restrict__ A, long lda,
                                          const double* __restrict__ Q, int ldq, int p, const double* Cin,
                                          double* C, long ldc, double alpha, double beta, long row0, int col0,
                                          float* C32 = nullptr) {
  // two LDS buffers of PJK rows of k: while the matrix cores work on one, the
  // next stage arrives in registers and is stored to the other (one barrier
  // per stage)
  // (rows padded by one double: 0.77 bank conflicts per LDS instruction at
  // the 1024^2 workload, the same with the stages stored [row][k]; a padding
  // of 16 measured 16.6 and a slower kernel)
  constexpr int PJK = PK / 2;
  __shared__ double As[2][PJK][PR + 1];
  __shared__ double Qs[2][PJK][PC + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  gram_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = gram_d4{0.0, 0.0, 0.0, 0.0};
  const int ar = tid & 63, ak = tid >> 6;  // A loader: row ar, k = ak + 4u
  const int qk = tid & 15, qc = tid >> 4;  // Q loader: k = qk, column qc + 16u
  const long grow = row0 + ar;
  const long growc = grow < nrows ? grow : nrows - 1;
  // loads are unconditional (indices clamped into range, out-of-range values
  // zeroed after) so that a stage's loads overlap
  double ra[PJK / 4], rq[PC / 16];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PJK / 4; ++u) {
      const int k = k0 + ak + 4 * u;
      const double v = A[(long)(k < m ? k : m - 1) * lda + growc];
      ra[u] = v * ((k < m && grow < nrows) ? 1.0 : 0.0);  // a select here becomes a branch per load
    }
    const int kq = k0 + qk;
    const int kqc = kq < m ? kq : m - 1;
#pragma unroll
    for (int u = 0; u < PC / 16; ++u) {
      const int c = col0 + qc + 16 * u;
      const double v = Q[(long)(c < p ? c : p - 1) * ldq + kqc];
      rq[u] = v * ((kq < m && c < p) ? 1.0 : 0.0);
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PJK / 4; ++u) As[buf][ak + 4 * u][ar] = ra[u];
#pragma unroll
    for (int u = 0; u < PC / 16; ++u) Qs[buf][qk][qc + 16 * u] = rq[u];
  };
  const int ci = lane & 15, ck = lane >> 4;
  const int nst = (m + PJK - 1) / PJK;
  if (nst > 0) {
    fetch(0);
    stage(0);
  }
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const int cb = s & 1;
    if (s + 1 < nst) fetch((s + 1) * PJK);
#pragma unroll
    for (int kk = 0; kk < PJK; kk += 4) {
      const double q0 = Qs[cb][kk + ck][wc * 32 + ci], q1 = Qs[cb][kk + ck][wc * 32 + 16 + ci];
      const double a0 = As[cb][kk + ck][wr * 32 + ci], a1 = As[cb][kk + ck][wr * 32 + 16 + ci];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(q0, a0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(q0, a1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(q1, a0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(q1, a1, acc[1][1], 0, 0, 0);
    }
    if (s + 1 < nst) stage(cb ^ 1);
    __syncthreads();
  }
  // beta != 0: every old value is read (from clamped addresses) before any
  // store, so that the reads are in flight together
  double old[2][2][4];
  if (beta != 0.0) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = col0 + wc * 32 + 16 * a + (lane >> 4) + 4 * v;
          const long r = row0 + wr * 32 + 16 * b + (lane & 15);
          old[a][b][v] = Cin[(long)(j < p ? j : p - 1) * ldc + (r < nrows ? r : nrows - 1)];
        }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = col0 + wc * 32 + 16 * a + (lane >> 4) + 4 * v;
        const long r = row0 + wr * 32 + 16 * b + (lane & 15);
        const double t = alpha * acc[a][b][v];
        const double y = beta == 0.0 ? t : fma(beta, old[a][b][v], t);
        if (j < p && r < nrows) {
          C[(long)j * ldc + r] = y;
          if (C32) C32[(long)j * ldc + r] = (float)y;
        }
      }
}

// (four waves per SIMD: the 1017 row tiles of a 255 x 255 mesh then fit in
// one round of 256 CUs x 4 workgroups)
__global__ __launch_bounds__(256, 4) void k_proj_mfma(long nrows, int m, const double* __restrict__ A, long lda,
                                                   const double* __restrict__ Q, int ldq, int p,
                                                   double* __restrict__ C, long ldc, double beta) {
  proj_tile(nrows, m, A, lda, Q, ldq, p, C, C, ldc, 1.0, beta, (long)blockIdx.x * PR, blockIdx.y * PC);
}

// Several independent products C_g = beta Cin_g + alpha A_g Q_g in one launch
// (blockIdx.z = g; tiles outside a product's shape return before any
// barrier).  Each tile is computed exactly as by a launch of its own.
__global__ __launch_bounds__(256, 4) void k_proj_grouped(ProjGroups gs, double alpha, double beta) {
  const ProjGroup& g = gs.g[blockIdx.z];
  const long row0 = (long)blockIdx.x * PR;
  const int col0 = blockIdx.y * PC;
  if (row0 >= g.nrows || col0 >= g.p || g.m <= 0) return;
  proj_tile(g.nrows, g.m, g.A, g.lda, g.Q, g.ldq, g.p, g.Cin, g.C, g.ldc, alpha, beta, row0, col0, g.C32);
}

// The projection tile on the float32 matrix cores for the first Gram-Schmidt
// sweep: A from its float32 copy, Q rounded to float32 as it is staged, A Q
// accumulated in float32, the update C = beta Cin + alpha (A Q) in float64.
__device__ __forceinline__ void proj_tile_f32(long nrows, int m, const float* __restrict__ A, long lda,
                                              const double* __restrict__ Q, int ldq, int p, const double* Cin,
                                              double* C, long ldc, double alpha, double beta, long row0, int col0) {
  __shared__ float As[PK][PR + 1];
  __shared__ float Qs[PK][PC + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  gram_f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = gram_f4{0.f, 0.f, 0.f, 0.f};
  const int ar = tid & 63, ak = tid >> 6;
  const int qk = tid & 31, qc = tid >> 5;
  const long grow = row0 + ar;
  const long growc = grow < nrows ? grow : nrows - 1;
  float ra[PK / 4], rq[PC / 8];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PK / 4; ++u) {
      const int k = k0 + ak + 4 * u;
      const float v = A[(long)(k < m ? k : m - 1) * lda + growc];
      ra[u] = v * ((k < m && grow < nrows) ? 1.f : 0.f);
    }
    const int kq = k0 + qk;
    const int kqc = kq < m ? kq : m - 1;
#pragma unroll
    for (int u = 0; u < PC / 8; ++u) {
      const int c = col0 + qc + 8 * u;
      const float v = (float)Q[(long)(c < p ? c : p - 1) * ldq + kqc];
      rq[u] = v * ((kq < m && c < p) ? 1.f : 0.f);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < m; k0 += PK) {
#pragma unroll
    for (int u = 0; u < PK / 4; ++u) As[ak + 4 * u][ar] = ra[u];
#pragma unroll
    for (int u = 0; u < PC / 8; ++u) Qs[qk][qc + 8 * u] = rq[u];
    __syncthreads();
    if (k0 + PK < m) fetch(k0 + PK);
    const int ci = lane & 15, ck = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < PK; kk += 4) {
      const float q0 = Qs[kk + ck][wc * 32 + ci], q1 = Qs[kk + ck][wc * 32 + 16 + ci];
      const float a0 = As[kk + ck][wr * 32 + ci], a1 = As[kk + ck][wr * 32 + 16 + ci];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(q0, a0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(q0, a1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(q1, a0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(q1, a1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  double old[2][2][4];
  if (beta != 0.0) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = col0 + wc * 32 + 16 * a + kF32Row(lane, v);
          const long r = row0 + wr * 32 + 16 * b + (lane & 15);
          old[a][b][v] = Cin[(long)(j < p ? j : p - 1) * ldc + (r < nrows ? r : nrows - 1)];
        }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = col0 + wc * 32 + 16 * a + kF32Row(lane, v);
        const long r = row0 + wr * 32 + 16 * b + (lane & 15);
        const double t = alpha * (double)acc[a][b][v];
        if (j < p && r < nrows) C[(long)j * ldc + r] = beta == 0.0 ? t : fma(beta, old[a][b][v], t);
      }
}

__global__ __launch_bounds__(256, 4) void k_proj_grouped_f32(ProjGroups gs, double alpha, double beta) {
  const ProjGroup& g = gs.g[blockIdx.z];
  const long row0 = (long)blockIdx.x * PR;
  const int col0 = blockIdx.y * PC;
  if (row0 >= g.nrows || col0 >= g.p || g.m <= 0) return;
  proj_tile_f32(g.nrows, g.m, g.A32, g.lda, g.Q, g.ldq, g.p, g.Cin, g.C, g.ldc, alpha, beta, row0, col0);
}

void proj_grouped(hipStream_t st, int count, const ProjGroup* groups, double alpha, double beta) {
  for (int g0 = 0; g0 < count; g0 += kProjGroupMax) {
    ProjGroups gs{};
    const int n = std::min(kProjGroupMax, count - g0);
    long rmax = 0;
    int pmax = 0;
    for (int i = 0; i < n; ++i) {
      gs.g[i] = groups[g0 + i];
      rmax = std::max(rmax, gs.g[i].nrows);
      pmax = std::max(pmax, gs.g[i].p);
    }
    if (rmax <= 0 || pmax <= 0) continue;
    dim3 grd((rmax + PR - 1) / PR, (pmax + PC - 1) / PC, n);
    if (gs.g[0].A32)  // a launch is all float32 or all float64 (the caller groups them)
      hipLaunchKernelGGL(k_proj_grouped_f32, grd, dim3(256), 0, st, gs, alpha, beta);
    else
      hipLaunchKernelGGL(k_proj_grouped, grd, dim3(256), 0, st, gs, alpha, beta);
  }
}

// A_g[i, i] += v (i < n_g) and dst_g = src_g (len_g doubles) for several
// matrices in one launch (blockIdx.y = g)
__global__ void k_add_diag_grouped(DiagGroups gs, double v) {
  const int g = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < gs.n[g]) gs.A[g][(long)i * gs.lda[g] + i] += v;
}
void add_diag_grouped(hipStream_t st, const DiagGroups& gs, int count, double v) {
  int nmax = 0;
  for (int g = 0; g < count; ++g) nmax = std::max(nmax, gs.n[g]);
  if (nmax <= 0 || count <= 0) return;
  hipLaunchKernelGGL(k_add_diag_grouped, dim3((nmax + 255) / 256, count), dim3(256), 0, st, gs, v);
}
__global__ void k_copy_grouped(CopyGroups gs) {
  const int g = blockIdx.y;
  const long n = gs.len[g];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    gs.dst[g][i] = gs.src[g][i];
}
void copy_grouped(hipStream_t st, const CopyGroups& gs, int count) {
  long nmax = 0;
  for (int g = 0; g < count; ++g) nmax = std::max(nmax, gs.len[g]);
  if (nmax <= 0 || count <= 0) return;
  const long blocks = std::min<long>((nmax + 255) / 256, 1024);
  hipLaunchKernelGGL(k_copy_grouped, dim3((unsigned)blocks, count), dim3(256), 0, st, gs);
}

template <>
void proj<double>(hipStream_t st, long nrows, int m, const double* A, long lda, const double* Q, int ldq, int p,
                  double* C, long ldc, double beta) {
  if (p <= 0) return;
  if (m <= 0) {
    if (beta == 0.0) axpby<double>(st, nrows, p, C, ldc, C, ldc, 0.0, 0.0);
    return;
  }
  dim3 grd((nrows + PR - 1) / PR, (p + PC - 1) / PC);
  hipLaunchKernelGGL(k_proj_mfma, grd, dim3(256), 0, st, nrows, m, A, lda, Q, ldq, p, C, ldc, beta);
}
template void proj<float>(hipStream_t, long, int, const float*, long, const double*, int, int, float*, long, double);

// ---------------------------------------------------------------------------
// Elementwise helpers
// ---------------------------------------------------------------------------
// Y[:,c] = s * mask .* X[:,c]
template <typename T>
__global__ void k_mask_scale(long nx, int ncols, const T* __restrict__ X, long ldx, T* __restrict__ Y, long ldy,
                             const uint8_t* __restrict__ mask, double s) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (idx >= nx) return;
  Y[(long)c * ldy + idx] = mask[idx] ? (T)(s * (double)X[(long)c * ldx + idx]) : T(0);
}
template <typename T>
void mask_scale(hipStream_t st, long nx, int ncols, const T* X, long ldx, T* Y, long ldy, const uint8_t* mask,
                double s) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL((k_mask_scale<T>), dim3((nx + 255) / 256, ncols), dim3(256), 0, st, nx, ncols, X, ldx, Y, ldy,
                     mask, s);
}
template void mask_scale<double>(hipStream_t, long, int, const double*, long, double*, long, const uint8_t*, double);
template void mask_scale<float>(hipStream_t, long, int, const float*, long, float*, long, const uint8_t*, double);

// X[:,c] = w .* X[:,c] (a per-node weight applied to every column)
__global__ void k_scale_nodes(long nx, double* __restrict__ X, long ldx, const double* __restrict__ w) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long c = blockIdx.y;
  if (idx >= nx) return;
  X[c * ldx + idx] *= w[idx];
}
void scale_nodes(hipStream_t st, long nx, int ncols, double* X, long ldx, const double* w) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_scale_nodes, dim3((nx + 255) / 256, ncols), dim3(256), 0, st, nx, X, ldx, w);
}

// A[i, i] += v (i < n), and A[j, i] = A[i, j] for i < j: the upper triangle
// copied to the lower one (column-major, leading dimension lda)
__global__ void k_add_diag(int n, double* A, long lda, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[(long)i * lda + i] += v;
}
__global__ void k_symmetrize_upper(int n, double* A, long lda) {
  const int i = blockIdx.x * 16 + threadIdx.x, j = blockIdx.y * 16 + threadIdx.y;
  if (i < n && j < n && i > j) A[(long)j * lda + i] = A[(long)i * lda + j];
}
// out[i] = sum_j A[i + j lda] B[i + j ldb] for i < n, j < r: the row-wise
// dot products of two column-major n x r matrices.  A workgroup takes 64 rows;
// its 16 waves each sum one sixteenth of the j range (ascending), and the 16
// partial sums are combined in a fixed order, so every run rounds alike.
constexpr int RD_ROWS = 64, RD_SEG = 16;
__global__ __launch_bounds__(RD_ROWS * RD_SEG) void k_row_dot(int n, int r, const double* __restrict__ A, long lda,
                                                            const double* __restrict__ B, long ldb,
                                                            double* __restrict__ out) {
  __shared__ double red[RD_SEG][RD_ROWS + 1];
  const int tx = threadIdx.x % RD_ROWS, ty = threadIdx.x / RD_ROWS;
  const int i = blockIdx.x * RD_ROWS + tx;
  const int ic = i < n ? i : n - 1;
  const int seg = (r + RD_SEG - 1) / RD_SEG;
  const int j0 = ty * seg, j1 = min(r, j0 + seg);
  double acc = 0.0;
  for (int j = j0; j < j1; ++j) acc = fma(A[ic + (long)j * lda], B[ic + (long)j * ldb], acc);
  red[ty][tx] = acc;
  __syncthreads();
  if (ty == 0 && i < n) {
    double t = red[0][tx];
#pragma unroll
    for (int y = 1; y < RD_SEG; ++y) t += red[y][tx];
    out[i] = t;
  }
}
void row_dot(hipStream_t st, int n, int r, const double* A, long lda, const double* B, long ldb, double* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_row_dot, dim3((n + RD_ROWS - 1) / RD_ROWS), dim3(RD_ROWS * RD_SEG), 0, st, n, r, A, lda, B, ldb,
                     out);
}
void add_diag(hipStream_t st, int n, double* A, long lda, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_add_diag, dim3((n + 255) / 256), dim3(256), 0, st, n, A, lda, v);
}
void symmetrize_upper(hipStream_t st, int n, double* A, long lda) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_symmetrize_upper, dim3((n + 15) / 16, (n + 15) / 16), dim3(16, 16), 0, st, n, A, lda);
}

// Y = a X + b Y (column blocks)
template <typename T>
__global__ void k_axpby(long nx, const T* __restrict__ X, long ldx, T* __restrict__ Y, long ldy, double a, double b) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (idx >= nx) return;
  T* y = Y + (long)c * ldy + idx;
  *y = (T)(a * (double)X[(long)c * ldx + idx] + (b == 0.0 ? 0.0 : b * (double)(*y)));
}
template <typename T>
void axpby(hipStream_t st, long nx, int ncols, const T* X, long ldx, T* Y, long ldy, double a, double b) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL((k_axpby<T>), dim3((nx + 255) / 256, ncols), dim3(256), 0, st, nx, X, ldx, Y, ldy, a, b);
}
template void axpby<double>(hipStream_t, long, int, const double*, long, double*, long, double, double);
template void axpby<float>(hipStream_t, long, int, const float*, long, float*, long, double, double);

// conversions
__global__ void k_d2f(long n, const double* __restrict__ x, float* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ void k_f2d(long n, const float* __restrict__ x, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}
void d2f(hipStream_t st, long n, const double* x, float* y) {
  if (n > 0) hipLaunchKernelGGL(k_d2f, dim3((n + 255) / 256), dim3(256), 0, st, n, x, y);
}
void f2d(hipStream_t st, long n, const float* x, double* y) {
  if (n > 0) hipLaunchKernelGGL(k_f2d, dim3((n + 255) / 256), dim3(256), 0, st, n, x, y);
}

// ---------------------------------------------------------------------------
// Posterior variance: D[x, t] = dprior[x] - sum_i d_i (sum_c A_i[x, c] B_i[t, c])^2
// The eigenvector factors are packed: A (nx x R) with all vectors' spatial
// columns side by side, Bt (R x nt) the temporal factors transposed, and
// seg[i] .. seg[i+1] the column range of vector i.  Each thread owns one
// node x and a run of time steps; the small factors of a time tile are staged
// in LDS.
// ---------------------------------------------------------------------------
constexpr int VT = 16;  // time steps per thread

__global__ __launch_bounds__(256) void k_post_var(long nx, int nt, int k, const int* __restrict__ seg,
                                                  const double* __restrict__ dcoef, const double* __restrict__ A,
                                                  long lda, const double* __restrict__ Bt, int R,
                                                  const double* __restrict__ dprior, double* __restrict__ D,
                                                  long ldd) {
  const long x = (long)blockIdx.x * 256 + threadIdx.x;
  const int t0 = blockIdx.y * VT;
  __shared__ double Bsh[64][VT];
  double acc[VT];
#pragma unroll
  for (int t = 0; t < VT; ++t) acc[t] = 0.0;
  for (int i = 0; i < k; ++i) {
    const int c0 = seg[i], c1 = seg[i + 1];
    const double di = dcoef[i];
    double v[VT];
#pragma unroll
    for (int t = 0; t < VT; ++t) v[t] = 0.0;
    for (int cb = c0; cb < c1; cb += 64) {
      const int cn = min(64, c1 - cb);
      __syncthreads();
      for (int p = threadIdx.x; p < 64 * VT; p += 256) {
        const int cc = p / VT, tt = p % VT;
        Bsh[cc][tt] = (cc < cn && t0 + tt < nt) ? Bt[(long)(t0 + tt) * R + cb + cc] : 0.0;
      }
      __syncthreads();
      if (x < nx) {
        for (int cc = 0; cc < cn; ++cc) {
          const double a = A[(long)(cb + cc) * lda + x];
#pragma unroll
          for (int t = 0; t < VT; ++t) v[t] += a * Bsh[cc][t];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < VT; ++t) acc[t] += di * v[t] * v[t];
  }
  if (x < nx) {
    const double dp = dprior[x];
#pragma unroll
    for (int t = 0; t < VT; ++t)
      if (t0 + t < nt) D[(long)(t0 + t) * ldd + x] = dp - acc[t];
  }
}

void post_variance(hipStream_t st, long nx, int nt, int k, const int* seg, const double* dcoef, const double* A,
                   long lda, const double* Bt, int R, const double* dprior, double* D, long ldd) {
  dim3 grd((nx + 255) / 256, (nt + VT - 1) / VT);
  hipLaunchKernelGGL(k_post_var, grd, dim3(256), 0, st, nx, nt, k, seg, dcoef, A, lda, Bt, R, dprior, D, ldd);
}

// ---------------------------------------------------------------------------
// Convection-diffusion with the wind along x2 (Sec. 6.3): the SUPG operator
// on the tensor mesh is L = D K1 (x) M1 + nu M1 (x) K1 + w C1 (x) M1 (first
// factor along x2, D = nu + delta w^2), so a L + b M is symmetric along x1
// and its x1 factors are diagonal in the sine basis.  Solves transform along
// x1, solve one tridiagonal system along x2 per sine mode, and transform
// back (fast diagonalization).
// ---------------------------------------------------------------------------

// Y[:,c] = sum over the 3 x 3 block of W_c[d2][|d1|] x(i + d1, j + d2): six
// weights per column (centre and side of the rows j - 1, j, j + 1), since
// the operator is symmetric along x1 but not along x2.
template <int S>
__global__ __launch_bounds__(256) void k_cd_stencil(int n, const double* __restrict__ X, long ldx,
                                                    double* __restrict__ Y, long ldy, const double* __restrict__ W,
                                                    int wstride) {
  const int col = blockIdx.z;
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j0 = (blockIdx.y * 4 + threadIdx.y) * S;
  if (i >= n || j0 >= n) return;
  const double* w = W + (long)wstride * col;
  const double c0 = w[0], s0 = w[1], c1 = w[2], s1 = w[3], c2 = w[4], s2 = w[5];
  const double* x = X + (long)col * ldx;
  double* y = Y + (long)col * ldy;
  const bool hl = i > 0, hr = i + 1 < n;
  auto row = [&](int j, double& m, double& lr) {
    if (j < 0 || j >= n) {
      m = lr = 0.0;
      return;
    }
    const double* p = x + (long)j * n + i;
    m = p[0];
    lr = (hl ? p[-1] : 0.0) + (hr ? p[1] : 0.0);
  };
  double m0, e0, m1, e1, m2, e2;
  row(j0 - 1, m0, e0);
  row(j0, m1, e1);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = j0 + s;
    if (j >= n) break;
    row(j + 1, m2, e2);
    y[(long)j * n + i] = (c0 * m0 + s0 * e0) + (c1 * m1 + s1 * e1) + (c2 * m2 + s2 * e2);
    m0 = m1; e0 = e1;
    m1 = m2; e1 = e2;
  }
}

void cd_stencil(hipStream_t st, int n, int ncols, const double* X, long ldx, double* Y, long ldy, const double* W,
                int wstride) {
  if (ncols <= 0 || n <= 0) return;
  constexpr int S = 8;
  dim3 blk(64, 4), grd((n + 63) / 64, (n + 4 * S - 1) / (4 * S), ncols);
  hipLaunchKernelGGL(k_cd_stencil<S>, grd, blk, 0, st, n, X, ldx, Y, ldy, W, wstride);
}

// Sine transform along x1 of every mesh row of ncols columns: Y[l][j] =
// sum_i X[l][i] S[i][j] for the lines l = (column c, row i2) at c ld + i2 n,
// with S the n x n orthonormal sine matrix (symmetric, its own inverse).  A
// dense product on the float64 matrix cores: 64 lines x 64 modes per
// workgroup, the k dimension staged through two LDS buffers of 16 (one
// barrier per stage).  The mode tiles of one line tile run on one XCD,
// dispatched one after another (workgroups 8 apart), so that its lines come
// from that XCD's L2 after the first.  X and Y must not overlap.
constexpr int SX_L = 64, SX_M = 64, SX_K = 16;

__global__ __launch_bounds__(256, 4) void k_sine_x1(int n, long nlines, int nmt, const double* __restrict__ X,
                                                     long ldx, double* __restrict__ Y, long ldy,
                                                     const double* __restrict__ S) {
  __shared__ double As[2][SX_K][SX_L + 1];
  __shared__ double Ss[2][SX_K][SX_M + 1];
  const long w = blockIdx.x, g = gridDim.x;
  const long full = g & ~7L;
  const long lw = w < full ? (w & 7) * (full >> 3) + (w >> 3) : w;
  const long l0 = (lw / nmt) * SX_L;
  const int j0 = (int)(lw % nmt) * SX_M;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  // A loader: k = tid & 15 of the lines (tid >> 4) + 16 u (16 lanes read 16
  // consecutive doubles of one line); S loader: mode tid & 63 of the k rows
  // (tid >> 6) + 4 u
  const int ak = tid & 15, al = tid >> 4;
  const int sj = tid & 63, sk = tid >> 6;
  const double* arow[4];
  double aval[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long l = l0 + al + 16 * u;
    const long lc = l < nlines ? l : nlines - 1;
    arow[u] = X + (lc / n) * ldx + (lc % n) * (long)n;
    aval[u] = l < nlines ? 1.0 : 0.0;
  }
  const int jj = j0 + sj;
  const int jjc = jj < n ? jj : n - 1;
  const double sval = jj < n ? 1.0 : 0.0;
  double ra[4], rs[4];
  auto fetch = [&](int k0) {
    const int k = k0 + ak;
    const int kc = k < n ? k : n - 1;
    const double kv = k < n ? 1.0 : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) ra[u] = arow[u][kc] * (aval[u] * kv);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ks = k0 + sk + 4 * u;
      const int ksc = ks < n ? ks : n - 1;
      rs[u] = S[(long)ksc * n + jjc] * (ks < n ? sval : 0.0);
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) As[buf][ak][al + 16 * u] = ra[u];
#pragma unroll
    for (int u = 0; u < 4; ++u) Ss[buf][sk + 4 * u][sj] = rs[u];
  };
  gram_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = gram_d4{0.0, 0.0, 0.0, 0.0};
  const int ci = lane & 15, ck = lane >> 4;
  const int nst = (n + SX_K - 1) / SX_K;
  fetch(0);
  stage(0);
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const int cb = s & 1;
    if (s + 1 < nst) fetch((s + 1) * SX_K);
#pragma unroll
    for (int kk = 0; kk < SX_K; kk += 4) {
      const double a0 = As[cb][kk + ck][wr * 32 + ci], a1 = As[cb][kk + ck][wr * 32 + 16 + ci];
      const double b0 = Ss[cb][kk + ck][wc * 32 + ci], b1 = Ss[cb][kk + ck][wc * 32 + 16 + ci];
      // first operand: lines, second: modes (the result's lane & 15 index,
      // contiguous in Y)
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (s + 1 < nst) stage(cb ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long l = l0 + wr * 32 + 16 * a + (lane >> 4) + 4 * v;
        const int j = j0 + wc * 32 + 16 * b + (lane & 15);
        if (l < nlines && j < n) Y[(l / n) * ldy + (l % n) * (long)n + j] = acc[a][b][v];
      }
}

void sine_x1(hipStream_t st, int n, int ncols, const double* X, long ldx, double* Y, long ldy, const double* S) {
  if (ncols <= 0 || n <= 0) return;
  const long nlines = (long)ncols * n;
  const int nmt = (n + SX_M - 1) / SX_M;
  const long nwg = (nlines + SX_L - 1) / SX_L * nmt;
  hipLaunchKernelGGL(k_sine_x1, dim3((unsigned)nwg), dim3(256), 0, st, n, nlines, nmt, X, ldx, Y, ldy, S);
}

// One tridiagonal system along x2 per (column c, sine mode j), solved in
// place in R by elimination without pivoting (the systems are strictly
// diagonally dominant: the streamwise part D K1 + s w C1 has non-positive
// off-diagonals and zero row sums when D >= h |w| / 2, which the Peclet rule
// gives, and the mass part adds a strict margin).  Mode j of column c with
// shift (a, b) = ab[2c..]: alpha = a mu_j, g = a nu kappa_j + b mu_j,
//   sub = -alpha (D/h + s w/2) + g h/6, diag = 2 alpha D/h + 4 g h/6,
//   sup = -alpha (D/h - s w/2) + g h/6.
// CP (same layout as R) receives the eliminated super-diagonal.  One thread
// per system, consecutive threads on consecutive modes (one contiguous row
// segment per step); loads run a chunk ahead of the arithmetic.
constexpr int TD_U = 8;

__global__ __launch_bounds__(256) void k_tridiag_x2(int n, long nsys, double* __restrict__ R, long ldr,
                                                    double* __restrict__ CP, long ldc,
                                                    const double* __restrict__ ab, const double* __restrict__ mu,
                                                    const double* __restrict__ kap, CdCoef k) {
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  if (g >= nsys) return;
  const int c = (int)(g / n), j = (int)(g % n);
  const double a = ab[2 * c], b = ab[2 * c + 1];
  const double al = a * mu[j], gm = a * k.nu * kap[j] + b * mu[j];
  const double sub = -al * (k.Dh + k.sw2) + gm * k.h6;
  const double dia = 2.0 * al * k.Dh + 4.0 * gm * k.h6;
  const double sup = -al * (k.Dh - k.sw2) + gm * k.h6;
  double* r = R + (long)c * ldr + j;
  double* cp = CP + (long)c * ldc + j;
  const long sn = n;
  // forward elimination: c'_i = sup / (diag - sub c'_{i-1}),
  // d'_i = (r_i - sub d'_{i-1}) / (diag - sub c'_{i-1})
  double cur[TD_U], nxt[TD_U];
#pragma unroll
  for (int u = 0; u < TD_U; ++u) cur[u] = r[(long)(u < n ? u : n - 1) * sn];
  double cprev = 0.0, dprev = 0.0;
  for (int i0 = 0; i0 < n; i0 += TD_U) {
#pragma unroll
    for (int u = 0; u < TD_U; ++u) {
      const int i = i0 + TD_U + u;
      nxt[u] = r[(long)(i < n ? i : n - 1) * sn];
    }
#pragma unroll
    for (int u = 0; u < TD_U; ++u) {
      const int i = i0 + u;
      if (i < n) {
        const double m = 1.0 / (dia - sub * cprev);
        cprev = sup * m;
        dprev = (cur[u] - sub * dprev) * m;
        cp[(long)i * sn] = cprev;
        r[(long)i * sn] = dprev;
      }
    }
#pragma unroll
    for (int u = 0; u < TD_U; ++u) cur[u] = nxt[u];
  }
  // back substitution z_i = d'_i - c'_i z_{i+1} (z_{n-1} = d'_{n-1} is in
  // place), chunks of rows below i loaded ahead
  double z = dprev;
  double dc[TD_U], cc[TD_U], dn[TD_U], cn[TD_U];
  auto load = [&](int top, double* dd, double* cv) {
#pragma unroll
    for (int u = 0; u < TD_U; ++u) {
      const int i = top - u;
      const long ic = (long)(i >= 0 ? i : 0) * sn;
      dd[u] = r[ic];
      cv[u] = cp[ic];
    }
  };
  load(n - 2, dc, cc);
  for (int top = n - 2; top >= 0; top -= TD_U) {
    load(top - TD_U, dn, cn);
#pragma unroll
    for (int u = 0; u < TD_U; ++u) {
      const int i = top - u;
      if (i >= 0) {
        z = dc[u] - cc[u] * z;
        r[(long)i * sn] = z;
      }
    }
#pragma unroll
    for (int u = 0; u < TD_U; ++u) {
      dc[u] = dn[u];
      cc[u] = cn[u];
    }
  }
}

void tridiag_x2(hipStream_t st, int n, int ncols, double* R, long ldr, double* CP, long ldc, const double* ab,
                const double* mu, const double* kap, const CdCoef& k) {
  if (ncols <= 0 || n <= 0) return;
  const long nsys = (long)ncols * n;
  hipLaunchKernelGGL(k_tridiag_x2, dim3((unsigned)((nsys + 255) / 256)), dim3(256), 0, st, n, nsys, R, ldr, CP, ldc,
                     ab, mu, kap, k);
}

}  // namespace lrp
