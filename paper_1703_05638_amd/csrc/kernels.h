// Launch wrappers for the device kernels (all asynchronous on the given stream).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <stdint.h>

namespace lrp {

// Y[:,c] = w0*centre + w1*edges + w2*corners of X[:,c] + w3*Z[:,c] with
// (w0..w3) = W[wstride*c .. +3] (W: device doubles; wstride 4: one set per
// column, 0: one set for all; Z may be null).
template <typename T>
void stencil(hipStream_t st, int n, int ncols, const T* X, long ldx, T* Y, long ldy, const T* Z, long ldz,
             const double* W, int wstride = 4);

// Multigrid passes; P: device, kMgStride doubles per column:
// {wc, we, wk, 0, alpha_0, beta_0/wc, alpha_1, beta_1/wc, ...} (Chebyshev steps).
constexpr int kMgStride = 12;
constexpr int kMgMaxSteps = 4;
template <typename T>
void mg_smooth_step(hipStream_t st, int n, int ncols, const T* Xc, const T* Xp, T* Xo, const T* B, long ld,
                    const double* P, int step);
template <typename T>
void mg_resid_restrict(hipStream_t st, int n, int ncols, const T* X, const T* B, long ld, T* Bc, long ldc,
                       const double* P);
template <typename T>
void mg_prolong_add(hipStream_t st, int n, int ncols, const T* E, long ldc, const T* Xi, T* Xo, long ld);
// Level-fused passes for n <= kMgFusedMaxN with kMgFusedNu smoother steps:
// down: X = smoothing from zero for A X = B, Bc = P^T (B - A X);
// up: Xo = smoothing from Xi + P E (acc: Xo += that).  Xo must not alias Xi.
constexpr int kMgFusedNu = 3;
constexpr int kMgFusedMaxN = 1023;
template <typename T>
void mg_down(hipStream_t st, int n, int ncols, const T* B, long ld, T* X, T* Bc, long ldc, const double* P);
template <typename T>
void mg_up(hipStream_t st, int n, int ncols, const T* Xi, const T* E, long ldc, const T* B, long ld, T* Xo,
           const double* P, bool acc = false);
template <typename T>
void mg_coarse_lds(hipStream_t st, int n0, int nlev, int ncols, const T* B, long ldb, T* X, long ldx,
                   const double* Pc, int nu1, int nu2);
constexpr int kCoarseLdsMaxN = 31;

int gram_chunks(long nrows, int m, int q);       // float instance (LDS kernel)
int gram_chunks_mfma(long nrows, int m, int q);  // double instance (FP64 MFMA kernel)
// Products of one launch: up to kProjGroupMax Gram products, projections,
// diagonal shifts or copies.
constexpr int kProjGroupMax = 8;
// One Gram product C = A^T B (A nrows x m, B nrows x q; C m x q with leading
// dimension ldc) and its partial-product scratch (gram_part_doubles()).
struct GramGroup {
  const double* A;
  const double* B;
  double* part;
  double* C;
  long lda, ldb, ldc;
  long rpc;    // rows per chunk, set by gram_mfma_partials
  int m, q;
  int nchunk;  // set by gram_mfma_partials
  // when set, A is read from this float32 copy instead (B still float64) and
  // the product runs on the float32 matrix cores with float32 accumulation
  // within a chunk (partial sums across chunks in float64)
  const float* A32 = nullptr;
  // when m2 > 0, the last m2 of the m columns of A are read from A2 (leading
  // dimension lda): C = [A | A2]^T B, rows m - m2 .. m - 1 from A2 (float64
  // products only)
  const double* A2 = nullptr;
  int m2 = 0;
};
// column sums of squares out_g[c] = sum_i C_g[i + c ld_g]^2 (i < rows_g,
// c < cols_g) for several small matrices in one launch, in a fixed order
struct ColGroup {
  const double* C;
  double* out;
  long ld;
  int rows, cols;
};
void col_sqnorms(hipStream_t st, int count, const ColGroup* groups);
// out[i] = c - c sum_j w[j] V[i + j ldv]^2 (i < nx, j < k): the posterior
// variance of the initial-condition problem from k eigenpairs, w = lam/(1+lam)
void ic_post_var(hipStream_t st, long nx, int k, const double* V, long ldv, const double* w, double c, double* out);
struct GramGroups {
  GramGroup g[kProjGroupMax];
  int nchunk_max;
};
struct SumGroup {
  const double* part;
  double* C;
  long ldc;
  int m, q, nchunk;
};
struct SumGroups {
  SumGroup g[kProjGroupMax];
};
// the two stages of gram<double> for several products: per-chunk partial
// products on the matrix cores (each product chunked by its own shape, so its
// result does not depend on the others), then their sums into each C
void gram_mfma_partials(hipStream_t st, long nrows, int count, GramGroup* groups);
void sum_partials_grouped(hipStream_t st, int count, const GramGroup* groups);
long gram_part_doubles(long nrows, int m, int q);
// tile height class of a Gram product with m columns of A: 64 gram_bm(m) rows
int gram_bm(int m);
// tile width class of a Gram product with q columns of B: 64 gram_bq(q) columns
int gram_bq(int q);
void sum_partials(hipStream_t st, int nchunk, long count, const double* part, double* C);
// C (device, m x q, double) = A^T B; part: device scratch of gram_chunks()*m*q
// doubles (gram_chunks_mfma() for T = double).
template <typename T>
void gram(hipStream_t st, long nrows, int m, const T* A, long lda, int q, const T* B, long ldb, double* C,
          double* part);
template <>
void gram<double>(hipStream_t st, long nrows, int m, const double* A, long lda, int q, const double* B, long ldb,
                  double* C, double* part);
// C = beta*C + A Q  (Q: device m x p double, leading dim ldq; C must not overlap A)
template <typename T>
void proj(hipStream_t st, long nrows, int m, const T* A, long lda, const double* Q, int ldq, int p, T* C, long ldc,
          double beta);
template <>
void proj<double>(hipStream_t st, long nrows, int m, const double* A, long lda, const double* Q, int ldq, int p,
                  double* C, long ldc, double beta);

// Several independent products C_g = beta Cin_g + alpha A_g Q_g (A_g nrows x m,
// Q_g m x p, C_g nrows x p, Cin_g may be C_g) on the matrix cores, up to
// kProjGroupMax per launch; each product is computed exactly as by proj.
struct ProjGroup {
  const double* A;
  const double* Q;
  const double* Cin;
  double* C;
  long lda, ldc, nrows;
  int ldq, m, p;
  // when set, A is read from this float32 copy and A Q runs on the float32
  // matrix cores (Q rounded to float32); the update of C stays float64
  const float* A32 = nullptr;
  // when set (float64 products), C is also written rounded to float32 here
  // (leading dimension ldc)
  float* C32 = nullptr;
};
struct ProjGroups {
  ProjGroup g[kProjGroupMax];
};
void proj_grouped(hipStream_t st, int count, const ProjGroup* groups, double alpha, double beta);
// A_g[i, i] += v for i < n_g; dst_g = src_g (len_g doubles); count <= kProjGroupMax
struct DiagGroups {
  double* A[kProjGroupMax];
  long lda[kProjGroupMax];
  int n[kProjGroupMax];
};
void add_diag_grouped(hipStream_t st, const DiagGroups& gs, int count, double v);
struct CopyGroups {
  const double* src[kProjGroupMax];
  double* dst[kProjGroupMax];
  long len[kProjGroupMax];
};
void copy_grouped(hipStream_t st, const CopyGroups& gs, int count);

template <typename T>
void mask_scale(hipStream_t st, long nx, int ncols, const T* X, long ldx, T* Y, long ldy, const uint8_t* mask,
                double s);
template <typename T>
void axpby(hipStream_t st, long nx, int ncols, const T* X, long ldx, T* Y, long ldy, double a, double b);
void scale_nodes(hipStream_t st, long nx, int ncols, double* X, long ldx, const double* w);
// out[i] = sum_j A[i + j lda] B[i + j ldb], i < n, j < r (row-wise dot products)
void row_dot(hipStream_t st, int n, int r, const double* A, long lda, const double* B, long ldb, double* out);
void add_diag(hipStream_t st, int n, double* A, long lda, double v);
void symmetrize_upper(hipStream_t st, int n, double* A, long lda);
void d2f(hipStream_t st, long n, const double* x, float* y);
void f2d(hipStream_t st, long n, const float* x, double* y);

void post_variance(hipStream_t st, long nx, int nt, int k, const int* seg, const double* dcoef, const double* A,
                   long lda, const double* Bt, int R, const double* dprior, double* D, long ldd);

// Static partial-product scratch of the Gram products for callers that cannot
// allocate: kGramScratchDoubles doubles per device, held until the process
// ends.  gram_scratch_setup() resolves the array's address on the current
// device (once per device, later calls return the cached address; nullptr on
// a HIP error); gram_scratch_device() returns it for the current device, or
// nullptr before setup there.
// Stencil strip-height autotuner: switch, and its table as text lines.
void set_stencil_autotune(bool on);
std::string stencil_autotune_report();
constexpr long kGramScratchDoubles = long(8) << 20;  // 64 MiB
double* gram_scratch_setup();
double* gram_scratch_device();

// Convection-diffusion with the wind along x2 (tensor mesh, x1 fastest).
// Y[:,c] = the 9-point stencil with weights W[wstride c .. + 5] = (centre,
// side) of the rows j - 1, j, j + 1 (symmetric along x1).
void cd_stencil(hipStream_t st, int n, int ncols, const double* X, long ldx, double* Y, long ldy, const double* W,
                int wstride);
// Y = X transformed along x1 by the n x n sine matrix S (device, symmetric,
// orthonormal) for every mesh row of ncols columns; X and Y distinct.
void sine_x1(hipStream_t st, int n, int ncols, const double* X, long ldx, double* Y, long ldy, const double* S);
// scalars of the x2 systems: D/h, s w / 2 (s = +1 for L, -1 for L^T), nu, h/6
struct CdCoef {
  double Dh, sw2, nu, h6;
};
// In place along x2 for every (column, sine mode): the tridiagonal system of
// mode j of column c with shift (a, b) = ab[2c..] (device), sine-mode mass
// and stiffness eigenvalues mu, kap (device, n); CP: scratch of R's shape.
void tridiag_x2(hipStream_t st, int n, int ncols, double* R, long ldr, double* CP, long ldc, const double* ab,
                const double* mu, const double* kap, const CdCoef& k);

}  // namespace lrp
