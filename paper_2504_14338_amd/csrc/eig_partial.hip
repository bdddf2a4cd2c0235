// Partial eigendecomposition for a prescribed r (arXiv:2504.14338, Sec. 3.4:
// only the r leading eigenpairs of D enter Qhat = Lambda_r^{1/2} U_r^T and
// T_r, Eqs. (6)-(8)).  Block subspace iteration with Rayleigh-Ritz
// (Rutishauser 1970; Saad, "Numerical Methods for Large Eigenvalue
// Problems", Sec. 5.2), all in float64 on the GPU:
//
//   X (k x p, p = block size > r)  <-  orthonormal basis of D X
//
// where the orthonormalization is shifted Cholesky QR (Fukaya, Kannan,
// Nakatsukasa, Yamamoto, Yanagisawa 2020): G = Y^T Y + sigma I = L L^T,
// X = Y L^{-T}, sigma = 11 (k p + p (p + 1)) u trace(Y^T Y), which stays
// stable however ill-conditioned Y is; before each Rayleigh-Ritz step two
// more, unshifted passes (their shifted CholeskyQR3) make X orthonormal to
// working precision.  Rayleigh-
// Ritz: H = X^T D X (p x p) is diagonalized by the library's dense
// eigensolver and X <- X W (Ritz vectors in descending order of Ritz value).
//
// Iteration count: the error of the j-th Ritz vector decays like
// (lambda_{p+1} / lambda_j)^m.  After m0 iterations a first Rayleigh-Ritz
// step computes the Ritz values only: rho = theta_p / theta_r bounds that
// rate for all j <= r, and the iteration continues until rho^m <= 1e-17,
// plus two extra steps, then ends with a second Rayleigh-Ritz step that
// computes the r leading Ritz vectors.  The shift damps directions whose
// share of the block is near its relative size (see the driver), which
// decides whether two products D (D X) may share one orthonormalization and
// whether the r-th direction survives the iteration at all.  When it does
// not, when rho is too close to 1 (more than kMaxIter iterations), or when r
// is too large for the block size, the full eigensolver runs instead.
//
// Products: D X and X^T (D X) use the cross-Gram kernel (D is symmetric, so
// D X = D^T X), Y^T Y the Gram kernel, X L^{-T} and X W the row-GEMM tile
// kernel; the p x p Cholesky factor and its inverse come from one
// workgroup with the packed triangles in LDS.
#include <cmath>
#include <utility>
#include <vector>

#include "common.hpp"

namespace dopinf {
int cross_gram_internal(hipStream_t st, const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n,
                        int64_t mx, int64_t my, double* C, int64_t ldc, void* ws, size_t ws_bytes,
                        const double* mean, const double* scale, int nvars, const int64_t* var_rows_h);
size_t cross_gram_workspace_internal(int64_t n, int64_t mx, int64_t my);
int gram_f64_internal(hipStream_t st, const double* X, int64_t n, int64_t m, int64_t ldx, const double* mean,
                      const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd, void* ws,
                      size_t ws_bytes);
size_t gram_f64_workspace_internal(int64_t n, int64_t m, int nvars);
int row_gemm_f64(hipStream_t st, const double* A, int64_t lda, int64_t m, int64_t K, const double* B, int64_t ldb,
                 int64_t ncol, double* C, int64_t ldc);
size_t eig_vectors_workspace(int64_t k, int r);
int eig_vectors_internal(hipStream_t st, const double* D, int64_t k, int64_t ldd, int r, double* lambda, int* info,
                         void* ws, size_t ws_bytes, double** Z);
int eig_values_internal(hipStream_t st, const double* D, int64_t k, int64_t ldd, double* lambda, int* info, void* ws,
                        size_t ws_bytes);
int form_qhat_internal(hipStream_t st, const double* Z, int64_t k, int r, const double* lambda, double* Qhat,
                       int64_t ldqh, double* Tr, int64_t ldtr, int* info);

namespace {

constexpr int PMAX = 128;     // largest block size (packed triangles in LDS)
constexpr int kM0 = 4;        // iterations before the first Rayleigh-Ritz step
constexpr int kMaxIter = 80;  // beyond this the full eigensolver is used
constexpr int CT = 1024;      // threads of the Cholesky workgroup

int block_size(int64_t k, int r) {
  int p = std::max(r + 16, 2 * r);
  p = (p + 15) / 16 * 16;
  if (p > PMAX) p = PMAX;
  if (p >= k) p = int(k) - 1;
  return p;
}

bool partial_applies(int64_t k, int r) {
  const int p = block_size(k, r);
  return k >= 64 && p >= r + 8;
}

// SplitMix64 (Steele, Lea, Flood 2014) of a counter, mapped to [-1, 1)
__device__ __forceinline__ double splitmix_unit(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return double(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(256) void init_block_kernel(double* X, int64_t k, int p) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e < k * p) X[e] = splitmix_unit(uint64_t(e));
}

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

// One workgroup: G + sigma I = Lt Dg Lt^T (G p x p symmetric, ld p; sigma =
// shift_coef * trace(G), 0 for plain Cholesky QR) by symmetric Gaussian
// elimination, so that L = Lt Dg^{1/2}, and Rinv = L^{-T} = Lt^{-T} Dg^{-1/2}
// (upper triangular, p x p, ld p, zeros below).  A non-positive or
// non-finite pivot sets *fail and leaves Rinv undefined.
//  * step j, one barrier: with the pivot a_jj and the multipliers
//    f_i = a_ij / a_jj (i > j), both final after step j - 1, the trailing
//    triangle is updated a_il -= f_i a_lj (j < l <= i), and the same row
//    operations applied to the identity give Z = Lt^{-1}: z_ic -= f_i z_jc
//    (c <= j), i.e. column-oriented forward substitution for all right-hand
//    sides at once.  Row i's i + 1 entries in the two packed triangles (LDS)
//    are split over 32 lanes; step j writes neither column j of A nor row j
//    of Z.
//  * Rinv[a][b] = z_ba / sqrt(a_bb) for b >= a.
__global__ __launch_bounds__(CT) void chol_inv_kernel(const double* __restrict__ G, int p, double shift_coef,
                                                      double* __restrict__ Rinv, int* fail) {
  extern __shared__ double lds[];
  double* A = lds;                    // packed lower triangle of the working matrix
  double* Z = lds + p * (p + 1) / 2;  // packed unit lower triangle of Lt^{-1}
  __shared__ double red[CT / 64];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int ty = tid >> 5, tx = tid & 31;  // 32 x 32 layout over (row, column)
  double tr = 0.0;
  for (int i = tid; i < p; i += CT) tr += G[int64_t(i) * p + i];
  tr = block_sum<CT>(tr, red);
  const double sigma = shift_coef * tr;
  for (int i = ty; i < p; i += CT / 32)
    for (int l = tx; l <= i; l += 32) {
      A[tri(i, l)] = G[int64_t(i) * p + l] + (i == l ? sigma : 0.0);
      Z[tri(i, l)] = (i == l) ? 1.0 : 0.0;
    }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    const double djj = A[tri(j, j)];
    const bool ok = (djj > 0.0) && isfinite(djj);
    if (tid == 0 && !ok) bad = 1;
    const double inv = ok ? 1.0 / djj : 0.0;
    for (int i = j + 1 + ty; i < p; i += CT / 32) {
      const double f = A[tri(i, j)] * inv;
      for (int c = tx; c <= i; c += 32) {
        if (c <= j)
          Z[tri(i, c)] -= f * Z[tri(j, c)];
        else
          A[tri(i, c)] -= f * A[tri(c, j)];
      }
    }
    __syncthreads();
  }
  for (int a = ty; a < p; a += CT / 32)
    for (int b = tx; b < p; b += 32) {
      double x = 0.0;
      if (b >= a) {
        const double dbb = A[tri(b, b)];
        x = Z[tri(b, a)] / sqrt(dbb > 0.0 ? dbb : 1.0);
      }
      Rinv[int64_t(a) * p + b] = x;
    }
  if (tid == 0 && bad) atomicExch(fail, 1);
}

// (H + H^T) / 2 in place (p x p)
__global__ __launch_bounds__(256) void symmetrize_kernel(double* H, int p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p * p) return;
  const int i = e / p, j = e % p;
  if (j < i) {
    const double v = 0.5 * (H[int64_t(i) * p + j] + H[int64_t(j) * p + i]);
    H[int64_t(i) * p + j] = v;
    H[int64_t(j) * p + i] = v;
  }
}

// Out (cols x rows, ld rows) = In^T for In rows x cols (ld ldin), first `cols` columns
__global__ __launch_bounds__(256) void transpose_kernel(const double* __restrict__ In, int64_t rows, int64_t cols,
                                                        int64_t ldin, double* __restrict__ Out) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t c = e / rows, r = e % rows;
  Out[e] = In[r * ldin + c];
}

__global__ void copy_vec_kernel(const double* __restrict__ a, double* __restrict__ b, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) b[i] = a[i];
}

__global__ void info_merge_kernel(const int* chol_fail, const int* eig_info, int* info) {
  if (threadIdx.x != 0) return;
  int v = *eig_info;
  if (*chol_fail && v == DOPINF_OK) v = DOPINF_E_NONFINITE;
  *info = v;
}

__global__ void zero_int_kernel(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

struct PartWs {
  double *X, *Y, *G, *Rinv, *H, *W, *theta, *Zf, *lam_full;
  int *fail, *einfo;
  void* cg;
  size_t cg_bytes;
  void* gw;
  size_t gw_bytes;
  void* ew;
  size_t ew_bytes;
};

PartWs carve_part(Carver& c, int64_t k, int r, int p) {
  PartWs w{};
  w.X = c.take<double>(size_t(k) * p);
  w.Y = c.take<double>(size_t(k) * p);
  w.G = c.take<double>(size_t(p) * p);
  w.Rinv = c.take<double>(size_t(p) * p);
  w.H = c.take<double>(size_t(p) * p);
  w.W = c.take<double>(size_t(p) * p);
  w.theta = c.take<double>(size_t(p));
  w.Zf = c.take<double>(size_t(r) * k);
  w.lam_full = c.take<double>(size_t(k));
  w.fail = c.take<int>(1);
  w.einfo = c.take<int>(1);
  w.cg_bytes = std::max(cross_gram_workspace_internal(k, k, p), cross_gram_workspace_internal(k, p, p));
  w.cg = c.take<char>(w.cg_bytes);
  w.gw_bytes = gram_f64_workspace_internal(k, p, 1);
  w.gw = c.take<char>(w.gw_bytes);
  w.ew_bytes = std::max(eig_vectors_workspace(p, p), eig_vectors_workspace(k, r));
  w.ew = c.take<char>(w.ew_bytes);
  return w;
}

size_t partial_workspace(int64_t k, int r) {
  Carver c(nullptr, 0);
  carve_part(c, k, r, block_size(k, r) > 0 ? block_size(k, r) : 1);
  return c.used;
}

// Xout <- orthonormal basis of span(Yin) by one Cholesky QR pass (shifted or
// not); Yin and Xout must differ
int cholqr(hipStream_t st, const PartWs& w, const double* Yin, double* Xout, int64_t k, int p, bool shifted) {
  int rc = gram_f64_internal(st, Yin, k, p, p, nullptr, nullptr, 0, nullptr, w.G, p, w.gw, w.gw_bytes);
  if (rc) return rc;
  const double u = 1.1102230246251565e-16;
  const double coef = shifted ? 11.0 * (double(k) * p + double(p) * (p + 1)) * u : 0.0;
  const size_t lds = size_t(p) * (p + 1) * sizeof(double);
  chol_inv_kernel<<<1, CT, lds, st>>>(w.G, p, coef, w.Rinv, w.fail);
  DOPINF_LAUNCHED();
  return row_gemm_f64(st, Yin, p, k, p, w.Rinv, p, p, Xout, p);
}

// D times the block: out = D in (D symmetric: the cross Gram D^T in)
int apply_d(hipStream_t st, const PartWs& w, const double* D, int64_t ldd, int64_t k, int p, const double* in,
            double* out) {
  return cross_gram_internal(st, D, ldd, in, p, k, k, p, out, p, w.cg, w.cg_bytes, nullptr, nullptr, 0, nullptr);
}

// subspace steps: X <- orth(D^m X), m = 1 or 2 (two products before one
// orthonormalization when the spread of the spectrum allows it)
int power_step(hipStream_t st, PartWs& w, const double* D, int64_t ldd, int64_t k, int p, int m) {
  int rc = apply_d(st, w, D, ldd, k, p, w.X, w.Y);
  if (rc) return rc;
  if (m == 2) {
    rc = apply_d(st, w, D, ldd, k, p, w.Y, w.X);
    if (rc) return rc;
    std::swap(w.X, w.Y);  // the product is in Y now
  }
  return cholqr(st, w, w.Y, w.X, k, p, true);
}

// X orthonormal to working precision (shifted CholeskyQR3: one shifted pass,
// two plain ones; the result ends in X), then H = X^T D X symmetrized
int project(hipStream_t st, PartWs& w, const double* D, int64_t ldd, int64_t k, int p) {
  int rc = cholqr(st, w, w.X, w.Y, k, p, true);
  if (!rc) rc = cholqr(st, w, w.Y, w.X, k, p, false);
  if (!rc) rc = cholqr(st, w, w.X, w.Y, k, p, false);
  if (rc) return rc;
  std::swap(w.X, w.Y);
  rc = apply_d(st, w, D, ldd, k, p, w.X, w.Y);  // Y = D X
  if (rc) return rc;
  rc = cross_gram_internal(st, w.X, p, w.Y, p, k, p, p, w.H, p, w.cg, w.cg_bytes, nullptr, nullptr, 0, nullptr);
  if (rc) return rc;
  symmetrize_kernel<<<(p * p + 255) / 256, 256, 0, st>>>(w.H, p);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

}  // namespace
}  // namespace dopinf

using namespace dopinf;

extern "C" size_t dopinf_reduce_topr_workspace(int64_t k, int r) {
  if (k <= 0 || r <= 0 || r > k) return 0;
  size_t full = dopinf_reduce_workspace(k, r) + size_t(k) * sizeof(double) + 512;
  if (!partial_applies(k, r)) return full;
  return std::max(full, partial_workspace(k, r));
}

extern "C" int dopinf_reduce_topr(void* stream, const double* D, int64_t k, int64_t ldd, int r, double* lambda,
                                  double* Tr, int64_t ldtr, double* Qhat, int64_t ldqh, int* info, int* iters_h,
                                  void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(D && lambda && Qhat && info, "D, lambda, Qhat and info must be non-NULL");
  DOPINF_REQUIRE(k >= 1 && k <= 65536 && ldd >= k && ldqh >= k, "need 1 <= k <= 65536, ldd >= k, ldqh >= k");
  DOPINF_REQUIRE(r >= 1 && r <= k, "need 1 <= r <= k");
  DOPINF_REQUIRE(!Tr || ldtr >= r, "ldtr must be >= r");
  const size_t need = dopinf_reduce_topr_workspace(k, r);
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (iters_h) *iters_h = 0;

  auto full_solver = [&]() -> int {
    // all eigenvalues into a k-vector of the workspace, the first r copied out
    Carver c(ws, ws_bytes);
    double* lam_all = c.take<double>(size_t(k));
    void* rws = c.take<char>(dopinf_reduce_workspace(k, r));
    int rc = dopinf_reduce(stream, D, k, ldd, r, 0.5, r, nullptr, lam_all, Tr, ldtr, Qhat, ldqh, info, rws,
                           dopinf_reduce_workspace(k, r));
    if (rc) return rc;
    copy_vec_kernel<<<1, 256, 0, st>>>(lam_all, lambda, r);
    DOPINF_LAUNCHED();
    return DOPINF_OK;
  };
  if (!partial_applies(k, r)) return full_solver();

  const int p = block_size(k, r);
  Carver c(ws, ws_bytes);
  PartWs w = carve_part(c, k, r, p);
  {
    const size_t lds = size_t(p) * (p + 1) * sizeof(double);
    if (lds > 65536)
      DOPINF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(chol_inv_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  }
  zero_int_kernel<<<1, 64, 0, st>>>(w.fail);
  DOPINF_LAUNCHED();
  init_block_kernel<<<unsigned((k * p + 255) / 256), 256, 0, st>>>(w.X, k, p);
  DOPINF_LAUNCHED();
  int rc = DOPINF_OK;
  for (int it = 0; it < kM0 && !rc; ++it) rc = power_step(st, w, D, ldd, k, p, 1);
  // first Rayleigh-Ritz step: the Ritz values only (they give the rate)
  if (!rc) rc = project(st, w, D, ldd, k, p);
  if (!rc) rc = eig_values_internal(st, w.H, p, p, w.theta, w.einfo, w.ew, w.ew_bytes);
  if (rc) return rc;
  // the convergence rate from the Ritz values (one host synchronization)
  std::vector<double> th(p);
  int flags[2] = {0, 0};
  DOPINF_HIP(hipMemcpyAsync(th.data(), w.theta, sizeof(double) * p, hipMemcpyDeviceToHost, st));
  DOPINF_HIP(hipMemcpyAsync(flags, w.fail, sizeof(int), hipMemcpyDeviceToHost, st));
  DOPINF_HIP(hipMemcpyAsync(flags + 1, w.einfo, sizeof(int), hipMemcpyDeviceToHost, st));
  DOPINF_HIP(hipStreamSynchronize(st));
  if (flags[0] || flags[1] != DOPINF_OK || !(th[r - 1] > 0.0) || !std::isfinite(th[0])) return full_solver();
  const double rho = std::max(th[p - 1], 0.0) / th[r - 1];
  int m_total = kM0 + 2;
  if (rho > 0.0) {
    if (rho >= 1.0) return full_solver();
    m_total = int(std::ceil(std::log(1e-17) / std::log(rho))) + 2;
  }
  if (m_total > kMaxIter) return full_solver();
  int m_more = std::max(m_total - kM0, 1);
  // The shift of the orthonormalization damps a direction whose share of
  // the block's norm, squared, is near sigma_rel = 11 (k p + p (p + 1)) u: a
  // product D^m X leaves the r-th direction a share (theta_r / theta_1)^m.
  // One product per orthonormalization needs that share squared far above
  // sigma_rel (else the full eigensolver runs); two products share one
  // orthonormalization only when the square of the two-product share is too.
  const double sig_rel = 11.0 * (double(k) * p + double(p) * (p + 1)) * 1.1102230246251565e-16;
  const double share = th[r - 1] / th[0];
  if (share * share < 1e2 * sig_rel) return full_solver();
  const bool pairs = share * share * share * share > 1e6 * sig_rel;
  int done = 0;
  while (done < m_more && !rc) {
    const int m = (pairs && m_more - done >= 2) ? 2 : 1;
    rc = power_step(st, w, D, ldd, k, p, m);
    done += m;
  }
  // final Rayleigh-Ritz step: the r leading Ritz pairs
  double* Z = nullptr;
  if (!rc) rc = project(st, w, D, ldd, k, p);
  if (!rc) rc = eig_vectors_internal(st, w.H, p, p, r, w.theta, w.einfo, w.ew, w.ew_bytes, &Z);
  if (rc) return rc;
  if (iters_h) *iters_h = kM0 + done;
  // W_r (p x r): column j = eigenvector j of H (row j of Z); U = X W_r (k x r
  // in Y, ld p); eigenvector rows Z_f (r x k) for the sign rule, Qhat and T_r
  transpose_kernel<<<unsigned((p * r + 255) / 256), 256, 0, st>>>(Z, r, p, p, w.W);
  DOPINF_LAUNCHED();
  rc = row_gemm_f64(st, w.X, p, k, p, w.W, r, r, w.Y, p);
  if (rc) return rc;
  transpose_kernel<<<unsigned((k * r + 255) / 256), 256, 0, st>>>(w.Y, k, r, p, w.Zf);
  DOPINF_LAUNCHED();
  info_merge_kernel<<<1, 64, 0, st>>>(w.fail, w.einfo, info);
  DOPINF_LAUNCHED();
  copy_vec_kernel<<<1, 256, 0, st>>>(w.theta, lambda, r);
  DOPINF_LAUNCHED();
  return form_qhat_internal(st, w.Zf, k, r, w.theta, Qhat, ldqh, Tr, ldtr, info);
}
