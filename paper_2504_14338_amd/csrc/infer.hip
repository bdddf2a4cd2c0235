// Step IV of dOpInf (arXiv:2504.14338, Sec. 3.5): the regularized operator
// inference problem of Eq. (12) on the data of Eq. (13), for one or many
// (r, beta1, beta2) candidates.
//
// Design:
//  * One data matrix E = [Qhat_1^T | quad(Qhat_1^T) | 1 | Qhat_2^T] is built
//    at the largest requested r and its Gram G_E = E^T E is formed by the
//    Step III Gram kernel.  For a smaller r, Dhat^T Dhat and Dhat^T Qhat_2^T
//    are index-submatrices of G_E (the same dot products), so one Gram serves
//    every reduced size.
//  * The normal matrix is factored in the permuted column order
//    [quadratic (s) | linear (r), constant (1)].  Its leading s x s block
//    G_qq + beta2 I depends on beta2 only, so its Cholesky factor L, the
//    solves [W | y] = L^{-1} [G_ql | B_q] and [P | Z] = L^{-T} [W | y], and
//    the products W^T [W | y] are computed once per (r, beta2).  Each pair
//    then factors the small Schur complement
//       S = G_ll + beta1 I - W^T W           ((r+1) x (r+1))
//    solves S X_l = B_l - W^T y and recovers X_q = Z - P X_l.  This is
//    Cholesky factorization of the same matrix under a symmetric permutation.
//  * The s x s factorization is blocked right-looking (64-wide panels): a
//    diagonal-block kernel also inverts its 64 x 64 triangle, a panel kernel
//    solves the rows below, and the trailing update runs on FP64 MFMA tiles.
//    Triangular solves then reduce to products with the stored diagonal
//    inverses.
#include <vector>

#include "common.hpp"

namespace dopinf {
int gram_f64_internal(hipStream_t st, const double* X, int64_t n, int64_t m, int64_t ldx, const double* mean,
                      const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd, void* ws,
                      size_t ws_bytes);
size_t gram_f64_workspace_internal(int64_t n, int64_t m, int nvars);
int cross_gram_internal(hipStream_t st, const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n,
                        int64_t mx, int64_t my, double* C, int64_t ldc, void* ws, size_t ws_bytes,
                        const double* mean, const double* scale, int nvars, const int64_t* var_rows_h);
size_t cross_gram_workspace_internal(int64_t n, int64_t mx, int64_t my);

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int NB = 64;         // panel width of the blocked Cholesky
constexpr int UCHUNK = 32;     // beta2 groups factored together

__host__ __device__ inline int64_t nquad(int64_t r) { return r * (r + 1) / 2; }
__host__ __device__ inline int64_t ncols(int64_t r) { return r + nquad(r) + 1; }

// column of E for the quadratic feature (i, j), i <= j, at r_max
__device__ __forceinline__ int64_t qcol_max(int i, int j, int rmax) {
  return rmax + int64_t(i) * rmax - int64_t(i) * (i - 1) / 2 + (j - i);
}

// (i, j) of quadratic index q in the ordering (0,0),(0,1),..,(0,r-1),(1,1),..
__device__ __forceinline__ void qpair(int64_t q, int r, int& i, int& j) {
  int ii = 0;
  int64_t off = 0;
  while (off + (r - ii) <= q) {
    off += r - ii;
    ++ii;
  }
  i = ii;
  j = ii + int(q - off);
}

// ---------------------------------------------------------------------------
// E = [Qhat_1^T | quad(Qhat_1^T) | 1 | Qhat_2^T] at r_max, (k-1) x m, ld lde
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void assemble_kernel(const double* __restrict__ Qhat, int64_t ldqh, int64_t k,
                                                       int rmax, double* __restrict__ E, int64_t lde) {
  const int64_t c = blockIdx.y;                    // column of E
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;  // row (time index of Qhat_1)
  if (t >= k - 1) return;
  const int64_t s = nquad(rmax);
  const int64_t d = rmax + s + 1;
  double v;
  if (c < rmax) {
    v = Qhat[c * ldqh + t];
  } else if (c < rmax + s) {
    int i, j;
    qpair(c - rmax, rmax, i, j);
    v = Qhat[int64_t(i) * ldqh + t] * Qhat[int64_t(j) * ldqh + t];
  } else if (c == rmax + s) {
    v = 1.0;
  } else {
    v = Qhat[(c - d) * ldqh + t + 1];
  }
  E[t * lde + c] = v;
}

// ---------------------------------------------------------------------------
// per (r, beta2) group: gather the quadratic block and right-hand sides
//   L[u]  (s x s, lower, ld s)   = G_qq + beta2_u I
//   R[u]  (s x (2r+1), ld 2r+1)  = [G_ql | G_q,rhs]
// ---------------------------------------------------------------------------
struct GroupGeom {
  int r, rmax;
  int64_t s, m;  // m = leading dimension of G_E
  int64_t dmax;
};

__device__ __forceinline__ int64_t gcol_q(const GroupGeom& g, int64_t q) {
  int i, j;
  qpair(q, g.r, i, j);
  return qcol_max(i, j, g.rmax);
}
// linear/constant index c in [0, r]: c < r linear column c, c == r constant
__device__ __forceinline__ int64_t gcol_l(const GroupGeom& g, int c) {
  return (c < g.r) ? c : (g.rmax + nquad(g.rmax));
}
__device__ __forceinline__ int64_t gcol_rhs(const GroupGeom& g, int c) { return g.dmax + c; }

__global__ __launch_bounds__(256) void gather_qq_kernel(const double* __restrict__ GE, GroupGeom geo,
                                                        const double* __restrict__ beta2u, double* __restrict__ L,
                                                        double* __restrict__ R) {
  const int u = blockIdx.z;
  const int64_t a = blockIdx.y;
  const int64_t s = geo.s;
  const int64_t ca = gcol_q(geo, a);
  const double* grow = GE + ca * geo.m;
  double* Lu = L + size_t(u) * s * s;
  const double b2 = beta2u[u];
  for (int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x; b <= a; b += int64_t(gridDim.x) * 256) {
    double v = grow[gcol_q(geo, b)];
    if (b == a) v += b2;
    Lu[a * s + b] = v;
  }
  const int w = 2 * geo.r + 1;
  double* Ru = R + size_t(u) * s * w;
  if (blockIdx.x == 0) {
    for (int c = threadIdx.x; c < w; c += 256) {
      const int64_t col = (c <= geo.r) ? gcol_l(geo, c) : gcol_rhs(geo, c - geo.r - 1);
      Ru[a * w + c] = grow[col];
    }
  }
}

// ---------------------------------------------------------------------------
// blocked Cholesky (lower, row-major, ld n), batched over blockIdx.z / .y
// ---------------------------------------------------------------------------
// Diagonal block at jb: factor in LDS with one wave (no workgroup barriers
// beyond the wave), write L_jj and the inverse of its triangle.
__global__ __launch_bounds__(256) void potf2_kernel(double* __restrict__ A, int64_t n, int64_t jb,
                                                    double* __restrict__ Linv, int* __restrict__ fail_flag) {
  __shared__ double T[NB][NB + 1];
  __shared__ double Ti[NB][NB + 1];
  __shared__ int bad;
  const int u = blockIdx.x;
  const int tid = threadIdx.x;
  double* Au = A + size_t(u) * n * n;
  const int nb = int(min<int64_t>(NB, n - jb));
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    double v = 0.0;
    if (i < nb && j <= i) v = Au[(jb + i) * n + jb + j];
    else if (i == j) v = 1.0;  // identity padding beyond the matrix
    T[i][j] = v;
    Ti[i][j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  // right-looking Cholesky of the 64 x 64 block
  for (int c = 0; c < NB; ++c) {
    const double piv = T[c][c];
    const bool okp = (piv > 0.0) && isfinite(piv);
    const double dc = sqrt(okp ? piv : 1.0);
    __syncthreads();
    if (tid == 0) {
      T[c][c] = dc;
      if (!okp) bad = 1;
    }
    if (tid > c && tid < NB) T[tid][c] /= dc;
    __syncthreads();
    const int rem = NB - 1 - c;
    for (int e = tid; e < rem * rem; e += 256) {
      const int i = c + 1 + e / rem, l = c + 1 + e % rem;
      if (l <= i) T[i][l] -= T[i][c] * T[l][c];
    }
    __syncthreads();
  }
  // inverse of the triangle: T Ti = I, right-looking over rows
  for (int i = 0; i < NB; ++i) {
    if (tid <= i) Ti[i][tid] /= T[i][i];
    __syncthreads();
    const int rem = NB - 1 - i, cols = i + 1;
    for (int e = tid; e < rem * cols; e += 256) {
      const int q = i + 1 + e / cols, c = e % cols;
      Ti[q][c] -= T[q][i] * Ti[i][c];
    }
    __syncthreads();
  }
  double* Lo = Linv + (size_t(u) * ((n + NB - 1) / NB) + jb / NB) * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    if (i < nb && j <= i) Au[(jb + i) * n + jb + j] = T[i][j];
    Lo[e] = Ti[i][j];
  }
  if (tid == 0 && bad) fail_flag[u] = 1;
}

// Rows below the diagonal block: A[i, jb:jb+nb] <- A[i, jb:jb+nb] L_jj^{-T}
// = A[i, :] Linv^T, one thread per row.
__global__ __launch_bounds__(256) void panel_kernel(double* __restrict__ A, int64_t n, int64_t jb,
                                                    const double* __restrict__ Linv) {
  __shared__ double Li[NB][NB + 1];
  const int u = blockIdx.y;
  double* Au = A + size_t(u) * n * n;
  const double* Lu = Linv + (size_t(u) * ((n + NB - 1) / NB) + jb / NB) * NB * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) Li[e / NB][e % NB] = Lu[e];
  __syncthreads();
  const int64_t i = jb + NB + int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int nb = int(min<int64_t>(NB, n - jb));
  double x[NB];
#pragma unroll
  for (int p = 0; p < NB; ++p) x[p] = (p < nb) ? Au[i * n + jb + p] : 0.0;
  for (int c = 0; c < nb; ++c) {
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < NB; ++p) s += x[p] * Li[c][p];
    Au[i * n + jb + c] = s;
  }
}

// Trailing update on FP64 MFMA: A[i][l] -= sum_p L[i][jb+p] L[l][jb+p] for
// i >= l >= jb+NB, 64 x 64 tiles (lower triangle of tiles), 4 waves of 32 x 32.
__global__ __launch_bounds__(256) void syrk_update_kernel(double* __restrict__ A, int64_t n, int64_t jb) {
  __shared__ double Pa[NB][NB + 2];
  __shared__ double Pb[NB][NB + 2];
  const int u = blockIdx.y;
  double* Au = A + size_t(u) * n * n;
  const int64_t j1 = jb + NB;
  const int t = blockIdx.x;
  int I = int((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int64_t r0 = j1 + int64_t(I) * 64, c0 = j1 + int64_t(J) * 64;
  for (int e = threadIdx.x; e < 64 * NB; e += 256) {
    const int rr = e / NB, p = e % NB;
    Pa[rr][p] = (r0 + rr < n) ? Au[(r0 + rr) * n + jb + p] : 0.0;
    Pb[rr][p] = (c0 + rr < n) ? Au[(c0 + rr) * n + jb + p] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < NB / 4; ++kk) {
    const int p = kk * 4 + (lane >> 4);
    double af[2], bf[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) af[i] = Pa[wm * 32 + i * 16 + (lane & 15)][p];
#pragma unroll
    for (int j = 0; j < 2; ++j) bf[j] = Pb[wn * 32 + j * 16 + (lane & 15)][p];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = r0 + wm * 32 + i * 16 + (lane >> 4) + 4 * e;  // MFMA f64 output layout
        const int64_t col = c0 + wn * 32 + j * 16 + (lane & 15);
        if (row < n && col <= row) Au[row * n + col] -= acc[i][j][e];
      }
}

// ---------------------------------------------------------------------------
// Triangular solves with the factored L (row-major lower, ld n) and its
// diagonal-block inverses, right-looking, per 64-row block J:
//   forward  (L Y = X):   Y_J = Linv_J X_J,    then X_T -= L_TJ Y_J   (T > J)
//   backward (L^T Y = X): Y_J = Linv_J^T X_J,  then X_T -= L_JT^T Y_J (T < J)
// X (n x w, ld w) holds the right-hand sides and is consumed; Y_J goes to
// Yout.  Both steps are 64 x 64 x 64 products on FP64 MFMA tiles with A and
// B staged in LDS: the diagonal solve once per (item, 64 columns), the update
// once per (coupled block row, 64 columns, item).
// ---------------------------------------------------------------------------
constexpr int TP = NB + 2;  // LDS pitch of the solve tiles

// acc += A . B for the wave's 32 x 32 quarter (2 x 2 blocks of 16 x 16)
__device__ __forceinline__ void tile_mma64(const double (*A)[TP], const double (*B)[TP], dbl4 (&acc)[2][2], int lane,
                                           int wm, int wn) {
#pragma unroll 4
  for (int kk = 0; kk < NB / 4; ++kk) {
    const int p = kk * 4 + (lane >> 4);
    double af[2], bf[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) af[i] = A[wm * 32 + i * 16 + (lane & 15)][p];
#pragma unroll
    for (int j = 0; j < 2; ++j) bf[j] = B[p][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
  }
}

// stage rows [r0, r0+64) x columns [c0, c0+64) of an n x w row-major matrix (zero outside)
__device__ __forceinline__ void stage_rhs(double (*B)[TP], const double* __restrict__ X, int64_t n, int64_t w,
                                          int64_t r0, int64_t c0) {
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int a = e / NB, c = e % NB;
    B[a][c] = (r0 + a < n && c0 + c < w) ? X[(r0 + a) * w + c0 + c] : 0.0;
  }
}

template <bool TRANS>
__global__ __launch_bounds__(256) void trsm_diag_kernel(const double* __restrict__ Linv, int64_t n,
                                                        const double* __restrict__ X, double* __restrict__ Y,
                                                        int64_t w, int64_t J) {
  __shared__ double A[NB][TP];
  __shared__ double B[NB][TP];
  const int u = blockIdx.y;
  const int64_t nblk = (n + NB - 1) / NB;
  const double* Li = Linv + (size_t(u) * nblk + J) * NB * NB;
  const double* Xu = X + size_t(u) * n * w;
  double* Yu = Y + size_t(u) * n * w;
  const int64_t c0 = int64_t(blockIdx.x) * NB, jb = J * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int a = e / NB, b = e % NB;
    A[a][b] = TRANS ? Li[b * NB + a] : Li[a * NB + b];
  }
  stage_rhs(B, Xu, n, w, jb, c0);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  tile_mma64(A, B, acc, lane, wm, wn);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = jb + wm * 32 + i * 16 + (lane >> 4) + 4 * e;  // MFMA f64 output layout
        const int64_t col = c0 + wn * 32 + j * 16 + (lane & 15);
        if (row < n && col < w) Yu[row * w + col] = acc[i][j][e];
      }
}

template <bool TRANS>
__global__ __launch_bounds__(256) void trsm_update_kernel(const double* __restrict__ L, int64_t n,
                                                          double* __restrict__ X, const double* __restrict__ Y,
                                                          int64_t w, int64_t J) {
  __shared__ double A[NB][TP];
  __shared__ double B[NB][TP];
  const int u = blockIdx.z;
  const double* Lu = L + size_t(u) * n * n;
  double* Xu = X + size_t(u) * n * w;
  const double* Yu = Y + size_t(u) * n * w;
  const int64_t T = TRANS ? int64_t(blockIdx.x) : J + 1 + int64_t(blockIdx.x);
  const int64_t tb = T * NB, jb = J * NB, c0 = int64_t(blockIdx.y) * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {  // A[a][b]: coefficient of Y_J row b in X_T row a
    const int a = e / NB, b = e % NB;
    double v = 0.0;
    if (tb + a < n && jb + b < n) v = TRANS ? Lu[(jb + b) * n + tb + a] : Lu[(tb + a) * n + jb + b];
    A[a][b] = v;
  }
  stage_rhs(B, Yu, n, w, jb, c0);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  tile_mma64(A, B, acc, lane, wm, wn);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = tb + wm * 32 + i * 16 + (lane >> 4) + 4 * e;
        const int64_t col = c0 + wn * 32 + j * 16 + (lane & 15);
        if (row < n && col < w) Xu[row * w + col] -= acc[i][j][e];
      }
}

int trsm_run(hipStream_t st, bool trans, const double* L, int64_t n, const double* Linv, double* X, double* Yout,
             int64_t w, int nu) {
  const int64_t nblk = (n + NB - 1) / NB;
  const unsigned nch = unsigned((w + NB - 1) / NB);
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t J = trans ? (nblk - 1 - b) : b;
    const unsigned ntrail = unsigned(trans ? J : (nblk - 1 - J));  // coupled block rows
    if (!trans)
      trsm_diag_kernel<false><<<dim3(nch, unsigned(nu)), 256, 0, st>>>(Linv, n, X, Yout, w, J);
    else
      trsm_diag_kernel<true><<<dim3(nch, unsigned(nu)), 256, 0, st>>>(Linv, n, X, Yout, w, J);
    DOPINF_LAUNCHED();
    if (ntrail == 0) continue;
    if (!trans)
      trsm_update_kernel<false><<<dim3(ntrail, nch, unsigned(nu)), 256, 0, st>>>(L, n, X, Yout, w, J);
    else
      trsm_update_kernel<true><<<dim3(ntrail, nch, unsigned(nu)), 256, 0, st>>>(L, n, X, Yout, w, J);
    DOPINF_LAUNCHED();
  }
  return DOPINF_OK;
}

// ---------------------------------------------------------------------------
// per pair: Schur complement solve and operator write-out
// CV[u] = W^T [W | y] ((r+1) x (2r+1)); R2[u] = [P | Z] (s x (2r+1))
// ---------------------------------------------------------------------------
struct PairArgs {
  const double* GE;
  GroupGeom geo;
  const double* CV;
  const double* R2;
  const int* ufail;
  const int* pair_u;     // pair -> local u index (within the chunk), -1: not in chunk
  const double* beta1;   // per pair
  double* O;             // group base, pair stride r*d
  int* status;           // group base
  double* XL;            // per pair: X_l ((r+1) x r), for the quadratic columns
  int n_pairs;
};

__global__ __launch_bounds__(256) void pair_solve_kernel(PairArgs a) {
  extern __shared__ double sm[];
  const int p = blockIdx.x;
  const int u = a.pair_u[p];
  if (u < 0) return;
  const GroupGeom& g = a.geo;
  const int r = g.r;
  const int r1 = r + 1;
  const int w = 2 * r + 1;
  const int64_t s = g.s;
  const int64_t d = ncols(r);
  double* S = sm;               // r1 x r1
  double* X = sm + r1 * r1;     // r1 x r  (rhs, then solution)
  __shared__ int bad;
  const double* CVu = a.CV + size_t(u) * r1 * w;
  const double b1 = a.beta1[p];
  for (int e = threadIdx.x; e < r1 * r1; e += 256) {
    const int i = e / r1, j = e % r1;
    double v = a.GE[gcol_l(g, i) * g.m + gcol_l(g, j)] - CVu[i * w + j];
    if (i == j) v += b1;
    S[e] = v;
  }
  for (int e = threadIdx.x; e < r1 * r; e += 256) {
    const int i = e / r, c = e % r;
    X[e] = a.GE[gcol_l(g, i) * g.m + gcol_rhs(g, c)] - CVu[i * w + r1 + c];
  }
  if (threadIdx.x == 0) bad = a.ufail[u];
  __syncthreads();
  // Cholesky of S (right-looking, in LDS)
  for (int c = 0; c < r1; ++c) {
    if (threadIdx.x == 0) {
      double piv = S[c * r1 + c];
      if (!(piv > 0.0) || !isfinite(piv)) {
        bad = 1;
        piv = 1.0;
      }
      S[c * r1 + c] = sqrt(piv);
    }
    __syncthreads();
    const double dc = S[c * r1 + c];
    for (int i = c + 1 + threadIdx.x; i < r1; i += 256) S[i * r1 + c] /= dc;
    __syncthreads();
    const int rem = r1 - c - 1;
    for (int e = threadIdx.x; e < rem * rem; e += 256) {
      const int i = c + 1 + e / rem, l = c + 1 + e % rem;
      if (l <= i) S[i * r1 + l] -= S[i * r1 + c] * S[l * r1 + c];
    }
    __syncthreads();
  }
  // forward (L Y = X) then backward (L^T X = Y) substitution, right-looking:
  // each step scales one row (all r columns at once) and updates the rest
  for (int i = 0; i < r1; ++i) {
    for (int c = threadIdx.x; c < r; c += 256) X[i * r + c] /= S[i * r1 + i];
    __syncthreads();
    const int rem = r1 - 1 - i;
    for (int e = threadIdx.x; e < rem * r; e += 256) {
      const int q = i + 1 + e / r, c = e % r;
      X[q * r + c] -= S[q * r1 + i] * X[i * r + c];
    }
    __syncthreads();
  }
  for (int i = r1 - 1; i >= 0; --i) {
    for (int c = threadIdx.x; c < r; c += 256) X[i * r + c] /= S[i * r1 + i];
    __syncthreads();
    for (int e = threadIdx.x; e < i * r; e += 256) {
      const int q = e / r, c = e % r;
      X[q * r + c] -= S[i * r1 + q] * X[i * r + c];
    }
    __syncthreads();
  }
  double* Op = a.O + size_t(p) * r * d;
  // linear and constant columns of O = X^T
  for (int e = threadIdx.x; e < r * r1; e += 256) {
    const int i = e / r1, c = e % r1;   // O row i, permuted column c
    const int64_t col = (c < r) ? c : (r + s);
    Op[i * d + col] = X[c * r + i];
  }
  // X_l for the quadratic columns X_q = Z - P X_l (opq_kernel)
  double* XLp = a.XL + size_t(p) * r1 * r;
  for (int e = threadIdx.x; e < r1 * r; e += 256) XLp[e] = X[e];
  if (threadIdx.x == 0) a.status[p] = bad ? DOPINF_E_NOTSPD : DOPINF_OK;
}

// Quadratic columns of O for every pair: O[i][r + q] = Z[q][i] - sum_c P[q][c] X_l[c][i]
// with [P | Z] = R2 of the pair's beta2 group.  Workgroup = (64 quadratic
// columns, 64 modes, pair); FP64 MFMA over K = r + 1 in chunks of 64; the tile
// goes through LDS so that rows of O are written contiguously.
__global__ __launch_bounds__(256) void opq_kernel(PairArgs a) {
  __shared__ double At[NB][TP];
  __shared__ double Bt[NB][TP];
  const int p = blockIdx.y;
  const int u = a.pair_u[p];
  if (u < 0) return;
  const int r = a.geo.r, r1 = r + 1, w = 2 * r + 1;
  const int64_t s = a.geo.s, d = ncols(r);
  const int64_t q0 = int64_t(blockIdx.x) * NB;
  const int i0 = int(blockIdx.z) * NB;
  const double* R2u = a.R2 + size_t(u) * s * w;
  const double* XLp = a.XL + size_t(p) * r1 * r;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < r1; k0 += NB) {
    __syncthreads();
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
      const int a_ = e / NB, b_ = e % NB;
      At[a_][b_] = (q0 + a_ < s && k0 + b_ < r1) ? R2u[(q0 + a_) * w + k0 + b_] : 0.0;        // P[q][c]
      Bt[a_][b_] = (k0 + a_ < r1 && i0 + b_ < r) ? XLp[(k0 + a_) * r + i0 + b_] : 0.0;       // X_l[c][i]
    }
    __syncthreads();
    tile_mma64(At, Bt, acc, lane, wm, wn);
  }
  __syncthreads();
  // C[q][i] -> At[i][q] (transposed) for row-contiguous writes of O
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int qq = wm * 32 + i * 16 + (lane >> 4) + 4 * e;  // MFMA f64 output layout
        const int ii = wn * 32 + j * 16 + (lane & 15);
        At[ii][qq] = acc[i][j][e];
      }
  __syncthreads();
  double* Op = a.O + size_t(p) * r * d;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int ii = e / NB, qq = e % NB;
    const int i = i0 + ii;
    const int64_t q = q0 + qq;
    if (i < r && q < s) Op[int64_t(i) * d + r + q] = R2u[q * w + r1 + i] - At[ii][qq];
  }
}

__global__ void zero_ints_kernel(int* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void copy_kernel(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) b[i] = a[i];
}

// ---------------------------------------------------------------------------
// host-side planning
// ---------------------------------------------------------------------------
struct InferLayout {
  int rmax;
  int64_t smax, dmax, m, lde, km1;
  size_t e_off, g_off, gram_off, gram_bytes;
  size_t chunk_off;  // per-chunk storage start
  size_t l_bytes, r_bytes, linv_bytes, cv_bytes;  // per u, at rmax
  size_t cg_bytes;   // cross gram partials
  size_t misc_off;
  size_t total;
};

InferLayout layout(int64_t k, int n_r, const int* r_list, int n_pairs) {
  InferLayout L{};
  int rmax = 0;
  for (int g = 0; g < n_r; ++g) rmax = r_list[g] > rmax ? r_list[g] : rmax;
  L.rmax = rmax;
  L.smax = nquad(rmax);
  L.dmax = ncols(rmax);
  L.m = L.dmax + rmax;
  L.lde = (L.m + 1) / 2 * 2;
  L.km1 = k - 1;
  Carver c(nullptr, 0);
  c.take<double>(size_t(L.km1) * L.lde);
  L.e_off = 0;
  L.g_off = c.used;
  c.take<double>(size_t(L.m) * L.m);
  L.gram_off = (c.used + 255) & ~size_t(255);
  L.gram_bytes = gram_f64_workspace_internal(L.km1, L.m, 1);
  c.take<char>(L.gram_bytes);
  const int64_t s = L.smax, w = 2 * rmax + 1, nblk = (s + NB - 1) / NB;
  L.l_bytes = size_t(s) * s * sizeof(double);
  L.r_bytes = size_t(s) * w * sizeof(double);
  L.linv_bytes = size_t(nblk) * NB * NB * sizeof(double);
  L.cv_bytes = size_t(rmax + 1) * w * sizeof(double);
  L.cg_bytes = 0;
  for (int g = 0; g < n_r; ++g) {
    const int64_t rg = r_list[g];
    const size_t b = cross_gram_workspace_internal(nquad(rg), rg + 1, 2 * rg + 1);
    if (b > L.cg_bytes) L.cg_bytes = b;
  }
  const int uc = n_pairs < UCHUNK ? n_pairs : UCHUNK;
  L.chunk_off = (c.used + 255) & ~size_t(255);
  c.take<char>(uc * L.l_bytes);
  c.take<char>(uc * L.r_bytes);
  c.take<char>(uc * L.r_bytes);
  c.take<char>(uc * L.r_bytes);
  c.take<char>(uc * L.linv_bytes);
  c.take<char>(uc * L.cv_bytes);
  c.take<char>(L.cg_bytes);
  L.misc_off = (c.used + 255) & ~size_t(255);
  c.take<double>(size_t(uc));       // beta2 per u
  c.take<int>(size_t(uc));          // fail flag per u
  c.take<int>(size_t(n_pairs));     // pair -> u
  c.take<double>(size_t(n_pairs));  // beta1 per pair
  c.take<double>(size_t(n_pairs) * (rmax + 1) * rmax);  // X_l per pair
  L.total = c.used;
  return L;
}

}  // namespace
}  // namespace dopinf

using namespace dopinf;

extern "C" size_t dopinf_operator_offset(int n_r, const int* r_list_h, int n_pairs, int item) {
  if (n_r <= 0 || !r_list_h || n_pairs <= 0 || item < 0) return 0;
  size_t off = 0;
  for (int g = 0; g < n_r; ++g) {
    const size_t per = size_t(r_list_h[g]) * size_t(ncols(r_list_h[g]));
    if (item < (g + 1) * n_pairs) return off + size_t(item - g * n_pairs) * per;
    off += per * size_t(n_pairs);
  }
  return off;
}

extern "C" size_t dopinf_infer_workspace(int64_t k, int n_r, const int* r_list_h, int n_pairs) {
  if (k < 2 || n_r <= 0 || !r_list_h || n_pairs <= 0) return 0;
  return layout(k, n_r, r_list_h, n_pairs).total;
}

extern "C" int dopinf_infer(void* stream, const double* Qhat, int64_t ldqh, int64_t k, int n_r, const int* r_list_h,
                            int n_pairs, const double* beta1_h, const double* beta2_h, double* O, int* status,
                            void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE(Qhat && O && status && r_list_h && beta1_h && beta2_h, "NULL argument");
  DOPINF_REQUIRE(k >= 2 && ldqh >= k, "need k >= 2 and ldqh >= k");
  DOPINF_REQUIRE(n_r >= 1 && n_pairs >= 1, "need n_r >= 1 and n_pairs >= 1");
  for (int g = 0; g < n_r; ++g) DOPINF_REQUIRE(r_list_h[g] >= 1 && r_list_h[g] <= 512, "r must be in [1, 512]");
  for (int p = 0; p < n_pairs; ++p)
    DOPINF_REQUIRE(beta1_h[p] >= 0.0 && beta2_h[p] >= 0.0, "regularization parameters must be >= 0");
  const InferLayout L = layout(k, n_r, r_list_h, n_pairs);
  if (!ws || ws_bytes < L.total) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total, ws_bytes);
  int dev = 0, maxlds = 0;
  DOPINF_HIP(hipGetDevice(&dev));
  DOPINF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  {
    const size_t need = size_t(L.rmax + 1) * (2 * L.rmax + 1) * sizeof(double) + 1024;
    DOPINF_REQUIRE(need <= size_t(maxlds), "r too large for the per-pair LDS solve");
    if (need > 65536)
      DOPINF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(pair_solve_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(need)));
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  double* E = reinterpret_cast<double*>(base + L.e_off);
  double* GE = reinterpret_cast<double*>(base + L.g_off);

  // E and its Gram
  {
    dim3 grid(unsigned((L.km1 + 255) / 256), unsigned(L.m));
    assemble_kernel<<<grid, 256, 0, st>>>(Qhat, ldqh, k, L.rmax, E, L.lde);
    DOPINF_LAUNCHED();
    int rc = gram_f64_internal(st, E, L.km1, L.m, L.lde, nullptr, nullptr, 0, nullptr, GE, L.m,
                               base + L.gram_off, L.gram_bytes);
    if (rc) return rc;
  }

  // distinct beta2 values (exact equality), in first-appearance order
  std::vector<double> b2u;
  std::vector<int> pair_uid(n_pairs);
  for (int p = 0; p < n_pairs; ++p) {
    int id = -1;
    for (size_t q = 0; q < b2u.size(); ++q)
      if (b2u[q] == beta2_h[p]) {
        id = int(q);
        break;
      }
    if (id < 0) {
      id = int(b2u.size());
      b2u.push_back(beta2_h[p]);
    }
    pair_uid[p] = id;
  }
  const int n_u = int(b2u.size());
  const int uc = n_pairs < UCHUNK ? n_pairs : UCHUNK;

  char* ch = base + L.chunk_off;
  Carver mc(base + L.misc_off, ws_bytes - L.misc_off);
  double* b2dev = mc.take<double>(size_t(uc));
  int* ufail = mc.take<int>(size_t(uc));
  int* pair_u = mc.take<int>(size_t(n_pairs));
  double* b1dev = mc.take<double>(size_t(n_pairs));
  double* XL = mc.take<double>(size_t(n_pairs) * (L.rmax + 1) * L.rmax);
  DOPINF_HIP(hipMemcpyAsync(b1dev, beta1_h, sizeof(double) * n_pairs, hipMemcpyHostToDevice, st));

  std::vector<int> pu(n_pairs);
  for (int g = 0; g < n_r; ++g) {
    GroupGeom geo{};
    geo.r = r_list_h[g];
    geo.rmax = L.rmax;
    geo.s = nquad(geo.r);
    geo.m = L.m;
    geo.dmax = L.dmax;
    const int64_t s = geo.s, w = 2 * geo.r + 1, r1 = geo.r + 1;
    const int64_t nblk = (s + NB - 1) / NB;
    // per-u storage at this r (packed tighter than at rmax)
    const size_t lb = size_t(s) * s * sizeof(double), rb = size_t(s) * w * sizeof(double);
    const size_t lib = size_t(nblk) * NB * NB * sizeof(double), cvb = size_t(r1) * w * sizeof(double);
    double* Lq = reinterpret_cast<double*>(ch);
    double* R = reinterpret_cast<double*>(ch + uc * lb);
    double* R2 = reinterpret_cast<double*>(ch + uc * (lb + rb));
    double* Rt = reinterpret_cast<double*>(ch + uc * (lb + 2 * rb));
    double* Linv = reinterpret_cast<double*>(ch + uc * (lb + 3 * rb));
    double* CV = reinterpret_cast<double*>(ch + uc * (lb + 3 * rb + lib));
    char* cgws = ch + uc * (lb + 3 * rb + lib + cvb);
    const size_t cgb = cross_gram_workspace_internal(s, r1, w);
    const size_t op_base = dopinf_operator_offset(n_r, r_list_h, n_pairs, g * n_pairs);

    for (int u0 = 0; u0 < n_u; u0 += uc) {
      const int nu = (n_u - u0) < uc ? (n_u - u0) : uc;
      for (int p = 0; p < n_pairs; ++p) pu[p] = (pair_uid[p] >= u0 && pair_uid[p] < u0 + nu) ? pair_uid[p] - u0 : -1;
      DOPINF_HIP(hipMemcpyAsync(b2dev, b2u.data() + u0, sizeof(double) * nu, hipMemcpyHostToDevice, st));
      DOPINF_HIP(hipMemcpyAsync(pair_u, pu.data(), sizeof(int) * n_pairs, hipMemcpyHostToDevice, st));
      // hipMemcpyAsync from pageable host memory returns after staging, so the
      // host vectors may be reused in the next iteration.
      zero_ints_kernel<<<1, 256, 0, st>>>(ufail, uc);
      DOPINF_LAUNCHED();
      {
        dim3 grid(unsigned((s + 255) / 256 > 64 ? 64 : (s + 255) / 256), unsigned(s), unsigned(nu));
        gather_qq_kernel<<<grid, 256, 0, st>>>(GE, geo, b2dev, Lq, R);
        DOPINF_LAUNCHED();
      }
      for (int64_t jb = 0; jb < s; jb += NB) {
        potf2_kernel<<<nu, 256, 0, st>>>(Lq, s, jb, Linv, ufail);
        DOPINF_LAUNCHED();
        const int64_t rest = s - jb - NB;
        if (rest > 0) {
          panel_kernel<<<dim3(unsigned((rest + 255) / 256), unsigned(nu)), 256, 0, st>>>(Lq, s, jb, Linv);
          DOPINF_LAUNCHED();
          const int64_t tt = (rest + 63) / 64;
          syrk_update_kernel<<<dim3(unsigned(tt * (tt + 1) / 2), unsigned(nu)), 256, 0, st>>>(Lq, s, jb);
          DOPINF_LAUNCHED();
        }
      }
      // [W | y] = L^{-1} [G_ql | B_q] into R2 (R consumed), then
      // [P | Z] = L^{-T} [W | y]: copy to R, solve into R2 ... so keep [W | y]:
      int rc2 = trsm_run(st, false, Lq, s, Linv, R, R2, w, nu);  // R2 = [W | y]
      if (rc2) return rc2;
      copy_kernel<<<1024, 256, 0, st>>>(R2, R, int64_t(nu) * s * w);  // R = [W | y]
      DOPINF_LAUNCHED();
      rc2 = trsm_run(st, true, Lq, s, Linv, R2, Rt, w, nu);  // Rt = [P | Z] (R2 consumed)
      if (rc2) return rc2;
      for (int u = 0; u < nu; ++u) {
        int rc = cross_gram_internal(st, R + size_t(u) * s * w, w, R + size_t(u) * s * w, w, s, r1, w,
                                     CV + size_t(u) * r1 * w, w, cgws, cgb, nullptr, nullptr, 0, nullptr);
        if (rc) return rc;
      }
      PairArgs pa{};
      pa.GE = GE;
      pa.geo = geo;
      pa.CV = CV;
      pa.R2 = Rt;
      pa.ufail = ufail;
      pa.pair_u = pair_u;
      pa.beta1 = b1dev;
      pa.O = O + op_base;
      pa.status = status + g * n_pairs;
      pa.n_pairs = n_pairs;
      pa.XL = XL;
      const size_t smem = size_t(r1) * (r1 + geo.r) * sizeof(double);
      pair_solve_kernel<<<n_pairs, 256, smem, st>>>(pa);
      DOPINF_LAUNCHED();
      opq_kernel<<<dim3(unsigned((s + NB - 1) / NB), unsigned(n_pairs), unsigned((geo.r + NB - 1) / NB)), 256, 0,
                   st>>>(pa);
      DOPINF_LAUNCHED();
    }
  }
  return DOPINF_OK;
}
