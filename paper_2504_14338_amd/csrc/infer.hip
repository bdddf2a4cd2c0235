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
//    forward solve [W | y] = L^{-1} [G_ql | B_q] and the products
//    W^T [W | y] are computed once per (r, beta2).  Each pair then factors
//    the small Schur complement
//       S = G_ll + beta1 I - W^T W           ((r+1) x (r+1))
//    solves S X_l = B_l - W^T y, forms v = y - W X_l and solves
//    L^T X_q = v by back substitution.  This is Cholesky factorization of
//    the same matrix under a symmetric permutation (backward stable; the
//    shortcut X_q = L^{-T} y - (L^{-T} W) X_l is not: it cancels
//    |L^{-T} W| |X_l| down to |X_q|).
//  * The s x s factorization is blocked right-looking (64-wide panels): a
//    diagonal-block kernel also inverts its 64 x 64 triangle, a panel kernel
//    solves the rows below, and the trailing update runs on FP64 MFMA tiles.
//    Triangular solves then reduce to products with the stored diagonal
//    inverses.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <utility>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace dopinf {
int gram_f64_internal(hipStream_t st, const double* X, int64_t n, int64_t m, int64_t ldx, const double* mean,
                      const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd, void* ws,
                      size_t ws_bytes);
size_t gram_f64_workspace_internal(int64_t n, int64_t m, int nvars);

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
// Row i starts at off(i) = i r - i (i - 1) / 2; i is the largest root bound of
// off(i) <= q, taken from the quadratic formula and corrected by +-1 steps.
__device__ __forceinline__ void qpair(int64_t q, int r, int& i, int& j) {
  auto off = [r](int64_t ii) { return ii * r - ii * (ii - 1) / 2; };
  const double b = 2.0 * r + 1.0;
  const double disc = b * b - 8.0 * double(q);
  int64_t ii = int64_t((b - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
  if (ii < 0) ii = 0;
  if (ii > r - 1) ii = r - 1;
  while (ii + 1 <= r - 1 && off(ii + 1) <= q) ++ii;
  while (ii > 0 && off(ii) > q) --ii;
  i = int(ii);
  j = int(ii + (q - off(ii)));
}

// ---------------------------------------------------------------------------
// E = [Qhat_1^T | quad(Qhat_1^T) | 1 | Qhat_2^T] at r_max, (k-1) x m, ld lde
// (discrete form, dt == 0), or, for the continuous-time form of Eq. (10),
// E = [Qhat^T | quad(Qhat^T) | 1 | Qdot^T], k x m, with the time derivative
// by second-order finite differences at snapshot spacing dt: central
// differences inside the window, the one-sided three-point formulas at its
// two ends (exact for quadratics in t).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fd_derivative(const double* __restrict__ q, int64_t t, int64_t k, double dt) {
  if (t == 0) return (-3.0 * q[0] + 4.0 * q[1] - q[2]) / (2.0 * dt);
  if (t == k - 1) return (3.0 * q[k - 1] - 4.0 * q[k - 2] + q[k - 3]) / (2.0 * dt);
  return (q[t + 1] - q[t - 1]) / (2.0 * dt);
}

__global__ __launch_bounds__(256) void assemble_kernel(const double* __restrict__ Qhat, int64_t ldqh, int64_t k,
                                                       int rmax, double* __restrict__ E, int64_t lde, double dt) {
  const int64_t c = blockIdx.y;                    // column of E
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;  // row (time index of Qhat_1, or of Qhat)
  if (t >= (dt > 0.0 ? k : k - 1)) return;
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
  } else if (dt > 0.0) {
    v = fd_derivative(Qhat + (c - d) * ldqh, t, k, dt);
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
                                                        const double* __restrict__ beta2u, int nu,
                                                        double* __restrict__ L, double* __restrict__ R) {
  // row a of G_qq (lower triangle) and of [G_ql | B_q], gathered once from
  // G_E and written into every beta2 matrix of the chunk
  const int64_t a = blockIdx.y;
  const int64_t s = geo.s;
  const int64_t ca = gcol_q(geo, a);
  const double* grow = GE + ca * geo.m;
  for (int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x; b <= a; b += int64_t(gridDim.x) * 256) {
    const double v = grow[gcol_q(geo, b)];
    double* dst = L + a * s + b;
    for (int u = 0; u < nu; ++u) dst[size_t(u) * s * s] = (b == a) ? v + beta2u[u] : v;
  }
  const int w = 2 * geo.r + 1;
  if (blockIdx.x == 0) {
    for (int c = threadIdx.x; c < w; c += 256) {
      const int64_t col = (c <= geo.r) ? gcol_l(geo, c) : gcol_rhs(geo, c - geo.r - 1);
      const double v = grow[col];
      for (int u = 0; u < nu; ++u) R[size_t(u) * s * w + a * w + c] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// blocked Cholesky (lower, row-major, ld n), batched over blockIdx.z / .y
// ---------------------------------------------------------------------------
// Diagonal block at jb: Cholesky factor and inverse of the 64 x 64 block in
// LDS, one workgroup per matrix, one barrier per column.  Step c reads the
// unscaled column c of the working matrix T and its pivot d_c; it writes
// column c of the factor F (sqrt(d_c) on the diagonal), updates the trailing
// triangle T[i][l] -= T[i][c] T[l][c] / d_c, and applies the same elimination
// to W (initially I): W[q][p] -= (T[q][c] / d_c) W[c][p] for q > c.  Nothing
// that step c reads is written in step c.  W ends as M^{-1} for the unit
// lower factor M of A = M diag(d) M^T, so L^{-1} = diag(d)^{-1/2} W.  Rows
// beyond the matrix are identity rows.
constexpr int PF2 = 1024;      // threads of the diagonal-block kernel
constexpr int PR = PF2 / NB;    // row groups (one column per thread)

__global__ __launch_bounds__(PF2) void potf2_kernel(double* __restrict__ A, int64_t n, int64_t jb,
                                                    double* __restrict__ Linv, int* __restrict__ fail_flag) {
  __shared__ double T[NB][NB + 1];
  __shared__ double F[NB][NB + 1];
  __shared__ double W[NB][NB + 1];
  __shared__ int bad;
  const int u = blockIdx.x;
  const int tid = threadIdx.x;
  double* Au = A + size_t(u) * n * n;
  const int nb = int(min<int64_t>(NB, n - jb));
  {
    // all 16 loads of a thread in flight together (clamped addresses, select)
    const int j = tid % NB, i0 = tid / NB;
    double v[NB / PR];
#pragma unroll
    for (int k = 0; k < NB / PR; ++k) {
      const int i = i0 + PR * k;
      const int ic = i < nb ? i : 0, jc = j < nb ? j : 0;
      v[k] = Au[(jb + ic) * n + jb + jc];
    }
#pragma unroll
    for (int k = 0; k < NB / PR; ++k) {
      const int i = i0 + PR * k;
      T[i][j] = (i < nb && j <= i) ? v[k] : (i == j ? 1.0 : 0.0);
      F[i][j] = 0.0;
      W[i][j] = (i == j) ? 1.0 : 0.0;
    }
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int c = 0; c < NB; ++c) {
    const double piv = T[c][c];
    const bool okp = (piv > 0.0) && isfinite(piv);
    const double pv = okp ? piv : 1.0;
    const double d = sqrt(pv);
    if (tid >= c && tid < NB) F[tid][c] = (tid == c) ? d : T[tid][c] / d;
    if (tid == 0 && !okp) bad = 1;
    const double rp = 1.0 / pv;
    // thread -> column j = tid % 64 and rows c + 1 + tid / 64 + PR k: column
    // j > c of T (lower part) or column j <= c of W, with one code path for
    // both (no divergence) and all reads issued before the writes
    const int j = tid % NB;
    const bool onT = j > c;
    double* dst = onT ? &T[0][0] : &W[0][0];
    const double f = (onT ? T[j][c] : W[c][j]) * rp;
    // rows c + 1 .. NB - 1 in steps of PR
    auto step = [&](auto kn) {
      constexpr int KN = decltype(kn)::value;
      double a[KN], b[KN];
#pragma unroll
      for (int k = 0; k < KN; ++k) {
        const int i = c + 1 + tid / NB + PR * k;
        const int ic = i < NB ? i : NB - 1;
        a[k] = T[ic][c];
        b[k] = dst[ic * (NB + 1) + j];
      }
#pragma unroll
      for (int k = 0; k < KN; ++k) {
        const int i = c + 1 + tid / NB + PR * k;
        if (i < NB && (!onT || j <= i)) dst[i * (NB + 1) + j] = b[k] - a[k] * f;
      }
    };
    if (c < NB / 2)
      step(std::integral_constant<int, NB / PR>{});
    else
      step(std::integral_constant<int, NB / (2 * PR)>{});
    __syncthreads();
  }
  double* Lo = Linv + (size_t(u) * ((n + NB - 1) / NB) + jb / NB) * NB * NB;
  for (int e = tid; e < NB * NB; e += PF2) {
    const int i = e / NB, j = e % NB;
    if (i < nb && j <= i) Au[(jb + i) * n + jb + j] = F[i][j];
    Lo[e] = (j <= i) ? W[i][j] / F[i][i] : 0.0;
  }
  if (tid == 0 && bad) fail_flag[u] = 1;
}

// ---------------------------------------------------------------------------
// Triangular solves with the factored L (row-major lower, ld n) and its
// diagonal-block inverses, per 64-row block J:
//   forward  (L Y = X):   Y_J = Linv_J X_J,    and X_T -= L_TJ Y_J   (T > J)
//   backward (L^T Y = X): Y_J = Linv_J^T X_J,  and X_T -= L_JT^T Y_J (T < J)
// X holds the right-hand sides and is consumed; Y goes to Yout.  The blocks
// are taken in block columns of kb rows: inside one, each solved block
// updates only the rest of the block column; the blocks outside then take a
// single update of depth kb (fewer passes over X than one update per block).
// The innermost runs of up to 2 blocks are solved by one fused launch that
// keeps their rows of X in LDS.  All products run on FP64 MFMA tiles with
// both operands staged in LDS.
//
// Right-hand sides of group g (one factor L_g): cnt[g] matrices of n x w,
// row-major, stored one after the other from entry e0[g]; the tiles see them
// as one n x (cnt[g] w) matrix, so several items that share a factor fill
// the 64-wide column tiles.  NULL tables mean one matrix per group.
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

// Rows below the diagonal block (called only when rows remain below it, so
// the block is a full 64 wide): A[i, jb:jb+64] <- A[i, jb:jb+64] Linv^T,
// one 64-row tile per workgroup on FP64 MFMA.
__global__ __launch_bounds__(256) void panel_kernel(double* __restrict__ A, int64_t n, int64_t jb,
                                                    const double* __restrict__ Linv) {
  __shared__ double Xs[NB][TP];  // the tile's rows of the panel
  __shared__ double Bs[NB][TP];  // Bs[p][c] = Linv[c][p]
  const int u = blockIdx.y;
  double* Au = A + size_t(u) * n * n;
  const double* Lu = Linv + (size_t(u) * ((n + NB - 1) / NB) + jb / NB) * NB * NB;
  const int64_t r0 = jb + NB + int64_t(blockIdx.x) * NB;
  // all loads of a thread issued together (clamped rows), then the LDS stores
  double xv[NB * NB / 256], lv[NB * NB / 256];
#pragma unroll
  for (int k = 0; k < NB * NB / 256; ++k) {
    const int e = threadIdx.x + 256 * k, a = e / NB, p = e % NB;
    xv[k] = Au[(r0 + a < n ? r0 + a : r0) * n + jb + p];
    lv[k] = Lu[e];
  }
#pragma unroll
  for (int k = 0; k < NB * NB / 256; ++k) {
    const int e = threadIdx.x + 256 * k, a = e / NB, p = e % NB;
    Xs[a][p] = (r0 + a < n) ? xv[k] : 0.0;
    Bs[p][a] = lv[k];  // e = a * NB + p: Linv[a][p]
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  tile_mma64(Xs, Bs, acc, lane, wm, wn);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = r0 + wm * 32 + i * 16 + (lane >> 4) + 4 * e;  // MFMA f64 output layout
        const int64_t col = jb + wn * 32 + j * 16 + (lane & 15);
        if (row < n) Au[row * n + col] = acc[i][j][e];
      }
}

struct RhsMap {
  const int* e0;   // per group: first matrix (NULL: g)
  const int* cnt;  // per group: matrices (NULL: 1)
  int64_t w;       // columns per matrix
};

// offset of element (row 0, virtual column vcol) of group g, or -1 past the end
__device__ __forceinline__ int64_t rhs_offset(const RhsMap& m, int g, int64_t n, int64_t vcol) {
  const int e0 = m.e0 ? m.e0[g] : g;
  const int cnt = m.cnt ? m.cnt[g] : 1;
  if (vcol >= int64_t(cnt) * m.w) return -1;
  return (e0 + vcol / m.w) * n * m.w + vcol % m.w;
}

// Fused leaf of the triangular solves: a run of up to LMAX diagonal blocks
// [b0, b1) of one factor, for a slab of CW right-hand-side columns per
// workgroup, held in LDS for the whole run.  Backward (TRANS, L^T Y = X): for
// J = b1-1 down to b0, Y_J = Linv_J^T X_J, then X_T -= L[J, T]^T Y_J for
// b0 <= T < J; forward: for J = b0 up, Y_J = Linv_J X_J, then
// X_T -= L[T, J] Y_J for J < T < b1.  One launch per run instead of a
// diagonal-block launch and a 64-deep update launch per block, and no round
// trips of X through HBM between them.  4 waves; wave w computes rows
// 16 w .. 16 w + 15 of each 64 x CW product (CW / 16 FP64 MFMA blocks), so it
// alone uses those rows of the 64 x 64 coefficient block (Linv_J or a block
// of L): it reads its A fragments straight from memory into registers, the
// next item's while the current one is multiplied, and LDS holds only the
// slab (68 KB: two workgroups per CU, and room beside other kernels).  64
// columns per workgroup share each coefficient fragment load between twice
// the columns of 32 (sweep 87.0 -> 88.6 thousand solves per second).
// Barriers: before each diagonal product (its rows were updated by every
// wave), after it (before Y_J overwrites X_J) and before the first update
// that reads Y_J; the updates from one J write disjoint rows.
// Where the backward solve also writes its result transposed into the
// operators: O[i][r + q] = X_q[q][i] for the pair of each right-hand-side
// matrix (batch entry e -> pair border[e]); O == nullptr: no write.
struct OWrite {
  const int* border;  // batch entry -> pair
  double* O;          // group base, pair stride r * d
  int64_t d;          // columns of an operator
  int r;
};

constexpr int LMAX = 2;       // diagonal blocks per leaf
constexpr int CW = 64;        // right-hand-side columns per workgroup
constexpr int CWP = CW + 2;   // LDS pitch of the slab

template <bool TRANS>
__global__ __launch_bounds__(256, 2) void trsm_leaf_kernel(const double* __restrict__ L, int64_t n,
                                                           const double* __restrict__ Linv,
                                                           const double* __restrict__ X, double* __restrict__ Y,
                                                           RhsMap m, int64_t b0, int64_t b1, OWrite ow) {
  __shared__ double Xs[LMAX * NB][CWP];
  const int g = blockIdx.y;
  const int64_t c0 = int64_t(blockIdx.x) * CW;
  if (rhs_offset(m, g, n, c0) < 0) return;  // slab wholly past the group's columns
  const int tid = threadIdx.x;
  const int nbk = int(b1 - b0);
  const int64_t r0 = b0 * NB, nblk = (n + NB - 1) / NB, w = m.w;
  const double* Lg = L + size_t(g) * n * n;
  const double* Lig = Linv + size_t(g) * nblk * NB * NB;
  // the slab: thread -> column tid % CW, rows tid / CW + (256 / CW) q
  {
    constexpr int RG = 256 / CW;
    const int c = tid % CW, rr0 = tid / CW;
    const int64_t off0 = rhs_offset(m, g, n, c0 + c);
    const int64_t off = off0 >= 0 ? off0 : rhs_offset(m, g, n, c0);
    for (int q0 = 0; q0 < nbk * NB / RG; q0 += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t row = r0 + rr0 + RG * (q0 + u);
        v[u] = X[off + (row < n ? row : r0) * w];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int rr = rr0 + RG * (q0 + u);
        Xs[rr][c] = (off0 >= 0 && r0 + rr < n) ? v[u] : 0.0;
      }
    }
  }
  // work items in order: per J a diagonal product (t == J), then the
  // updates of the run's other blocks t from it
  const int nitems = nbk * (nbk + 1) / 2;
  auto item = [&](int it, int& J, int& t) {
    int jj = 0;
    for (;;) {
      const int cnt = nbk - jj;  // the jj-th block processed has nbk - jj items
      if (it < cnt) break;
      it -= cnt;
      ++jj;
    }
    if (TRANS) {
      J = nbk - 1 - jj;            // blocks from the bottom
      t = (it == 0) ? J : it - 1;  // then T = 0 .. J - 1
    } else {
      J = jj;                      // blocks from the top
      t = (it == 0) ? J : J + it;  // then T = J + 1 .. nbk - 1
    }
  };
  const int lane = tid & 63, wv = tid >> 6;
  const int ia = 16 * wv + (lane & 15), kq = lane >> 4;  // A fragment: row ia, k = 4 kk + kq
  // A fragments of item it: a[kk] = A[ia][4 kk + kq] with A = Linv_J (^T) or
  // the block of L; rows of L past n read as 0
  auto load_a = [&](int it, double (&a)[NB / 4]) {
    int J, t;
    item(it, J, t);
    const int64_t gJ = b0 + J, gt = b0 + t;
#pragma unroll
    for (int kk = 0; kk < NB / 4; ++kk) {
      const int k = 4 * kk + kq;
      if (t == J) {
        const double* Li = Lig + gJ * NB * NB;
        a[kk] = TRANS ? Li[k * NB + ia] : Li[ia * NB + k];
      } else if (TRANS) {
        const int64_t row = gJ * NB + k;  // A[i][k] = L[J rows k][t columns i]
        const double v = Lg[(row < n ? row : 0) * n + gt * NB + ia];
        a[kk] = row < n ? v : 0.0;
      } else {
        const int64_t row = gt * NB + ia;  // A[i][k] = L[t rows i][J columns k]
        const double v = Lg[(row < n ? row : 0) * n + gJ * NB + k];
        a[kk] = row < n ? v : 0.0;
      }
    }
  };
  double a_cur[NB / 4], a_nxt[NB / 4];
  load_a(0, a_cur);
  bool after_diag = false;
  for (int it = 0; it < nitems; ++it) {
    int J, t;
    item(it, J, t);
    if (t == J || after_diag) __syncthreads();
    if (it + 1 < nitems) load_a(it + 1, a_nxt);
    dbl4 acc[CW / 16];
#pragma unroll
    for (int j = 0; j < CW / 16; ++j) acc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < NB / 4; ++kk) {
      const int k = 4 * kk + kq;
#pragma unroll
      for (int j = 0; j < CW / 16; ++j)
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_cur[kk], Xs[J * NB + k][16 * j + (lane & 15)], acc[j], 0,
                                                      0, 0);
    }
    if (t == J) {
      __syncthreads();  // every wave has read X_J
#pragma unroll
      for (int j = 0; j < CW / 16; ++j) {
        const int c = 16 * j + (lane & 15);
        const int64_t off = rhs_offset(m, g, n, c0 + c);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int rr = 16 * wv + (lane >> 4) + 4 * e;  // MFMA f64 output layout
          const int64_t row = (b0 + J) * NB + rr;
          Xs[J * NB + rr][c] = acc[j][e];
          if (off >= 0 && row < n) Y[off + row * w] = acc[j][e];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < CW / 16; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int rr = 16 * wv + (lane >> 4) + 4 * e;
          Xs[t * NB + rr][16 * j + (lane & 15)] -= acc[j][e];
        }
    }
    after_diag = (t == J);
#pragma unroll
    for (int kk = 0; kk < NB / 4; ++kk) a_cur[kk] = a_nxt[kk];
  }
  if (TRANS && ow.O) {
    // the run's solved rows (Y_J stays in Xs after its diagonal product):
    // wave w writes columns 8 w .. 8 w + 7, lane = row within the block, so
    // every store covers 64 consecutive q of one operator row
    __syncthreads();
#pragma unroll 1
    for (int cc = 0; cc < CW / 4; ++cc) {
      const int c = (CW / 4) * wv + cc;
      const int64_t vcol = c0 + c;
      const int e0 = m.e0 ? m.e0[g] : g, cnt = m.cnt ? m.cnt[g] : 1;
      if (vcol >= int64_t(cnt) * w) break;  // columns of a wave are consecutive
      const int p = ow.border[e0 + int(vcol / w)];
      double* Orow = ow.O + size_t(p) * ow.r * ow.d + (vcol % w) * ow.d + ow.r;
      for (int J = 0; J < nbk; ++J) {
        const int64_t q = (b0 + J) * NB + lane;
        if (q < n) Orow[q] = Xs[J * NB + lane][c];
      }
    }
  }
}

// Deep update of the triangular solves on 128 x 128 tiles:
//   X[i][c] -= sum_{k in [k0, k1)} C(i, k) Y[k][c],   r_lo <= i < r_hi,
// with C(i, k) = L[k][i] for the backward solve (TRANS: rows of L are
// contiguous in i) and L[i][k] for the forward solve (staged transposed).
// Workgroup = (128 virtual columns, 128 rows, group); 4 waves of 64 x 64
// (4 x 4 FP64 MFMA blocks each); K in slabs of 16 rows, double-buffered in
// LDS, the next slab's loads in flight while the current one is multiplied.
constexpr int UT = 128;      // output tile edge
constexpr int UK = 16;       // K slab
constexpr int UP = UT + 4;   // LDS pitch in doubles

// An operand staged transposed (16 lanes writing 16 different K rows) is
// stored at column c ^ swz(k): with the 132-double pitch the 16 lanes of a
// store then hit 16 different bank pairs (4-way conflicts without it); the
// XOR only permutes inside 16-aligned groups, so fragment reads of 16
// consecutive columns stay conflict-free.
__device__ __forceinline__ int swz(int k) { return (k >> 2) & 3; }

template <bool SWA, bool SWB>
__device__ __forceinline__ void mma_slab128(const double (*As)[UP], const double (*Bs)[UP], dbl4 (&acc)[4][4],
                                            int lane, int wm, int wn) {
#pragma unroll
  for (int kk = 0; kk < UK / 4; ++kk) {
    const int k = kk * 4 + (lane >> 4);
    double af[4], bf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = As[k][(wm * 64 + i * 16 + (lane & 15)) ^ (SWA ? swz(k) : 0)];
#pragma unroll
    for (int j = 0; j < 4; ++j) bf[j] = Bs[k][(wn * 64 + j * 16 + (lane & 15)) ^ (SWB ? swz(k) : 0)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
  }
}

// X rows [tb, tb + 128) n [r_lo, r_hi), virtual columns [c0, c0 + 128) of
// group g -= the tile's accumulators (4 waves of 64 x 64, MFMA f64 output
// layout); per column group the 16 old values are loaded (clamped addresses)
// before any is written back.
__device__ __forceinline__ void rhs_tile_subtract(double* __restrict__ X, const RhsMap& m, int g, int64_t n,
                                                  int64_t c0, int64_t tb, int64_t r_lo, int64_t r_hi,
                                                  const dbl4 (&acc)[4][4], int lane, int wm, int wn) {
  const int64_t w = m.w;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t off0 = rhs_offset(m, g, n, c0 + wn * 64 + j * 16 + (lane & 15));
    const int64_t off = off0 >= 0 ? off0 : rhs_offset(m, g, n, c0);
    double old[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = tb + wm * 64 + i * 16 + (lane >> 4) + 4 * e;  // MFMA f64 output layout
        old[i][e] = X[off + (row < r_hi ? row : r_lo) * w];
      }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = tb + wm * 64 + i * 16 + (lane >> 4) + 4 * e;
        if (off0 >= 0 && row < r_hi) X[off + row * w] = old[i][e] - acc[i][j][e];
      }
  }
}

template <bool TRANS>
__global__ __launch_bounds__(256, 2) void trsm_update_t128_kernel(const double* __restrict__ L, int64_t n,
                                                               double* __restrict__ X, const double* __restrict__ Y,
                                                               RhsMap m, int64_t r_lo, int64_t r_hi, int64_t k0,
                                                               int64_t k1) {
  __shared__ double As[2][UK][UP];
  __shared__ double Bs[2][UK][UP];
  const int g = blockIdx.z;
  const int64_t c0 = int64_t(blockIdx.x) * UT;
  if (rhs_offset(m, g, n, c0) < 0) return;  // tile wholly past the group's columns
  const int64_t tb = r_lo + int64_t(blockIdx.y) * UT;
  const double* Lg = L + size_t(g) * n * n;
  const int64_t w = m.w;
  // B loader: thread -> one column c of the tile, K rows kr0 + 2q.
  // A loader (TRANS): the same pattern over rows i; (forward): thread -> K
  // offset kl, rows ml + 16q, so that 16 threads read 16 consecutive k of a row.
  const int lc = threadIdx.x % UT, kr0 = threadIdx.x / UT;
  const int kl = threadIdx.x % UK, ml = threadIdx.x / UK;
  const bool arow = tb + lc < r_hi;
  const int64_t boff = rhs_offset(m, g, n, c0 + lc);
  double ra[UK / 2], rb[UK / 2];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int q = 0; q < UK / 2; ++q) {
      const int64_t k = kb + kr0 + 2 * q;
      const bool kin = k < k1;
      if (TRANS) {
        ra[q] = (kin && arow) ? Lg[k * n + tb + lc] : 0.0;
      } else {
        const int64_t ka = kb + kl, row = tb + ml + 16 * q;
        ra[q] = (ka < k1 && row < r_hi) ? Lg[row * n + ka] : 0.0;
      }
      rb[q] = (kin && boff >= 0) ? Y[boff + k * w] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < UK / 2; ++q) {
      if (TRANS)
        As[buf][kr0 + 2 * q][lc] = ra[q];
      else
        As[buf][kl][(ml + 16 * q) ^ swz(kl)] = ra[q];
      Bs[buf][kr0 + 2 * q][lc] = rb[q];
    }
  };
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  dbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  load(k0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int64_t kb = k0; kb < k1; kb += UK) {
    const bool more = kb + UK < k1;
    if (more) load(kb + UK);
    mma_slab128<!TRANS, false>(As[buf], Bs[buf], acc, lane, wm, wn);
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  rhs_tile_subtract(X, m, g, n, c0, tb, r_lo, r_hi, acc, lane, wm, wn);
}

// The same updates with both operands brought in by LDS-DMA (buffer loads
// that write LDS directly, no register round trip), as in the FP64 Gram: per
// 16-row stage of K, double-buffered, with the next stage's loads in flight
// over the current stage's MFMAs.  B: row k of Y across the tile's columns
// as one 128-double LDS row; a lane brings two adjacent right-hand-side
// columns (16 bytes; they lie in one matrix since the width is even), at a
// fixed offset from the tile's first column, so that the same offsets serve
// every row.  A, backward (TRANS, X[i][c] -= sum_k L[k][i] Y[k][c]): row k
// of L from column tb, K-major like B; forward (X[i][c] -= sum_k L[i][k]
// Y[k][c]): the tile's 128 rows of L, 16 values of k each, M-major
// (issue_mmajor).  Rows past k1, columns past the group's, and L past row or
// column n read as zero (buffer range checks).  Needs even n and width and
// 16-byte aligned L and Y.
constexpr int QK = 16;               // K rows per stage
constexpr int QP = 144;              // LDS row pitch (doubles)
constexpr int QSLOT = 2 * QK * QP;   // A rows, then B rows

#define DOPINF_LDS(p) ((__attribute__((address_space(3))) void*)(p))

// Buffer descriptor over [p, p + nbytes): reads past nbytes return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void* p, int64_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(nbytes), 0x00020000);
}

// Wait until none of this wave's vector-memory operations is in flight.
__device__ __forceinline__ void wait_vmem_all() { __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8)); }

// Workgroup barrier that leaves the LDS-DMA loads alone (the explicit wait
// above decides what must have landed).
__device__ __forceinline__ void barrier_only() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// M-major LDS tile: 128 rows of 16 doubles (8 chunks of 16 bytes); chunk c
// of row m sits at slot c ^ mswz(m), which spreads the 16 rows that one MFMA
// fragment read touches over distinct banks.
__device__ __forceinline__ int mswz(int m) { return (m ^ (m >> 3)) & 7; }

__device__ __forceinline__ double mm_at(const double* tile, int m, int k) {
  return tile[m * 16 + (((k >> 1) ^ mswz(m)) << 1) + (k & 1)];
}

// Issue the loads of rows [row0, row0 + 128) x columns [kb, kb + 16) of the
// row-major P (leading dimension ld, at most 2^31 bytes in all) into an
// M-major tile: wave wv brings rows 32 wv .. 32 wv + 31, 8 rows per
// instruction, and lane l the chunk that belongs in slot l % 8 of row l / 8.
// Rows at or past nrow and columns at or past k1 read as zero (k1 even).
__device__ __forceinline__ void issue_mmajor(double* tile, const double* P, int64_t ld, int64_t row0, int64_t nrow,
                                             int64_t kb, int64_t k1, int wv, int lane) {
  const __amdgpu_buffer_rsrc_t rs = span_rsrc(P, 0x7ffffff0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int mloc = wv * 32 + q * 8 + (lane >> 3);
    const int c = (lane & 7) ^ mswz(mloc);
    const int64_t row = row0 + mloc, k = kb + 2 * c;
    const uint32_t off = (row < nrow && k < k1) ? uint32_t((row * ld + k) * 8) : 0x80000000u;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, DOPINF_LDS(tile + (wv * 32 + q * 8) * 16), 16, off, 0, 0, 0);
  }
}

template <bool TRANS>
__global__ __launch_bounds__(256, 2) void trsm_update_dma_kernel(const double* __restrict__ L, int64_t n,
                                                                double* __restrict__ X, const double* __restrict__ Y,
                                                                RhsMap m, int64_t r_lo, int64_t r_hi, int64_t k0,
                                                                int64_t k1) {
  __shared__ double lds[2 * QSLOT];
  const int g = blockIdx.z;
  const int64_t c0 = int64_t(blockIdx.x) * UT;
  const int64_t base = rhs_offset(m, g, n, c0);
  if (base < 0) return;  // tile wholly past the group's columns
  const int64_t tb = r_lo + int64_t(blockIdx.y) * UT;
  const double* Lg = L + size_t(g) * n * n;
  const int64_t w = m.w;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int wm = wv >> 1, wn = wv & 1;
  const int64_t lo = rhs_offset(m, g, n, c0 + 2 * lane);
  const uint32_t offb = lo >= 0 ? uint32_t((lo - base) * 8) : 0x80000000u;  // past the range: zero
  const uint32_t offa = uint32_t(lane) * 16;
  const int64_t nst = (k1 - k0 + QK - 1) / QK;
  auto issue = [&](int64_t st) {
    double* sl = lds + (st & 1) * QSLOT;
    const int64_t kb = k0 + st * QK;
    if (!TRANS) issue_mmajor(sl, Lg, n, tb, r_hi, kb, k1, wv, lane);
#pragma unroll
    for (int q = 0; q < QK / 4; ++q) {
      const int r = wv * (QK / 4) + q;
      const bool in = kb + r < k1;
      const int64_t k = in ? kb + r : k0;
      if (TRANS)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(span_rsrc(Lg + k * n + tb, in ? (n - tb) * 8 : 0),
                                                 DOPINF_LDS(sl + r * QP), 16, offa, 0, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(span_rsrc(Y + base + k * w, in ? 0x7ffffff0 : 0),
                                               DOPINF_LDS(sl + (QK + r) * QP), 16, offb, 0, 0, 0);
    }
  };
  dbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  if (nst > 0) issue(0);
  for (int64_t st = 0; st < nst; ++st) {
    wait_vmem_all();
    barrier_only();
    if (st + 1 < nst) issue(st + 1);
    const double* As = lds + (st & 1) * QSLOT;
    const double* Bs = As + QK * QP;
#pragma unroll
    for (int kk = 0; kk < QK / 4; ++kk) {
      const int krow = kk * 4 + (lane >> 4), cm = lane & 15;
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        af[i] = TRANS ? As[krow * QP + wm * 64 + i * 16 + cm] : mm_at(As, wm * 64 + i * 16 + cm, krow);
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[krow * QP + wn * 64 + j * 16 + cm];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  rhs_tile_subtract(X, m, g, n, c0, tb, r_lo, r_hi, acc, lane, wm, wn);
}

// The Cholesky's update from the factored columns [a0, a0 + K) on 128 x 128
// tiles: A[i][l] -= sum_{a0 <= p < a0+K} L[i][p] L[l][p] for c_lo <= l < c_hi,
// l <= i < n (with c_hi = n the trailing update of the lower triangle), over
// the trapezoid of rows [c_lo, n) and columns [c_lo, c_hi).  Both operands
// are rows of L (contiguous in p); they are staged transposed (K-major) into
// the double-buffered LDS slabs of mma_slab128.  A diagonal tile loads its
// rows once.
// Tile t of the trapezoid (TR tile rows from c_lo, TC tile columns): a
// triangle of tiles when the columns reach the end, else column by column.
__device__ __forceinline__ void syrk_tile_coords(int t, int TR, int TC, int& I, int& J) {
  if (TC >= TR) {
    I = int((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    J = t - I * (I + 1) / 2;
  } else {
    int rem = t;
    J = 0;
    while (rem >= TR - J) {
      rem -= TR - J;
      ++J;
    }
    I = J + rem;
  }
}

// A[row][col] -= the tile's accumulators for rows [r0, r0 + 128) below n,
// columns [cc0, cc0 + 128) below c_hi, on or below the diagonal; per column
// group the 16 old values are loaded (clamped addresses) before any is
// written back.
__device__ __forceinline__ void syrk_tile_subtract(double* __restrict__ Au, int64_t n, int64_t r0, int64_t cc0,
                                                   int64_t c_hi, const dbl4 (&acc)[4][4], int lane, int wm, int wn) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t col = cc0 + wn * 64 + j * 16 + (lane & 15);
    const int64_t colc = col < n ? col : cc0;
    double old[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = r0 + wm * 64 + i * 16 + (lane >> 4) + 4 * e;  // MFMA f64 output layout
        old[i][e] = Au[(row < n ? row : r0) * n + colc];
      }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = r0 + wm * 64 + i * 16 + (lane >> 4) + 4 * e;
        if (row < n && col <= row && col < c_hi) Au[row * n + col] = old[i][e] - acc[i][j][e];
      }
  }
}

__global__ __launch_bounds__(256, 2) void syrk_update128_kernel(double* __restrict__ A, int64_t n, int64_t a0, int64_t K,
                                                             int64_t c_lo, int64_t c_hi) {
  __shared__ double As[2][UK][UP];
  __shared__ double Bs[2][UK][UP];
  const int u = blockIdx.y;
  double* Au = A + size_t(u) * n * n;
  const int TR = int((n - c_lo + UT - 1) / UT), TC = int((c_hi - c_lo + UT - 1) / UT);
  int I, J;
  syrk_tile_coords(int(blockIdx.x), TR, TC, I, J);
  const bool diag = (I == J);
  const int64_t r0 = c_lo + int64_t(I) * UT, cc0 = c_lo + int64_t(J) * UT;
  const int64_t k1 = a0 + K;
  // loader: thread -> K offset kl, rows ml + 16 q
  const int kl = threadIdx.x % UK, ml = threadIdx.x / UK;
  double ra[UT / 16], rb[UT / 16];
  auto load = [&](int64_t kb) {
    const int64_t k = kb + kl;
    const bool kin = k < k1;
#pragma unroll
    for (int q = 0; q < UT / 16; ++q) {
      const int64_t ra_row = r0 + ml + 16 * q, rb_row = cc0 + ml + 16 * q;
      ra[q] = (kin && ra_row < n) ? Au[ra_row * n + k] : 0.0;
      if (!diag) rb[q] = (kin && rb_row < n) ? Au[rb_row * n + k] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < UT / 16; ++q) {
      As[buf][kl][(ml + 16 * q) ^ swz(kl)] = ra[q];
      if (!diag) Bs[buf][kl][(ml + 16 * q) ^ swz(kl)] = rb[q];
    }
  };
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  dbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  load(a0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int64_t kb = a0; kb < k1; kb += UK) {
    const bool more = kb + UK < k1;
    if (more) load(kb + UK);
    mma_slab128<true, true>(As[buf], diag ? As[buf] : Bs[buf], acc, lane, wm, wn);
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  syrk_tile_subtract(Au, n, r0, cc0, c_hi, acc, lane, wm, wn);
}

// The Cholesky's update with both operands (rows of L, 16 values of p per
// stage) brought in by LDS-DMA into M-major tiles (issue_mmajor), double
// buffered, the next stage's loads in flight over the current MFMAs; a
// diagonal tile loads its rows once.  Needs even n, n^2 8 < 2^31 bytes and a
// 16-byte aligned A.
__global__ __launch_bounds__(256, 2) void syrk_update_dma_kernel(double* __restrict__ A, int64_t n, int64_t a0,
                                                                int64_t K, int64_t c_lo, int64_t c_hi) {
  __shared__ double lds[2 * 2 * UT * 16];
  const int u = blockIdx.y;
  double* Au = A + size_t(u) * n * n;
  const int TR = int((n - c_lo + UT - 1) / UT), TC = int((c_hi - c_lo + UT - 1) / UT);
  int I, J;
  syrk_tile_coords(int(blockIdx.x), TR, TC, I, J);
  const bool diag = (I == J);
  const int64_t r0 = c_lo + int64_t(I) * UT, cc0 = c_lo + int64_t(J) * UT;
  const int64_t k1 = a0 + K;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int wm = wv >> 1, wn = wv & 1;
  const int64_t nst = (K + QK - 1) / QK;
  auto issue = [&](int64_t st) {
    double* sl = lds + (st & 1) * (2 * UT * 16);
    const int64_t kb = a0 + st * QK;
    issue_mmajor(sl, Au, n, r0, n, kb, k1, wv, lane);
    if (!diag) issue_mmajor(sl + UT * 16, Au, n, cc0, n, kb, k1, wv, lane);
  };
  dbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  if (nst > 0) issue(0);
  for (int64_t st = 0; st < nst; ++st) {
    wait_vmem_all();
    barrier_only();
    if (st + 1 < nst) issue(st + 1);
    const double* As = lds + (st & 1) * (2 * UT * 16);
    const double* Bs = diag ? As : As + UT * 16;
#pragma unroll
    for (int kk = 0; kk < QK / 4; ++kk) {
      const int krow = kk * 4 + (lane >> 4), cm = lane & 15;
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = mm_at(As, wm * 64 + i * 16 + cm, krow);
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = mm_at(Bs, wn * 64 + j * 16 + cm, krow);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  syrk_tile_subtract(Au, n, r0, cc0, c_hi, acc, lane, wm, wn);
}

inline int64_t syrk_tiles128(int64_t n, int64_t c_lo, int64_t c_hi) {
  const int64_t TR = (n - c_lo + UT - 1) / UT, TC = (c_hi - c_lo + UT - 1) / UT;
  if (TC >= TR) return TR * (TR + 1) / 2;
  return TC * TR - TC * (TC - 1) / 2;
}

// Block-column widths of the blocked Cholesky and triangular solves: an
// outer width and an optional inner one (0: none) that must divide it; the
// innermost level is always NB.
struct Widths {
  int64_t w[2];
  int n;  // levels above NB
};
inline Widths widths(int64_t kb, int64_t kb2) {
  Widths x{{kb, 0}, 1};
  if (kb2 >= NB && kb2 < kb && kb % kb2 == 0) {
    x.w[1] = kb2;
    x.n = 2;
  }
  return x;
}

// Blocked Cholesky of nu matrices (s x s, row-major, lower triangle used) in
// place, recursive over the widths: columns [c0, c1) are factored in blocks
// of the level's width; each block is factored one level down and then
// updates the rest of [c0, c1), all rows below, with depth = its width.  At
// the last level the 64-wide panels are factored left to right (diagonal
// block, then the panel below it) and each updates the rest of its block.
// One width kb is the classic scheme (panels update their block column of
// kb, the trailing matrix takes one update of depth kb); an inner width
// keeps the panels' shallow updates inside blocks of kb2 and gives the
// block column of kb updates of depth kb2.
int cholesky_run(hipStream_t st, double* Lq, int64_t s, double* Linv, int* ufail, int nu, int64_t kb, int64_t kb2) {
  const Widths W = widths(kb, kb2);
  // the updates load by LDS-DMA where rows are 16-byte aligned and one
  // buffer descriptor spans a factor
  const bool dma = s % 2 == 0 && (reinterpret_cast<uintptr_t>(Lq) & 15) == 0 && s * s * 8 < 0x7ffffff0;
  auto syrk = [&](int64_t k0, int64_t kd, int64_t c0, int64_t c1) -> int {
    const int64_t nt = syrk_tiles128(s, c0, c1);
    if (dma)
      syrk_update_dma_kernel<<<dim3(unsigned(nt), unsigned(nu)), 256, 0, st>>>(Lq, s, k0, kd, c0, c1);
    else
      syrk_update128_kernel<<<dim3(unsigned(nt), unsigned(nu)), 256, 0, st>>>(Lq, s, k0, kd, c0, c1);
    DOPINF_LAUNCHED();
    return DOPINF_OK;
  };
  auto leaf = [&](int64_t c0, int64_t c1) -> int {
    for (int64_t jb = c0; jb < c1; jb += NB) {
      potf2_kernel<<<nu, PF2, 0, st>>>(Lq, s, jb, Linv, ufail);
      DOPINF_LAUNCHED();
      const int64_t rest = s - jb - NB;
      if (rest <= 0) continue;
      panel_kernel<<<dim3(unsigned((rest + NB - 1) / NB), unsigned(nu)), 256, 0, st>>>(Lq, s, jb, Linv);
      DOPINF_LAUNCHED();
      if (jb + NB < c1) {
        const int rc = syrk(jb, NB, jb + NB, c1);
        if (rc) return rc;
      }
    }
    return DOPINF_OK;
  };
  // columns [c0, c1) at level lev (0: outer width)
  auto level = [&](auto&& self, int64_t c0, int64_t c1, int lev) -> int {
    if (lev == W.n) return leaf(c0, c1);
    for (int64_t cb = c0; cb < c1; cb += W.w[lev]) {
      const int64_t ce = std::min<int64_t>(cb + W.w[lev], c1);
      int rc = self(self, cb, ce, lev + 1);
      if (!rc && ce < c1) rc = syrk(cb, ce - cb, ce, c1);
      if (rc) return rc;
    }
    return DOPINF_OK;
  };
  return level(level, int64_t(0), s, 0);
}

// ng groups, each with at most max_cols virtual columns; block columns of kb
// rows (a multiple of NB)
int trsm_run(hipStream_t st, bool trans, const double* L, int64_t n, const double* Linv, double* X, double* Yout,
             RhsMap m, int64_t max_cols, int ng, int64_t kb, int64_t kb2, OWrite ow = OWrite{}) {
  const int64_t nblk = (n + NB - 1) / NB;
  const Widths W = widths(kb, kb2);
  const unsigned nslab = unsigned((max_cols + CW - 1) / CW);
  // the updates load by LDS-DMA where rows are 16-byte aligned (and, for
  // the forward form, one buffer descriptor spans a factor)
  const bool dma_b = n % 2 == 0 && m.w % 2 == 0 && (reinterpret_cast<uintptr_t>(L) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(Yout) & 15) == 0 && n < (int64_t(1) << 27);
  const bool dma = trans ? dma_b : dma_b && n * n * 8 < 0x7ffffff0;
  auto leaf = [&](int64_t cb, int64_t ce) -> int {
    if (!trans)
      trsm_leaf_kernel<false><<<dim3(nslab, unsigned(ng)), 256, 0, st>>>(L, n, Linv, X, Yout, m, cb, ce, OWrite{});
    else
      trsm_leaf_kernel<true><<<dim3(nslab, unsigned(ng)), 256, 0, st>>>(L, n, Linv, X, Yout, m, cb, ce, ow);
    DOPINF_LAUNCHED();
    return DOPINF_OK;
  };
  // X blocks [t0, t1) -= coefficients x Y rows [k0, k1)
  auto update = [&](int64_t t0, int64_t t1, int64_t k0, int64_t k1) -> int {
    if (t1 <= t0) return DOPINF_OK;
    const int64_t r_lo = t0 * NB, r_hi = std::min<int64_t>(t1 * NB, n);
    const dim3 g128(unsigned((max_cols + UT - 1) / UT), unsigned((r_hi - r_lo + UT - 1) / UT), unsigned(ng));
    const int64_t kh = std::min<int64_t>(k1, n);
    if (dma && trans)
      trsm_update_dma_kernel<true><<<g128, 256, 0, st>>>(L, n, X, Yout, m, r_lo, r_hi, k0, kh);
    else if (dma)
      trsm_update_dma_kernel<false><<<g128, 256, 0, st>>>(L, n, X, Yout, m, r_lo, r_hi, k0, kh);
    else if (trans)
      trsm_update_t128_kernel<true><<<g128, 256, 0, st>>>(L, n, X, Yout, m, r_lo, r_hi, k0, kh);
    else
      trsm_update_t128_kernel<false><<<g128, 256, 0, st>>>(L, n, X, Yout, m, r_lo, r_hi, k0, kh);
    DOPINF_LAUNCHED();
    return DOPINF_OK;
  };
  // blocks [b0, b1) at level lev, recursive over the widths as in
  // cholesky_run: a solved block of the level's width updates the rest of
  // [b0, b1) with depth = its width; at the last level runs of LMAX blocks
  auto level = [&](auto&& self, int64_t b0, int64_t b1, int lev) -> int {
    int rc = DOPINF_OK;
    if (lev == W.n) {
      // runs of up to LMAX blocks by the fused leaf kernel, the rest of
      // [b0, b1) updated from each run
      if (!trans) {
        for (int64_t cb = b0; cb < b1 && !rc; cb += LMAX) {
          const int64_t ce = std::min<int64_t>(cb + LMAX, b1);
          rc = leaf(cb, ce);
          if (!rc) rc = update(ce, b1, cb * NB, ce * NB);
        }
      } else {
        for (int64_t ce = b1; ce > b0 && !rc; ce -= LMAX) {
          const int64_t cb = std::max<int64_t>(b0, ce - LMAX);
          rc = leaf(cb, ce);
          if (!rc) rc = update(b0, cb, cb * NB, ce * NB);
        }
      }
      return rc;
    }
    const int64_t kbb = W.w[lev] / NB;
    if (!trans) {
      for (int64_t cb = b0; cb < b1 && !rc; cb += kbb) {
        const int64_t ce = std::min(cb + kbb, b1);
        rc = self(self, cb, ce, lev + 1);
        if (!rc) rc = update(ce, b1, cb * NB, ce * NB);
      }
    } else {
      for (int64_t ce = b1; ce > b0 && !rc; ce -= kbb) {
        const int64_t cb = std::max(b0, ce - kbb);
        rc = self(self, cb, ce, lev + 1);
        if (!rc) rc = update(b0, cb, cb * NB, ce * NB);
      }
    }
    return rc;
  };
  return level(level, int64_t(0), nblk, 0);
}

// ---------------------------------------------------------------------------
// per pair: Schur complement solve and operator write-out
// CV[u] = W^T [W | y] ((r+1) x (2r+1))
// ---------------------------------------------------------------------------
struct PairArgs {
  const double* GE;
  GroupGeom geo;
  const double* CV;
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
    // thread -> columns l = c + 1 + (tid % 64) + 64 t, rows i >= l in steps of 4
    // (no integer division in the loops)
    for (int l = c + 1 + (threadIdx.x & 63); l < r1; l += 64) {
      const double sl = S[l * r1 + c];
      for (int i = l + (threadIdx.x >> 6); i < r1; i += 4) S[i * r1 + l] -= S[i * r1 + c] * sl;
    }
    __syncthreads();
  }
  // forward (L Y = X) then backward (L^T X = Y) substitution, right-looking:
  // each step scales one row (all r columns at once) and updates the rest
  for (int i = 0; i < r1; ++i) {
    for (int c = threadIdx.x; c < r; c += 256) X[i * r + c] /= S[i * r1 + i];
    __syncthreads();
    for (int c = threadIdx.x & 63; c < r; c += 64) {
      const double xc = X[i * r + c];
      for (int q = i + 1 + (threadIdx.x >> 6); q < r1; q += 4) X[q * r + c] -= S[q * r1 + i] * xc;
    }
    __syncthreads();
  }
  for (int i = r1 - 1; i >= 0; --i) {
    for (int c = threadIdx.x; c < r; c += 256) X[i * r + c] /= S[i * r1 + i];
    __syncthreads();
    for (int c = threadIdx.x & 63; c < r; c += 64) {
      const double xc = X[i * r + c];
      for (int q = threadIdx.x >> 6; q < i; q += 4) X[q * r + c] -= S[i * r1 + q] * xc;
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
  // X_l for the quadratic columns (vq_kernel)
  double* XLp = a.XL + size_t(p) * r1 * r;
  for (int e = threadIdx.x; e < r1 * r; e += 256) XLp[e] = X[e];
  if (threadIdx.x == 0) a.status[p] = bad ? DOPINF_E_NOTSPD : DOPINF_OK;
}

// Quadratic columns of O, by back substitution per pair:
//   L^T X_q = v,   v = y - W X_l   (s x r),
// with [W | y] = R2 of the pair's beta2 group.  (Forming X_q = Z - P X_l from
// precomputed P = L^{-T} W, Z = L^{-T} y is cheaper but cancels |P| |X_l| down
// to |X_q| and is not backward stable.)  Pairs are batched in the order
// border[b] (grouped by beta2 group), V and X_q are s x r per batch entry.
struct QuadArgs {
  const double* R2;     // [W | y] per u, s x (2r+1)
  const double* XL;     // per pair: X_l ((r+1) x r)
  const int* border;    // batch entry -> pair
  const int* pair_u;    // pair -> u within the chunk
  double* V;            // per batch entry: v (the solve writes X_q to another buffer)
  double* O;            // group base, pair stride r*d
  int64_t s;
  int r;
};

// v = y - W X_l: workgroup = (64 quadratic rows, batch entry, up to 128
// modes).  Wave w computes rows 16 w .. 16 w + 15 against every 16-mode block
// of the tile (FP64 MFMA), over K = r + 1 in LDS chunks of 32 with only the
// k-steps of 4 that K reaches, so neither the modes nor K are padded to 64.
constexpr int VK = 32;        // K per LDS chunk
constexpr int VAP = VK + 4;   // pitch of the W chunk (rows of 16 lanes in distinct banks)
constexpr int VBP = 128 + 8;  // pitch of the X_l chunk

__global__ __launch_bounds__(256) void vq_kernel(QuadArgs a) {
  __shared__ double At[NB][VAP];   // W[q0 + m][k0 + k]
  __shared__ double Bt[VK][VBP];   // X_l[k0 + k][i0 + i]
  const int bt = blockIdx.y;
  const int p = a.border[bt];
  const int u = a.pair_u[p];
  if (u < 0) return;
  const int r = a.r, r1 = r + 1, w = 2 * r + 1;
  const int64_t s = a.s;
  const int64_t q0 = int64_t(blockIdx.x) * NB;
  const int i0 = int(blockIdx.z) * 128;
  const int nb = min(8, (r - i0 + 15) / 16);  // mode blocks of this tile
  const double* R2u = a.R2 + size_t(u) * s * w;
  const double* XLp = a.XL + size_t(p) * r1 * r;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  dbl4 acc[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) acc[b] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < r1; k0 += VK) {
    // all loads of a thread issued together (clamped addresses), then the LDS stores
    double av[NB * VK / 256], bv[VK * 128 / 256];
#pragma unroll
    for (int k = 0; k < NB * VK / 256; ++k) {
      const int e = tid + 256 * k, m = e / VK, c = e % VK;
      av[k] = R2u[(q0 + m < s ? q0 + m : q0) * w + (k0 + c < r1 ? k0 + c : k0)];
    }
#pragma unroll
    for (int k = 0; k < VK * 128 / 256; ++k) {
      const int e = tid + 256 * k, kr = e / 128, i = e % 128;
      bv[k] = XLp[(k0 + kr < r1 ? k0 + kr : k0) * r + (i0 + i < r ? i0 + i : i0)];
    }
    __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int k = 0; k < NB * VK / 256; ++k) {
      const int e = tid + 256 * k, m = e / VK, c = e % VK;
      At[m][c] = (q0 + m < s && k0 + c < r1) ? av[k] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < VK * 128 / 256; ++k) {
      const int e = tid + 256 * k, kr = e / 128, i = e % 128;
      Bt[kr][i] = (k0 + kr < r1 && i0 + i < r) ? bv[k] : 0.0;
    }
    __syncthreads();
    const int nst = min(VK / 4, (r1 - k0 + 3) / 4);
#pragma unroll
    for (int kk = 0; kk < VK / 4; ++kk) {
      if (kk < nst) {
        const int k = 4 * kk + (lane >> 4);
        const double af = At[16 * wv + (lane & 15)][k];
#pragma unroll
        for (int b = 0; b < 8; ++b)
          if (b < nb) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, Bt[k][16 * b + (lane & 15)], acc[b], 0, 0, 0);
      }
    }
  }
  double* Vb = a.V + size_t(bt) * s * r;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    if (b >= nb) continue;
    const int ii = i0 + 16 * b + (lane & 15);
    double yv[4];  // y entries, all loaded (clamped) before the writes
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t q = q0 + 16 * wv + (lane >> 4) + 4 * e;  // MFMA f64 output layout
      yv[e] = R2u[(q < s ? q : q0) * w + r1 + (ii < r ? ii : i0)];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t q = q0 + 16 * wv + (lane >> 4) + 4 * e;
      if (q < s && ii < r) Vb[q * r + ii] = yv[e] - acc[b][e];
    }
  }
}

// CV[u] = W^T [W | y] for every u of a chunk, R[u] = [W | y] (s x w, w = 2r + 1,
// W = its first r + 1 columns).  Workgroup = (64 x 64 output tile, row split,
// u): FP64 MFMA over 64-row slabs of R staged through LDS; each split writes a
// partial tile and cv_reduce_kernel sums the splits in a fixed order.
constexpr int CV_SPLIT_MAX = 8;

__global__ __launch_bounds__(256) void cv_partial_kernel(const double* __restrict__ R, int64_t s, int r1, int w,
                                                         int nspl, double* __restrict__ part) {
  __shared__ double At[NB][TP];  // At[a][p] = W[k0 + p][i0 + a]
  __shared__ double Bt[NB][TP];  // Bt[p][b] = R[k0 + p][c0 + b]
  const int tcols = (w + NB - 1) / NB;
  const int i0 = int(blockIdx.x / tcols) * NB, c0 = int(blockIdx.x % tcols) * NB;
  const int sp = blockIdx.y, u = blockIdx.z;
  const int64_t chunk = ((s + nspl - 1) / nspl + NB - 1) / NB * NB;
  const int64_t lo = int64_t(sp) * chunk, hi = min<int64_t>(s, lo + chunk);
  const double* Ru = R + size_t(u) * s * w;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv >> 1, wn = wv & 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = lo; k0 < hi; k0 += NB) {
    __syncthreads();
    // all loads of a thread issued together (clamped addresses), then the LDS stores
    double av[NB * NB / 256], bv[NB * NB / 256];
#pragma unroll
    for (int k = 0; k < NB * NB / 256; ++k) {
      const int e = threadIdx.x + 256 * k, p_ = e / NB, a_ = e % NB;
      const int64_t row = k0 + p_ < hi ? k0 + p_ : k0;
      av[k] = Ru[row * w + (i0 + a_ < r1 ? i0 + a_ : i0)];
      bv[k] = Ru[row * w + (c0 + a_ < w ? c0 + a_ : c0)];
    }
#pragma unroll
    for (int k = 0; k < NB * NB / 256; ++k) {
      const int e = threadIdx.x + 256 * k, p_ = e / NB, a_ = e % NB;
      const bool in = k0 + p_ < hi;
      At[a_][p_] = (in && i0 + a_ < r1) ? av[k] : 0.0;
      Bt[p_][a_] = (in && c0 + a_ < w) ? bv[k] : 0.0;
    }
    __syncthreads();
    tile_mma64(At, Bt, acc, lane, wm, wn);
  }
  double* Pp = part + (size_t(u) * nspl + sp) * size_t(r1) * w;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = i0 + wm * 32 + i * 16 + (lane >> 4) + 4 * e;  // MFMA f64 output layout
        const int col = c0 + wn * 32 + j * 16 + (lane & 15);
        if (row < r1 && col < w) Pp[size_t(row) * w + col] = acc[i][j][e];
      }
}

__global__ void cv_reduce_kernel(const double* __restrict__ part, int64_t per, int nspl, int64_t total,
                                 double* __restrict__ CV) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < total; i += int64_t(gridDim.x) * 256) {
    const int64_t u = i / per, e = i % per;
    const double* pp = part + size_t(u) * nspl * per + e;
    double acc = 0.0;
    for (int sp = 0; sp < nspl; ++sp) acc += pp[size_t(sp) * per];
    CV[i] = acc;
  }
}

int cv_splits(int64_t s, int r1, int w, int nu) {
  const int tiles = ((r1 + NB - 1) / NB) * ((w + NB - 1) / NB);
  int n = 2048 / (tiles * nu);
  const int64_t slabs = (s + NB - 1) / NB;
  if (n > slabs) n = int(slabs);
  if (n > CV_SPLIT_MAX) n = CV_SPLIT_MAX;
  return n < 1 ? 1 : n;
}

__global__ void zero_ints_kernel(int* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}


// ---------------------------------------------------------------------------
// host-side planning
// ---------------------------------------------------------------------------
struct InferLayout {
  int rmax, uc, n_r;
  int64_t smax, dmax, m, lde, km1;
  size_t e_off, g_off, gram_off, gram_bytes;
  std::vector<size_t> grp_off;  // per group: start of its chunk storage
  size_t misc_off;
  size_t total;
};

// Per-group storage of one chunk of beta2 groups, at the group's own r; the
// groups have separate regions so that they can run concurrently.
struct ChunkBufs {
  GroupGeom geo;
  int64_t s, w, r1;
  double *Lq, *R, *R2, *Linv, *CV, *part, *V, *Xq, *XL;
  int* ufail;
};

ChunkBufs carve_chunk(Carver& cc, int r, int rmax, int64_t m, int64_t dmax, int uc, int n_pairs) {
  ChunkBufs b{};
  b.geo.r = r;
  b.geo.rmax = rmax;
  b.geo.s = nquad(r);
  b.geo.m = m;
  b.geo.dmax = dmax;
  b.s = b.geo.s;
  b.w = 2 * r + 1;
  b.r1 = r + 1;
  const int64_t nblk = (b.s + NB - 1) / NB;
  b.Lq = cc.take<double>(size_t(uc) * b.s * b.s);
  b.R = cc.take<double>(size_t(uc) * b.s * b.w);
  b.R2 = cc.take<double>(size_t(uc) * b.s * b.w);
  b.Linv = cc.take<double>(size_t(uc) * nblk * NB * NB);
  b.CV = cc.take<double>(size_t(uc) * b.r1 * b.w);
  b.part = cc.take<double>(size_t(uc) * CV_SPLIT_MAX * b.r1 * b.w);
  b.V = cc.take<double>(size_t(n_pairs) * b.s * r);
  b.Xq = cc.take<double>(size_t(n_pairs) * b.s * r);
  b.XL = cc.take<double>(size_t(n_pairs) * b.r1 * r);
  b.ufail = cc.take<int>(size_t(uc));
  return b;
}

// Every table the kernels read from host data (beta values, the pair -> beta2
// group map of every chunk) has a fixed place in the workspace, written once
// by infer_upload; infer_enqueue then issues kernels only, so a stream capture
// of it replays without host memory.
struct MiscPtrs {
  double* b2dev;  // distinct beta2 values (n_u <= n_pairs)
  int* pair_u;    // per chunk: pair -> u within the chunk, -1 outside
  int* border;    // per chunk: batch entry -> pair (pairs of the chunk, by u)
  int* ue0;       // per chunk: first batch entry of u
  int* ucnt;      // per chunk: batch entries of u
  double* b1dev;  // per pair
};

// erows: rows of the data matrix E (k - 1 for the discrete form, k for the
// continuous-time form)
InferLayout layout(int64_t k, int n_r, const int* r_list, int n_pairs, int64_t erows) {
  InferLayout L{};
  L.n_r = n_r;
  int rmax = 0;
  for (int g = 0; g < n_r; ++g) rmax = r_list[g] > rmax ? r_list[g] : rmax;
  L.rmax = rmax;
  L.uc = n_pairs < UCHUNK ? n_pairs : UCHUNK;
  L.smax = nquad(rmax);
  L.dmax = ncols(rmax);
  L.m = L.dmax + rmax;
  L.lde = (L.m + 1) / 2 * 2;
  L.km1 = erows;
  Carver c(nullptr, 0);
  c.take<double>(size_t(L.km1) * L.lde);
  L.e_off = 0;
  L.g_off = c.used;
  c.take<double>(size_t(L.m) * L.m);
  L.gram_off = (c.used + 255) & ~size_t(255);
  L.gram_bytes = gram_f64_workspace_internal(L.km1, L.m, 1);
  c.take<char>(L.gram_bytes);
  const int uc = L.uc;
  L.grp_off.resize(n_r);
  for (int g = 0; g < n_r; ++g) {
    L.grp_off[g] = (c.used + 255) & ~size_t(255);
    Carver cg(nullptr, 0);
    carve_chunk(cg, r_list[g], rmax, L.m, L.dmax, uc, n_pairs);
    c.take<char>(cg.used);
  }
  L.misc_off = (c.used + 255) & ~size_t(255);
  const int max_chunks = (n_pairs + uc - 1) / uc;
  c.take<double>(size_t(n_pairs));                    // distinct beta2
  c.take<int>(size_t(max_chunks) * n_pairs);          // pair -> u, per chunk
  c.take<int>(size_t(max_chunks) * n_pairs);          // batch entry -> pair, per chunk
  c.take<int>(size_t(max_chunks) * uc);               // first batch entry per u, per chunk
  c.take<int>(size_t(max_chunks) * uc);               // batch entries per u, per chunk
  c.take<double>(size_t(n_pairs));                    // beta1 per pair
  L.total = c.used;
  return L;
}

MiscPtrs misc_ptrs(const InferLayout& L, void* ws, int n_pairs) {
  Carver mc(static_cast<char*>(ws) + L.misc_off, L.total - L.misc_off);
  MiscPtrs m{};
  const int max_chunks = (n_pairs + L.uc - 1) / L.uc;
  m.b2dev = mc.take<double>(size_t(n_pairs));
  m.pair_u = mc.take<int>(size_t(max_chunks) * n_pairs);
  m.border = mc.take<int>(size_t(max_chunks) * n_pairs);
  m.ue0 = mc.take<int>(size_t(max_chunks) * L.uc);
  m.ucnt = mc.take<int>(size_t(max_chunks) * L.uc);
  m.b1dev = mc.take<double>(size_t(n_pairs));
  return m;
}

struct InferPlan {
  InferLayout L;
  int64_t k;
  double dt = 0.0;  // > 0: continuous-time form (derivative data at spacing dt)
  int n_r, n_pairs;
  std::vector<int> r_list;
  std::vector<double> beta1, b2u;  // per pair; distinct beta2 in first-appearance order
  std::vector<int> pu;             // n_chunks x n_pairs
  std::vector<int> border;         // n_chunks x n_pairs (the first nbc[c] entries used)
  std::vector<int> ue0, ucnt;      // n_chunks x uc
  std::vector<int> nbc, npu_max;   // per chunk: pairs, most pairs of one u
  int n_u, n_chunks;
  // With several reduced sizes, each group runs on a stream of its own
  // (forked from the caller's stream after the data Gram and joined back at
  // the end; a stream capture turns this into parallel graph branches).
  std::vector<hipStream_t> gst;
  std::vector<hipEvent_t> gev;
  hipEvent_t fork = nullptr;
  InferPlan() = default;
  InferPlan(const InferPlan&) = delete;
  InferPlan& operator=(const InferPlan&) = delete;
  ~InferPlan() {
    for (hipEvent_t x : gev) (void)hipEventDestroy(x);
    if (fork) (void)hipEventDestroy(fork);
  }
};

// Streams of the group fork: created once per host thread and device
// (default priority, non-blocking) and kept for the life of the process, so
// that a call neither pays for creating them nor shares them with a call on
// another host thread.  Events are per call.  Every such stream is also
// entered in a process-wide list, and an exit handler (registered after the
// HIP runtime has loaded, so it runs before the runtime's own teardown)
// destroys them: no stream of the library is left for the runtime to tear
// down at process exit, after profiling tools have finalized.
//
// A process has GPU_MAX_HW_QUEUES hardware queues (4 unless set), and streams
// beyond that share them: two groups whose streams land on one queue run one
// after the other (measured: r = 60 and r = 80 on one queue, eager sweep
// 74 ms).  So at most (queues - 1) group streams are used, the caller's
// stream keeping one queue: the largest groups get a stream each and the
// smallest groups share the last one.
std::mutex g_stream_mu;
std::vector<std::pair<int, hipStream_t>> g_all_streams;

void destroy_pool_streams() {
  std::lock_guard<std::mutex> lock(g_stream_mu);
  int cur = 0;
  const bool have_dev = hipGetDevice(&cur) == hipSuccess;
  for (auto& ds : g_all_streams) {
    if (hipSetDevice(ds.first) != hipSuccess) continue;
    (void)hipStreamSynchronize(ds.second);
    (void)hipStreamDestroy(ds.second);
  }
  g_all_streams.clear();
  if (have_dev) (void)hipSetDevice(cur);
}

// Up to `want` streams of the calling thread's pool on the current device,
// at most (hardware queues - 1); *got receives how many.
int pool_streams_impl(int want, std::vector<hipStream_t>*& out, int* got) {
  *got = 0;
  int hwq = 4;
  if (const char* e = std::getenv("GPU_MAX_HW_QUEUES")) {
    const int v = std::atoi(e);
    if (v >= 1) hwq = v;
  }
  const int ns = std::min(want, hwq - 1);
  if (ns < 1) return DOPINF_OK;
  int dev = 0;
  DOPINF_HIP(hipGetDevice(&dev));
  static thread_local std::vector<std::vector<hipStream_t>> pool;
  if (int(pool.size()) <= dev) pool.resize(dev + 1);
  std::vector<hipStream_t>& mine = pool[dev];
  while (int(mine.size()) < ns) {
    hipStream_t x = nullptr;
    DOPINF_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    mine.push_back(x);
    std::lock_guard<std::mutex> lock(g_stream_mu);
    static const bool registered = (std::atexit(destroy_pool_streams) == 0);
    (void)registered;
    g_all_streams.emplace_back(dev, x);
  }
  out = &mine;
  *got = ns;
  return DOPINF_OK;
}

int infer_streams(InferPlan& P) {
  if (P.n_r < 2 || !P.gst.empty()) return DOPINF_OK;
  std::vector<hipStream_t>* pool = nullptr;
  int ns = 0;
  const int rc = pool_streams_impl(P.n_r, pool, &ns);
  if (rc) return rc;
  if (ns < 2) return DOPINF_OK;  // no fork: the groups run on the caller's stream
  std::vector<hipStream_t>& mine = *pool;
  DOPINF_HIP(hipEventCreateWithFlags(&P.fork, hipEventDisableTiming));
  for (int g = 0; g < P.n_r; ++g) {
    // rank by decreasing r (ties: lower index first)
    int rank = 0;
    for (int q = 0; q < P.n_r; ++q) rank += (P.r_list[q] > P.r_list[g]) || (P.r_list[q] == P.r_list[g] && q < g);
    P.gst.push_back(mine[std::min(rank, ns - 1)]);
    hipEvent_t e = nullptr;
    DOPINF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    P.gev.push_back(e);
  }
  return DOPINF_OK;
}

// block-column widths (outer, inner) of the s x s Cholesky and of the
// triangular solves with its factor: the tuned values, else (256, none)
struct Kb {
  int64_t w, w2;
};
Kb chol_kb(int64_t s) {
  const int v = tune::get(DOPINF_TUNE_CHOL_KB, s);
  return Kb{v > 0 ? v : 4 * NB, tune::get(DOPINF_TUNE_CHOL_KB2, s)};
}
Kb trsm_kb(int64_t s) {
  const int v = tune::get(DOPINF_TUNE_TRSM_KB, s);
  return Kb{v > 0 ? v : 4 * NB, tune::get(DOPINF_TUNE_TRSM_KB2, s)};
}

int infer_plan(int64_t k, int64_t ldqh, int n_r, const int* r_list_h, int n_pairs, const double* beta1_h,
               const double* beta2_h, size_t ws_bytes, const void* ws, InferPlan& P, double dt = 0.0) {
  DOPINF_REQUIRE(r_list_h && beta1_h && beta2_h, "NULL argument");
  DOPINF_REQUIRE(k >= 2 && ldqh >= k, "need k >= 2 and ldqh >= k");
  DOPINF_REQUIRE(n_r >= 1 && n_pairs >= 1, "need n_r >= 1 and n_pairs >= 1");
  for (int g = 0; g < n_r; ++g) DOPINF_REQUIRE(r_list_h[g] >= 1 && r_list_h[g] <= 512, "r must be in [1, 512]");
  for (int p = 0; p < n_pairs; ++p)
    DOPINF_REQUIRE(beta1_h[p] >= 0.0 && beta2_h[p] >= 0.0, "regularization parameters must be >= 0");
  if (dt != 0.0) DOPINF_REQUIRE(dt > 0.0 && std::isfinite(dt) && k >= 3, "continuous form: need dt > 0 and k >= 3");
  P.dt = dt;
  P.L = layout(k, n_r, r_list_h, n_pairs, dt > 0.0 ? k : k - 1);
  if (!ws || ws_bytes < P.L.total)
    return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", P.L.total, ws_bytes);
  int dev = 0, maxlds = 0;
  DOPINF_HIP(hipGetDevice(&dev));
  DOPINF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  {
    const size_t need = size_t(P.L.rmax + 1) * (2 * P.L.rmax + 1) * sizeof(double) + 1024;
    DOPINF_REQUIRE(need <= size_t(maxlds), "r too large for the per-pair LDS solve");
    if (need > 65536)
      DOPINF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(pair_solve_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(need)));
  }
  P.k = k;
  P.n_r = n_r;
  P.n_pairs = n_pairs;
  P.r_list.assign(r_list_h, r_list_h + n_r);
  P.beta1.assign(beta1_h, beta1_h + n_pairs);
  // distinct beta2 values (exact equality), in first-appearance order
  std::vector<int> pair_uid(n_pairs);
  P.b2u.clear();
  for (int p = 0; p < n_pairs; ++p) {
    int id = -1;
    for (size_t q = 0; q < P.b2u.size(); ++q)
      if (P.b2u[q] == beta2_h[p]) {
        id = int(q);
        break;
      }
    if (id < 0) {
      id = int(P.b2u.size());
      P.b2u.push_back(beta2_h[p]);
    }
    pair_uid[p] = id;
  }
  P.n_u = int(P.b2u.size());
  const int uc = P.L.uc;
  P.n_chunks = (P.n_u + uc - 1) / uc;
  P.pu.assign(size_t(P.n_chunks) * n_pairs, -1);
  P.border.assign(size_t(P.n_chunks) * n_pairs, 0);
  P.ue0.assign(size_t(P.n_chunks) * uc, 0);
  P.ucnt.assign(size_t(P.n_chunks) * uc, 0);
  P.nbc.assign(P.n_chunks, 0);
  P.npu_max.assign(P.n_chunks, 0);
  for (int c = 0; c < P.n_chunks; ++c) {
    const int u0 = c * uc;
    for (int p = 0; p < n_pairs; ++p)
      if (pair_uid[p] >= u0 && pair_uid[p] < u0 + uc) P.pu[size_t(c) * n_pairs + p] = pair_uid[p] - u0;
    // batch order: by u, then by pair, so that entries sharing a factor are adjacent
    int nb = 0;
    for (int u = 0; u < uc; ++u) {
      P.ue0[size_t(c) * uc + u] = nb;
      for (int p = 0; p < n_pairs; ++p)
        if (P.pu[size_t(c) * n_pairs + p] == u) P.border[size_t(c) * n_pairs + nb++] = p;
      const int cnt = nb - P.ue0[size_t(c) * uc + u];
      P.ucnt[size_t(c) * uc + u] = cnt;
      if (cnt > P.npu_max[c]) P.npu_max[c] = cnt;
    }
    P.nbc[c] = nb;
  }
  return DOPINF_OK;
}

// Host tables into the workspace.  hipMemcpyAsync from pageable memory
// returns once the source has been staged, so the plan may be dropped after.
int infer_upload(hipStream_t st, const InferPlan& P, void* ws) {
  const MiscPtrs m = misc_ptrs(P.L, ws, P.n_pairs);
  DOPINF_HIP(hipMemcpyAsync(m.b2dev, P.b2u.data(), sizeof(double) * P.n_u, hipMemcpyHostToDevice, st));
  DOPINF_HIP(hipMemcpyAsync(m.pair_u, P.pu.data(), sizeof(int) * P.pu.size(), hipMemcpyHostToDevice, st));
  DOPINF_HIP(hipMemcpyAsync(m.border, P.border.data(), sizeof(int) * P.border.size(), hipMemcpyHostToDevice, st));
  DOPINF_HIP(hipMemcpyAsync(m.ue0, P.ue0.data(), sizeof(int) * P.ue0.size(), hipMemcpyHostToDevice, st));
  DOPINF_HIP(hipMemcpyAsync(m.ucnt, P.ucnt.data(), sizeof(int) * P.ucnt.size(), hipMemcpyHostToDevice, st));
  DOPINF_HIP(hipMemcpyAsync(m.b1dev, P.beta1.data(), sizeof(double) * P.n_pairs, hipMemcpyHostToDevice, st));
  return DOPINF_OK;
}

// E and its Gram G_E
int infer_gram(hipStream_t st, const InferPlan& P, const double* Qhat, int64_t ldqh, void* ws) {
  const InferLayout& L = P.L;
  char* base = static_cast<char*>(ws);
  double* E = reinterpret_cast<double*>(base + L.e_off);
  double* GE = reinterpret_cast<double*>(base + L.g_off);
  dim3 grid(unsigned((L.km1 + 255) / 256), unsigned(L.m));
  assemble_kernel<<<grid, 256, 0, st>>>(Qhat, ldqh, P.k, L.rmax, E, L.lde, P.dt);
  DOPINF_LAUNCHED();
  return gram_f64_internal(st, E, L.km1, L.m, L.lde, nullptr, nullptr, 0, nullptr, GE, L.m, base + L.gram_off,
                           L.gram_bytes);
}

ChunkBufs chunk_bufs(const InferPlan& P, int g, void* ws) {
  const InferLayout& L = P.L;
  Carver cc(static_cast<char*>(ws) + L.grp_off[g], ~size_t(0));
  return carve_chunk(cc, P.r_list[g], L.rmax, L.m, L.dmax, L.uc, P.n_pairs);
}

// the chunk's beta2 groups: G_qq + beta2 I gathered and factored with block
// columns of width kb
int chunk_factor(hipStream_t st, const InferPlan& P, const ChunkBufs& b, int c, int nu, Kb kb, void* ws) {
  const MiscPtrs m = misc_ptrs(P.L, ws, P.n_pairs);
  const double* GE = reinterpret_cast<const double*>(static_cast<char*>(ws) + P.L.g_off);
  zero_ints_kernel<<<1, 256, 0, st>>>(b.ufail, P.L.uc);
  DOPINF_LAUNCHED();
  dim3 grid(unsigned((b.s + 255) / 256 > 64 ? 64 : (b.s + 255) / 256), unsigned(b.s));
  gather_qq_kernel<<<grid, 256, 0, st>>>(GE, b.geo, m.b2dev + size_t(c) * P.L.uc, nu, b.Lq, b.R);
  DOPINF_LAUNCHED();
  return cholesky_run(st, b.Lq, b.s, b.Linv, b.ufail, nu, kb.w, kb.w2);
}

// [W | y] = L^{-1} [G_ql | B_q], CV = W^T [W | y], and per pair the Schur
// complement solve for X_l (linear and constant columns of O, and XL)
int chunk_linear(hipStream_t st, const InferPlan& P, const ChunkBufs& b, int g, int c, int nu, Kb kb, double* O,
                 int* status, void* ws) {
  const MiscPtrs m = misc_ptrs(P.L, ws, P.n_pairs);
  const double* GE = reinterpret_cast<const double*>(static_cast<char*>(ws) + P.L.g_off);
  const int64_t s = b.s, w = b.w, r1 = b.r1;
  int rc = trsm_run(st, false, b.Lq, s, b.Linv, b.R, b.R2, RhsMap{nullptr, nullptr, w}, w, nu, kb.w, kb.w2);
  if (rc) return rc;
  {
    const int nspl = cv_splits(s, int(r1), int(w), nu);
    const unsigned tiles = unsigned(((r1 + NB - 1) / NB) * ((w + NB - 1) / NB));
    cv_partial_kernel<<<dim3(tiles, unsigned(nspl), unsigned(nu)), 256, 0, st>>>(b.R2, s, int(r1), int(w), nspl,
                                                                               b.part);
    DOPINF_LAUNCHED();
    const int64_t total = int64_t(nu) * r1 * w;
    cv_reduce_kernel<<<unsigned((total + 255) / 256), 256, 0, st>>>(b.part, r1 * w, nspl, total, b.CV);
    DOPINF_LAUNCHED();
  }
  PairArgs pa{};
  pa.GE = GE;
  pa.geo = b.geo;
  pa.CV = b.CV;
  pa.ufail = b.ufail;
  pa.pair_u = m.pair_u + size_t(c) * P.n_pairs;
  pa.beta1 = m.b1dev;
  pa.O = O + dopinf_operator_offset(P.n_r, P.r_list.data(), P.n_pairs, g * P.n_pairs);
  pa.status = status + g * P.n_pairs;
  pa.n_pairs = P.n_pairs;
  pa.XL = b.XL;
  const size_t smem = size_t(r1) * (r1 + b.geo.r) * sizeof(double);
  pair_solve_kernel<<<P.n_pairs, 256, smem, st>>>(pa);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

QuadArgs quad_args(const InferPlan& P, const ChunkBufs& b, int g, int c, double* O, void* ws) {
  const MiscPtrs m = misc_ptrs(P.L, ws, P.n_pairs);
  QuadArgs qa{};
  qa.R2 = b.R2;
  qa.XL = b.XL;
  qa.border = m.border + size_t(c) * P.n_pairs;
  qa.pair_u = m.pair_u + size_t(c) * P.n_pairs;
  qa.V = b.V;
  qa.O = O ? O + dopinf_operator_offset(P.n_r, P.r_list.data(), P.n_pairs, g * P.n_pairs) : nullptr;
  qa.s = b.s;
  qa.r = b.geo.r;
  return qa;
}

// v = y - W X_l per pair, then L^T X_q = v with the pairs of each beta2 group
// side by side as one right-hand side; the solve's leaves also write X_q into
// the quadratic columns of O (O == nullptr: X_q only)
int chunk_quad_solve(hipStream_t st, const InferPlan& P, const ChunkBufs& b, int g, int c, int nu, Kb kb,
                     double* O, void* ws) {
  const MiscPtrs m = misc_ptrs(P.L, ws, P.n_pairs);
  const QuadArgs qa = quad_args(P, b, g, c, O, ws);
  vq_kernel<<<dim3(unsigned((b.s + NB - 1) / NB), unsigned(P.nbc[c]), unsigned((b.geo.r + 127) / 128)), 256, 0, st>>>(
      qa);
  DOPINF_LAUNCHED();
  const RhsMap rm{m.ue0 + size_t(c) * P.L.uc, m.ucnt + size_t(c) * P.L.uc, b.geo.r};
  const OWrite ow{qa.border, qa.O, ncols(b.geo.r), b.geo.r};
  return trsm_run(st, true, b.Lq, b.s, b.Linv, b.V, b.Xq, rm, int64_t(P.npu_max[c]) * b.geo.r, nu, kb.w, kb.w2,
                  ow);
}

int infer_enqueue(hipStream_t st, const InferPlan& P, const double* Qhat, int64_t ldqh, double* O, int* status,
                  void* ws) {
  int rc = infer_gram(st, P, Qhat, ldqh, ws);
  if (rc) return rc;
  const int uc = P.L.uc;
  const bool forked = !P.gst.empty();
  if (forked) DOPINF_HIP(hipEventRecord(P.fork, st));
  // Order of issue.  Eagerly, smallest r first: issued largest first, the
  // smaller groups started only once the largest had drained part of its
  // queue.  Under capture, largest r first: a graph's branches start in
  // capture order, and the largest group is the longest chain.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  DOPINF_HIP(hipStreamIsCapturing(st, &cap));
  const bool largest_first = cap == hipStreamCaptureStatusActive;
  for (int gi0 = 0; gi0 < P.n_r && !rc; ++gi0) {
    const int gi = largest_first ? P.n_r - 1 - gi0 : gi0;
    int g = gi;
    if (forked) {  // g: the group of rank gi in increasing r
      g = 0;
      for (int h = 0; h < P.n_r; ++h) {
        int rank = 0;
        for (int q = 0; q < P.n_r; ++q) rank += (P.r_list[q] < P.r_list[h]) || (P.r_list[q] == P.r_list[h] && q < h);
        if (rank == gi) g = h;
      }
    }
    hipStream_t sg = forked ? P.gst[g] : st;
    if (forked) DOPINF_HIP(hipStreamWaitEvent(sg, P.fork, 0));
    const ChunkBufs b = chunk_bufs(P, g, ws);
    const Kb kc = chol_kb(b.s), kt = trsm_kb(b.s);
    for (int c = 0; c < P.n_chunks && !rc; ++c) {
      const int nu = (P.n_u - c * uc) < uc ? (P.n_u - c * uc) : uc;
      rc = chunk_factor(sg, P, b, c, nu, kc, ws);
      if (!rc) rc = chunk_linear(sg, P, b, g, c, nu, kt, O, status, ws);
      if (rc || P.nbc[c] == 0) continue;
      rc = chunk_quad_solve(sg, P, b, g, c, nu, kt, O, ws);
    }
    if (forked) {
      // join even after an error, so that no forked work is left outside
      const hipError_t e1 = hipEventRecord(P.gev[g], sg);
      const hipError_t e2 = hipStreamWaitEvent(st, P.gev[g], 0);
      if (!rc && (e1 != hipSuccess || e2 != hipSuccess)) rc = fail(DOPINF_E_HIP, "joining the group streams failed");
    }
  }
  return rc;
}

}  // namespace

// The pool streams for other grouped launches of the library (the rollout
// groups): up to `want` of them into out[]; returns how many (0 on error,
// with the error message set).
int pool_streams(int want, hipStream_t* out) {
  std::vector<hipStream_t>* pool = nullptr;
  int ns = 0;
  if (pool_streams_impl(want, pool, &ns) != DOPINF_OK) return 0;
  for (int i = 0; i < ns; ++i) out[i] = (*pool)[i];
  return ns;
}

// Candidate block-column widths (outer, inner; inner 0: one level), for the
// beta2-group Cholesky and for the triangular solves with its factor.
constexpr int kKbCand[][2] = {{64, 0},    {128, 0},    {256, 0},    {512, 0},
                              {512, 128}, {1024, 128}, {1024, 256}, {2048, 256}};
constexpr int kNumKbCand = 8;

// Minimum over two timed runs of fn (after one warm-up run) on stream st.
template <class F>
int time_min(hipStream_t st, hipEvent_t e0, hipEvent_t e1, F&& fn, float& out) {
  out = -1.f;
  for (int rep = 0; rep < 3; ++rep) {
    DOPINF_HIP(hipEventRecord(e0, st));
    const int rc = fn();
    if (rc) return rc;
    DOPINF_HIP(hipEventRecord(e1, st));
    DOPINF_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    DOPINF_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (rep > 0 && (out < 0.f || ms < out)) out = ms;
  }
  return DOPINF_OK;
}

// For every group, on the first beta2 chunk with the sweep's own data: time
// the factorization (gather + Cholesky) at every width and keep the fastest;
// then, with that factor, time the per-pair back substitution (v rebuilt
// every run, since the solve consumes it) at every depth and keep the
// fastest.  The stored values are then used by the complete infer that ends
// the call.
int infer_autotune(hipStream_t st, const InferPlan& P, const double* Qhat, int64_t ldqh, double* O, int* status,
                   void* ws, float* times_h) {
  int rc = infer_upload(st, P, ws);
  if (!rc) rc = infer_gram(st, P, Qhat, ldqh, ws);
  if (rc) return rc;
  hipEvent_t e0, e1;
  DOPINF_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(DOPINF_E_HIP, "hipEventCreate failed");
  }
  const int uc = P.L.uc;
  const int nu = P.n_u < uc ? P.n_u : uc;
  for (int g = 0; g < P.n_r && !rc; ++g) {
    const ChunkBufs b = chunk_bufs(P, g, ws);
    float* tg = times_h ? times_h + size_t(g) * 2 * kNumKbCand : nullptr;
    if (tg)
      for (int ci = 0; ci < 2 * kNumKbCand; ++ci) tg[ci] = 0.f;
    // widths already in a persisted table (DOPINF_TUNE_CACHE) are not timed again
    if (tune::persisted() && tune::get(DOPINF_TUNE_CHOL_KB, b.s) > 0 && tune::get(DOPINF_TUNE_TRSM_KB, b.s) > 0)
      continue;
    int best = -1;
    float best_t = 0.f;
    for (int ci = 0; ci < kNumKbCand && !rc; ++ci) {
      float t = 0.f;
      const Kb kb{kKbCand[ci][0], kKbCand[ci][1]};
      rc = time_min(st, e0, e1, [&] { return chunk_factor(st, P, b, 0, nu, kb, ws); }, t);
      if (tg) tg[ci] = t;
      if (!rc && (best < 0 || t < best_t)) {
        best = ci;
        best_t = t;
      }
    }
    if (rc) break;
    tune::set(DOPINF_TUNE_CHOL_KB, b.s, kKbCand[best][0]);
    tune::set(DOPINF_TUNE_CHOL_KB2, b.s, kKbCand[best][1]);
    rc = chunk_factor(st, P, b, 0, nu, chol_kb(b.s), ws);
    if (!rc) rc = chunk_linear(st, P, b, g, 0, nu, trsm_kb(b.s), O, status, ws);
    if (rc || P.nbc[0] == 0) continue;
    best = -1;
    for (int ci = 0; ci < kNumKbCand && !rc; ++ci) {
      float t = 0.f;
      const Kb kb{kKbCand[ci][0], kKbCand[ci][1]};
      rc = time_min(st, e0, e1, [&] { return chunk_quad_solve(st, P, b, g, 0, nu, kb, nullptr, ws); }, t);
      if (tg) tg[kNumKbCand + ci] = t;
      if (!rc && (best < 0 || t < best_t)) {
        best = ci;
        best_t = t;
      }
    }
    if (!rc) {
      tune::set(DOPINF_TUNE_TRSM_KB, b.s, kKbCand[best][0]);
      tune::set(DOPINF_TUNE_TRSM_KB2, b.s, kKbCand[best][1]);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!rc) rc = infer_enqueue(st, P, Qhat, ldqh, O, status, ws);
  return rc;
}

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
  return layout(k, n_r, r_list_h, n_pairs, k - 1).total;
}

extern "C" int dopinf_infer(void* stream, const double* Qhat, int64_t ldqh, int64_t k, int n_r, const int* r_list_h,
                            int n_pairs, const double* beta1_h, const double* beta2_h, double* O, int* status,
                            void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(Qhat && O && status, "NULL argument");
  InferPlan P;
  int rc = infer_plan(k, ldqh, n_r, r_list_h, n_pairs, beta1_h, beta2_h, ws_bytes, ws, P);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = infer_upload(st, P, ws);
  if (!rc) rc = infer_streams(P);
  if (rc) return rc;
  return infer_enqueue(st, P, Qhat, ldqh, O, status, ws);
}

extern "C" size_t dopinf_infer_continuous_workspace(int64_t k, int n_r, const int* r_list_h, int n_pairs) {
  if (k < 3 || n_r <= 0 || !r_list_h || n_pairs <= 0) return 0;
  return layout(k, n_r, r_list_h, n_pairs, k).total;
}

extern "C" int dopinf_infer_continuous(void* stream, const double* Qhat, int64_t ldqh, int64_t k, double dt, int n_r,
                                       const int* r_list_h, int n_pairs, const double* beta1_h,
                                       const double* beta2_h, double* O, int* status, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(Qhat && O && status, "NULL argument");
  DOPINF_REQUIRE(dt > 0.0 && std::isfinite(dt), "dt must be finite and > 0");
  InferPlan P;
  int rc = infer_plan(k, ldqh, n_r, r_list_h, n_pairs, beta1_h, beta2_h, ws_bytes, ws, P, dt);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = infer_upload(st, P, ws);
  if (!rc) rc = infer_streams(P);
  if (rc) return rc;
  return infer_enqueue(st, P, Qhat, ldqh, O, status, ws);
}

extern "C" int dopinf_autotune_infer(void* stream, const double* Qhat, int64_t ldqh, int64_t k, int n_r,
                                     const int* r_list_h, int n_pairs, const double* beta1_h, const double* beta2_h,
                                     double* O, int* status, void* ws, size_t ws_bytes, float* times_h) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(Qhat && O && status, "NULL argument");
  InferPlan P;
  int rc = infer_plan(k, ldqh, n_r, r_list_h, n_pairs, beta1_h, beta2_h, ws_bytes, ws, P);
  if (rc) return rc;
  return infer_autotune(static_cast<hipStream_t>(stream), P, Qhat, ldqh, O, status, ws, times_h);
}

extern "C" int dopinf_autotune_candidates(int param, int* values_h, int max_values) {
  DOPINF_REQUIRE(param == DOPINF_TUNE_CHOL_KB || param == DOPINF_TUNE_TRSM_KB || param == DOPINF_TUNE_CHOL_KB2 ||
                     param == DOPINF_TUNE_TRSM_KB2,
                 "unknown tuning parameter %d", param);
  const int col = (param == DOPINF_TUNE_CHOL_KB2 || param == DOPINF_TUNE_TRSM_KB2) ? 1 : 0;
  for (int i = 0; i < kNumKbCand && i < max_values && values_h; ++i) values_h[i] = kKbCand[i][col];
  return kNumKbCand;
}

// ---------------------------------------------------------------------------
// the sweep (infer + rollout) as one instantiated graph
// ---------------------------------------------------------------------------
struct dopinf_sweep_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" size_t dopinf_sweep_workspace(int64_t k, int n_r, const int* r_list_h, int n_pairs) {
  const size_t a = dopinf_infer_workspace(k, n_r, r_list_h, n_pairs);
  const size_t b = dopinf_rollout_workspace(n_r, r_list_h, n_pairs, k);
  if (!a || !b) return 0;
  return round_up(a, 256) + b;
}

extern "C" int dopinf_sweep_create(void* stream, const double* Qhat, int64_t ldqh, int64_t k, int n_r,
                                   const int* r_list_h, int n_pairs, const double* beta1_h, const double* beta2_h,
                                   int n_states, double max_growth, unsigned flags, double* O, int* status,
                                   double* train_err, double* growth, int* outcome, int* best, void* ws,
                                   size_t ws_bytes, dopinf_sweep_t* sweep_out) {
  DOPINF_REQUIRE(sweep_out, "NULL sweep_out");
  *sweep_out = nullptr;
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(stream, "the null stream cannot be captured; pass a stream created by the caller");
  DOPINF_REQUIRE(Qhat && O && status && train_err && growth && outcome && best, "NULL argument");
  DOPINF_REQUIRE((flags & ~DOPINF_SWEEP_AUTOTUNE) == 0, "unknown flag bits");
  DOPINF_REQUIRE(n_states >= 1 && max_growth > 0.0, "need n_states >= 1 and max_growth > 0");
  const size_t need = dopinf_sweep_workspace(k, n_r, r_list_h, n_pairs);
  DOPINF_REQUIRE(need > 0, "invalid sizes");
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  const size_t ia = round_up(dopinf_infer_workspace(k, n_r, r_list_h, n_pairs), 256);
  char* wsi = static_cast<char*>(ws);
  char* wsr = wsi + ia;
  InferPlan P;
  int rc = infer_plan(k, ldqh, n_r, r_list_h, n_pairs, beta1_h, beta2_h, ia, wsi, P);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (flags & DOPINF_SWEEP_AUTOTUNE) {
    rc = infer_autotune(st, P, Qhat, ldqh, O, status, wsi, nullptr);
    if (rc) return rc;
  }
  rc = infer_upload(st, P, wsi);
  if (!rc) rc = infer_streams(P);
  if (rc) return rc;
  DOPINF_HIP(hipStreamSynchronize(st));
  DOPINF_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
  rc = infer_enqueue(st, P, Qhat, ldqh, O, status, wsi);
  if (!rc)
    rc = dopinf_rollout(stream, n_r, r_list_h, n_pairs, O, Qhat, ldqh, nullptr, k, n_states, max_growth,
                        DOPINF_ROLLOUT_ONE_WG,
                        status, nullptr, train_err, growth, outcome, best, wsr, ws_bytes - ia);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(st, &graph);
  if (rc || ec != hipSuccess) {
    if (ec == hipSuccess && graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return rc ? rc : fail(DOPINF_E_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(DOPINF_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
  }
  *sweep_out = new dopinf_sweep_s{graph, exec};
  return DOPINF_OK;
}

extern "C" int dopinf_sweep_launch(dopinf_sweep_t sweep, void* stream) {
  DOPINF_REQUIRE(sweep && sweep->exec, "NULL sweep");
  DOPINF_HIP(hipGraphLaunch(sweep->exec, static_cast<hipStream_t>(stream)));
  return DOPINF_OK;
}

extern "C" int dopinf_sweep_destroy(dopinf_sweep_t sweep) {
  if (!sweep) return DOPINF_OK;
  const hipError_t a = sweep->exec ? hipGraphExecDestroy(sweep->exec) : hipSuccess;
  const hipError_t b = sweep->graph ? hipGraphDestroy(sweep->graph) : hipSuccess;
  delete sweep;
  if (a != hipSuccess || b != hipSuccess) return fail(DOPINF_E_HIP, "destroying the sweep graph failed");
  return DOPINF_OK;
}
