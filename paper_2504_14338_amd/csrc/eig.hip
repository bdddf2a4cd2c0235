// Step III of dOpInf (arXiv:2504.14338, Sec. 3.4): eigenpairs of the Gram
// matrix D (Eq. (6)), the retained-energy rank (Eq. (9)) and the reduced data
// Qhat = Lambda_r^{1/2} U_r^T = T_r^T D (Eq. (8)) without the POD basis.
//
// Pipeline on one GPU (all float64):
//  1. Householder reduction D = P T P^T to symmetric tridiagonal T, as ONE
//     cooperative persistent kernel: workgroup g owns rows g, g+P, g+2P, ...
//     of the trailing matrix (kept in LDS when they fit, else in the
//     workspace).  Per column j: the owner of row j forms the reflector, a
//     device-wide barrier publishes it, every workgroup forms its entries of
//     p = tau * A v plus a partial v^T p, a second barrier, then every
//     workgroup applies the rank-2 update A -= v w^T + w v^T to its rows.
//     Orders up to 128 are reduced by one workgroup with the matrix in LDS.
//  2. All k eigenvalues of T by multisection: one wave per eigenvalue, the
//     64 lanes evaluate Sturm counts at 64 interior points per round.
//  3. The top r eigenvectors of T by inverse iteration with partial-pivoting
//     LU of T - lambda I (one wave per cluster, factors in LDS).  As in
//     LAPACK's inverse-iteration routine xSTEIN, neighbouring eigenvalues
//     closer than a separation tolerance form a cluster whose vectors are
//     orthogonalized (modified Gram-Schmidt) against the cluster's earlier
//     vectors inside every iteration.  Vectors computed one by one lose
//     orthogonality like u ||T|| / gap; the tolerance 1e-5 ||T|| keeps that
//     loss below ~1e-11 between clusters (xSTEIN's more conservative 1e-3
//     ||T|| chains dozens of well-separated eigenvalues of a decaying
//     spectrum into one cluster, which one wave then has to walk alone).
//  4. Back-transformation u = P z (reflectors applied in reverse order), one
//     workgroup per vector with z in LDS.
//  5. Sign rule and Qhat / T_r formation.
#include "common.hpp"
#include "xwg_sync.hpp"

namespace dopinf {
namespace {

constexpr int TNT = 256;            // threads of the tridiagonalization kernel
constexpr int TCH = 8;              // rows reduced together in phase 2

using xwg::drain_then_sync;
using xwg::ld_dev;
using xwg::st_dev;
using xwg::wait_ge;

__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks, unsigned& gen, int* abort_flag) {
  return xwg::team_barrier(bar, nblocks, gen, abort_flag);
}

__global__ void zero_words_kernel(unsigned* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// 1. tridiagonalization
// ---------------------------------------------------------------------------
struct TridArgs {
  const double* D;  // input, ldd
  int64_t ldd;
  double* A;        // workspace k x k: rows owned in global mode; row j = v_j
  int64_t k;
  int P;
  int in_lds;
  int rows_max;     // max rows owned by one workgroup
  double* d;        // k diagonal
  double* e;        // k-1 off-diagonal
  double* tau;      // k
  double* p;        // 2 x k (double-buffered by column parity)
  double* part;     // 2 x P
  unsigned* bar;    // barrier counter
  unsigned* vflag;  // number of published reflectors
  int* abort_flag;
};

// Householder reflector of row j (owned by this workgroup): publishes v_j
// (row j of A, v_j[j+1] = 1), tau_j, d_j, e_j, then raises vflag to j+1.
__device__ void make_reflector(const TridArgs& a, double* row, int64_t j, double* red) {
  const int64_t k = a.k;
  const int tid = threadIdx.x;
  double ss = 0.0;
  for (int64_t l = j + 2 + tid; l < k; l += TNT) ss += row[l] * row[l];
  ss = block_sum<TNT>(ss, red);
  const double alpha = row[j + 1];
  double beta, tj, scal;
  if (ss == 0.0) {
    beta = alpha;
    tj = 0.0;
    scal = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + ss), alpha);
    tj = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
  const double dj = row[j];
  __syncthreads();  // row may alias v_j's storage: everything read before it is overwritten
  double* vout = a.A + j * k;
  for (int64_t l = j + 2 + tid; l < k; l += TNT) st_dev(vout + l, (tj == 0.0) ? 0.0 : row[l] * scal);
  if (tid == 0) {
    st_dev(vout + j + 1, 1.0);
    st_dev(a.tau + j, tj);
    a.d[j] = dj;
    a.e[j] = beta;
  }
  drain_then_sync();
  if (tid == 0) __hip_atomic_store(a.vflag, unsigned(j + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(TNT) void sytrd_kernel(TridArgs a) {
  extern __shared__ double lds_rows[];
  __shared__ double red[TNT / 64][TCH];
  __shared__ double bc[4];
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t k = a.k;
  const int P = a.P;
  unsigned gen = 0;

  auto row_ptr = [&](int q) -> double* {
    const int64_t i = g + int64_t(q) * P;
    return a.in_lds ? (lds_rows + int64_t(q) * k) : (a.A + i * k);
  };
  const int nown = int((k - g + P - 1) / P) > 0 ? int((k - g + P - 1) / P) : 0;

  for (int q = 0; q < nown; ++q) {  // load owned rows of D
    const int64_t i = g + int64_t(q) * P;
    double* dst = row_ptr(q);
    for (int64_t l = tid; l < k; l += TNT) dst[l] = a.D[i * a.ldd + l];
  }
  __syncthreads();
  if (k >= 2 && g == 0) make_reflector(a, row_ptr(0), 0, &red[0][0]);

  for (int64_t j = 0; j + 1 < k; ++j) {
    if (!wait_ge(a.vflag, unsigned(j + 1), a.abort_flag)) return;  // v_j published
    const double tj = ld_dev(a.tau + j);
    const double* v = a.A + j * k;
    const int par = int(j & 1);
    double* pj = a.p + par * k;
    double* partj = a.part + par * P;
    const int q0 = int((j + 1 - g + P - 1) / P) > 0 ? int((j + 1 - g + P - 1) / P) : 0;  // first owned row > j
    const bool owns_next = (j + 2 < k) && ((j + 1) % P == g);
    if (tj == 0.0) {  // H_j = I: nothing to update.  The barrier keeps every
      // workgroup within one column of the others, which the double-buffered
      // p / partial sums rely on.
      if (!grid_barrier(a.bar, P, gen, a.abort_flag)) return;
      if (owns_next) make_reflector(a, row_ptr(int((j + 1) / P)), j + 1, &red[0][0]);
      continue;
    }
    // ---- phase 2: p_i = tau * A[i, j+1:] . v[j+1:] for owned rows i > j --
    double mypart = 0.0;
    for (int qb = q0; qb < nown; qb += TCH) {
      const int nq = min(TCH, nown - qb);
      double acc[TCH];
#pragma unroll
      for (int u = 0; u < TCH; ++u) acc[u] = 0.0;
      for (int64_t l = j + 1 + tid; l < k; l += TNT) {
        const double vl = ld_dev(v + l);
#pragma unroll
        for (int u = 0; u < TCH; ++u)
          if (u < nq) acc[u] += row_ptr(qb + u)[l] * vl;
      }
#pragma unroll
      for (int u = 0; u < TCH; ++u) acc[u] = wave_sum(acc[u]);
      __syncthreads();
      if ((tid & 63) == 0) {
#pragma unroll
        for (int u = 0; u < TCH; ++u) red[tid >> 6][u] = acc[u];
      }
      __syncthreads();
      if (tid == 0) {
        for (int u = 0; u < nq; ++u) {
          double sacc = 0.0;
#pragma unroll
          for (int ww = 0; ww < TNT / 64; ++ww) sacc += red[ww][u];
          const int64_t i = g + int64_t(qb + u) * P;
          const double pi = tj * sacc;
          st_dev(pj + i, pi);
          mypart += ld_dev(v + i) * pi;
        }
      }
    }
    if (tid == 0) st_dev(partj + g, mypart);
    if (!grid_barrier(a.bar, P, gen, a.abort_flag)) return;  // p complete

    // ---- K = tau/2 * v^T p, partial sums reduced in a fixed order ----------
    {
      double s = 0.0;
      for (int q = tid; q < P; q += TNT) s += ld_dev(partj + q);
      s = block_sum<TNT>(s, &red[0][0]);
      if (tid == 0) bc[0] = 0.5 * tj * s;
      __syncthreads();
    }
    const double K = bc[0];
    // ---- phase 3: rank-2 update; the next reflector's row goes first ------
    auto update_row = [&](int q) {
      const int64_t i = g + int64_t(q) * P;
      double* row = row_ptr(q);
      const double vi = ld_dev(v + i);
      const double wi = ld_dev(pj + i) - K * vi;
      for (int64_t l = j + 1 + tid; l < k; l += TNT) {
        const double vl = ld_dev(v + l);
        const double wl = ld_dev(pj + l) - K * vl;
        row[l] -= vi * wl + wi * vl;
      }
    };
    int qn = -1;
    if (owns_next) {
      qn = int((j + 1) / P);
      update_row(qn);
      __syncthreads();
      make_reflector(a, row_ptr(qn), j + 1, &red[0][0]);
    }
    for (int q = q0; q < nown; ++q)
      if (q != qn) update_row(q);
    __syncthreads();
  }
  if (k >= 1 && (k - 1) % P == g) {
    const double* row = row_ptr(int((k - 1) / P));
    if (tid == 0) {
      a.d[k - 1] = row[k - 1];
      a.tau[k - 1] = 0.0;
    }
  }
}

// Same reduction with the owned rows in LDS and each thread's slice of v_j
// and w_j = p_j - K v_j held in registers for the whole column: v and p are
// read from global memory once per column (one parallel round of loads each)
// instead of once per owned row, and the owned rows' v_i, p_i sit in LDS.
// Thread t handles the columns l = j + 1 + t + TNT m, m < NM (k <= NM TNT).
template <int NM>
__global__ __launch_bounds__(TNT) void sytrd_reg_kernel(TridArgs a) {
  extern __shared__ double lds_rows[];
  __shared__ double red[TNT / 64][TCH];
  __shared__ double bc[4];
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t k = a.k;
  const int P = a.P;
  unsigned gen = 0;
  double* vown = lds_rows + int64_t(a.rows_max) * k;   // v_i of owned rows
  double* pown = vown + a.rows_max;                    // p_i of owned rows

  auto row_ptr = [&](int q) -> double* { return lds_rows + int64_t(q) * k; };
  const int nown = int((k - g + P - 1) / P) > 0 ? int((k - g + P - 1) / P) : 0;

  for (int q = 0; q < nown; ++q) {
    const int64_t i = g + int64_t(q) * P;
    double* dst = row_ptr(q);
    for (int64_t l = tid; l < k; l += TNT) dst[l] = a.D[i * a.ldd + l];
  }
  __syncthreads();
  if (k >= 2 && g == 0) make_reflector(a, row_ptr(0), 0, &red[0][0]);

  for (int64_t j = 0; j + 1 < k; ++j) {
    if (!wait_ge(a.vflag, unsigned(j + 1), a.abort_flag)) return;  // v_j published
    const double tj = ld_dev(a.tau + j);
    const double* v = a.A + j * k;
    const int par = int(j & 1);
    double* pj = a.p + par * k;
    double* partj = a.part + par * P;
    const int q0 = int((j + 1 - g + P - 1) / P) > 0 ? int((j + 1 - g + P - 1) / P) : 0;  // first owned row > j
    const bool owns_next = (j + 2 < k) && ((j + 1) % P == g);
    if (tj == 0.0) {  // H_j = I: nothing to update (the barrier keeps the columns in step)
      if (!grid_barrier(a.bar, P, gen, a.abort_flag)) return;
      if (owns_next) make_reflector(a, row_ptr(int((j + 1) / P)), j + 1, &red[0][0]);
      continue;
    }
    // this thread's entries of v_j, all loads in flight together (clamped
    // addresses, selected after); the owned rows' v_i by a separate load
    double vr[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const int64_t l = j + 1 + tid + int64_t(TNT) * m;
      const double x = ld_dev(v + (l < k ? l : j + 1));
      vr[m] = (l < k) ? x : 0.0;
    }
    for (int q = q0 + tid; q < nown; q += TNT) vown[q] = ld_dev(v + g + int64_t(q) * P);
    __syncthreads();
    // ---- p_i = tau * A[i, j+1:] . v[j+1:] for owned rows i > j ----------------
    double mypart = 0.0;
    for (int qb = q0; qb < nown; qb += TCH) {
      const int nq = min(TCH, nown - qb);
      double acc[TCH];
#pragma unroll
      for (int u = 0; u < TCH; ++u) acc[u] = 0.0;
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const int64_t l = j + 1 + tid + int64_t(TNT) * m;
        if (l < k) {
#pragma unroll
          for (int u = 0; u < TCH; ++u)
            if (u < nq) acc[u] += row_ptr(qb + u)[l] * vr[m];
        }
      }
#pragma unroll
      for (int u = 0; u < TCH; ++u) acc[u] = wave_sum(acc[u]);
      __syncthreads();
      if ((tid & 63) == 0) {
#pragma unroll
        for (int u = 0; u < TCH; ++u) red[tid >> 6][u] = acc[u];
      }
      __syncthreads();
      if (tid < nq) {
        double sacc = 0.0;
#pragma unroll
        for (int ww = 0; ww < TNT / 64; ++ww) sacc += red[ww][tid];
        const int q = qb + tid;
        const double pi = tj * sacc;
        st_dev(pj + g + int64_t(q) * P, pi);
        pown[q] = pi;
      }
      __syncthreads();
      if (tid == 0)
        for (int u = 0; u < nq; ++u) mypart += vown[qb + u] * pown[qb + u];
    }
    if (tid == 0) st_dev(partj + g, mypart);
    if (!grid_barrier(a.bar, P, gen, a.abort_flag)) return;  // p complete

    // ---- K = tau/2 * v^T p, partial sums reduced in a fixed order ----------
    {
      double sp = 0.0;
      for (int q = tid; q < P; q += TNT) sp += ld_dev(partj + q);
      sp = block_sum<TNT>(sp, &red[0][0]);
      if (tid == 0) bc[0] = 0.5 * tj * sp;
      __syncthreads();
    }
    const double K = bc[0];
    double wr[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const int64_t l = j + 1 + tid + int64_t(TNT) * m;
      const double pl = ld_dev(pj + (l < k ? l : j + 1));
      wr[m] = (l < k) ? pl - K * vr[m] : 0.0;
    }
    // ---- rank-2 update; the next reflector's row goes first ----------------
    auto update_row = [&](int q) {
      double* row = row_ptr(q);
      const double vi = vown[q];
      const double wi = pown[q] - K * vi;
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const int64_t l = j + 1 + tid + int64_t(TNT) * m;
        if (l < k) row[l] -= vi * wr[m] + wi * vr[m];
      }
    };
    int qn = -1;
    if (owns_next) {
      qn = int((j + 1) / P);
      update_row(qn);
      __syncthreads();
      make_reflector(a, row_ptr(qn), j + 1, &red[0][0]);
    }
    for (int q = q0; q < nown; ++q)
      if (q != qn) update_row(q);
    __syncthreads();
  }
  if (k >= 1 && (k - 1) % P == g) {
    const double* row = row_ptr(int((k - 1) / P));
    if (tid == 0) {
      a.d[k - 1] = row[k - 1];
      a.tau[k - 1] = 0.0;
    }
  }
}

// Same reduction for k <= SK by one workgroup holding the whole matrix in LDS
// (row stride k + 1 doubles spreads neighbouring rows over the banks).  The
// Rayleigh-Ritz matrices of the partial eigensolver are this small, and at
// this size the device-wide barriers of the cooperative kernel cost far more
// than the arithmetic.  Per column, four workgroup barriers: wave 0 forms the
// reflector from row j; p = tau A v with 8 lanes per row; wave 0 forms
// K = tau / 2 v^T p and w = p - K v; every thread applies the rank-2 update
// A -= v w^T + w v^T to the trailing block.  Outputs as the cooperative
// kernel's: v_j in row j of Aout (entry j + 1 = 1), tau, d, e.
constexpr int SK = 128;
constexpr int STN = 1024;

size_t sytrd_small_lds(int64_t k) { return (size_t(k) * size_t(k + 1) + 2 * size_t(k)) * sizeof(double); }

__global__ __launch_bounds__(STN) void sytrd_small_kernel(const double* __restrict__ D, int64_t ldd, int k,
                                                          double* __restrict__ Aout, double* __restrict__ d,
                                                          double* __restrict__ e, double* __restrict__ tau) {
  extern __shared__ double sm[];
  __shared__ double bc;  // tau_j
  const int ld = k + 1;
  double* A = sm;          // k x k, row stride ld
  double* v = A + k * ld;  // v_j, entries j + 1 .. k - 1
  double* pw = v + k;      // p, then w = p - K v
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = wv; i < k; i += STN / 64)
    for (int l = lane; l < k; l += 64) A[i * ld + l] = D[int64_t(i) * ldd + l];
  __syncthreads();
  for (int j = 0; j + 1 < k; ++j) {
    if (wv == 0) {
      const double* row = A + j * ld;
      double ss = 0.0;
      for (int l = j + 2 + lane; l < k; l += 64) ss += row[l] * row[l];
      ss = lane_value(wave_sum(ss), 0);  // one rounding for every lane
      const double alpha = row[j + 1];
      double beta, tj, scal;
      if (ss == 0.0) {
        beta = alpha;
        tj = 0.0;
        scal = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + ss), alpha);
        tj = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      for (int l = j + 2 + lane; l < k; l += 64) {
        const double x = (tj == 0.0) ? 0.0 : row[l] * scal;
        v[l] = x;
        Aout[int64_t(j) * k + l] = x;
      }
      if (lane == 0) {
        v[j + 1] = 1.0;
        Aout[int64_t(j) * k + j + 1] = 1.0;
        tau[j] = tj;
        d[j] = row[j];
        e[j] = beta;
        bc = tj;
      }
    }
    __syncthreads();
    const double tj = bc;
    {  // p_i = tau A[i, j+1:] . v[j+1:], rows i > j, 8 lanes per row
      const int i = j + 1 + (tid >> 3), part = tid & 7;
      double s = 0.0;
      if (i < k) {
        const double* row = A + i * ld;
        for (int l = j + 1 + part; l < k; l += 8) s += row[l] * v[l];
      }
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      if (i < k && part == 0) pw[i] = tj * s;
    }
    __syncthreads();
    if (wv == 0) {
      double s = 0.0;
      for (int i = j + 1 + lane; i < k; i += 64) s += v[i] * pw[i];
      const double K = 0.5 * tj * lane_value(wave_sum(s), 0);
      for (int i = j + 1 + lane; i < k; i += 64) pw[i] -= K * v[i];
    }
    __syncthreads();
    for (int i = j + 1 + wv; i < k; i += STN / 64) {
      const double vi = v[i], wi = pw[i];
      double* row = A + i * ld;
      for (int l = j + 1 + lane; l < k; l += 64) row[l] -= vi * pw[l] + wi * v[l];
    }
    __syncthreads();
  }
  if (tid == 0) {
    d[k - 1] = A[(k - 1) * ld + k - 1];
    tau[k - 1] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// 2. eigenvalues of T by multisection (one wave per eigenvalue)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int64_t k, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) <= pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int64_t i = 1; i < k; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) <= pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

__global__ void tri_prep_kernel(const double* d, const double* e, int64_t k, double* e2, double* bounds) {
  // bounds[0] = gl, bounds[1] = gu, bounds[2] = pivmin, bounds[3] = tnorm,
  // bounds[4] = nonfinite flag.  One block.
  __shared__ double red[4];
  double gl = INFINITY, gu = -INFINITY, emax = 0.0, bad = 0.0;
  for (int64_t i = threadIdx.x; i < k; i += blockDim.x) {
    const double el = (i > 0) ? fabs(e[i - 1]) : 0.0;
    const double er = (i + 1 < k) ? fabs(e[i]) : 0.0;
    gl = fmin(gl, d[i] - el - er);
    gu = fmax(gu, d[i] + el + er);
    if (i + 1 < k) {
      e2[i] = e[i] * e[i];
      emax = fmax(emax, e2[i]);
    }
    if (!isfinite(d[i]) || (i + 1 < k && !isfinite(e[i]))) bad = 1.0;
  }
  auto bred = [&](double v, bool mx) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      double w = __shfl_xor(v, o, 64);
      v = mx ? fmax(v, w) : fmin(v, w);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
    for (int i = 1; i < int(blockDim.x / 64); ++i) r = mx ? fmax(r, red[i]) : fmin(r, red[i]);
    return r;
  };
  gl = bred(gl, false);
  gu = bred(gu, true);
  emax = bred(emax, true);
  bad = bred(bad, true);
  if (threadIdx.x == 0) {
    const double tnorm = fmax(fabs(gl), fabs(gu));
    const double eps = 2.220446049250313e-16;
    const double safemin = 2.2250738585072014e-308;
    const double pad = 2.0 * eps * tnorm * double(k) + 2.0 * safemin;
    bounds[0] = gl - pad;
    bounds[1] = gu + pad;
    bounds[2] = safemin * fmax(1.0, emax);
    bounds[3] = tnorm;
    bounds[4] = bad;
  }
}

// lambda_desc[k-1-m] = m-th smallest eigenvalue.  With LDS_MODE the
// workgroup first copies d and e2 into LDS, so the Sturm recurrence (one
// dependent step per row) reads LDS instead of waiting on the cache.
template <bool LDS_MODE>
__global__ __launch_bounds__(256) void tri_bisect_kernel(const double* dg, const double* e2g, int64_t k,
                                                         const double* bounds, double* lambda_desc) {
  extern __shared__ double tri_lds[];
  const double* d = dg;
  const double* e2 = e2g;
  if (LDS_MODE) {
    for (int64_t i = threadIdx.x; i < k; i += 256) {
      tri_lds[i] = dg[i];
      tri_lds[k + i] = (i + 1 < k) ? e2g[i] : 0.0;
    }
    __syncthreads();
    d = tri_lds;
    e2 = tri_lds + k;
  }
  const int64_t m = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (m >= k) return;
  double lo = bounds[0], hi = bounds[1];
  const double pivmin = bounds[2];
  const double tnorm = bounds[3];
  const double eps = 2.220446049250313e-16;
  for (int it = 0; it < 64; ++it) {
    const double width = hi - lo;
    if (width <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin || width <= 4.0 * eps * eps * tnorm) break;
    const double x = lo + width * double(lane + 1) / 65.0;
    const int c = sturm_count(d, e2, k, x, pivmin);
    // largest lane with count <= m moves lo; smallest lane with count > m moves hi
    const unsigned long long below = __ballot(c <= m);
    const unsigned long long above = __ballot(c > m);
    double nlo = lo, nhi = hi;
    if (below) {
      const int lb = 63 - __clzll(below);
      nlo = __shfl(x, lb, 64);
    }
    if (above) {
      const int la = __ffsll(above) - 1;
      nhi = __shfl(x, la, 64);
    }
    if (nlo == lo && nhi == hi) break;  // no progress representable
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) lambda_desc[k - 1 - m] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// 3. inverse iteration for the top r eigenvectors of T
// ---------------------------------------------------------------------------
__device__ __forceinline__ double hash_unit(uint64_t x) {
  // SplitMix64 finalizer (Steele, Lea, Flood 2014) mapped to [-1, 1)
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return double(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// One wave per cluster of the top-r eigenvalues (descending order).  The LU
// factors of T - lambda I (u0, u1, u2, multipliers, swaps) and the iterate
// live in LDS when they fit (LDS_MODE), else in a per-cluster global scratch;
// the recurrences run on lane 0, reductions use the whole wave.
template <bool LDS_MODE>
__global__ __launch_bounds__(64) void tri_invit_kernel(const double* d, const double* e, int64_t k, int r,
                                                       const double* lambda_desc, const double* bounds,
                                                       double* Z /* r x k */, double* scratch,
                                                       unsigned char* swaps) {
  extern __shared__ double lds[];
  const int j0 = blockIdx.x;
  const int lane = threadIdx.x;
  const double tnorm = bounds[3];
  const double eps = 2.220446049250313e-16;
  const double ctol = 1e-5 * fmax(tnorm, 1e-300);  // cluster separation (header)
  if (j0 > 0 && fabs(lambda_desc[j0 - 1] - lambda_desc[j0]) <= ctol) return;  // not first of its cluster
  int j1 = j0 + 1;
  while (j1 < r && fabs(lambda_desc[j1 - 1] - lambda_desc[j1]) <= ctol) ++j1;

  double* base = LDS_MODE ? lds : scratch + size_t(j0) * 5 * k;
  double* u0 = base;
  double* u1 = u0 + k;
  double* u2 = u1 + k;
  double* mu = u2 + k;
  double* z = mu + k;
  unsigned char* sw = LDS_MODE ? reinterpret_cast<unsigned char*>(z + k) : swaps + size_t(j0) * k;
  const double piv_floor = eps * fmax(tnorm, 1e-300);

  for (int j = j0; j < j1; ++j) {
    const double lam = lambda_desc[j];
    if (lane == 0) {
      // LU with partial pivoting of T - lam I (rows i, i+1 at elimination step i)
      double x = d[0] - lam;
      double y = (k > 1) ? e[0] : 0.0;
      for (int64_t i = 0; i + 1 < k; ++i) {
        const double sub = e[i];
        const double dn = d[i + 1] - lam;
        const double sup = (i + 2 < k) ? e[i + 1] : 0.0;
        if (fabs(sub) > fabs(x)) {
          const double m = x / sub;
          u0[i] = sub;
          u1[i] = dn;
          u2[i] = sup;
          mu[i] = m;
          sw[i] = 1;
          x = y - m * dn;
          y = -m * sup;
        } else {
          double piv = x;
          if (fabs(piv) < piv_floor) piv = copysign(piv_floor, piv == 0.0 ? 1.0 : piv);
          const double m = sub / piv;
          u0[i] = piv;
          u1[i] = y;
          u2[i] = 0.0;
          mu[i] = m;
          sw[i] = 0;
          x = dn - m * y;
          y = sup;
        }
      }
      double piv = x;
      if (fabs(piv) < piv_floor) piv = copysign(piv_floor, piv == 0.0 ? 1.0 : piv);
      u0[k - 1] = piv;
      u1[k - 1] = 0.0;
      u2[k - 1] = 0.0;
    }
    __syncthreads();
    for (int64_t i = lane; i < k; i += 64) {
      if (fabs(u0[i]) < piv_floor) u0[i] = copysign(piv_floor, u0[i] == 0.0 ? 1.0 : u0[i]);
      z[i] = hash_unit(uint64_t(i) * 1315423911ull + uint64_t(j) * 2654435761ull + 7);
    }
    __syncthreads();
    for (int it = 0; it < 5; ++it) {
      // orthogonalize against earlier members of the cluster (modified Gram-Schmidt)
      for (int p = j0; p < j; ++p) {
        const double* zp = Z + size_t(p) * k;
        double dot = 0.0;
        for (int64_t i = lane; i < k; i += 64) dot += zp[i] * z[i];
        dot = wave_sum(dot);
        for (int64_t i = lane; i < k; i += 64) z[i] -= dot * zp[i];
        __syncthreads();
      }
      if (lane == 0) {
        double zc = z[0];
        for (int64_t i = 0; i + 1 < k; ++i) {  // row swaps and multipliers
          double zn = z[i + 1];
          if (sw[i]) {
            const double t = zc;
            zc = zn;
            zn = t;
          }
          z[i] = zc;
          zc = zn - mu[i] * zc;
        }
        z[k - 1] = zc;
        // back substitution, two super-diagonals
        double x2 = 0.0, x1 = z[k - 1] / u0[k - 1];
        z[k - 1] = x1;
        for (int64_t i = k - 2; i >= 0; --i) {
          const double xi = (z[i] - u1[i] * x1 - u2[i] * x2) / u0[i];
          z[i] = xi;
          x2 = x1;
          x1 = xi;
        }
      }
      __syncthreads();
      double amax = 0.0;
      for (int64_t i = lane; i < k; i += 64) amax = fmax(amax, fabs(z[i]));
      amax = wave_max(amax);
      if (!(amax > 0.0) || !isfinite(amax)) amax = 1.0;
      double nrm = 0.0;
      for (int64_t i = lane; i < k; i += 64) {
        const double v = z[i] / amax;
        z[i] = v;
        nrm += v * v;
      }
      nrm = sqrt(wave_sum(nrm));
      for (int64_t i = lane; i < k; i += 64) z[i] /= nrm;
      __syncthreads();
    }
    for (int p = j0; p < j; ++p) {  // final orthogonalization in the cluster
      const double* zp = Z + size_t(p) * k;
      double dot = 0.0;
      for (int64_t i = lane; i < k; i += 64) dot += zp[i] * z[i];
      dot = wave_sum(dot);
      double nrm = 0.0;
      for (int64_t i = lane; i < k; i += 64) {
        const double v = z[i] - dot * zp[i];
        z[i] = v;
        nrm += v * v;
      }
      nrm = sqrt(wave_sum(nrm));
      for (int64_t i = lane; i < k; i += 64) z[i] /= nrm;
      __syncthreads();
    }
    double* zo = Z + size_t(j) * k;
    for (int64_t i = lane; i < k; i += 64) zo[i] = z[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 4. back-transformation u = H_0 H_1 ... H_{k-3} z (one workgroup per vector)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void backtransform_kernel(const double* A /* row j: v_j */, const double* tau,
                                                            int64_t k, double* Z /* r x k in/out */) {
  extern __shared__ double zs[];
  __shared__ double red[4];
  double* zg = Z + size_t(blockIdx.x) * k;
  for (int64_t i = threadIdx.x; i < k; i += 256) zs[i] = zg[i];
  __syncthreads();
  for (int64_t j = k - 2; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    const double* v = A + j * k;
    double s = 0.0;
    for (int64_t l = j + 1 + threadIdx.x; l < k; l += 256) s += v[l] * zs[l];
    s = block_sum<256>(s, red);
    const double f = tj * s;
    for (int64_t l = j + 1 + threadIdx.x; l < k; l += 256) zs[l] -= f * v[l];
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < k; i += 256) zg[i] = zs[i];
}

// Blocked form (k <= 2048): the reflectors go in blocks of 32,
// H_{j0} H_{j0+1} ... H_{j0+31} = I - V T V^T (compact WY; T upper
// triangular with T[i][i] = tau_i and T[0:i, i] = -tau_i T[0:i, 0:i] V^T v_i),
// applied from the last block to the first, so each vector takes one
// 32-wide dot pass, one T product and one update pass per block instead of
// one reduction per reflector.  Row j of A holds v_j from column j + 1 on
// (earlier columns are not written), so every read is masked by l > j.
constexpr int BTB = 32;

__global__ __launch_bounds__(256) void bt_tfactor_kernel(const double* __restrict__ A, const double* __restrict__ tau,
                                                         int64_t k, double* __restrict__ Tb) {
  __shared__ double Vs[BTB][64 + 1];
  __shared__ double G[BTB][BTB + 1];
  __shared__ double T[BTB][BTB + 1];
  __shared__ double taus[BTB];
  const int tid = threadIdx.x;
  const int64_t j0 = int64_t(blockIdx.x) * BTB;
  const int nref = int(min<int64_t>(BTB, (k - 1) - j0));  // reflectors j0 .. j0 + nref - 1 (j <= k - 2)
  double g[BTB * BTB / 256];
#pragma unroll
  for (int q = 0; q < BTB * BTB / 256; ++q) g[q] = 0.0;
  for (int64_t c0 = j0 + 1; c0 < k; c0 += 64) {
    double x[BTB * 64 / 256];
#pragma unroll
    for (int q = 0; q < BTB * 64 / 256; ++q) {  // loads in flight together (clamped)
      const int e = tid + 256 * q, i = e / 64;
      const int64_t l = c0 + e % 64, j = j0 + i;
      x[q] = A[(i < nref ? j : j0) * k + (l < k ? l : k - 1)];
    }
#pragma unroll
    for (int q = 0; q < BTB * 64 / 256; ++q) {
      const int e = tid + 256 * q, i = e / 64;
      const int64_t l = c0 + e % 64, j = j0 + i;
      Vs[i][e % 64] = (i < nref && l < k && l > j) ? x[q] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < BTB * BTB / 256; ++q) {
      const int e = tid + 256 * q, i = e / BTB, i2 = e % BTB;
      double acc = g[q];
      for (int cc = 0; cc < 64; ++cc) acc += Vs[i][cc] * Vs[i2][cc];
      g[q] = acc;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < BTB * BTB / 256; ++q) {
    const int e = tid + 256 * q;
    G[e / BTB][e % BTB] = g[q];
    T[e / BTB][e % BTB] = 0.0;
  }
  if (tid < BTB) taus[tid] = (tid < nref) ? tau[j0 + tid] : 0.0;
  __syncthreads();
  for (int i = 0; i < BTB; ++i) {
    if (tid < i) {
      double acc = 0.0;
      for (int c = tid; c < i; ++c) acc += T[tid][c] * G[c][i];
      T[tid][i] = -taus[i] * acc;
    } else if (tid == i) {
      T[i][i] = taus[i];
    }
    __syncthreads();
  }
  double* Tout = Tb + size_t(blockIdx.x) * BTB * BTB;
  for (int e = tid; e < BTB * BTB; e += 256) Tout[e] = T[e / BTB][e % BTB];
}

// one workgroup per vector; thread t keeps z[t + 256 m] in registers
template <int NZ>
__global__ __launch_bounds__(256) void bt_apply_kernel(const double* __restrict__ A, const double* __restrict__ Tb,
                                                       int64_t k, double* __restrict__ Z) {
  __shared__ double red[4][BTB];
  __shared__ double sv[BTB], sp[BTB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* zg = Z + size_t(blockIdx.x) * k;
  double z[NZ];
#pragma unroll
  for (int m = 0; m < NZ; ++m) {
    const int64_t l = tid + 256 * int64_t(m);
    const double x = zg[l < k ? l : 0];
    z[m] = (l < k) ? x : 0.0;
  }
  const int nblk = int((k - 1 + BTB - 1) / BTB);
  for (int b = nblk - 1; b >= 0; --b) {
    const int64_t j0 = int64_t(b) * BTB;
    const int nref = int(min<int64_t>(BTB, (k - 1) - j0));
    double s[BTB];
#pragma unroll
    for (int i = 0; i < BTB; ++i) s[i] = 0.0;
#pragma unroll
    for (int m = 0; m < NZ; ++m) {
      const int64_t l = tid + 256 * int64_t(m);
      if (j0 + 1 > int64_t(m) * 256 + 255) continue;  // this lane group's columns all lie left of the block
      double x[BTB];
#pragma unroll
      for (int i = 0; i < BTB; ++i) x[i] = A[(j0 + (i < nref ? i : 0)) * k + (l < k ? l : k - 1)];
#pragma unroll
      for (int i = 0; i < BTB; ++i)
        if (i < nref && l < k && l > j0 + i) s[i] += x[i] * z[m];
    }
#pragma unroll
    for (int i = 0; i < BTB; ++i) {
      const double t = wave_sum(s[i]);
      if (lane == 0) red[wv][i] = t;
    }
    __syncthreads();
    if (tid < BTB) sv[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
    if (tid < BTB) {
      const double* Tt = Tb + size_t(b) * BTB * BTB + size_t(tid) * BTB;
      double acc = 0.0;
      for (int c = tid; c < BTB; ++c) acc += Tt[c] * sv[c];
      sp[tid] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NZ; ++m) {
      const int64_t l = tid + 256 * int64_t(m);
      if (j0 + 1 > int64_t(m) * 256 + 255) continue;
      double x[BTB];
#pragma unroll
      for (int i = 0; i < BTB; ++i) x[i] = A[(j0 + (i < nref ? i : 0)) * k + (l < k ? l : k - 1)];
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < BTB; ++i)
        if (i < nref && l < k && l > j0 + i) acc += x[i] * sp[i];
      z[m] -= acc;
    }
  }
#pragma unroll
  for (int m = 0; m < NZ; ++m) {
    const int64_t l = tid + 256 * int64_t(m);
    if (l < k) zg[l] = z[m];
  }
}

// ---------------------------------------------------------------------------
// 5. sign rule, Qhat = sqrt(lambda_j) u_j^T, T_r = u_j / sqrt(lambda_j)
// ---------------------------------------------------------------------------
struct Top2 {
  double a1;
  int64_t i1;
  double a2;
  int64_t i2;
};

__device__ __forceinline__ bool better(double a, int64_t i, double b, int64_t j) {
  return a > b || (a == b && i < j);
}

__device__ __forceinline__ Top2 merge2(Top2 x, Top2 y) {
  Top2 r;
  if (better(x.a1, x.i1, y.a1, y.i1)) {
    r.a1 = x.a1;
    r.i1 = x.i1;
    if (better(x.a2, x.i2, y.a1, y.i1)) {
      r.a2 = x.a2;
      r.i2 = x.i2;
    } else {
      r.a2 = y.a1;
      r.i2 = y.i1;
    }
  } else {
    r.a1 = y.a1;
    r.i1 = y.i1;
    if (better(y.a2, y.i2, x.a1, x.i1)) {
      r.a2 = y.a2;
      r.i2 = y.i2;
    } else {
      r.a2 = x.a1;
      r.i2 = x.i1;
    }
  }
  return r;
}

__global__ __launch_bounds__(256) void form_qhat_kernel(const double* Z /* r x k eigenvectors */, int64_t k, int r,
                                                        const double* lambda_desc, double* Qhat, int64_t ldqh,
                                                        double* Tr, int64_t ldtr, int* info) {
  __shared__ Top2 tops[4];
  __shared__ double red[4];
  __shared__ double bc;
  const int j = blockIdx.x;
  const double* u = Z + size_t(j) * k;
  Top2 t{-1.0, INT64_MAX, -1.0, INT64_MAX};
  for (int64_t i = threadIdx.x; i < k; i += 256) {
    Top2 c{fabs(u[i]), i, -1.0, INT64_MAX};
    t = merge2(t, c);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    Top2 other;
    other.a1 = __shfl_xor(t.a1, o, 64);
    other.i1 = __shfl_xor(t.i1, o, 64);
    other.a2 = __shfl_xor(t.a2, o, 64);
    other.i2 = __shfl_xor(t.i2, o, 64);
    t = merge2(t, other);
  }
  if ((threadIdx.x & 63) == 0) tops[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    Top2 b = tops[0];
    for (int w = 1; w < 4; ++w) b = merge2(b, tops[w]);
    double sg = (u[b.i1] >= 0.0) ? 1.0 : -1.0;
    bc = sg;
    if (b.i2 != INT64_MAX && (b.a1 - b.a2) <= 1e-8 * b.a1 && u[b.i1] * u[b.i2] < 0.0) bc = 2.0;  // near tie
  }
  __syncthreads();
  double sg = bc;
  if (sg == 2.0) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < k; i += 256) s += double(i + 1) * u[i];
    s = block_sum<256>(s, red);
    sg = (s >= 0.0) ? 1.0 : -1.0;
  }
  const double lam = lambda_desc[j];
  // an eigenvalue at or below k * u * lambda_1 is numerically zero
  if (threadIdx.x == 0 && !(lam > double(k) * 2.220446049250313e-16 * lambda_desc[0])) atomicMax(info, DOPINF_E_RANK);
  const double sl = sqrt(lam);
  const double isl = 1.0 / sl;
  for (int64_t i = threadIdx.x; i < k; i += 256) {
    const double ui = sg * u[i];
    Qhat[size_t(j) * ldqh + i] = sl * ui;
    if (Tr) Tr[i * ldtr + j] = ui * isl;
  }
}

__global__ void finite_check_kernel(const double* bounds, const int* abort_flag, int* info) {
  if (threadIdx.x == 0) {
    int v = DOPINF_OK;
    if (bounds[4] != 0.0) v = DOPINF_E_NONFINITE;
    if (*abort_flag) v = DOPINF_E_TIMEOUT;
    *info = v;
  }
}

__global__ void energy_rank_kernel(const double* lambda_desc, int64_t k, double tau, int* r_out) {
  if (threadIdx.x != 0) return;
  double total = 0.0;
  for (int64_t i = 0; i < k; ++i) total += lambda_desc[i];
  double c = 0.0;
  int64_t r = k;
  for (int64_t i = 0; i < k; ++i) {
    c += lambda_desc[i];
    if (c / total > tau) {
      r = i + 1;
      break;
    }
  }
  *r_out = int(r);
}

struct EigPlan {
  int P;
  int in_lds;
  int rows_max;
  size_t lds_bytes;
  const void* kern;
};

int plan_sytrd(int64_t k, EigPlan& pl) {
  int dev = 0;
  DOPINF_HIP(hipGetDevice(&dev));
  int ncu = 0, coop = 0;
  DOPINF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  DOPINF_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) return fail(DOPINF_E_HIP, "device does not support cooperative launches");
  int maxlds = 0;
  DOPINF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  int P = ncu;
  if (P > k) P = int(k);
  if (P < 1) P = 1;
  pl.P = P;
  pl.rows_max = int((k + P - 1) / P);
  const size_t need = size_t(pl.rows_max) * size_t(k) * sizeof(double);
  const size_t static_lds = 2048;
  pl.in_lds = (need + static_lds <= size_t(maxlds)) ? 1 : 0;
  pl.lds_bytes = pl.in_lds ? need : 0;
  pl.kern = reinterpret_cast<const void*>(sytrd_kernel);
  // rows in LDS plus the owned rows' v_i, p_i: register form for k <= 16 TNT
  const size_t need_reg = need + 2 * size_t(pl.rows_max) * sizeof(double);
  if (k <= 16 * TNT && need_reg + static_lds <= size_t(maxlds)) {
    pl.in_lds = 1;
    pl.lds_bytes = need_reg;
    pl.kern = (k <= 8 * TNT) ? reinterpret_cast<const void*>(sytrd_reg_kernel<8>)
                             : reinterpret_cast<const void*>(sytrd_reg_kernel<16>);
  }
  if (pl.in_lds)
    DOPINF_HIP(hipFuncSetAttribute(pl.kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(pl.lds_bytes)));
  int nb = 0;
  DOPINF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pl.kern, TNT, pl.lds_bytes));
  if (nb < 1) return fail(DOPINF_E_HIP, "tridiagonalization kernel cannot be resident");
  return DOPINF_OK;
}

struct EigWs {
  double* A;
  double* d;
  double* e;
  double* e2;
  double* tau;
  double* p;
  double* part;
  double* bounds;
  double* Z;
  double* scratch;
  double* tblk;  // T factors of the blocked back-transformation
  unsigned char* swaps;
  unsigned* words;  // [0] barrier, [1] abort, [2] r_out, [3] published reflectors
};

EigWs carve_eig(void* ws, size_t bytes, int64_t k, int r_max, int P, Carver& c) {
  (void)bytes;
  EigWs w;
  w.A = c.take<double>(size_t(k) * k);
  w.d = c.take<double>(size_t(k));
  w.e = c.take<double>(size_t(k));
  w.e2 = c.take<double>(size_t(k));
  w.tau = c.take<double>(size_t(k));
  w.p = c.take<double>(size_t(2 * k));
  w.part = c.take<double>(size_t(2 * (P > 0 ? P : 1024)));
  w.bounds = c.take<double>(8);
  w.Z = c.take<double>(size_t(r_max) * k);
  w.scratch = c.take<double>(size_t(r_max) * 5 * k);
  w.tblk = c.take<double>(size_t((k + BTB - 1) / BTB) * BTB * BTB);
  w.swaps = c.take<unsigned char>(size_t(r_max) * k);
  w.words = c.take<unsigned>(8);
  (void)ws;
  return w;
}

}  // namespace
}  // namespace dopinf

using namespace dopinf;

extern "C" size_t dopinf_reduce_workspace(int64_t k, int r_max) {
  if (k <= 0 || r_max <= 0) return 0;
  Carver c(nullptr, 0);
  carve_eig(nullptr, 0, k, r_max, 1024, c);
  return c.used;
}

namespace dopinf {
namespace {

// Tridiagonalization, all eigenvalues (descending, into lambda) and the
// finiteness / time-out status (into info) of the symmetric k x k matrix D.
int eig_values_stage(hipStream_t st, const double* D, int64_t k, int64_t ldd, double* lambda, int* info,
                     const EigWs& w, const EigPlan& pl) {
  zero_words_kernel<<<1, 64, 0, st>>>(w.words, 8);
  DOPINF_LAUNCHED();
  TridArgs ta{};
  ta.D = D;
  ta.ldd = ldd;
  ta.A = w.A;
  ta.k = k;
  ta.P = pl.P;
  ta.in_lds = pl.in_lds;
  ta.rows_max = pl.rows_max;
  ta.d = w.d;
  ta.e = w.e;
  ta.tau = w.tau;
  ta.p = w.p;
  ta.part = w.part;
  ta.bar = w.words;
  ta.vflag = w.words + 3;
  ta.abort_flag = reinterpret_cast<int*>(w.words + 1);
  if (k <= SK) {
    const size_t lb = sytrd_small_lds(k);
    if (lb > 65536)
      DOPINF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(sytrd_small_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lb)));
    sytrd_small_kernel<<<1, STN, lb, st>>>(D, ldd, int(k), w.A, w.d, w.e, w.tau);
    DOPINF_LAUNCHED();
  } else {
    void* args[] = {&ta};
    DOPINF_HIP(hipLaunchCooperativeKernel(pl.kern, dim3(pl.P), dim3(TNT), args, unsigned(pl.lds_bytes), st));
  }
  tri_prep_kernel<<<1, 256, 0, st>>>(w.d, w.e, k, w.e2, w.bounds);
  DOPINF_LAUNCHED();
  {
    int devb = 0, maxldsb = 0;
    DOPINF_HIP(hipGetDevice(&devb));
    DOPINF_HIP(hipDeviceGetAttribute(&maxldsb, hipDeviceAttributeMaxSharedMemoryPerBlock, devb));
    const size_t tl = size_t(2 * k) * sizeof(double);
    if (tl + 1024 <= size_t(maxldsb)) {
      if (tl > 65536)
        DOPINF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(tri_bisect_kernel<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(tl)));
      tri_bisect_kernel<true><<<unsigned((k + 3) / 4), 256, tl, st>>>(w.d, w.e2, k, w.bounds, lambda);
    } else {
      tri_bisect_kernel<false><<<unsigned((k + 3) / 4), 256, 0, st>>>(w.d, w.e2, k, w.bounds, lambda);
    }
  }
  DOPINF_LAUNCHED();
  finite_check_kernel<<<1, 64, 0, st>>>(w.bounds, reinterpret_cast<int*>(w.words + 1), info);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

// The top r eigenvectors of D into w.Z (r x k, one per row), from the
// tridiagonal form and the eigenvalues of eig_values_stage.
int eig_vectors_stage(hipStream_t st, int64_t k, int r, const double* lambda, const EigWs& w) {
  {
    int maxlds = 0, devi = 0;
    DOPINF_HIP(hipGetDevice(&devi));
    DOPINF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, devi));
    const size_t lb = size_t(k) * (5 * sizeof(double) + 1) + 64;
    if (lb <= size_t(maxlds)) {
      if (lb > 65536)
        DOPINF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(tri_invit_kernel<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lb)));
      tri_invit_kernel<true><<<unsigned(r), 64, lb, st>>>(w.d, w.e, k, r, lambda, w.bounds, w.Z, w.scratch, w.swaps);
    } else {
      tri_invit_kernel<false><<<unsigned(r), 64, 0, st>>>(w.d, w.e, k, r, lambda, w.bounds, w.Z, w.scratch, w.swaps);
    }
    DOPINF_LAUNCHED();
  }
  if (k >= 2 && k <= 2048) {
    const unsigned nblk = unsigned((k - 1 + BTB - 1) / BTB);
    bt_tfactor_kernel<<<nblk, 256, 0, st>>>(w.A, w.tau, k, w.tblk);
    DOPINF_LAUNCHED();
    bt_apply_kernel<8><<<unsigned(r), 256, 0, st>>>(w.A, w.tblk, k, w.Z);
    DOPINF_LAUNCHED();
  } else {
    const size_t zl = size_t(k) * sizeof(double);
    if (zl > 65536)
      DOPINF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(backtransform_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(zl)));
    backtransform_kernel<<<unsigned(r), 256, zl, st>>>(w.A, w.tau, k, w.Z);
    DOPINF_LAUNCHED();
  }
  return DOPINF_OK;
}

}  // namespace

// All eigenvalues (descending) and the top r eigenvectors (rows of *Z, r x k,
// inside ws) of the symmetric k x k matrix D; info as for dopinf_reduce.
size_t eig_vectors_workspace(int64_t k, int r) { return dopinf_reduce_workspace(k, r); }

int eig_vectors_internal(hipStream_t st, const double* D, int64_t k, int64_t ldd, int r, double* lambda, int* info,
                         void* ws, size_t ws_bytes, double** Z) {
  EigPlan pl{};
  int rc = plan_sytrd(k, pl);
  if (rc) return rc;
  Carver c(ws, ws_bytes);
  EigWs w = carve_eig(ws, ws_bytes, k, r, 1024, c);
  rc = eig_values_stage(st, D, k, ldd, lambda, info, w, pl);
  if (!rc) rc = eig_vectors_stage(st, k, r, lambda, w);
  *Z = w.Z;
  return rc;
}

// All eigenvalues (descending) of the symmetric k x k matrix D, no vectors;
// workspace eig_vectors_workspace(k, 1).
int eig_values_internal(hipStream_t st, const double* D, int64_t k, int64_t ldd, double* lambda, int* info, void* ws,
                        size_t ws_bytes) {
  EigPlan pl{};
  int rc = plan_sytrd(k, pl);
  if (rc) return rc;
  Carver c(ws, ws_bytes);
  EigWs w = carve_eig(ws, ws_bytes, k, 1, 1024, c);
  return eig_values_stage(st, D, k, ldd, lambda, info, w, pl);
}

// Sign rule, Qhat = Lambda_r^{1/2} U_r^T and T_r = U_r Lambda_r^{-1/2} from
// the eigenvector rows Z (r x k) and the descending eigenvalues.
int form_qhat_internal(hipStream_t st, const double* Z, int64_t k, int r, const double* lambda, double* Qhat,
                       int64_t ldqh, double* Tr, int64_t ldtr, int* info) {
  form_qhat_kernel<<<unsigned(r), 256, 0, st>>>(Z, k, r, lambda, Qhat, ldqh, Tr, ldtr, info);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

}  // namespace dopinf

extern "C" int dopinf_reduce(void* stream, const double* D, int64_t k, int64_t ldd, int r_req, double tau,
                             int r_max, int* r_out_h, double* lambda, double* Tr, int64_t ldtr, double* Qhat,
                             int64_t ldqh, int* info, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(D && lambda && Qhat && info, "D, lambda, Qhat and info must be non-NULL");
  DOPINF_REQUIRE(k >= 1 && ldd >= k && ldqh >= k, "need k >= 1, ldd >= k, ldqh >= k");
  DOPINF_REQUIRE(k <= 65536, "k > 65536 is not supported");
  DOPINF_REQUIRE(r_max >= 1 && r_max <= k, "need 1 <= r_max <= k");
  DOPINF_REQUIRE(r_req >= 0 && r_req <= r_max, "need 0 <= r_req <= r_max");
  DOPINF_REQUIRE(r_req > 0 || (tau > 0.0 && tau < 1.0), "energy threshold tau must be in (0, 1)");
  DOPINF_REQUIRE(!Tr || ldtr >= r_max, "ldtr must be >= r_max");
  const size_t need = dopinf_reduce_workspace(k, r_max);
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  EigPlan pl{};
  int rc = plan_sytrd(k, pl);
  if (rc) return rc;
  Carver c(ws, ws_bytes);
  EigWs w = carve_eig(ws, ws_bytes, k, r_max, 1024, c);
  rc = eig_values_stage(st, D, k, ldd, lambda, info, w, pl);
  if (rc) return rc;

  int r = r_req;
  if (r == 0) {
    int* r_dev = reinterpret_cast<int*>(w.words + 2);
    energy_rank_kernel<<<1, 64, 0, st>>>(lambda, k, tau, r_dev);
    DOPINF_LAUNCHED();
    int r_h = 0;
    DOPINF_HIP(hipMemcpyAsync(&r_h, r_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    DOPINF_HIP(hipStreamSynchronize(st));
    if (r_h > r_max) return fail(DOPINF_E_RANK, "energy criterion needs r = %d > r_max = %d", r_h, r_max);
    r = r_h;
  }
  if (r_out_h) *r_out_h = r;
  rc = eig_vectors_stage(st, k, r, lambda, w);
  if (rc) return rc;
  return form_qhat_internal(st, w.Z, k, r, lambda, Qhat, ldqh, Tr, ldtr, info);
}
