// Step IV of dOpInf (arXiv:2504.14338, Sec. 3.5): rollouts of the discrete
// quadratic ROM of Eq. (11) over the trial horizon, the training error, the
// growth bound and the selection of the best candidate.
//
// One workgroup rolls out one candidate: the state and the feature vector
// [q, quad(q), 1] live in LDS, the operator rows stream from L2 (each wave
// reduces several rows at a time), and the score (finiteness, running
// maximum of the relative training error, running maximum deviation from the
// training mean) is accumulated while stepping, so the trajectory never has
// to be stored.  A candidate stops as soon as its failure is certain: the
// growth statistic is a running maximum, so crossing the bound (or meeting a
// non-finite value) is final and the selection is unchanged.
#include "common.hpp"

namespace dopinf {
namespace {

constexpr int RT = 1024;  // threads per rollout workgroup (16 waves)
constexpr int RPW = 2;    // operator rows reduced together by one wave
constexpr int CU8 = 8;    // independent operator loads per lane per row in flight

__host__ __device__ inline int64_t nquad(int64_t r) { return r * (r + 1) / 2; }
__host__ __device__ inline int64_t ncols(int64_t r) { return r + nquad(r) + 1; }

// training statistics of group r: mean m_i over t < k_train (one workgroup per
// mode) and the per-mode maximum |Qhat[i,t] - m_i|
__global__ __launch_bounds__(256) void train_stats_kernel(const double* __restrict__ Qhat, int64_t ldqh,
                                                          int64_t k_train, double* __restrict__ mean,
                                                          double* __restrict__ maxdev) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const double* q = Qhat + int64_t(i) * ldqh;
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < k_train; t += 256) s += q[t];
  s = block_sum<256>(s, red);
  const double m = s / double(k_train);
  double mx = 0.0;
  for (int64_t t = threadIdx.x; t < k_train; t += 256) mx = fmax(mx, fabs(q[t] - m));
  mx = wave_max(mx);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mean[i] = m;
    maxdev[i] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  }
}

struct RollArgs {
  int r;
  int64_t s, d;
  const double* O;       // group base, item stride r*d
  const double* Qhat;
  int64_t ldqh;
  int64_t k_train;
  int n_states;
  double max_growth;
  int full;
  const double* mean;    // r
  const double* maxdev;  // r
  const int* solve_status;  // group base or null
  double* traj;          // group base or null, item stride n_states*r
  double* train_err;     // group base
  double* growth;
  int* outcome;
};

__global__ __launch_bounds__(RT) void rollout_kernel(RollArgs a) {
  extern __shared__ double sm[];
  const int p = blockIdx.x;
  const int r = a.r;
  const int64_t s = a.s, d = a.d;
  double* f = sm;                  // d features: [q | quad(q) | 1]
  double* qn = sm + d;             // r next state
  double* mean = qn + r;           // r
  unsigned short* qi = reinterpret_cast<unsigned short*>(mean + r);
  unsigned short* qj = qi + s;
  __shared__ double red[RT / 64][4];
  __shared__ int stop_sh;
  __shared__ double dev0_sh;

  const double* Op = a.O + size_t(p) * r * d;
  double* trj = a.traj ? a.traj + size_t(p) * a.n_states * r : nullptr;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  if (a.solve_status && a.solve_status[p] != DOPINF_OK) {
    if (tid == 0) {
      a.outcome[p] = DOPINF_ITEM_SOLVE;
      a.train_err[p] = NAN;
      a.growth[p] = NAN;
    }
    if (trj)
      for (int64_t e = tid; e < int64_t(a.n_states) * r; e += RT) trj[e] = NAN;
    return;
  }
  // quadratic index map and training mean
  for (int64_t c = tid; c < s; c += RT) {
    int ii = 0;
    int64_t off = 0;
    while (off + (r - ii) <= c) {
      off += r - ii;
      ++ii;
    }
    qi[c] = static_cast<unsigned short>(ii);
    qj[c] = static_cast<unsigned short>(ii + (c - off));
  }
  for (int i = tid; i < r; i += RT) {
    mean[i] = a.mean[i];
    f[i] = a.Qhat[int64_t(i) * a.ldqh];  // state 0 = first training snapshot
  }
  if (tid == 0) {
    double md = 0.0;
    for (int i = 0; i < r; ++i) md = fmax(md, a.maxdev[i]);
    dev0_sh = md;
  }
  __syncthreads();
  const double maxdev = dev0_sh;

  double run_err = 0.0;   // max over t of ||q_t - qhat_t||^2 / ||qhat_t||^2  (thread 0)
  double run_dev = 0.0;   // max over t, i of |q_t[i] - m_i|                  (thread 0)
  int oc = DOPINF_ITEM_PASS;
  int t_done = a.n_states;
  for (int t = 0; t < a.n_states; ++t) {
    // ---- score state t (held in f[0:r]) ----
    double e2 = 0.0, n2 = 0.0, dv = 0.0, bad = 0.0;
    for (int i = tid; i < r; i += RT) {
      const double x = f[i];
      if (!isfinite(x)) bad = 1.0;
      dv = fmax(dv, fabs(x - mean[i]));
      if (t < a.k_train) {
        const double h = a.Qhat[int64_t(i) * a.ldqh + t];
        e2 += (x - h) * (x - h);
        n2 += h * h;
      }
      if (trj) trj[int64_t(t) * r + i] = x;
    }
    // r <= RT is not required: reduce over the block
    e2 = wave_sum(e2);
    n2 = wave_sum(n2);
    dv = wave_max(dv);
    bad = wave_max(bad);
    if (lane == 0) {
      red[w][0] = e2;
      red[w][1] = n2;
      red[w][2] = dv;
      red[w][3] = bad;
    }
    __syncthreads();
    if (tid == 0) {
      double E2 = 0.0, N2 = 0.0, DV = 0.0, BAD = 0.0;
      for (int q = 0; q < RT / 64; ++q) {
        E2 += red[q][0];
        N2 += red[q][1];
        DV = fmax(DV, red[q][2]);
        BAD = fmax(BAD, red[q][3]);
      }
      int stop = 0;
      if (BAD != 0.0) {
        oc = DOPINF_ITEM_NONFINITE;
        stop = 1;
      } else {
        run_dev = fmax(run_dev, DV);
        if (t < a.k_train) run_err = fmax(run_err, E2 / N2);
        if (run_dev / maxdev >= a.max_growth && oc == DOPINF_ITEM_PASS) {
          oc = DOPINF_ITEM_GROWTH;
          if (!a.full) stop = 1;
        }
      }
      stop_sh = stop;
    }
    __syncthreads();
    if (stop_sh) {
      t_done = t + 1;
      break;
    }
    if (t + 1 == a.n_states) break;
    // ---- features of state t ----
    for (int64_t c = tid; c < s; c += RT) f[r + c] = f[qi[c]] * f[qj[c]];
    if (tid == 0) f[d - 1] = 1.0;
    __syncthreads();
    // ---- next state: q_{t+1}[i] = O[i, :] . f ----
    // each wave owns rows w*RPW + 16*RPW*m; per lane CU8 x RPW loads are issued
    // before their FMAs so that enough L2 traffic is in flight per CU
    for (int i0 = w * RPW; i0 < r; i0 += (RT / 64) * RPW) {
      double acc[RPW];
#pragma unroll
      for (int u = 0; u < RPW; ++u) acc[u] = 0.0;
      int64_t c = lane;
      for (; c + 64 * (CU8 - 1) < d; c += 64 * CU8) {
        double ov[RPW][CU8];
#pragma unroll
        for (int u = 0; u < RPW; ++u)
#pragma unroll
          for (int q = 0; q < CU8; ++q) ov[u][q] = (i0 + u < r) ? Op[int64_t(i0 + u) * d + c + 64 * q] : 0.0;
#pragma unroll
        for (int q = 0; q < CU8; ++q) {
          const double fc = f[c + 64 * q];
#pragma unroll
          for (int u = 0; u < RPW; ++u) acc[u] += ov[u][q] * fc;
        }
      }
      for (; c < d; c += 64) {
        const double fc = f[c];
#pragma unroll
        for (int u = 0; u < RPW; ++u)
          if (i0 + u < r) acc[u] += Op[int64_t(i0 + u) * d + c] * fc;
      }
#pragma unroll
      for (int u = 0; u < RPW; ++u) {
        const double v = wave_sum(acc[u]);
        if (lane == 0 && i0 + u < r) qn[i0 + u] = v;
      }
    }
    __syncthreads();
    for (int i = tid; i < r; i += RT) f[i] = qn[i];
    __syncthreads();
  }
  if (trj)
    for (int64_t e = int64_t(t_done) * r + tid; e < int64_t(a.n_states) * r; e += RT) trj[e] = NAN;
  if (tid == 0) {
    a.outcome[p] = oc;
    a.train_err[p] = (oc == DOPINF_ITEM_NONFINITE) ? NAN : sqrt(run_err);
    a.growth[p] = (oc == DOPINF_ITEM_NONFINITE) ? NAN : run_dev / maxdev;
  }
}

// best[g] = argmin train_err over passing items of group g (first on ties)
__global__ void select_kernel(const double* __restrict__ train_err, const int* __restrict__ outcome, int n_pairs,
                              int* __restrict__ best) {
  const int g = blockIdx.x;
  if (threadIdx.x != 0) return;
  int b = -1;
  double be = 0.0;
  for (int p = 0; p < n_pairs; ++p) {
    const int it = g * n_pairs + p;
    if (outcome[it] != DOPINF_ITEM_PASS) continue;
    if (b < 0 || train_err[it] < be) {
      b = it;
      be = train_err[it];
    }
  }
  best[g] = b;
}

}  // namespace
}  // namespace dopinf

using namespace dopinf;

extern "C" size_t dopinf_traj_offset(int n_r, const int* r_list_h, int n_pairs, int n_states, int item) {
  if (n_r <= 0 || !r_list_h || n_pairs <= 0 || n_states <= 0 || item < 0) return 0;
  size_t off = 0;
  for (int g = 0; g < n_r; ++g) {
    const size_t per = size_t(r_list_h[g]) * size_t(n_states);
    if (item < (g + 1) * n_pairs) return off + size_t(item - g * n_pairs) * per;
    off += per * size_t(n_pairs);
  }
  return off;
}

extern "C" size_t dopinf_rollout_workspace(int n_r, const int* r_list_h, int /*n_pairs*/, int64_t /*k_train*/) {
  if (n_r <= 0 || !r_list_h) return 0;
  int rmax = 0;
  for (int g = 0; g < n_r; ++g) rmax = r_list_h[g] > rmax ? r_list_h[g] : rmax;
  Carver c(nullptr, 0);
  for (int g = 0; g < n_r; ++g) {
    c.take<double>(size_t(rmax));
    c.take<double>(size_t(rmax));
  }
  return c.used;
}

extern "C" int dopinf_rollout(void* stream, int n_r, const int* r_list_h, int n_pairs, const double* O,
                              const double* Qhat, int64_t ldqh, int64_t k_train, int n_states, double max_growth,
                              unsigned flags, const int* solve_status, double* traj, double* train_err,
                              double* growth, int* outcome, int* best, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE(O && Qhat && train_err && growth && outcome && best && r_list_h, "NULL argument");
  DOPINF_REQUIRE(n_r >= 1 && n_pairs >= 1 && n_states >= 1, "need n_r, n_pairs, n_states >= 1");
  DOPINF_REQUIRE(k_train >= 1 && ldqh >= k_train, "need k_train >= 1 and ldqh >= k_train");
  DOPINF_REQUIRE(max_growth > 0.0, "max_growth must be > 0");
  DOPINF_REQUIRE((flags & ~DOPINF_ROLLOUT_FULL) == 0, "unknown flag bits");
  for (int g = 0; g < n_r; ++g) DOPINF_REQUIRE(r_list_h[g] >= 1 && r_list_h[g] <= 512, "r must be in [1, 512]");
  const size_t need = dopinf_rollout_workspace(n_r, r_list_h, n_pairs, k_train);
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  int dev = 0, maxlds = 0;
  DOPINF_HIP(hipGetDevice(&dev));
  DOPINF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws, ws_bytes);
  for (int g = 0; g < n_r; ++g) {
    const int r = r_list_h[g];
    const int64_t s = nquad(r), d = ncols(r);
    double* mean = c.take<double>(size_t(r > 0 ? r : 1));
    double* maxdev = c.take<double>(size_t(r > 0 ? r : 1));
    train_stats_kernel<<<r, 256, 0, st>>>(Qhat, ldqh, k_train, mean, maxdev);
    DOPINF_LAUNCHED();
    const size_t smem = size_t(d + 2 * r) * sizeof(double) + size_t(2 * s) * sizeof(unsigned short) + 64;
    DOPINF_REQUIRE(smem + 1024 <= size_t(maxlds), "r too large for the rollout workgroup");
    if (smem > 65536)
      DOPINF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(rollout_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(smem)));
    RollArgs ra{};
    ra.r = r;
    ra.s = s;
    ra.d = d;
    ra.O = O + dopinf_operator_offset(n_r, r_list_h, n_pairs, g * n_pairs);
    ra.Qhat = Qhat;
    ra.ldqh = ldqh;
    ra.k_train = k_train;
    ra.n_states = n_states;
    ra.max_growth = max_growth;
    ra.full = (flags & DOPINF_ROLLOUT_FULL) ? 1 : 0;
    ra.mean = mean;
    ra.maxdev = maxdev;
    ra.solve_status = solve_status ? solve_status + g * n_pairs : nullptr;
    ra.traj = traj ? traj + dopinf_traj_offset(n_r, r_list_h, n_pairs, n_states, g * n_pairs) : nullptr;
    ra.train_err = train_err + g * n_pairs;
    ra.growth = growth + g * n_pairs;
    ra.outcome = outcome + g * n_pairs;
    rollout_kernel<<<n_pairs, RT, smem, st>>>(ra);
    DOPINF_LAUNCHED();
  }
  select_kernel<<<n_r, 64, 0, st>>>(train_err, outcome, n_pairs, best);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}
