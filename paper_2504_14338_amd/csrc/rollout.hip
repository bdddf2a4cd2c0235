// Step IV of dOpInf (arXiv:2504.14338, Sec. 3.5): rollouts of the discrete
// quadratic ROM of Eq. (11) over the trial horizon, the training error, the
// growth bound and the selection of the best candidate.
//
// Many candidates (the regularization sweep): one workgroup rolls out one
// candidate: the state and the feature vector [q, quad(q), 1] live in LDS,
// the operator rows stream from L2 (each wave reduces several rows at a
// time).
//
// Few candidates (the plain run): a team of P co-resident workgroups rolls
// out one candidate.  Wave w of team member p owns operator row p*8 + w and
// keeps it in registers for the whole rollout, so no operator byte moves
// after the start; every step each member builds the features of the full
// state in LDS, forms its 8 next-state entries, publishes them with
// device-scope stores and meets the others at a counter barrier, then reads
// the full next state back.
//
// In both forms the score (finiteness, running maximum of the relative
// training error, running maximum deviation from the training mean) is
// accumulated while stepping, so the trajectory never has to be stored, and a
// candidate stops as soon as its failure is certain: the growth statistic is
// a running maximum, so crossing the bound (or meeting a non-finite value) is
// final and the selection is unchanged.  Team members score the same state
// with the same code and so take the same decision without talking.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "xwg_sync.hpp"

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
  int n_items;           // candidates of the group
  unsigned* queue;       // persistent grid: next-candidate counter (zeroed), or null
  double dt;             // > 0: continuous-time ROM stepped by RK4 with this step
  const double* q0;      // initial states of the group's items (r each), or null: Qhat[:, 0]
  const double* mean;    // r
  const double* maxdev;  // r
  const int* solve_status;  // group base or null
  double* traj;          // group base or null, item stride n_states*r
  double* train_err;     // group base
  double* growth;
  int* outcome;
};

// The ROM's map of the state in f[0:r]: builds the features f = [q |
// quad(q) | 1] in LDS, then qn[i] = O[i, :] . f for every row i.  Each wave
// owns rows w*RPW + 16*RPW*m; per lane CU8 x RPW operator loads are issued
// before their FMAs so that enough L2 traffic is in flight per CU.  Ends
// with a workgroup barrier (qn complete, f no longer read).
__device__ __forceinline__ void rom_map(const double* __restrict__ Op, double* f, double* qn, int r, int64_t s,
                                        int64_t d, const unsigned short* qi, const unsigned short* qj, int tid,
                                        int lane, int w) {
  for (int64_t c = tid; c < s; c += RT) f[r + c] = f[qi[c]] * f[qj[c]];
  if (tid == 0) f[d - 1] = 1.0;
  __syncthreads();
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
}

// RK4 = false: the discrete ROM of Eq. (11), q_{t+1} = O [q | quad(q) | 1].
// RK4 = true: the continuous-time ROM of Eq. (10), dq/dt = O [q | quad(q) | 1],
// advanced by one classical fourth-order Runge-Kutta step of a.dt per state.
template <bool RK4>
__device__ void rollout_item(const RollArgs& a, const int p) {
  extern __shared__ double sm[];
  const int r = a.r;
  const int64_t s = a.s, d = a.d;
  double* f = sm;                  // d features: [q | quad(q) | 1]
  double* qn = sm + d;             // r next state (RK4: the stage's right-hand side)
  double* mean = qn + r;           // r
  double* q0s = mean + r;          // RK4: r, the state at the start of the step
  double* ksum = q0s + (RK4 ? r : 0);  // RK4: r, k1 + 2 k2 + 2 k3 + k4
  unsigned short* qi = reinterpret_cast<unsigned short*>(ksum + (RK4 ? r : 0));
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
    f[i] = a.q0 ? a.q0[int64_t(p) * r + i] : a.Qhat[int64_t(i) * a.ldqh];  // state 0
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
    if constexpr (RK4) {
      for (int i = tid; i < r; i += RT) q0s[i] = f[i];
      for (int stage = 0; stage < 4; ++stage) {
        // f[0:r] holds the stage state; qn receives its right-hand side
        rom_map(Op, f, qn, r, s, d, qi, qj, tid, lane, w);
        for (int i = tid; i < r; i += RT) {
          const double kv = qn[i];
          ksum[i] = (stage == 0) ? kv : ksum[i] + ((stage == 3) ? kv : 2.0 * kv);
          if (stage < 3) f[i] = q0s[i] + ((stage == 2) ? a.dt : 0.5 * a.dt) * kv;
        }
        __syncthreads();
      }
      for (int i = tid; i < r; i += RT) f[i] = q0s[i] + (a.dt / 6.0) * ksum[i];
      __syncthreads();
    } else {
      rom_map(Op, f, qn, r, s, d, qi, qj, tid, lane, w);
      for (int i = tid; i < r; i += RT) f[i] = qn[i];
      __syncthreads();
    }
  }
  if (trj)
    for (int64_t e = int64_t(t_done) * r + tid; e < int64_t(a.n_states) * r; e += RT) trj[e] = NAN;
  if (tid == 0) {
    a.outcome[p] = oc;
    a.train_err[p] = (oc == DOPINF_ITEM_NONFINITE) ? NAN : sqrt(run_err);
    a.growth[p] = (oc == DOPINF_ITEM_NONFINITE) ? NAN : run_dev / maxdev;
  }
}

// One workgroup per candidate (a.queue == nullptr: candidate = blockIdx.x),
// or a persistent grid of resident workgroups that take candidates from a
// device counter until all are taken: a workgroup whose candidate stopped
// early (failure decided) takes the next one at once.  Every workgroup
// leaves when the counter passes n_items, so the grid always drains.
template <bool RK4>
__global__ __launch_bounds__(RT) void rollout_kernel(RollArgs a) {
  if (!a.queue) {
    rollout_item<RK4>(a, blockIdx.x);
    return;
  }
  __shared__ int item_sh;
  for (;;) {
    __syncthreads();  // the previous candidate is done with item_sh and LDS
    if (threadIdx.x == 0) item_sh = int(atomicAdd(a.queue, 1u));
    __syncthreads();
    const int p = item_sh;
    if (p >= a.n_items) break;
    rollout_item<RK4>(a, p);
  }
}


// ---- team rollout -------------------------------------------------------------

constexpr int TW = 8;     // waves per team workgroup = operator rows per member
constexpr int TNT = TW * 64;
constexpr int TNJ_MAX = 64;  // operator entries per lane: d <= 64 * 64

struct TeamArgs {
  RollArgs a;
  int P;              // members per team
  int n_items;
  double* xbuf;       // per item: 2 x r exchange slots
  unsigned* bar;      // per item: step counter
  int* abort_flag;
};

// The team groups of one call (reduced sizes with the same operator width
// class) in one cooperative launch: group g owns workgroups
// [off[g], off[g + 1]), a multiple of 8 each.
constexpr int kMaxTeamGroups = 8;
struct TeamSet {
  TeamArgs g[kMaxTeamGroups];
  int off[kMaxTeamGroups + 1];
  int n_g;
};
static_assert(sizeof(TeamSet) <= 4096, "kernel arguments are limited to 4 KB");

__global__ void zero_u32_kernel(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// RK4 = true: the continuous-time ROM stepped by classical RK4; each of the
// four stages publishes the members' entries of its right-hand side and
// passes one team barrier (the exchange slots alternate with the barrier
// count), then every member forms the next stage state from the full vector.
template <int TNJ, bool RK4>
__global__ __launch_bounds__(TNT) void rollout_team_kernel(TeamSet ts) {
  extern __shared__ double sm[];
  int grp = 0;
  while (grp + 1 < ts.n_g && int(blockIdx.x) >= ts.off[grp + 1]) ++grp;
  const TeamArgs& ta = ts.g[grp];
  const RollArgs& a = ta.a;
  // each team on one XCD: workgroup b runs on XCD b % 8 (the dispatcher
  // deals workgroups to the 8 XCDs in turn), so team i of a group takes its
  // workgroups 8 (P (i / 8) + m) + i % 8, m < P (the group's first workgroup
  // is a multiple of 8), and its counter barrier and exchange stay inside one
  // L2 (1.06 against 1.35 us per barrier across XCDs); workgroups past the
  // group's last team leave at once
  const int lb = int(blockIdx.x) - ts.off[grp];
  const int item = ((lb >> 3) / ta.P) * 8 + (lb & 7);
  const int pm = (lb >> 3) % ta.P;
  if (item >= ta.n_items) return;
  const int r = a.r;
  const int64_t s = a.s, d = a.d;
  const int64_t dpad = int64_t(TNJ) * 64;
  double* f = sm;                  // dpad features [q | quad(q) | 1 | 0...]
  double* mean = f + dpad;         // r
  double* q0s = mean + r;          // RK4: r, the state at the start of the step
  double* ksum = q0s + (RK4 ? r : 0);  // RK4: r, k1 + 2 k2 + 2 k3 + k4
  unsigned short* qi = reinterpret_cast<unsigned short*>(ksum + (RK4 ? r : 0));
  unsigned short* qj = qi + s;
  __shared__ double red[TW][4];
  __shared__ int stop_sh;
  __shared__ double dev0_sh;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int row = pm * TW + w;
  const int i_lo = pm * TW;
  const int i_hi = (i_lo + TW < r) ? i_lo + TW : r;
  const double* Op = a.O + size_t(item) * r * d;
  double* trj = a.traj ? a.traj + size_t(item) * a.n_states * r : nullptr;
  double* xb = ta.xbuf + size_t(item) * 2 * r;
  unsigned* bar = ta.bar + item;

  if (a.solve_status && a.solve_status[item] != DOPINF_OK) {
    if (pm == 0 && tid == 0) {
      a.outcome[item] = DOPINF_ITEM_SOLVE;
      a.train_err[item] = NAN;
      a.growth[item] = NAN;
    }
    if (trj)
      for (int64_t e = tid; e < int64_t(a.n_states) * (i_hi - i_lo); e += TNT)
        trj[(e / (i_hi - i_lo)) * r + i_lo + e % (i_hi - i_lo)] = NAN;
    return;
  }
  for (int64_t c = tid; c < s; c += TNT) {
    int ii = 0;
    int64_t off = 0;
    while (off + (r - ii) <= c) {
      off += r - ii;
      ++ii;
    }
    qi[c] = static_cast<unsigned short>(ii);
    qj[c] = static_cast<unsigned short>(ii + (c - off));
  }
  for (int64_t c = d + tid; c < dpad; c += TNT) f[c] = 0.0;
  if (tid == 0) f[d - 1] = 1.0;
  for (int i = tid; i < r; i += TNT) {
    mean[i] = a.mean[i];
    f[i] = a.q0 ? a.q0[int64_t(item) * r + i] : a.Qhat[int64_t(i) * a.ldqh];
  }
  if (tid == 0) {
    double md = 0.0;
    for (int i = 0; i < r; ++i) md = fmax(md, a.maxdev[i]);
    dev0_sh = md;
  }
  // this wave's operator row, resident in registers for the whole rollout
  double o[TNJ];
#pragma unroll
  for (int j = 0; j < TNJ; ++j) {
    const int64_t c = lane + 64 * j;
    o[j] = (row < r && c < d) ? Op[int64_t(row) * d + c] : 0.0;
  }
  __syncthreads();
  const double maxdev = dev0_sh;

  double run_err = 0.0, run_dev = 0.0;
  int oc = DOPINF_ITEM_PASS;
  int t_done = a.n_states;
  unsigned gen = 0;
  // training snapshot of the state being scored, fetched one step ahead
  double h = (tid < r && 0 < a.k_train) ? a.Qhat[int64_t(tid) * a.ldqh] : 0.0;
  for (int t = 0; t < a.n_states; ++t) {
    double e2 = 0.0, n2 = 0.0, dv = 0.0, bad = 0.0;
    if (tid < r) {
      const double x = f[tid];
      if (!isfinite(x)) bad = 1.0;
      dv = fabs(x - mean[tid]);
      if (t < a.k_train) {
        e2 = (x - h) * (x - h);
        n2 = h * h;
      }
      if (trj && tid >= i_lo && tid < i_hi) trj[int64_t(t) * r + tid] = x;
    }
    // quadratic features of state t (read by the first evaluation below),
    // formed in the same phase as the scores: both only read f[0:r)
    if (t + 1 < a.n_states)
      for (int64_t c = tid; c < s; c += TNT) f[r + c] = f[qi[c]] * f[qj[c]];
    // the state's entries sit in lanes tid < r: for r <= 64 wave 0 alone
    // reduces them (DPP sums, no cross-wave step); else every wave, then
    // thread 0 over the waves
    double E2 = 0.0, N2 = 0.0, DV = 0.0, BAD = 0.0;
    if (r <= 64) {
      if (w == 0) {
        E2 = wave_sum_dpp(e2);
        N2 = wave_sum_dpp(n2);
        DV = wave_max_dpp(dv);
        BAD = wave_max_dpp(bad);
      }
    } else {
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
        for (int q = 0; q < TW; ++q) {
          E2 += red[q][0];
          N2 += red[q][1];
          DV = fmax(DV, red[q][2]);
          BAD = fmax(BAD, red[q][3]);
        }
      }
    }
    if (tid == 0) {
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
    // one evaluation of the ROM map at the state in f[0:r): this wave's entry
    // goes to the exchange slot of barrier round gen, and after the barrier
    // every member reads the whole vector from it
    // (the features of the step's first evaluation are already in f; the
    // constant feature f[d-1] = 1 is set once)
    auto exchange = [&](double& kv, bool features, bool last) -> bool {
      if (features) {
        for (int64_t c = tid; c < s; c += TNT) f[r + c] = f[qi[c]] * f[qj[c]];
        __syncthreads();
      }
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < TNJ; ++j) acc += o[j] * f[lane + 64 * j];
      acc = wave_sum_dpp(acc);
      double* slot = xb + ((gen + 1) & 1) * r;
      if (lane == 0 && row < r) xwg::st_dev(slot + row, acc);
      if (!xwg::team_barrier(bar, unsigned(ta.P), gen, ta.abort_flag)) return false;
      // the next training snapshot after the step's last barrier (whose
      // drain would otherwise wait for it), in flight with the exchange load
      if (last) h = (tid < r && t + 1 < a.k_train) ? a.Qhat[int64_t(tid) * a.ldqh + t + 1] : 0.0;
      kv = (tid < r) ? xwg::ld_dev(slot + tid) : 0.0;
      return true;
    };
    bool ok = true;
    if constexpr (RK4) {
      if (tid < r) q0s[tid] = f[tid];
      for (int stage = 0; stage < 4 && ok; ++stage) {
        double kv = 0.0;
        ok = exchange(kv, stage > 0, stage == 3);
        if (ok && tid < r) {
          ksum[tid] = (stage == 0) ? kv : ksum[tid] + ((stage == 3) ? kv : 2.0 * kv);
          if (stage < 3) f[tid] = q0s[tid] + ((stage == 2) ? a.dt : 0.5 * a.dt) * kv;
        }
        __syncthreads();
      }
      if (ok && tid < r) f[tid] = q0s[tid] + (a.dt / 6.0) * ksum[tid];
    } else {
      double kv = 0.0;
      ok = exchange(kv, false, true);
      if (ok && tid < r) f[tid] = kv;
    }
    if (!ok) {
      oc = DOPINF_ITEM_TIMEOUT;
      t_done = t + 1;
      break;
    }
    __syncthreads();
  }
  if (trj)
    for (int64_t e = tid; e < int64_t(a.n_states - t_done) * (i_hi - i_lo); e += TNT)
      trj[(t_done + e / (i_hi - i_lo)) * r + i_lo + e % (i_hi - i_lo)] = NAN;
  if (pm == 0 && tid == 0) {
    const bool nan_out = (oc == DOPINF_ITEM_NONFINITE) || (oc == DOPINF_ITEM_TIMEOUT);
    a.outcome[item] = oc;
    a.train_err[item] = nan_out ? NAN : sqrt(run_err);
    a.growth[item] = nan_out ? NAN : run_dev / maxdev;
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

namespace dopinf {
int pool_streams(int want, hipStream_t* out);

namespace {

// Team form for group of size r with n_pairs items: co-resident teams of
// ceil(r / 8) workgroups while the teams fit on the chip at once (up to 128
// workgroups for the discrete map; RK4, which makes four team exchanges per
// step and reads its operator four times per step in the one-workgroup form,
// takes teams up to one workgroup per CU).
constexpr int kTeamMaxWorkgroups = 128;
constexpr int kTeamMaxWorkgroupsRK4 = 256;
int team_size(int r, int n_pairs, unsigned flags, bool rk4) {
  if (flags & DOPINF_ROLLOUT_ONE_WG) return 0;
  if (ncols(r) > int64_t(64) * TNJ_MAX) return 0;
  const int P = (r + TW - 1) / TW;
  return (int64_t(P) * n_pairs <= (rk4 ? kTeamMaxWorkgroupsRK4 : kTeamMaxWorkgroups)) ? P : 0;
}

struct RollWs {
  double* mean;
  double* maxdev;
  double* xbuf;
  unsigned* words;   // n_pairs counters + abort flag + the persistent grid's counter
};

RollWs carve_group(Carver& c, int r, int n_pairs) {
  RollWs w;
  w.mean = c.take<double>(size_t(r));
  w.maxdev = c.take<double>(size_t(r));
  w.xbuf = c.take<double>(size_t(n_pairs) * 2 * size_t(r));
  w.words = c.take<unsigned>(size_t(n_pairs) + 2);
  return w;
}

}  // namespace
}  // namespace dopinf

extern "C" size_t dopinf_rollout_workspace(int n_r, const int* r_list_h, int n_pairs, int64_t /*k_train*/) {
  if (n_r <= 0 || !r_list_h || n_pairs <= 0) return 0;
  Carver c(nullptr, 0);
  for (int g = 0; g < n_r; ++g) carve_group(c, r_list_h[g] > 0 ? r_list_h[g] : 1, n_pairs);
  return c.used;
}

namespace dopinf {
namespace {

int check_rollout_args(int n_r, const int* r_list_h, int n_pairs, const double* O, const double* Qhat,
                       int64_t ldqh, int64_t k_train, int n_states, double max_growth, unsigned flags,
                       const double* train_err, const double* growth, const int* outcome, const int* best) {
  DOPINF_REQUIRE(O && Qhat && train_err && growth && outcome && best && r_list_h, "NULL argument");
  DOPINF_REQUIRE(n_r >= 1 && n_pairs >= 1 && n_states >= 1, "need n_r, n_pairs, n_states >= 1");
  DOPINF_REQUIRE(k_train >= 1 && ldqh >= k_train, "need k_train >= 1 and ldqh >= k_train");
  DOPINF_REQUIRE(max_growth > 0.0, "max_growth must be > 0");
  DOPINF_REQUIRE((flags & ~(DOPINF_ROLLOUT_FULL | DOPINF_ROLLOUT_ONE_WG)) == 0, "unknown flag bits");
  for (int g = 0; g < n_r; ++g) DOPINF_REQUIRE(r_list_h[g] >= 1 && r_list_h[g] <= 512, "r must be in [1, 512]");
  return DOPINF_OK;
}

// The launches of a rollout call on a checked argument set, with its scratch
// (dopinf_rollout_workspace bytes) at `ws`.
// Events of one call's group fork, destroyed when the call returns (a
// recorded event is released once it completes).
struct ForkEvents {
  std::vector<hipEvent_t> ev;
  ~ForkEvents() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  int make(hipEvent_t* out) {
    DOPINF_HIP(hipEventCreateWithFlags(out, hipEventDisableTiming));
    ev.push_back(*out);
    return DOPINF_OK;
  }
};

// fork: with several reduced sizes each group's launches go to a library
// stream of its own (forked from st, joined back before the selection), so
// the groups' rollouts overlap (a stream capture turns this into parallel
// graph branches); the allocation-free entry point keeps everything on st,
// and so do calls with a group in the cooperative team form.
int rollout_launch(hipStream_t st, int n_r, const int* r_list_h, int n_pairs, const double* O,
                   const double* Qhat, int64_t ldqh, int64_t k_train, int n_states, double max_growth,
                   unsigned flags, const int* solve_status, double* traj, double* train_err, double* growth,
                   int* outcome, int* best, void* ws, size_t ws_bytes, double dt = 0.0,
                   const double* q0 = nullptr, bool fork = true) {
  int dev = 0, maxlds = 0;
  DOPINF_HIP(hipGetDevice(&dev));
  DOPINF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // every argument error is raised before anything is enqueued; groups that
  // run as cooperative teams keep the caller's stream (the runtime runs
  // cooperative launches one at a time, and two partly resident team grids
  // must never wait on each other)
  for (int g = 0; g < n_r; ++g) {
    const int r = r_list_h[g];
    const size_t smem = size_t(ncols(r) + (dt > 0.0 ? 4 : 2) * r) * sizeof(double) +
                        size_t(2 * nquad(r)) * sizeof(unsigned short) + 64;
    DOPINF_REQUIRE(smem + 1024 <= size_t(maxlds), "r too large for the rollout workgroup");
    if (team_size(r, n_pairs, flags, dt > 0.0) > 0) fork = false;
  }
  hipStream_t gs[8];
  int ns = 0;
  ForkEvents fe;
  if (fork && n_r >= 2) {
    ns = pool_streams(std::min(n_r, 8), gs);
    if (ns >= 2) {
      hipEvent_t f = nullptr;
      int rc = fe.make(&f);
      if (rc) return rc;
      DOPINF_HIP(hipEventRecord(f, st));
      for (int i = 0; i < ns; ++i) DOPINF_HIP(hipStreamWaitEvent(gs[i], f, 0));
    } else {
      ns = 0;
    }
  }
  Carver c(ws, ws_bytes);
  struct Pending {
    TeamArgs ta;
    size_t smem, tsm;
    RollWs w;
    hipStream_t sg;
  };
  std::vector<Pending> teams32, teams64;
  // the one-workgroup form: more candidates than resident workgroups take a
  // persistent grid with a work counter, else one workgroup per candidate
  auto one_wg_launch = [&](RollArgs ra, size_t smem, const RollWs& w, hipStream_t sg) -> int {
    const bool rk4 = dt > 0.0;
    const void* one_wg = rk4 ? reinterpret_cast<const void*>(rollout_kernel<true>)
                             : reinterpret_cast<const void*>(rollout_kernel<false>);
    int per_cu = 0, ncu = 0;
    DOPINF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, one_wg, RT, smem));
    DOPINF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int resident = std::max(1, per_cu) * std::max(1, ncu);
    int grid = n_pairs;
    ra.n_items = n_pairs;
    ra.queue = nullptr;
    if (n_pairs > resident) {
      ra.queue = w.words + n_pairs + 1;
      zero_u32_kernel<<<1, 64, 0, sg>>>(ra.queue, 1);
      DOPINF_LAUNCHED();
      grid = resident;
    }
    if (rk4)
      rollout_kernel<true><<<grid, RT, smem, sg>>>(ra);
    else
      rollout_kernel<false><<<grid, RT, smem, sg>>>(ra);
    DOPINF_LAUNCHED();
    return DOPINF_OK;
  };
  for (int g = 0; g < n_r; ++g) {
    const int r = r_list_h[g];
    // the largest groups get a stream each, the smallest share the last one
    int rank = 0;
    for (int q = 0; q < n_r; ++q) rank += (r_list_h[q] > r) || (r_list_h[q] == r && q < g);
    const hipStream_t sg = ns ? gs[std::min(rank, ns - 1)] : st;
    const int64_t s = nquad(r), d = ncols(r);
    const RollWs w = carve_group(c, r, n_pairs);
    double* mean = w.mean;
    double* maxdev = w.maxdev;
    train_stats_kernel<<<r, 256, 0, sg>>>(Qhat, ldqh, k_train, mean, maxdev);
    DOPINF_LAUNCHED();
    const bool rk4 = dt > 0.0;
    const size_t smem =
        size_t(d + (rk4 ? 4 : 2) * r) * sizeof(double) + size_t(2 * s) * sizeof(unsigned short) + 64;
    DOPINF_REQUIRE(smem + 1024 <= size_t(maxlds), "r too large for the rollout workgroup");
    const void* one_wg = rk4 ? reinterpret_cast<const void*>(rollout_kernel<true>)
                             : reinterpret_cast<const void*>(rollout_kernel<false>);
    if (smem > 65536)
      DOPINF_HIP(hipFuncSetAttribute(one_wg, hipFuncAttributeMaxDynamicSharedMemorySize, int(smem)));
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
    ra.dt = dt;
    ra.q0 = q0 ? q0 + dopinf_traj_offset(n_r, r_list_h, n_pairs, 1, g * n_pairs) : nullptr;
    ra.mean = mean;
    ra.maxdev = maxdev;
    ra.solve_status = solve_status ? solve_status + g * n_pairs : nullptr;
    ra.traj = traj ? traj + dopinf_traj_offset(n_r, r_list_h, n_pairs, n_states, g * n_pairs) : nullptr;
    ra.train_err = train_err + g * n_pairs;
    ra.growth = growth + g * n_pairs;
    ra.outcome = outcome + g * n_pairs;
    const int P = team_size(r, n_pairs, flags, rk4);
    if (P > 0) {
      const int tnj = (d <= 64 * 32) ? 32 : 64;
      zero_u32_kernel<<<(n_pairs + 1 + 255) / 256, 256, 0, sg>>>(w.words, n_pairs + 1);
      DOPINF_LAUNCHED();
      Pending pg{};
      pg.ta.a = ra;
      pg.ta.P = P;
      pg.ta.n_items = n_pairs;
      pg.ta.xbuf = w.xbuf;
      pg.ta.bar = w.words;
      pg.ta.abort_flag = reinterpret_cast<int*>(w.words + n_pairs);
      pg.smem = smem;
      pg.tsm = size_t(int64_t(tnj) * 64 + (rk4 ? 3 : 1) * r) * sizeof(double) +
               size_t(2 * s) * sizeof(unsigned short) + 64;
      pg.w = w;
      pg.sg = sg;
      (tnj == 32 ? teams32 : teams64).push_back(pg);
    } else {
      int rc = one_wg_launch(ra, smem, w, sg);
      if (rc) return rc;
    }
  }
  // the team groups of each operator width class in one cooperative launch
  // (the runtime runs cooperative launches one after the other); if the
  // runtime cannot make a whole set co-resident, group by group, and a group
  // it cannot place runs in the one-workgroup form
  for (int cls = 0; cls < 2; ++cls) {
    const std::vector<Pending>& v = cls ? teams64 : teams32;
    const void* kern = dt > 0.0 ? (cls ? reinterpret_cast<const void*>(rollout_team_kernel<64, true>)
                                       : reinterpret_cast<const void*>(rollout_team_kernel<32, true>))
                                : (cls ? reinterpret_cast<const void*>(rollout_team_kernel<64, false>)
                                       : reinterpret_cast<const void*>(rollout_team_kernel<32, false>));
    for (size_t c0 = 0; c0 < v.size(); c0 += kMaxTeamGroups) {
      const size_t c1 = std::min(v.size(), c0 + kMaxTeamGroups);
      auto launch_set = [&](size_t a0, size_t a1) -> bool {
        TeamSet ts{};
        ts.n_g = int(a1 - a0);
        int off = 0;
        size_t tsm = 0;
        for (size_t q = a0; q < a1; ++q) {
          ts.g[q - a0] = v[q].ta;
          ts.off[q - a0] = off;
          off += 8 * v[q].ta.P * ((v[q].ta.n_items + 7) / 8);
          tsm = std::max(tsm, v[q].tsm);
        }
        ts.off[a1 - a0] = off;
        void* args[] = {&ts};
        if (hipLaunchCooperativeKernel(kern, dim3(unsigned(off)), dim3(TNT), args, unsigned(tsm), st) ==
            hipSuccess)
          return true;
        (void)hipGetLastError();
        return false;
      };
      if (launch_set(c0, c1)) continue;
      for (size_t q = c0; q < c1; ++q) {
        if (c1 - c0 > 1 && launch_set(q, q + 1)) continue;
        int rc = one_wg_launch(v[q].ta.a, v[q].smem, v[q].w, v[q].sg);
        if (rc) return rc;
      }
    }
  }
  for (int i = 0; i < ns; ++i) {
    hipEvent_t j = nullptr;
    int rc = fe.make(&j);
    if (rc) return rc;
    DOPINF_HIP(hipEventRecord(j, gs[i]));
    DOPINF_HIP(hipStreamWaitEvent(st, j, 0));
  }
  select_kernel<<<n_r, 64, 0, st>>>(train_err, outcome, n_pairs, best);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}

// Scratch of the allocation-free rollout: one copy per GPU, alive until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host it names a stand-in, not device memory); it passes the device address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kRolloutScratchBytes = size_t(4) << 20;
__device__ __align__(256) unsigned char scratch[kRolloutScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call made with that device current.
int scratch_address(void** out) {
  int dev = 0;
  DOPINF_HIP(hipGetDevice(&dev));
  DOPINF_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    DOPINF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    DOPINF_REQUIRE(p != nullptr, "no device address for the rollout scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DOPINF_OK;
}

}  // namespace
}  // namespace dopinf

extern "C" int dopinf_rollout(void* stream, int n_r, const int* r_list_h, int n_pairs, const double* O,
                              const double* Qhat, int64_t ldqh, const double* q0, int64_t k_train, int n_states,
                              double max_growth, unsigned flags, const int* solve_status, double* traj,
                              double* train_err, double* growth, int* outcome, int* best, void* ws,
                              size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  int rc = check_rollout_args(n_r, r_list_h, n_pairs, O, Qhat, ldqh, k_train, n_states, max_growth, flags, train_err,
                              growth, outcome, best);
  if (rc) return rc;
  const size_t need = dopinf_rollout_workspace(n_r, r_list_h, n_pairs, k_train);
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  return rollout_launch(static_cast<hipStream_t>(stream), n_r, r_list_h, n_pairs, O, Qhat, ldqh, k_train, n_states,
                        max_growth, flags, solve_status, traj, train_err, growth, outcome, best, ws, ws_bytes, 0.0,
                        q0);
}

extern "C" int dopinf_rollout_continuous(void* stream, int n_r, const int* r_list_h, int n_pairs, const double* O,
                                         const double* Qhat, int64_t ldqh, int64_t k_train, int n_states, double dt,
                                         double max_growth, unsigned flags, const int* solve_status, double* traj,
                                         double* train_err, double* growth, int* outcome, int* best, void* ws,
                                         size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  int rc = check_rollout_args(n_r, r_list_h, n_pairs, O, Qhat, ldqh, k_train, n_states, max_growth, flags, train_err,
                              growth, outcome, best);
  if (rc) return rc;
  DOPINF_REQUIRE(dt > 0.0 && std::isfinite(dt), "dt must be finite and > 0");
  const size_t need = dopinf_rollout_workspace(n_r, r_list_h, n_pairs, k_train);
  if (!ws || ws_bytes < need) return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  return rollout_launch(static_cast<hipStream_t>(stream), n_r, r_list_h, n_pairs, O, Qhat, ldqh, k_train, n_states,
                        max_growth, flags, solve_status, traj, train_err, growth, outcome, best, ws, ws_bytes, dt);
}

extern "C" size_t dopinf_rollout_noalloc_max_bytes(void) { return dopinf::kRolloutScratchBytes; }

extern "C" int dopinf_rollout_noalloc(void* stream, int n_r, const int* r_list_h, int n_pairs, const double* O,
                                      const double* Qhat, int64_t ldqh, int64_t k_train, int n_states,
                                      double max_growth, unsigned flags, const int* solve_status, double* traj,
                                      double* train_err, double* growth, int* outcome, int* best) {
  int rc = check_rollout_args(n_r, r_list_h, n_pairs, O, Qhat, ldqh, k_train, n_states, max_growth, flags, train_err,
                              growth, outcome, best);
  if (rc) return rc;
  const size_t need = dopinf_rollout_workspace(n_r, r_list_h, n_pairs, k_train);
  if (need > dopinf::kRolloutScratchBytes)
    return fail(DOPINF_E_WORKSPACE, "rollout needs %zu bytes of scratch, the allocation-free form holds %zu", need,
                dopinf::kRolloutScratchBytes);
  void* ws = nullptr;
  rc = dopinf::scratch_address(&ws);
  if (rc) return rc;
  return rollout_launch(static_cast<hipStream_t>(stream), n_r, r_list_h, n_pairs, O, Qhat, ldqh, k_train, n_states,
                        max_growth, flags, solve_status, traj, train_err, growth, outcome, best, ws,
                        dopinf::kRolloutScratchBytes, 0.0, nullptr, false);
}
