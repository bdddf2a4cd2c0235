// Step II of dOpInf (arXiv:2504.14338, Sec. 3.3): per-row temporal mean and
// per-variable max-abs scale of the centered snapshots.
//
// HBM-bound: one wavefront streams one row (k contiguous elements, coalesced
// 512-B loads per wave instruction), holds it in registers when k <= 64*NV,
// and reduces sum and max |x - mean| across the 64 lanes.  Per-variable maxima
// come from a deterministic two-stage max over the per-row maxima (max is
// exact, so the result is independent of order).
//
// Non-finite data: a row holding NaN or Inf gets a NaN row maximum, and every
// max here propagates NaN (fmax would drop it), so the variable's scale is
// NaN, as the plain definition gives it; the call's status word then reads
// DOPINF_E_NONFINITE.
#include "common.hpp"

namespace dopinf {
namespace {

constexpr int kRowsPerBlock = 4;  // one 64-lane wave per row

template <class T>
__device__ __forceinline__ double ld(const T* p) { return static_cast<double>(*p); }

// max that keeps NaN once it has been seen (either argument)
__device__ __forceinline__ double max_nan(double a, double b) { return (a != a || b > a || b != b) ? (a != a ? a : b) : a; }

__device__ __forceinline__ double wave_max_nan(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max_nan(v, __shfl_xor(v, o, 64));
  return v;
}

// NV > 0: the row is kept in registers (k <= 64*NV); NV == 0: re-read.
template <class T, int NV>
__global__ __launch_bounds__(256) void row_stats_kernel(
    const T* __restrict__ Q, int64_t n, int64_t k, int64_t ldq, int center,
    double* __restrict__ mean, double* __restrict__ rowmax) {
  const int lane = threadIdx.x & 63;
  const int64_t row = int64_t(blockIdx.x) * kRowsPerBlock + (threadIdx.x >> 6);
  if (row >= n) return;
  const T* q = Q + row * ldq;
  double mu = 0.0;
  double m = 0.0;
  if constexpr (NV > 0) {
    double v[NV];
    double s = 0.0;
    // every load reads a valid address (clamped) and the value is selected
    // after it, so the NV loads of a lane are in flight together
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int64_t t = lane + 64 * j;
      const double x = ld(q + (t < k ? t : 0));
      v[j] = (t < k) ? x : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) s += v[j];
    s = wave_sum(s);
    mu = center ? s / static_cast<double>(k) : 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      int64_t t = lane + 64 * j;
      if (t < k) m = max_nan(m, fabs(v[j] - mu));
    }
  } else {
    double s = 0.0;
    for (int64_t t = lane; t < k; t += 64) s += ld(q + t);
    s = wave_sum(s);
    mu = center ? s / static_cast<double>(k) : 0.0;
    for (int64_t t = lane; t < k; t += 64) m = max_nan(m, fabs(ld(q + t) - mu));
  }
  // an infinite value with a finite mean gives an infinite deviation; with
  // centering the mean is then infinite too and the deviation NaN: either way
  // the row is flagged by a NaN maximum
  m = wave_max_nan(m);
  if (isinf(m) || isinf(mu)) m = NAN;
  if (lane == 0) {
    mean[row] = mu;
    rowmax[row] = m;
  }
}

struct VarRanges {
  int nvars;
  int64_t row0[DOPINF_MAX_VARS + 1];
  int chunk0[DOPINF_MAX_VARS + 1];  // prefix sum of chunks per variable
};

constexpr int kChunkRows = 16384;

__device__ __forceinline__ int find_var(const VarRanges& vr, int chunk) {
  int v = 0;
  while (v + 1 < vr.nvars && chunk >= vr.chunk0[v + 1]) ++v;
  return v;
}

// Stage 1: max of rowmax over one chunk of rows of one variable.
__global__ __launch_bounds__(256) void var_max_partial_kernel(
    const double* __restrict__ rowmax, VarRanges vr, double* __restrict__ part) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  const int v = find_var(vr, c);
  const int64_t lo = vr.row0[v] + int64_t(c - vr.chunk0[v]) * kChunkRows;
  const int64_t hi = min(vr.row0[v + 1], lo + kChunkRows);
  double m = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) m = max_nan(m, rowmax[i]);
  m = wave_max_nan(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[c] = max_nan(max_nan(red[0], red[1]), max_nan(red[2], red[3]));
}

// Stage 2: one wave per variable; zero range -> scale 1 and a flag; a NaN
// maximum (non-finite data in the variable) -> scale NaN and the status word
// DOPINF_E_NONFINITE (set, never cleared, by any variable).
__global__ void var_max_final_kernel(const double* __restrict__ part, VarRanges vr,
                                     int do_scale, double* __restrict__ scale,
                                     int* __restrict__ zero_range, int* __restrict__ info) {
  const int v = blockIdx.x;
  double m = 0.0;
  for (int c = vr.chunk0[v] + threadIdx.x; c < vr.chunk0[v + 1]; c += 64) m = max_nan(m, part[c]);
  m = wave_max_nan(m);
  if (threadIdx.x == 0) {
    int zr = 0;
    double s = 1.0;
    if (m != m) {
      if (info) atomicExch(info, DOPINF_E_NONFINITE);
      if (do_scale) s = m;
    } else if (do_scale) {
      if (m == 0.0) {
        zr = 1;
      } else {
        s = m;
      }
    }
    scale[v] = s;
    if (zero_range) zero_range[v] = zr;
  }
}

__global__ void set_info_kernel(int* info) {
  if (threadIdx.x == 0) *info = DOPINF_OK;
}

template <class T>
__global__ __launch_bounds__(256) void apply_kernel(T* __restrict__ Q, int64_t n, int64_t k,
                                                    int64_t ldq, const double* __restrict__ mean,
                                                    const double* __restrict__ scale, VarRanges vr) {
  const int64_t row = int64_t(blockIdx.x) * kRowsPerBlock + (threadIdx.x >> 6);
  if (row >= n) return;
  int v = 0;
  while (v + 1 < vr.nvars && row >= vr.row0[v + 1]) ++v;
  const double mu = mean[row];
  const double s = scale[v];
  T* q = Q + row * ldq;
  for (int64_t t = threadIdx.x & 63; t < k; t += 64) q[t] = static_cast<T>((ld(q + t) - mu) / s);
}

// Lifting (Sec. 3.3): output variable j, cell i, snapshot t from the input
// variables' values at the same cell and snapshot.  One wave per output row.
struct LiftSpec {
  int n_out;
  int op[DOPINF_MAX_VARS], a[DOPINF_MAX_VARS], b[DOPINF_MAX_VARS];
};

__global__ __launch_bounds__(256) void lift_kernel(const double* __restrict__ Q, int64_t n_cells, int64_t k,
                                                   int64_t ldq, LiftSpec sp, double* __restrict__ L, int64_t ldl) {
  const int64_t row = int64_t(blockIdx.x) * kRowsPerBlock + (threadIdx.x >> 6);
  if (row >= int64_t(sp.n_out) * n_cells) return;
  const int j = int(row / n_cells);
  const int64_t i = row - int64_t(j) * n_cells;
  const double* qa = Q + (int64_t(sp.a[j]) * n_cells + i) * ldq;
  const double* qb = Q + (int64_t(sp.b[j]) * n_cells + i) * ldq;
  double* out = L + row * ldl;
  const int op = sp.op[j];
  for (int64_t t = threadIdx.x & 63; t < k; t += 64) {
    const double x = qa[t];
    double y;
    if (op == DOPINF_LIFT_PRODUCT)
      y = x * qb[t];
    else if (op == DOPINF_LIFT_RECIPROCAL)
      y = 1.0 / x;
    else
      y = x;
    out[t] = y;
  }
}

VarRanges make_ranges(int nvars, const int64_t* var_rows_h) {
  VarRanges vr{};
  vr.nvars = nvars;
  int c = 0;
  for (int v = 0; v <= nvars; ++v) {
    vr.row0[v] = var_rows_h[v];
    vr.chunk0[v] = c;
    if (v < nvars) c += int((var_rows_h[v + 1] - var_rows_h[v] + kChunkRows - 1) / kChunkRows);
  }
  return vr;
}

template <class T>
void launch_row_stats(hipStream_t st, const T* Q, int64_t n, int64_t k, int64_t ldq, int center,
                      double* mean, double* rowmax) {
  dim3 grid(unsigned((n + kRowsPerBlock - 1) / kRowsPerBlock));
  if (k <= 64 * 8)
    row_stats_kernel<T, 8><<<grid, 256, 0, st>>>(Q, n, k, ldq, center, mean, rowmax);
  else if (k <= 64 * 16)
    row_stats_kernel<T, 16><<<grid, 256, 0, st>>>(Q, n, k, ldq, center, mean, rowmax);
  else if (k <= 64 * 32)
    row_stats_kernel<T, 32><<<grid, 256, 0, st>>>(Q, n, k, ldq, center, mean, rowmax);
  else
    row_stats_kernel<T, 0><<<grid, 256, 0, st>>>(Q, n, k, ldq, center, mean, rowmax);
}

}  // namespace

int check_var_rows(int64_t n, int nvars, const int64_t* var_rows_h) {
  DOPINF_REQUIRE(nvars >= 1 && nvars <= DOPINF_MAX_VARS, "nvars must be in [1, %d]", DOPINF_MAX_VARS);
  DOPINF_REQUIRE(var_rows_h != nullptr, "var_rows_h is NULL");
  DOPINF_REQUIRE(var_rows_h[0] == 0 && var_rows_h[nvars] == n, "var_rows_h must start at 0 and end at n");
  for (int v = 0; v < nvars; ++v)
    DOPINF_REQUIRE(var_rows_h[v + 1] > var_rows_h[v], "var_rows_h must be strictly increasing");
  return DOPINF_OK;
}

}  // namespace dopinf

using namespace dopinf;

extern "C" size_t dopinf_preprocess_workspace(int64_t n, int64_t /*k*/, int nvars) {
  if (n <= 0 || nvars <= 0) return 0;
  Carver c(nullptr, 0);
  c.take<double>(size_t(n));
  c.take<double>(size_t(n / kChunkRows + nvars + 1));
  return c.used;
}

extern "C" int dopinf_preprocess(void* stream, int dtype, void* Q, int64_t n, int64_t k, int64_t ldq,
                                 int nvars, const int64_t* var_rows_h, unsigned flags, double* mean,
                                 double* scale, int* zero_range, int* info, void* ws, size_t ws_bytes) {
  DOPINF_REQUIRE_WS_ALIGNED(ws);
  DOPINF_REQUIRE(dtype == DOPINF_F64 || dtype == DOPINF_F32, "dtype must be DOPINF_F64 or DOPINF_F32");
  DOPINF_REQUIRE(Q && mean && scale, "Q, mean and scale must be non-NULL");
  DOPINF_REQUIRE(n >= 1 && k >= 1 && ldq >= k, "need n >= 1, k >= 1, ldq >= k");
  DOPINF_REQUIRE((flags & ~7u) == 0, "unknown flag bits");
  int rc = check_var_rows(n, nvars, var_rows_h);
  if (rc) return rc;
  const size_t need = dopinf_preprocess_workspace(n, k, nvars);
  if (!ws || ws_bytes < need)
    return fail(DOPINF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Carver c(ws, ws_bytes);
  double* rowmax = c.take<double>(size_t(n));
  double* part = c.take<double>(size_t(n / kChunkRows + nvars + 1));
  VarRanges vr = make_ranges(nvars, var_rows_h);
  const int center = (flags & DOPINF_CENTER) ? 1 : 0;
  if (info) {
    set_info_kernel<<<1, 64, 0, st>>>(info);
    DOPINF_LAUNCHED();
  }
  if (dtype == DOPINF_F64)
    launch_row_stats(st, static_cast<const double*>(Q), n, k, ldq, center, mean, rowmax);
  else
    launch_row_stats(st, static_cast<const float*>(Q), n, k, ldq, center, mean, rowmax);
  DOPINF_LAUNCHED();
  var_max_partial_kernel<<<vr.chunk0[nvars], 256, 0, st>>>(rowmax, vr, part);
  DOPINF_LAUNCHED();
  var_max_final_kernel<<<nvars, 64, 0, st>>>(part, vr, (flags & DOPINF_SCALE) ? 1 : 0, scale, zero_range, info);
  DOPINF_LAUNCHED();
  if (flags & DOPINF_APPLY) {
    dim3 grid(unsigned((n + kRowsPerBlock - 1) / kRowsPerBlock));
    if (dtype == DOPINF_F64)
      apply_kernel<double><<<grid, 256, 0, st>>>(static_cast<double*>(Q), n, k, ldq, mean, scale, vr);
    else
      apply_kernel<float><<<grid, 256, 0, st>>>(static_cast<float*>(Q), n, k, ldq, mean, scale, vr);
    DOPINF_LAUNCHED();
  }
  return DOPINF_OK;
}

extern "C" int dopinf_lift(void* stream, const double* Q, int64_t n_cells, int64_t k, int64_t ldq, int nvars_in,
                           int n_out, const int* spec_h, double* L, int64_t ldl) {
  DOPINF_REQUIRE(Q && L && spec_h, "Q, L and spec_h must be non-NULL");
  DOPINF_REQUIRE(n_cells >= 1 && k >= 1 && ldq >= k && ldl >= k, "need n_cells, k >= 1, ldq >= k, ldl >= k");
  DOPINF_REQUIRE(nvars_in >= 1 && n_out >= 1 && n_out <= DOPINF_MAX_VARS,
                 "need nvars_in >= 1 and 1 <= n_out <= %d", DOPINF_MAX_VARS);
  LiftSpec sp{};
  sp.n_out = n_out;
  for (int j = 0; j < n_out; ++j) {
    const int op = spec_h[3 * j], a = spec_h[3 * j + 1], b = spec_h[3 * j + 2];
    DOPINF_REQUIRE(op == DOPINF_LIFT_COPY || op == DOPINF_LIFT_PRODUCT || op == DOPINF_LIFT_RECIPROCAL,
                   "lifting output %d: unknown op %d", j, op);
    DOPINF_REQUIRE(a >= 0 && a < nvars_in, "lifting output %d: variable %d outside [0, %d)", j, a, nvars_in);
    DOPINF_REQUIRE(op != DOPINF_LIFT_PRODUCT || (b >= 0 && b < nvars_in),
                   "lifting output %d: variable %d outside [0, %d)", j, b, nvars_in);
    sp.op[j] = op;
    sp.a[j] = a;
    sp.b[j] = (op == DOPINF_LIFT_PRODUCT) ? b : a;
  }
  const int64_t rows = int64_t(n_out) * n_cells;
  hipStream_t st = static_cast<hipStream_t>(stream);
  lift_kernel<<<unsigned((rows + kRowsPerBlock - 1) / kRowsPerBlock), 256, 0, st>>>(Q, n_cells, k, ldq, sp, L, ldl);
  DOPINF_LAUNCHED();
  return DOPINF_OK;
}
