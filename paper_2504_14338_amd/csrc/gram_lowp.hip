// Reduced-precision forms of the Step III Gram matrix (arXiv:2504.14338,
// Eq. (5)) for float32-stored snapshots:
//  * FP32: v_mfma_f32_16x16x4_f32 on the transformed float32 values.
//  * BF16X3: each transformed value x is split into hi = bf16_rn(x) and
//    lo = bf16_rn(x - hi); D ~ H^T H + H^T L + L^T H (the lo*lo term is
//    dropped), three v_mfma_f32_16x16x32_bf16 per block (split method of
//    Henry, Tang and Heinecke, ARITH 2019, in its three-product form).
// Both accumulate in float32 over slabs of 512 rows and add each slab into
// float64 accumulators; splits are summed in float64 by the shared reduction
// kernel.  Tiling, split-K and XCD-aware ordering follow the float64 kernel;
// the centering / scaling transform is evaluated in float64 on load and then
// rounded to float32 (and split for BF16X3).
#include "common.hpp"
#include "gram_plan.hpp"

namespace dopinf {
int gram_reduce_launch(hipStream_t st, const double* part, int nsplit, int ntiles, int tiles_y, int triangle,
                       int64_t mx, int64_t my, double* C, int64_t ldc);
int check_var_rows(int64_t n, int nvars, const int64_t* var_rows_h);

namespace {

using gramplan::SplitPlan;

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int BT = 128;
constexpr int NTH = 256;
constexpr int KC = 32;           // rows per LDS stage
constexpr int SLAB_STAGES = 16;  // 512 rows accumulated in float32 before the float64 add
constexpr int PADF = 4;          // float32 panel row padding (floats)
constexpr int LDF = BT + PADF;
constexpr int LDB = KC + 8;      // bf16 transposed panel: column-major rows, 80-byte stride

struct LowpArgs {
  const float* Q;
  int64_t ldq;
  int64_t m;
  int ntiles;
  const double* mean;
  const double* scale;
  double* part;
};

// round-to-nearest-even float32 -> bfloat16 bits (NaN kept quiet)
__device__ __forceinline__ unsigned short bf16_rn_bits(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<unsigned short>((u >> 16) | 0x40);
  const unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned short b) { return __uint_as_float(unsigned(b) << 16); }

// f32 16x16 MFMA output layout: lane l, element e -> row 4 (l / 16) + e, column l % 16
__device__ __forceinline__ int out_row(int lane, int e) { return 4 * (lane >> 4) + e; }

template <int ALGO>
__global__ __launch_bounds__(NTH, 1) void gram_lowp_kernel(LowpArgs g, SplitPlan sp) {
  // FP32: two float panels per buffer; BF16X3: hi and lo transposed panels
  constexpr size_t F32_BYTES = size_t(2) * 2 * KC * LDF * sizeof(float);
  constexpr size_t B16_BYTES = size_t(2) * 2 * 2 * BT * LDB * sizeof(unsigned short);
  __shared__ __attribute__((aligned(16))) unsigned char smem[ALGO == 0 ? F32_BYTES : B16_BYTES];

  int t, s;
  {
    const int bid = blockIdx.x;
    if (sp.xcd_map) {
      const int xcd = bid & 7;
      const int local = bid >> 3;
      s = (local / g.ntiles) * 8 + xcd;
      t = local % g.ntiles;
    } else {
      s = bid / g.ntiles;
      t = bid % g.ntiles;
    }
  }
  int I, J;
  gramplan::tri_coords(t, I, J);
  int64_t lo, hi;
  int v;
  gramplan::split_range(sp, s, KC, lo, hi, v);
  const int64_t a0 = int64_t(I) * BT, b0 = int64_t(J) * BT;
  const double inv = g.scale ? 1.0 / g.scale[v] : 1.0;
  const bool vec = ((g.ldq & 3) == 0) && ((reinterpret_cast<uintptr_t>(g.Q) & 15) == 0);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  // staging: thread -> 2 consecutive rows x 8 columns of each panel
  const int srow = (tid >> 4) * 2;   // 0..30
  const int scol = (tid & 15) * 8;   // 0..120

  flt4 acc[4][4];
  double acc64[4][4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < 4; ++e) acc64[i][j][e] = 0.0;
    }

  const int64_t nst = (hi - lo + KC - 1) / KC;
  float xa[2][8], xb[2][8];

  auto load8 = [&](int64_t row, int64_t col0, float (&x)[8]) {
    if (row < hi) {
      const float* p = g.Q + row * g.ldq + col0;
      if (vec && col0 + 8 <= g.m) {
        const float4 u0 = reinterpret_cast<const float4*>(p)[0];
        const float4 u1 = reinterpret_cast<const float4*>(p)[1];
        x[0] = u0.x; x[1] = u0.y; x[2] = u0.z; x[3] = u0.w;
        x[4] = u1.x; x[5] = u1.y; x[6] = u1.z; x[7] = u1.w;
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = (col0 + u < g.m) ? p[u] : 0.f;
      }
      const double mu = g.mean ? g.mean[row] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        x[u] = (col0 + u < g.m) ? static_cast<float>((static_cast<double>(x[u]) - mu) * inv) : 0.f;
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = 0.f;
    }
  };
  auto fetch = [&](int64_t st) {
    const int64_t row = lo + st * KC + srow;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      load8(row + q, a0 + scol, xa[q]);
      load8(row + q, b0 + scol, xb[q]);
    }
  };
  auto stash = [&](int buf) {
    if constexpr (ALGO == 0) {
      float* P = reinterpret_cast<float*>(smem) + size_t(buf) * 2 * KC * LDF;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          P[(srow + q) * LDF + scol + u] = xa[q][u];
          P[KC * LDF + (srow + q) * LDF + scol + u] = xb[q][u];
        }
    } else {
      unsigned short* P = reinterpret_cast<unsigned short*>(smem) + size_t(buf) * 4 * BT * LDB;
      // [panel A hi | A lo | B hi | B lo], each BT x LDB, element (row, col) at col*LDB + row
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        unsigned int ha = 0, la = 0, hb = 0, lb = 0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const unsigned short h1 = bf16_rn_bits(xa[q][u]);
          const unsigned short l1 = bf16_rn_bits(xa[q][u] - bf16_bits_to_float(h1));
          const unsigned short h2 = bf16_rn_bits(xb[q][u]);
          const unsigned short l2 = bf16_rn_bits(xb[q][u] - bf16_bits_to_float(h2));
          ha |= unsigned(h1) << (16 * q);
          la |= unsigned(l1) << (16 * q);
          hb |= unsigned(h2) << (16 * q);
          lb |= unsigned(l2) << (16 * q);
        }
        const int off = (scol + u) * LDB + srow;  // even -> 4-byte aligned
        *reinterpret_cast<unsigned int*>(P + 0 * BT * LDB + off) = ha;
        *reinterpret_cast<unsigned int*>(P + 1 * BT * LDB + off) = la;
        *reinterpret_cast<unsigned int*>(P + 2 * BT * LDB + off) = hb;
        *reinterpret_cast<unsigned int*>(P + 3 * BT * LDB + off) = lb;
      }
    }
  };

  if (nst > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  for (int64_t st = 0; st < nst; ++st) {
    const int buf = int(st & 1);
    if (st + 1 < nst) fetch(st + 1);
    if constexpr (ALGO == 0) {
      const float* A = reinterpret_cast<const float*>(smem) + size_t(buf) * 2 * KC * LDF;
      const float* B = A + KC * LDF;
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
        const int krow = kk * 4 + (lane >> 4);
        const int cm = lane & 15;
        float af[4], bf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = A[krow * LDF + wm * 64 + i * 16 + cm];
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = B[krow * LDF + wn * 64 + j * 16 + cm];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    } else {
      const unsigned short* P = reinterpret_cast<const unsigned short*>(smem) + size_t(buf) * 4 * BT * LDB;
      const int cm = lane & 15;
      const int kq = (lane >> 4) * 8;  // this lane's 8 consecutive rows of the stage
      bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = wm * 64 + i * 16 + cm;
        ah[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(P + 0 * BT * LDB + col * LDB + kq));
        al[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(P + 1 * BT * LDB + col * LDB + kq));
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = wn * 64 + j * 16 + cm;
        bh[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(P + 2 * BT * LDB + col * LDB + kq));
        bl[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(P + 3 * BT * LDB + col * LDB + kq));
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    if (st + 1 < nst) stash(buf ^ 1);
    if ((st + 1) % SLAB_STAGES == 0 || st + 1 == nst) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int e = 0; e < 4; ++e) acc64[i][j][e] += static_cast<double>(acc[i][j][e]);
          acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
        }
    }
    __syncthreads();
  }

  double* out = g.part + (size_t(s) * g.ntiles + t) * (BT * BT);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = wm * 64 + i * 16 + out_row(lane, e);
        const int cc = wn * 64 + j * 16 + (lane & 15);
        out[rr * BT + cc] = acc64[i][j][e];
      }
}

size_t part_bytes(int nsplit, int ntiles) { return size_t(nsplit) * ntiles * BT * BT * sizeof(double); }
int tiles_of(int64_t m) { return int((m + BT - 1) / BT); }

}  // namespace
}  // namespace dopinf

using namespace dopinf;

size_t gram_lowp_workspace(int /*algo*/, int64_t n, int64_t k) {
  const int T = tiles_of(k);
  const int ntiles = T * (T + 1) / 2;
  return part_bytes(gramplan::choose_splits(n, ntiles) + DOPINF_MAX_VARS + 8, ntiles);
}

int gram_lowp(hipStream_t st, int algo, const float* Q, int64_t n, int64_t k, int64_t ldq, const double* mean,
              const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd, void* ws,
              size_t ws_bytes) {
  const int T = tiles_of(k);
  const int ntiles = T * (T + 1) / 2;
  int64_t one_var[2] = {0, n};
  if (!var_rows_h) {
    nvars = 1;
    var_rows_h = one_var;
  }
  SplitPlan sp = gramplan::make_plan(n, nvars, var_rows_h, gramplan::choose_splits(n, ntiles), KC);
  if (!ws || ws_bytes < part_bytes(sp.nsplit, ntiles))
    return fail(DOPINF_E_WORKSPACE, "gram workspace of %zu bytes needed, %zu given", part_bytes(sp.nsplit, ntiles),
                ws_bytes);
  LowpArgs g{};
  g.Q = Q;
  g.ldq = ldq;
  g.m = k;
  g.ntiles = ntiles;
  g.mean = mean;
  g.scale = scale;
  g.part = static_cast<double*>(ws);
  dim3 grid(unsigned(sp.nsplit) * unsigned(ntiles));
  if (algo == DOPINF_GRAM_NATIVE)
    gram_lowp_kernel<0><<<grid, NTH, 0, st>>>(g, sp);
  else
    gram_lowp_kernel<1><<<grid, NTH, 0, st>>>(g, sp);
  DOPINF_LAUNCHED();
  return gram_reduce_launch(st, g.part, sp.nsplit, ntiles, T, 1, k, k, D, ldd);
}
