// Reduced-precision forms of the Step III Gram matrix (arXiv:2504.14338,
// Eq. (5)) for float32-stored snapshots:
//  * FP32:   v_mfma_f32_16x16x4_f32 on the transformed float32 values.
//  * BF16X3: x = hi + lo with hi = bf16_rn(x), lo = bf16_rn(x - hi);
//            D ~ H^T H + H^T L + L^T H (three v_mfma_f32_16x16x32_bf16).
//  * BF16X6: x = hi + mid + lo (three-way split); six products
//            hh + hm + mh + mm + hl + lh, accurate to about float32.
//  (Split methods of Henry, Tang and Heinecke, ARITH 2019.)
//
// Two passes:
//  1. pack: one HBM-bound pass applies centering and scaling (in float64,
//     then rounded), splits into bfloat16 parts where needed, and writes the
//     parts in a K-blocked layout [row block of 32][column][32 rows], zero
//     padded.  Every later load of an element (about k/128 times) is then a
//     plain copy instead of a transform.
//  2. MFMA: 128 x 128 lower-triangle tiles, split-K over row blocks, 4 waves x
//     (4 x 4 blocks of 16 x 16), one 32-row block per LDS stage copied from
//     the packed layout (contiguous 128 x 32 chunks), double buffered;
//     float32 accumulation over slabs of 512 rows, slabs added into float64
//     accumulators; split partials summed in float64 by the shared kernel.
#include "common.hpp"
#include "gram_plan.hpp"

namespace dopinf {
int gram_reduce_launch(hipStream_t st, const double* part, int nsplit, int ntiles, int tiles_y, int triangle,
                       int64_t mx, int64_t my, double* C, int64_t ldc);

namespace {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int BT = 128;
constexpr int NTH = 256;
constexpr int KB = 32;           // rows per packed block = rows per LDS stage
constexpr int SLAB_STAGES = 16;  // 512 rows accumulated in float32 before the float64 add
constexpr int LDC16 = KB + 8;    // LDS column stride (bf16 elements): 80 bytes
constexpr int LDC32 = KB + 4;    // LDS column stride (floats): 144 bytes

__device__ __forceinline__ unsigned short bf16_rn_bits(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<unsigned short>((u >> 16) | 0x40);
  const unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short b) { return __uint_as_float(unsigned(b) << 16); }

struct PackArgs {
  const float* Q;
  int64_t ldq, n, k, kp;  // kp: padded column count (multiple of BT)
  const double* mean;
  const double* scale;
  int nvars;
  int64_t row0[DOPINF_MAX_VARS + 1];
  int algo;               // 0 FP32, 1 BF16X3, 2 BF16X6
  float* pf;              // FP32 part
  unsigned short* p0;     // hi
  unsigned short* p1;     // lo (x3) / mid (x6)
  unsigned short* p2;     // lo (x6)
};

// One workgroup packs a 32-row block x 128 columns: reads rows (coalesced),
// transposes through LDS, writes [col][32] chunks (coalesced).
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
  __shared__ float tile[KB][BT + 1];
  const int64_t blk = blockIdx.x;
  const int64_t c0 = int64_t(blockIdx.y) * BT;
  const int tid = threadIdx.x;
  for (int e = tid; e < KB * BT; e += 256) {
    const int rr = e / BT, cc = e % BT;
    const int64_t row = blk * KB + rr, col = c0 + cc;
    float v = 0.f;
    if (row < a.n && col < a.k) {
      int vv = 0;
      while (vv + 1 < a.nvars && row >= a.row0[vv + 1]) ++vv;
      const double mu = a.mean ? a.mean[row] : 0.0;
      const double inv = a.scale ? 1.0 / a.scale[vv] : 1.0;
      v = static_cast<float>((static_cast<double>(a.Q[row * a.ldq + col]) - mu) * inv);
    }
    tile[rr][cc] = v;
  }
  __syncthreads();
  // output element (col cc, row rr) at ((blk * kp + c0 + cc) * 32 + rr)
  for (int e = tid; e < KB * BT; e += 256) {
    const int cc = e / KB, rr = e % KB;
    const float x = tile[rr][cc];
    const size_t o = (size_t(blk) * a.kp + c0 + cc) * KB + rr;
    if (a.algo == 0) {
      a.pf[o] = x;
    } else {
      const unsigned short h = bf16_rn_bits(x);
      const float r1 = x - bf16_to_f(h);
      const unsigned short m = bf16_rn_bits(r1);
      a.p0[o] = h;
      a.p1[o] = m;
      if (a.algo == 2) a.p2[o] = bf16_rn_bits(r1 - bf16_to_f(m));
    }
  }
}

struct MmaArgs {
  int64_t nb;     // row blocks
  int64_t kp;
  int ntiles, nsplit, xcd_map;
  int64_t blocks_per_split;
  const float* pf;
  const unsigned short* p0;
  const unsigned short* p1;
  const unsigned short* p2;
  double* part;
};

// f32 16x16 MFMA output layout: lane l, element e -> row 4 (l / 16) + e, column l % 16
__device__ __forceinline__ int out_row(int lane, int e) { return 4 * (lane >> 4) + e; }

template <int ALGO>
__global__ __launch_bounds__(NTH, 1) void gram_packed_kernel(MmaArgs g) {
  constexpr int NPART = ALGO == 0 ? 1 : (ALGO == 1 ? 2 : 3);
  constexpr size_t F32_STAGE = size_t(2) * BT * LDC32 * sizeof(float);              // A and B panels
  constexpr size_t B16_STAGE = size_t(2) * NPART * BT * LDC16 * sizeof(unsigned short);
  constexpr size_t STAGE = ALGO == 0 ? F32_STAGE : B16_STAGE;
  __shared__ __attribute__((aligned(16))) unsigned char smem[2 * STAGE];

  int t, s;
  {
    const int bid = blockIdx.x;
    if (g.xcd_map) {
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
  const int64_t b_lo = int64_t(s) * g.blocks_per_split;
  const int64_t b_hi = min(g.nb, b_lo + g.blocks_per_split);
  const int64_t nst = b_hi > b_lo ? b_hi - b_lo : 0;
  const int64_t a0 = int64_t(I) * BT, c0 = int64_t(J) * BT;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;

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

  // staging: each panel part is a contiguous chunk of 128 columns x 32 rows;
  // thread -> (column tid / 2, half of the 32 rows) = 16 bytes per bf16 part
  // load (or 64 bytes per float32 part)
  uint4 ra[NPART][4], rb[NPART][4];  // FP32: 4 x 16 B per panel; bf16: 2 x 16 B per part
  const int scol = tid >> 1;          // 0..127
  const int shalf = tid & 1;          // rows 0..15 or 16..31
  auto fetch = [&](int64_t st) {
    const int64_t blk = b_lo + st;
#pragma unroll
    for (int q = 0; q < NPART; ++q) {
      if constexpr (ALGO == 0) {
        const float* base = g.pf + (size_t(blk) * g.kp) * KB;
        const uint4* pa = reinterpret_cast<const uint4*>(base + (a0 + scol) * KB + shalf * 16);
        const uint4* pb = reinterpret_cast<const uint4*>(base + (c0 + scol) * KB + shalf * 16);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ra[q][u] = pa[u];
          rb[q][u] = pb[u];
        }
      } else {
        const unsigned short* P = q == 0 ? g.p0 : (q == 1 ? g.p1 : g.p2);
        const unsigned short* base = P + (size_t(blk) * g.kp) * KB;
        ra[q][0] = *reinterpret_cast<const uint4*>(base + (a0 + scol) * KB + shalf * 8);
        ra[q][1] = *reinterpret_cast<const uint4*>(base + (a0 + scol) * KB + 16 + shalf * 8);
        rb[q][0] = *reinterpret_cast<const uint4*>(base + (c0 + scol) * KB + shalf * 8);
        rb[q][1] = *reinterpret_cast<const uint4*>(base + (c0 + scol) * KB + 16 + shalf * 8);
      }
    }
  };
  auto stash = [&](int buf) {
    unsigned char* S = smem + size_t(buf) * STAGE;
    if constexpr (ALGO == 0) {
      float* A = reinterpret_cast<float*>(S);
      float* B = A + BT * LDC32;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        *reinterpret_cast<uint4*>(A + scol * LDC32 + shalf * 16 + 4 * u) = ra[0][u];
        *reinterpret_cast<uint4*>(B + scol * LDC32 + shalf * 16 + 4 * u) = rb[0][u];
      }
    } else {
      unsigned short* base = reinterpret_cast<unsigned short*>(S);
#pragma unroll
      for (int q = 0; q < NPART; ++q) {
        unsigned short* A = base + size_t(q) * BT * LDC16;
        unsigned short* B = base + size_t(NPART + q) * BT * LDC16;
        *reinterpret_cast<uint4*>(A + scol * LDC16 + shalf * 8) = ra[q][0];
        *reinterpret_cast<uint4*>(A + scol * LDC16 + 16 + shalf * 8) = ra[q][1];
        *reinterpret_cast<uint4*>(B + scol * LDC16 + shalf * 8) = rb[q][0];
        *reinterpret_cast<uint4*>(B + scol * LDC16 + 16 + shalf * 8) = rb[q][1];
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
    const unsigned char* S = smem + size_t(buf) * STAGE;
    const int cm = lane & 15;
    if constexpr (ALGO == 0) {
      const float* A = reinterpret_cast<const float*>(S);
      const float* B = A + BT * LDC32;
#pragma unroll
      for (int kk = 0; kk < KB / 4; ++kk) {
        const int krow = kk * 4 + (lane >> 4);
        float af[4], bf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = A[(wm * 64 + i * 16 + cm) * LDC32 + krow];
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = B[(wn * 64 + j * 16 + cm) * LDC32 + krow];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    } else {
      const unsigned short* base = reinterpret_cast<const unsigned short*>(S);
      const int kq = (lane >> 4) * 8;
      bf16x8 a[NPART][4], b[NPART][4];
#pragma unroll
      for (int q = 0; q < NPART; ++q) {
        const unsigned short* A = base + size_t(q) * BT * LDC16;
        const unsigned short* B = base + size_t(NPART + q) * BT * LDC16;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          a[q][i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(A + (wm * 64 + i * 16 + cm) * LDC16 + kq));
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[q][j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const us8*>(B + (wn * 64 + j * 16 + cm) * LDC16 + kq));
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // smallest products first
          if constexpr (ALGO == 2) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], acc[i][j], 0, 0, 0);
          }
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
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

int tiles_of(int64_t m) { return int((m + BT - 1) / BT); }
int nparts(int algo) { return algo == DOPINF_GRAM_NATIVE ? 1 : (algo == DOPINF_GRAM_BF16X3 ? 2 : 3); }
size_t part_elt(int algo) { return algo == DOPINF_GRAM_NATIVE ? 4 : 2; }

struct LowpPlan {
  int64_t nb, kp;
  int T, ntiles, nsplit;
  int64_t bps;
  size_t pack_bytes, part_bytes;
};

LowpPlan plan(int algo, int64_t n, int64_t k) {
  LowpPlan p{};
  p.nb = (n + KB - 1) / KB;
  p.T = tiles_of(k);
  p.kp = int64_t(p.T) * BT;
  p.ntiles = p.T * (p.T + 1) / 2;
  int target = gramplan::choose_splits(n, p.ntiles);
  if (target < 1) target = 1;
  p.bps = (p.nb + target - 1) / target;
  p.nsplit = int((p.nb + p.bps - 1) / p.bps);
  p.pack_bytes = round_up(size_t(p.nb) * p.kp * KB * part_elt(algo), 256) * nparts(algo);
  p.part_bytes = size_t(p.nsplit) * p.ntiles * BT * BT * sizeof(double);
  return p;
}

}  // namespace
}  // namespace dopinf

using namespace dopinf;

size_t gram_lowp_workspace(int algo, int64_t n, int64_t k) {
  const LowpPlan p = plan(algo, n, k);
  return p.pack_bytes + p.part_bytes + 256;
}

int gram_lowp(hipStream_t st, int algo, const float* Q, int64_t n, int64_t k, int64_t ldq, const double* mean,
              const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd, void* ws,
              size_t ws_bytes) {
  const LowpPlan p = plan(algo, n, k);
  const size_t need = p.pack_bytes + p.part_bytes;
  if (!ws || ws_bytes < need)
    return fail(DOPINF_E_WORKSPACE, "gram workspace of %zu bytes needed, %zu given", need, ws_bytes);
  char* base = static_cast<char*>(ws);
  const size_t one = p.pack_bytes / nparts(algo);
  PackArgs pa{};
  pa.Q = Q;
  pa.ldq = ldq;
  pa.n = n;
  pa.k = k;
  pa.kp = p.kp;
  pa.mean = mean;
  pa.scale = scale;
  pa.algo = algo;
  if (var_rows_h && nvars >= 1) {
    pa.nvars = nvars;
    for (int v = 0; v <= nvars; ++v) pa.row0[v] = var_rows_h[v];
  } else {
    pa.nvars = 1;
    pa.row0[0] = 0;
    pa.row0[1] = n;
  }
  pa.pf = reinterpret_cast<float*>(base);
  pa.p0 = reinterpret_cast<unsigned short*>(base);
  pa.p1 = reinterpret_cast<unsigned short*>(base + one);
  pa.p2 = reinterpret_cast<unsigned short*>(base + 2 * one);
  pack_kernel<<<dim3(unsigned(p.nb), unsigned(p.T)), 256, 0, st>>>(pa);
  DOPINF_LAUNCHED();
  MmaArgs g{};
  g.nb = p.nb;
  g.kp = p.kp;
  g.ntiles = p.ntiles;
  g.nsplit = p.nsplit;
  g.xcd_map = (p.nsplit % 8 == 0) ? 1 : 0;
  g.blocks_per_split = p.bps;
  g.pf = pa.pf;
  g.p0 = pa.p0;
  g.p1 = pa.p1;
  g.p2 = pa.p2;
  g.part = reinterpret_cast<double*>(base + p.pack_bytes);
  dim3 grid(unsigned(p.nsplit) * unsigned(p.ntiles));
  if (algo == DOPINF_GRAM_NATIVE)
    gram_packed_kernel<0><<<grid, NTH, 0, st>>>(g);
  else if (algo == DOPINF_GRAM_BF16X3)
    gram_packed_kernel<1><<<grid, NTH, 0, st>>>(g);
  else
    gram_packed_kernel<2><<<grid, NTH, 0, st>>>(g);
  DOPINF_LAUNCHED();
  return gram_reduce_launch(st, g.part, p.nsplit, p.ntiles, p.T, 1, k, k, D, ldd);
}
