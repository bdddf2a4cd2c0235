// Int8 fixed-point form of the Step III Gram matrix (arXiv:2504.14338,
// Eq. (5)) for float32-stored snapshots: DOPINF_GRAM_I8X6.
//
// Each transformed value x = (q - mean) / scale of column j is scaled by
// 127 / a_j, where a_j = max_i |x_ij| is the column's max-abs, and written as
// three signed int8 slices in radix 254 (round to nearest at every step):
//   x 127 / a_j = t1 + t2 / 254 + t3 / 254^2 + d,   |t_s| <= 127,
//   |d| <= 0.5 / 254^2.
// The Gram keeps the six slice products whose radix weight is at most
// 254^-2 and sums them per weight ("level") in int32 on
// v_mfma_i32_16x16x64_i8:
//   L0 = T1^T T1,  L1 = T1^T T2 + T2^T T1,  L2 = T1^T T3 + T2^T T2 + T3^T T1,
//   D_jl ~ a_j a_l / 127^2 (L0 + (L1 + L2 / 254) / 254).
// Integer products and sums are exact: a row adds at most 3 x 127^2 to a
// level, so a split of at most MAXB x 64 rows stays below 2^31.  The only
// rounding is the splitting (the dropped products and d: at most ~3.9e-3 in
// units of (127 / a)^2 per product, i.e. |dD_jl| <= 2.5e-7 a_j a_l per row)
// and the final float64 combination.  The splitting of a product into
// limbs of fixed-point integers and exact integer matrix products follows
// the scheme of Ozaki, Ogita, Oishi and Rump (Numer. Algorithms 2012) as used
// for integer matrix engines by Ootomo, Ozaki and Yokota (IJHPCA 2024).
//
// Three passes:
//  1. colmax: a_j over all rows (float64 transform, bit-pattern atomic max;
//     a non-finite value makes a_j NaN, so that D's row and column j are NaN);
//  2. pack: the three slices in a K-blocked layout [row block of 64][column]
//     [64 rows], the four 16-byte slots of a column XORed with column bits 2-3
//     (the bfloat16 layout of the FP32/BF16 forms with one-byte elements:
//     sixteen consecutive columns reading one logical slot hit sixteen
//     different bank groups);
//  3. MFMA: 256 x 128 tiles covering the lower triangle, split-K over row
//     blocks, 8 waves (two per SIMD) x (4 x 4 blocks of 16 x 16) x 3 levels
//     of int32 accumulators; a row block of a panel is one contiguous chunk
//     per slice (16 KB for the 256 columns, 8 KB for the 128) brought into LDS
//     by LDS-DMA, double buffered; the split's float64 partial is formed once
//     at the end and the splits are summed in float64 by the shared
//     reduction.
#include "common.hpp"

namespace dopinf {
int gram_reduce_launch(hipStream_t st, const double* part, int nsplit, int ntiles, int tiles_y, int triangle,
                       int64_t mx, int64_t my, double* C, int64_t ldc);

namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int IT = 128;          // output tile edge
constexpr int IK = 64;           // rows per packed block = K of one MFMA = rows per LDS stage
constexpr int NSL = 3;           // slices
constexpr int MAXB = 640;        // row blocks per split: 3 x 127^2 x 640 x 64 < 2^31
constexpr int NTH = 256;
constexpr double TOP = 127.0;    // bound of the first slice
constexpr double RADIX = 254.0;  // weight ratio of consecutive slices

struct XArgs {
  const float* Q;
  int64_t ldq, n, k;
  const double* mean;   // per row (NULL: none)
  const double* scale;  // per variable (NULL: none)
  int nvars;
  int64_t row0[DOPINF_MAX_VARS + 1];
};

__device__ __forceinline__ double rinv_of(const XArgs& a, int v) { return a.scale ? 1.0 / a.scale[v] : 1.0; }

typedef float flt4 __attribute__((ext_vector_type(4)));

// Values of row r at columns c .. c + CPT - 1: one 16-byte load when VEC
// (Q 16-byte aligned, ldq a multiple of 4) and the columns lie inside k,
// else one load per column inside k (0 past it).
template <bool VEC, int CPT>
__device__ __forceinline__ void load_cols(const XArgs& a, int64_t r, int64_t c, float (&q)[CPT]) {
  const float* row = a.Q + r * a.ldq + c;
  if (VEC && CPT == 4 && c + 4 <= a.k) {
    const flt4 v = *reinterpret_cast<const flt4*>(row);
#pragma unroll
    for (int e = 0; e < CPT; ++e) q[e] = v[e];
  } else {
#pragma unroll
    for (int e = 0; e < CPT; ++e) q[e] = c + e < a.k ? row[e] : 0.f;
  }
}

// a_j = max_i |x_ij| over the workgroup's rows, folded into amax (the bit
// patterns of non-negative doubles order like the values; NaN above all).
// Thread -> CPT consecutive columns; 8 rows' loads in flight together.
template <bool VEC>
__global__ __launch_bounds__(NTH) void colmax_kernel(XArgs a, int64_t rows_per_wg,
                                                     unsigned long long* __restrict__ amax) {
  constexpr int CPT = VEC ? 4 : 1;
  const int64_t c = (int64_t(blockIdx.x) * NTH + threadIdx.x) * CPT;
  const int64_t r0 = int64_t(blockIdx.y) * rows_per_wg;
  const int64_t r1 = min(a.n, r0 + rows_per_wg);
  if (c >= a.k || r0 >= r1) return;
  int v = 0;
  while (v + 1 < a.nvars && r0 >= a.row0[v + 1]) ++v;
  double rinv = rinv_of(a, v);
  double m[CPT];
  bool bad[CPT];
#pragma unroll
  for (int e = 0; e < CPT; ++e) {
    m[e] = 0.0;
    bad[e] = false;
  }
  for (int64_t rb = r0; rb < r1; rb += 8) {
    float q[8][CPT];
#pragma unroll
    for (int u = 0; u < 8; ++u) load_cols<VEC, CPT>(a, rb + u < r1 ? rb + u : rb, c, q[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t r = rb + u;
      if (r >= r1) break;
      if (r >= a.row0[v + 1] && v + 1 < a.nvars) {
        while (v + 1 < a.nvars && r >= a.row0[v + 1]) ++v;
        rinv = rinv_of(a, v);
      }
      const double mu = a.mean ? a.mean[r] : 0.0;
#pragma unroll
      for (int e = 0; e < CPT; ++e) {
        const double x = fabs((static_cast<double>(q[u][e]) - mu) * rinv);
        bad[e] |= !(x <= 1.7976931348623157e308);
        m[e] = x > m[e] ? x : m[e];
      }
    }
  }
#pragma unroll
  for (int e = 0; e < CPT; ++e)
    if (c + e < a.k)
      atomicMax(amax + c + e,
                bad[e] ? 0x7ff8000000000000ull : static_cast<unsigned long long>(__double_as_longlong(m[e])));
}

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Three slices of xs in [-127, 127]: xs = t1 + t2 / 254 + t3 / 254^2 + d.
__device__ __forceinline__ void split3(double xs, int& t1, int& t2, int& t3) {
  const double a = rint(xs);
  const double e = (xs - a) * RADIX;
  const double b = rint(e);
  const double c = rint((e - b) * RADIX);
  t1 = int(fmin(fmax(a, -TOP), TOP));
  t2 = int(fmin(fmax(b, -TOP), TOP));
  t3 = int(fmin(fmax(c, -TOP), TOP));
}

struct PackArgs {
  XArgs x;
  int64_t kp;             // padded column count (multiple of IT)
  const double* amax;     // kp column max-abs values (0 past k)
  unsigned char* p;       // slice s at p + s * slice_bytes
  int64_t slice_bytes;
};

constexpr int PW = IK / 4 + 1;  // LDS pitch of a column in 32-bit words (16 + 1: stores conflict at most 2-way)

// One workgroup packs a 64-row block x 128 columns: thread -> columns
// 4 (tid % 32) .. + 3 and the row quads tid / 32 and tid / 32 + 8 (eight
// 16-byte loads in flight when VEC), each column's quad of rows stored as
// one 32-bit word per slice into a column-major LDS tile, then whole 16-byte
// slots written out.
template <bool VEC>
__global__ __launch_bounds__(NTH) void pack_i8_kernel(PackArgs a) {
  __shared__ unsigned t8[NSL][IT][PW];
  __shared__ double rmu[IK], rinv[IK], cs[IT];
  const int64_t blk = blockIdx.x;
  const int64_t c0 = int64_t(blockIdx.y) * IT;
  const int tid = threadIdx.x;
  const XArgs& x = a.x;
  if (tid < IK) {
    const int64_t row = blk * IK + tid;
    const int64_t rowc = row < x.n ? row : x.n - 1;
    int vv = 0;
    while (vv + 1 < x.nvars && rowc >= x.row0[vv + 1]) ++vv;
    rmu[tid] = x.mean ? x.mean[rowc] : 0.0;
    rinv[tid] = rinv_of(x, vv);
  } else if (tid < IK + IT) {
    const double am = a.amax[c0 + tid - IK];
    cs[tid - IK] = (am > 0.0 && am <= 1.7976931348623157e308) ? TOP / am : 0.0;
  }
  const int cq = tid % 32, rq0 = tid / 32;
  float q[2][4][4];  // [row quad][row of the quad][column]
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = blk * IK + 4 * (rq0 + 8 * h) + e;
      load_cols<VEC, 4>(x, row < x.n ? row : x.n - 1, c0 + 4 * cq, q[h][e]);
    }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int rq = rq0 + 8 * h;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int cc = 4 * cq + c;
      const double sc = cs[cc];
      const bool cin = c0 + cc < x.k;
      unsigned w[NSL] = {0u, 0u, 0u};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = 4 * rq + e;
        const bool in = cin && blk * IK + rr < x.n;
        const double xs = in ? (static_cast<double>(q[h][e][c]) - rmu[rr]) * rinv[rr] * sc : 0.0;
        int t[NSL];
        split3(xs, t[0], t[1], t[2]);
#pragma unroll
        for (int sl = 0; sl < NSL; ++sl) w[sl] |= (unsigned(t[sl]) & 0xffu) << (8 * e);
      }
#pragma unroll
      for (int sl = 0; sl < NSL; ++sl) t8[sl][cc][rq] = w[sl];
    }
  }
  __syncthreads();
  // 3 slices x 128 columns x 4 slots
#pragma unroll
  for (int i = 0; i < NSL * IT * 4 / NTH; ++i) {
    const int t = tid + NTH * i, sl = t / (IT * 4), cw = (t / 4) % IT, g = t & 3;
    const u32x4 v = {t8[sl][cw][4 * g], t8[sl][cw][4 * g + 1], t8[sl][cw][4 * g + 2], t8[sl][cw][4 * g + 3]};
    unsigned char* dst =
        a.p + sl * a.slice_bytes + (size_t(blk) * a.kp + c0 + cw) * IK + ((g ^ ((cw >> 2) & 3)) << 4);
    *reinterpret_cast<u32x4*>(dst) = v;
  }
}

struct MmaArgs {
  int64_t nb, kp;
  int T;                       // 128-column tiles of D (the reduction's tile grid)
  int nwide;                   // 256 x 128 tiles per split
  int nsplit, xcd_map;
  int64_t bps;                 // row blocks per split
  const unsigned char* p;      // slices
  int64_t slice_bytes;
  const double* amax;
  double* part;                // per split, the T (T + 1) / 2 lower 128 x 128 tiles
};

// A workgroup of 8 waves computes a 256 x 128 tile: rows [256 I, 256 I + 256)
// (panel A) by columns [128 J, 128 J + 128) (panel B), J <= 2 I + 1, i.e.
// the 128 x 128 tiles (2 I, J) and (2 I + 1, J) of the lower triangle (the
// upper one is skipped when J = 2 I + 1).  Row I holds 2 I + 2 tiles (fewer
// only in the last row when T is odd), so tile t lies in row
// I = floor((sqrt(4 t + 1) - 1) / 2), J = t - I (I + 1).  Wave w computes
// rows 64 (w / 2) .. + 63 and columns 64 (w % 2) .. + 63 of the tile: one wave
// per SIMD pair shares a panel row, and two waves per SIMD hide each other's
// LDS reads.
constexpr int MT = 512;                  // threads per workgroup
constexpr int COLB = IK;                 // bytes of one column of a block (one slice)
constexpr int PA_BYTES = 2 * IT * COLB;  // panel A slice of a block (256 columns)
constexpr int PB_BYTES = IT * COLB;      // panel B slice of a block (128 columns)
constexpr int STAGE = NSL * (PA_BYTES + PB_BYTES);
constexpr int CHUNKS = STAGE / 1024;     // 1 KB LDS-DMA chunks per stage
constexpr int NSTAGE = 2;
static_assert(CHUNKS % (MT / 64) == 0, "chunks per wave");

#define DOPINF_LDS(p) ((__attribute__((address_space(3))) void*)(p))

__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void* p, int nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, nbytes, 0x00020000);
}

// Wait until at most N of this wave's vector-memory operations are in flight.
template <int N>
__device__ __forceinline__ void wait_vmem() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

__device__ __forceinline__ void barrier_only() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// i32 16x16 MFMA output layout: lane l, element e -> row 4 (l / 16) + e, column l % 16
__device__ __forceinline__ int out_row(int lane, int e) { return 4 * (lane >> 4) + e; }

__global__ __launch_bounds__(MT, 1) void gram_i8_kernel(MmaArgs g) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[NSTAGE * STAGE];
  int t, s;
  {
    const int bid = blockIdx.x;
    if (g.xcd_map) {  // each XCD walks its own splits, all tiles of a split together
      const int xcd = bid & 7, local = bid >> 3;
      s = (local / g.nwide) * 8 + xcd;
      t = local % g.nwide;
    } else {
      s = bid / g.nwide;
      t = bid % g.nwide;
    }
  }
  int I = int((sqrt(4.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) <= t) ++I;
  while (I * (I + 1) > t) --I;
  const int J = t - I * (I + 1);
  const int64_t b_lo = int64_t(s) * g.bps;
  const int64_t b_hi = min(g.nb, b_lo + g.bps);
  const int64_t nst = b_hi > b_lo ? b_hi - b_lo : 0;
  const int64_t a0 = int64_t(I) * 2 * IT, c0 = int64_t(J) * IT;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int wm = w >> 1, wn = w & 1;
  // the 128 x 128 tile of D this wave's quadrant belongs to
  const int sub = 2 * I + (wm >> 1);
  const bool live = sub < g.T && J <= sub;
  const uint32_t voff = uint32_t(lane) * 16;
  // stage layout: A slices (16 chunks each), then B slices (8 chunks each);
  // wave w issues chunks w, w + 8, ...
  auto issue = [&](int64_t st) {
    unsigned char* S = smem + (st % NSTAGE) * STAGE;
    const size_t blk = size_t(b_lo + st);
#pragma unroll
    for (int t = 0; t < CHUNKS / (MT / 64); ++t) {
      const int q = w + (MT / 64) * t;
      const bool isa = q < NSL * (PA_BYTES / 1024);
      const int qa = isa ? q : q - NSL * (PA_BYTES / 1024);
      const int sl = isa ? qa / (PA_BYTES / 1024) : qa / (PB_BYTES / 1024);
      const int qc = isa ? qa % (PA_BYTES / 1024) : qa % (PB_BYTES / 1024);
      const unsigned char* src =
          g.p + sl * g.slice_bytes + (blk * size_t(g.kp) + size_t(isa ? a0 : c0)) * COLB + qc * 1024;
      const __amdgpu_buffer_rsrc_t rs = span_rsrc(src, 1024);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, DOPINF_LDS(S + q * 1024), 16, voff, 0, 0, 0);
    }
  };
  i32x4 acc[3][4][4];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[l][i][j] = i32x4{0, 0, 0, 0};
  const int cm = lane & 15, gq = lane >> 4;
  const int o = 16 * (gq ^ ((cm >> 2) & 3));
  if (nst > 0) issue(0);
  for (int64_t st = 0; st < nst; ++st) {
    wait_vmem<0>();
    barrier_only();
    // the other buffer was read in iteration st - 1, which every wave has left
    if (st + 1 < nst) issue(st + 1);
    if (!live) continue;  // wave-uniform: the quadrant lies above the diagonal or past k
    const unsigned char* SA = smem + (st % NSTAGE) * STAGE;
    const unsigned char* SB = SA + NSL * PA_BYTES;
    i32x4 fa[NSL][4], fb[NSL][4];
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        fa[sl][i] = *reinterpret_cast<const i32x4*>(SA + sl * PA_BYTES + (wm * 64 + i * 16 + cm) * COLB + o);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        fb[sl][j] = *reinterpret_cast<const i32x4*>(SB + sl * PB_BYTES + (wn * 64 + j * 16 + cm) * COLB + o);
    }
    // products in the outer loop: 16 independent blocks lie between two
    // products into one accumulator
    constexpr int PA[6] = {0, 0, 1, 0, 1, 2}, PB[6] = {0, 1, 0, 2, 1, 0}, LV[6] = {0, 1, 1, 2, 2, 2};
#pragma unroll
    for (int pr = 0; pr < 6; ++pr)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[LV[pr]][i][j] =
              __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[PA[pr]][i], fb[PB[pr]][j], acc[LV[pr]][i][j], 0, 0, 0);
  }
  if (!live) return;
  const int ntiles = g.T * (g.T + 1) / 2;
  double* out = g.part + (size_t(s) * ntiles + size_t(sub) * (sub + 1) / 2 + J) * (IT * IT);
  const int r0 = (wm & 1) * 64;  // rows of the quadrant within its 128 x 128 tile
  constexpr double INV = 1.0 / (TOP * TOP);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int cc = wn * 64 + j * 16 + (lane & 15);
    const double ac = g.amax[c0 + cc] * INV;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = r0 + i * 16 + out_row(lane, e);
        const double v = (static_cast<double>(acc[2][i][j][e]) / RADIX + static_cast<double>(acc[1][i][j][e])) / RADIX +
                         static_cast<double>(acc[0][i][j][e]);
        out[rr * IT + cc] = v * (g.amax[int64_t(sub) * IT + rr] * ac);
      }
  }
}

struct I8Plan {
  int64_t nb, kp;
  int T, T2, ntiles, nwide, nsplit;
  int64_t bps;
  size_t slice_bytes, amax_bytes, part_bytes;
};

I8Plan plan(int64_t n, int64_t k) {
  I8Plan p{};
  p.nb = (n + IK - 1) / IK;
  p.T = int((k + IT - 1) / IT);
  p.T2 = (p.T + 1) / 2;
  p.kp = int64_t(p.T2) * 2 * IT;
  p.ntiles = p.T * (p.T + 1) / 2;
  p.nwide = p.T2 * (p.T2 + 1) - (p.T % 2);
  // about 8192 workgroups, at least nb / MAXB splits (exact int32 sums), a
  // multiple of 8 (XCD map) and, where it costs at most a quarter more, whole
  // rounds of the resident workgroups (one per CU: 144 KB of LDS)
  int ncu = 0;
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 0;
  }
  int64_t target = (8192 + p.nwide - 1) / p.nwide;
  const int64_t need = (p.nb + MAXB - 1) / MAXB;
  if (target < need) target = need;
  if (target > p.nb) target = p.nb;
  if (target >= 8) target = (target + 7) / 8 * 8;
  if (ncu > 0 && target >= 8) {
    int64_t a = p.nwide, b = ncu;
    while (b) {
      const int64_t r = a % b;
      a = b;
      b = r;
    }
    const int64_t step = ncu / a;
    const int64_t up = (target + step - 1) / step * step;
    if (up <= target + target / 4) target = up;
  }
  if (target < 1) target = 1;
  p.bps = (p.nb + target - 1) / target;
  p.nsplit = int((p.nb + p.bps - 1) / p.bps);
  p.slice_bytes = round_up(size_t(p.nb) * p.kp * IK, 256);
  p.amax_bytes = round_up(size_t(p.kp) * sizeof(double), 256);
  p.part_bytes = size_t(p.nsplit) * p.ntiles * IT * IT * sizeof(double);
  return p;
}

}  // namespace

size_t gram_i8_workspace(int64_t n, int64_t k) {
  const I8Plan p = plan(n, k);
  return NSL * p.slice_bytes + p.amax_bytes + p.part_bytes + 256;
}

int gram_i8(hipStream_t st, const float* Q, int64_t n, int64_t k, int64_t ldq, const double* mean,
            const double* scale, int nvars, const int64_t* var_rows_h, double* D, int64_t ldd, void* ws,
            size_t ws_bytes) {
  const I8Plan p = plan(n, k);
  const size_t need = NSL * p.slice_bytes + p.amax_bytes + p.part_bytes;
  if (!ws || ws_bytes < need)
    return fail(DOPINF_E_WORKSPACE, "gram workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (p.bps > MAXB) return fail(DOPINF_E_ARG, "too many rows for the int8 Gram (%lld)", (long long)n);
  char* base = static_cast<char*>(ws);
  unsigned char* slices = reinterpret_cast<unsigned char*>(base);
  unsigned long long* amax = reinterpret_cast<unsigned long long*>(base + NSL * p.slice_bytes);
  double* part = reinterpret_cast<double*>(base + NSL * p.slice_bytes + p.amax_bytes);
  XArgs x{};
  x.Q = Q;
  x.ldq = ldq;
  x.n = n;
  x.k = k;
  x.mean = mean;
  x.scale = scale;
  if (var_rows_h && nvars >= 1) {
    x.nvars = nvars;
    for (int v = 0; v <= nvars; ++v) x.row0[v] = var_rows_h[v];
  } else {
    x.nvars = 1;
    x.row0[0] = 0;
    x.row0[1] = n;
  }
  zero_u64_kernel<<<unsigned((p.kp + 255) / 256), 256, 0, st>>>(amax, p.kp);
  DOPINF_LAUNCHED();
  // 16-byte row loads where every row start is 16-byte aligned
  const bool vec = reinterpret_cast<uintptr_t>(Q) % 16 == 0 && ldq % 4 == 0;
  // about 8 row chunks per CU and column group
  const int64_t col_groups = (k + NTH * (vec ? 4 : 1) - 1) / (NTH * (vec ? 4 : 1));
  int64_t chunks = (2048 + col_groups - 1) / col_groups;
  int64_t rows_per_wg = (n + chunks - 1) / chunks;
  rows_per_wg = (rows_per_wg + 7) / 8 * 8;
  if (rows_per_wg < 64) rows_per_wg = 64;
  chunks = (n + rows_per_wg - 1) / rows_per_wg;
  if (vec)
    colmax_kernel<true><<<dim3(unsigned(col_groups), unsigned(chunks)), NTH, 0, st>>>(x, rows_per_wg, amax);
  else
    colmax_kernel<false><<<dim3(unsigned(col_groups), unsigned(chunks)), NTH, 0, st>>>(x, rows_per_wg, amax);
  DOPINF_LAUNCHED();
  PackArgs pa{};
  pa.x = x;
  pa.kp = p.kp;
  pa.amax = reinterpret_cast<const double*>(amax);
  pa.p = slices;
  pa.slice_bytes = int64_t(p.slice_bytes);
  if (vec)
    pack_i8_kernel<true><<<dim3(unsigned(p.nb), unsigned(p.kp / IT)), NTH, 0, st>>>(pa);
  else
    pack_i8_kernel<false><<<dim3(unsigned(p.nb), unsigned(p.kp / IT)), NTH, 0, st>>>(pa);
  DOPINF_LAUNCHED();
  MmaArgs g{};
  g.nb = p.nb;
  g.kp = p.kp;
  g.T = p.T;
  g.nwide = p.nwide;
  g.nsplit = p.nsplit;
  g.xcd_map = (p.nsplit % 8 == 0) ? 1 : 0;
  g.bps = p.bps;
  g.p = slices;
  g.slice_bytes = int64_t(p.slice_bytes);
  g.amax = pa.amax;
  g.part = part;
  gram_i8_kernel<<<dim3(unsigned(p.nsplit) * unsigned(p.nwide)), MT, 0, st>>>(g);
  DOPINF_LAUNCHED();
  return gram_reduce_launch(st, part, p.nsplit, p.ntiles, p.T, 1, k, k, D, ldd);
}

}  // namespace dopinf
